// Device code of the substructuring Schur-complement solver (gfx950).
//
// Every per-row product is computed by one aligned group of G lanes (the
// whole 64-lane wavefront, or half of it for the interface rows): lane l of
// the group takes the row entries l, l+G, l+2G, ... in order and the G
// partial sums are combined by an xor butterfly.  A row's result therefore
// depends only on the row and on the column of right-hand sides it belongs
// to -- never on how many right-hand sides share the launch, or on the launch
// shape -- which is what makes a request's result identical alone and inside
// a batch.
//
// Dot products are reduced deterministically: fixed row chunks are reduced
// in a fixed order (a wave butterfly over 64 rows, or rows in order), and the
// chunk partials by a fixed two-level tree in the last workgroup to finish
// (no floating-point atomics).
//
// Vectors use the "DD layout": interface vectors are n_gamma x ld and
// interior vectors NI x ld, row-major with the right-hand-side index fastest
// (ld = batch width, a power of two <= 64), so a row's entries for all
// right-hand sides are one contiguous segment.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dd {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kRowsE = 64;    // rows per chunk in the element-wise kernels
constexpr int kMaxLd = 64;    // widest right-hand-side batch

__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
// The same butterfly within aligned groups of G lanes (G a power of two <= 64):
// every lane of a group receives the group's sum.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// ---------------------------------------------------------------- state --
// Per-column CG state, one array of kMaxLd entries per field.
struct ColState {
  double *rz;       // r^T z
  double *alpha;    // step length of the current iteration
  double *beta;     // direction update of the current iteration
  double *stop2;    // (tol * ||b||)^2
  double *nrm2;     // scratch norms
  int *active;      // 1 while the column iterates
  int *iters;       // iterations taken
  int *flag;        // [0]: breakdown (p^T S p <= 0) seen; [1]: iterate (persistent launch);
                    // [2], [3]: residual replacement (below)
  // three-launch iteration: values of iteration k in slot k & 1 (a launch
  // reads the previous iteration's slot while its workgroup 0 writes the
  // current one), and the per-column breakdown marks of the step length
  double *rz2;      // 2 x kMaxLd
  int *act2;        // 2 x kMaxLd
  int *bd;          // kMaxLd
  // split update of the tiled iteration: the state a step started from and
  // its breakdown marks (written by the update, read by the direction launch)
  double *rz_prev;  // kMaxLd
  int *act_prev;    // kMaxLd
  int *brk;         // kMaxLd
  // residual replacement (mixed tiled solve): r.r at the start or at the last
  // replacement; flag[2]: some column is due for the next one (all iterating
  // columns are then replaced together: one FP64 product serves the batch),
  // flag[3]: this step replaced
  double *ref2;     // kMaxLd
};


// Partial-sum buffers and completion counters of the reductions.
struct RedBuf {
  double *part0;       // chunk partials, dot 0  (max_chunks x kMaxLd)
  double *part1;       // chunk partials, dot 1
  double *part2;       // chunk partials of p^T q from the interface-row kernel
  double *part3;       // group sums of part2 (kPGroup chunks per group)
  unsigned *counter;   // last-workgroup counters (one per reduction site)
  unsigned *gcount;    // one completion counter per chunk group (kCounterStride apart)
};

// Two-level reduction of the interface-row chunk partials: groups of kPGroup
// consecutive chunks are summed by the wave butterfly (chunk m of the group
// in lane m; missing chunks of the last group add zeros) into part3 by the
// last workgroup of the group to finish; consumers sum the group values with
// partials_sum.  Per-group counters keep same-address atomics to kPGroup per
// counter instead of one per workgroup of the whole grid.
constexpr int kPGroup = 64;
constexpr int kCounterStride = 32;    // counters 128 bytes apart

// ---------------------------------------------------------------- trees --
// Column partial of a chunk: rows 0..63 of lds (stride ld) reduced by the
// xor butterfly of one wave (a fixed tree, the same for every ld).
__device__ __forceinline__ double chunk64_sum(const double *lds, int ld, int c) {
  return wave_sum(lds[lane_id() * ld + c]);
}

// chunk64_sum of two dots for a whole chunk held in registers: element
// threadIdx.x + k * kBlock of a chunk of width ld = 4 E (E >= 4) is row
// threadIdx.x / ld + (64 / E) k, column threadIdx.x % ld, with a[k] and b[k]
// its terms of the two dots.  The butterfly pairs rows m and m + 32 first,
// then m and m + 16, ..., m and m + 1; the levels of distance 64 / E and more
// pair values of one thread (k and k + h) and are added in registers, the
// rest by one thread per (column, dot) from LDS, in the same pairs, so every
// sum has the bits of chunk64_sum.  The sums go to outa[c] and outb[c] by
// device-coherent stores (not waited for).  lds: 2 kBlock doubles.
template <int E>
__device__ __forceinline__ void chunk64_sums2(double (&a)[E], double (&b)[E], double *lds, double *outa,
                                              double *outb) {
  static_assert(E >= 4 && (E & (E - 1)) == 0, "one chunk of 16 or more columns per workgroup");
  constexpr int LD = 4 * E, R = 64 / E;
#pragma unroll
  for (int h = E / 2; h >= 1; h /= 2)
#pragma unroll
    for (int k = 0; k < h; ++k) {
      a[k] += a[k + h];
      b[k] += b[k + h];
    }
  lds[threadIdx.x] = a[0];
  lds[kBlock + threadIdx.x] = b[0];
  __syncthreads();
  if (threadIdx.x < 2 * LD) {
    const int t = threadIdx.x / LD, c = threadIdx.x % LD;
    const double *s = lds + t * kBlock + c;
    double u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = s[r * LD];
#pragma unroll
    for (int h = R / 2; h >= 1; h /= 2)
#pragma unroll
      for (int r = 0; r < h; ++r) u[r] += u[r + h];
    __hip_atomic_store((t ? outb : outa) + c, u[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Chunk partials cross workgroups (and XCDs, whose L2 caches are not kept
// coherent with each other).  They are written with device-coherent (sc1)
// stores and read with device-coherent loads; the writing thread waits for
// its store to complete (s_waitcnt vmcnt(0)) before the workgroup counts
// itself done.  No L2 write-back or invalidate is needed.
__device__ __forceinline__ void store_partial(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0) expcnt(7) lgkmcnt(15)
}
__device__ __forceinline__ double load_partial(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Final reduction of P chunk partials for column c by one wave: lane t sums
// partials t, t+64, ... in order, then the butterfly.  Fixed for a given P.
// Loads are issued in batches of 8 so they overlap.
__device__ __forceinline__ double partials_sum(const double *part, int P, int ld, int c) {
  double s = 0.0;
  for (int i0 = lane_id(); i0 < P; i0 += 8 * kWave) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int i = i0 + u * kWave;
      v[u] = i < P ? load_partial(part + (size_t)i * ld + c) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  return wave_sum(s);
}

// Two reductions of the same shape at once (their loads overlap).
__device__ __forceinline__ void partials_sum2(const double *pa, const double *pb, int P, int ld,
                                              int c, double &ra, double &rb) {
  double sa = 0.0, sb = 0.0;
  for (int i0 = lane_id(); i0 < P; i0 += 8 * kWave) {
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int i = i0 + u * kWave;
      va[u] = i < P ? load_partial(pa + (size_t)i * ld + c) : 0.0;
      vb[u] = i < P ? load_partial(pb + (size_t)i * ld + c) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sa += va[u];
      sb += vb[u];
    }
  }
  ra = wave_sum(sa);
  rb = wave_sum(sb);
}

// partials_sum / partials_sum2 for NC consecutive columns c0 .. c0+NC-1 at
// once (columns >= c0 + nc read as zero): every column is summed exactly as the
// one-column forms sum it (lane t adds partials t, t+64, ... in increasing order,
// then the butterfly), only the loads of the columns overlap, so wide batches
// pay one memory round trip per batch of kBatch partials instead of one per
// column.
// COH = false: plain loads, for partials written by an earlier launch (a
// kernel boundary makes them visible; plain loads then hit in every XCD's L2
// instead of all workgroups of the launch reading the same few lines from
// memory).
// B: batches of kWave partials whose loads are issued together (registers:
// B * NC doubles; the sums do not depend on B).
template <int NC, bool COH = true, int B = 4>
__device__ __forceinline__ void partials_sum_cols(const double *part, int P, int ld, int c0, int nc,
                                                  double (&out)[NC]) {
  double s[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) s[c] = 0.0;
  for (int i0 = lane_id(); i0 < P; i0 += B * kWave) {
    double v[B][NC];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = i0 + u * kWave;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double *a = part + (size_t)i * ld + c0 + c;
        v[u][c] = (i < P && c < nc) ? (COH ? load_partial(a) : *a) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += v[u][c];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = wave_sum(s[c]);
}

template <int NC, int B = 4>
__device__ __forceinline__ void partials_sum2_cols(const double *pa, const double *pb, int P, int ld,
                                                   int c0, int nc, double (&ra)[NC], double (&rb)[NC]) {
  double sa[NC], sb[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) sa[c] = sb[c] = 0.0;
  for (int i0 = lane_id(); i0 < P; i0 += B * kWave) {
    double va[B][NC], vb[B][NC];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = i0 + u * kWave;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const bool ok = i < P && c < nc;
        va[u][c] = ok ? load_partial(pa + (size_t)i * ld + c0 + c) : 0.0;
        vb[u][c] = ok ? load_partial(pb + (size_t)i * ld + c0 + c) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        sa[c] += va[u][c];
        sb[c] += vb[u][c];
      }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    ra[c] = wave_sum(sa[c]);
    rb[c] = wave_sum(sb[c]);
  }
}

// Last-workgroup election after every workgroup stored its partials (with
// store_partial).  The counter is reset by the elected workgroup.
__device__ __forceinline__ bool last_block(unsigned *counter, int *lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *lds_flag = (prev == gridDim.x - 1);
  }
  __syncthreads();
  return *lds_flag != 0;
}

__device__ __forceinline__ void reset_counter(unsigned *counter) {
  __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last of `members` workgroups to arrive at counter (after storing partials).
__device__ __forceinline__ bool last_of(unsigned *counter, unsigned members, int *lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *lds_flag = (prev == members - 1);
  }
  __syncthreads();
  return *lds_flag != 0;
}

// Group sums (as chunk_group_sum) of every column c < ld, written to
// out[g * ld + c] by device-coherent stores: wave wv of nw takes 8 columns per
// pass, issues all their loads before the butterflies and all stores before a
// single wait for completion (one memory round trip per pass, not one load and
// one store round trip per column).
__device__ __forceinline__ void group_sums_store(const double *part, int P, int ld, int g,
                                                 double *out, int wv, int nw, bool wait = true) {
  constexpr int NC = 8;
  const int m = g * kPGroup + lane_id();
  for (int c0 = wv * NC; c0 < ld; c0 += nw * NC) {
    double v[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u)
      v[u] = (c0 + u < ld && m < P) ? __hip_atomic_load(part + (size_t)m * ld + c0 + u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                    : 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) v[u] = wave_sum(v[u]);
    if (lane_id() == 0)
#pragma unroll
      for (int u = 0; u < NC; ++u)
        if (c0 + u < ld)
          __hip_atomic_store(out + (size_t)g * ld + c0 + u, v[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (wait) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the group sums are stored
}

// Sum of chunk partials g*kPGroup .. g*kPGroup+63 (those < P) of column c.
__device__ __forceinline__ double chunk_group_sum(const double *part, int P, int ld, int c, int g) {
  const int m = g * kPGroup + lane_id();
  double v = m < P ? load_partial(part + (size_t)m * ld + c) : 0.0;
  return wave_sum(v);
}

// ----------------------------------------------------------- row products --
// Source of gathered vector entries, fixed at compile time (OTF):
//   0  a plain vector x;
//   1  the CG direction formed on the fly, z + beta * pp (beta per column);
//   2  the preconditioned residual of the next CG iterate formed on the fly,
//      dinv_j * (x - alpha q) for columns with upd != 0 and dinv_j * x for the
//      others (x = the previous residual, alpha = beta[] per column; dinv
//      nullptr: no preconditioner).
struct Src {
  const double *x;       // plain vector (kind 0); previous residual (kind 2)
  const double *z;       // kind 1: z + beta * pp
  const double *pp;
  const double *beta;    // kind 1: beta; kind 2: step lengths alpha
  const double *q;       // kind 2: S p of the previous iteration
  const double *dinv;    // kind 2: 1 / diagonal of the preconditioner (nullptr: none)
  const int *upd;        // kind 2: 1 if column c takes the step
  const float *x32 = nullptr;   // FP32 copy of x (kind 0), gathered instead of x when given
};

// FP32 copies of the vectors that the FP32-data products of the mixed inner
// solve gather (K_IG z, K_IG D^{-1} q in K1; K_GG p, K_GI w in K3).  Each is
// written next to its FP64 vector by the launch that produces it and read, in
// place of that vector, by the gathers of the next launch: half the gathered
// bytes, with rounding at the level of the FP32 matrix entries.  The Krylov
// vectors, their updates and every dot product stay FP64.  All nullptr: the
// gathers read the FP64 vectors.
struct Gather32 {
  const float *z_old;   // z_{k-1}                (read by K1's rows)
  float *z;             // z_k                    (written by K1's slices)
  const float *qd;      // D^{-1} q_{k-1}         (read by K1's rows)
  float *p;             // p_k                    (written by K2's slices, read by K3)
  float *w;             // w_k                    (written by K2's rows, read by K3)
  float *qd_out;        // D^{-1} q_k             (written by K3)
};

template <int C, bool OTF>
__device__ __forceinline__ void src_load(const Src &s, size_t off, const double (&bt)[C],
                                         double (&out)[C]) {
  if (OTF) {
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = fma(bt[c], s.pp[off + c], s.z[off + c]);
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c) out[c] = s.x[off + c];
  }
}

template <int C, int OTF>
__device__ __forceinline__ void src_beta(const Src &s, int cp, double (&bt)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) bt[c] = OTF ? s.beta[cp + c] : 0.0;
}

// Kind 2 entry of row j.  The residual update and the preconditioner are the
// exact operations the iteration's own update of row j performs, so every
// gathered value equals the stored one bit for bit.  q is loaded for every
// column and ignored where the column takes no step (q may then be stale).
template <int C>
__device__ __forceinline__ void src_load_z(const Src &s, int j, int ld, int cp, const double (&a)[C],
                                           const bool (&up)[C], double (&out)[C]) {
  const size_t off = (size_t)j * ld + cp;
  const double d = s.dinv ? s.dinv[j] : 1.0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double r = s.x[off + c], qv = s.q[off + c];
    const double rn = up[c] ? fma(-a[c], qv, r) : r;
    out[c] = s.dinv ? d * rn : rn;
  }
}

// acc[c] += sum_k val[k] * x[col[k]][cp + c] over the row, lane-strided.
// A row is processed by an aligned group of G lanes (G = 64: the whole wave;
// G = 32: half a wave, two rows per wave).  Lane s of the group visits its
// entries k = b+s, b+s+G, b+s+2G, ... in increasing order.  The loop handles U
// slots per pass with masked loads: a slot past the row end adds
// fma(0, 0, acc) = acc exactly, so the sum is bit-identical to the plain
// strided loop for every U.  The column indices and values of the next pass
// are loaded while the current pass's gathers are in flight, so a pass costs
// about one memory round trip instead of two (PIPE; costs registers).
template <int C> struct Unroll { static constexpr int U = C == 1 ? 8 : (C <= 4 ? 4 : (C <= 8 ? 2 : 1)); };

template <int U, int G, typename VT>
__device__ __forceinline__ void load_slots(int k, int e, const int *__restrict__ col,
                                           const VT *__restrict__ val, double (&v)[U],
                                           int (&cc)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    int idx = k + u * G;
    bool ok = idx < e;
    v[u] = ok ? (double)val[idx] : 0.0;
    cc[u] = ok ? col[idx] : -1;
  }
}

template <int C, typename VT, int OTF, int U = Unroll<C>::U, int G = kWave, bool PIPE = false,
          bool F32 = false>
__device__ __forceinline__ void csr_row_acc(int b, int e, const int *__restrict__ col,
                                            const VT *__restrict__ val, const Src &x, int ld,
                                            int cp, double (&acc)[C]) {
  double bt[C];
  src_beta<C, OTF>(x, cp, bt);
  bool up[C];
#pragma unroll
  for (int c = 0; c < C; ++c) up[c] = OTF == 2 ? x.upd[cp + c] != 0 : false;
  int k = b + (lane_id() & (G - 1));
  double vn[U];
  int cn[U];
  if (PIPE) load_slots<U, G>(k, e, col, val, vn, cn);
  while (k < e) {
    if (!PIPE) load_slots<U, G>(k, e, col, val, vn, cn);
    double v[U];
    double xv[U][C];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = vn[u];
      if (cn[u] >= 0) {
        if constexpr (F32) {               // FP32 copy of a plain vector
          const size_t off = (size_t)cn[u] * ld + cp;
#pragma unroll
          for (int c = 0; c < C; ++c) xv[u][c] = (double)x.x32[off + c];
        } else if constexpr (OTF == 2) src_load_z<C>(x, cn[u], ld, cp, bt, up, xv[u]);
        else src_load<C, OTF != 0>(x, (size_t)cn[u] * ld + cp, bt, xv[u]);
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) xv[u][c] = 0.0;
      }
    }
    k += U * G;
    if (PIPE) load_slots<U, G>(k, e, col, val, vn, cn);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = tfma(v[u], xv[u][c], acc[c]);
  }
}

// Two-part row: entries [b, s) gather from x1 into acc1, entries [s, e) from
// x2 into acc2, in one masked loop (each accumulator sees its entries in
// increasing order; slots of the other part add exact zeros).
template <int C, typename VT, bool OTF1, int U = Unroll<C>::U, int G = kWave, bool PIPE = false,
          bool F32 = false>
__device__ __forceinline__ void csr_row_acc2(int b, int s, int e, const int *__restrict__ col,
                                             const VT *__restrict__ val, const Src &x1,
                                             const Src &x2, int ld, int cp, double (&acc1)[C],
                                             double (&acc2)[C], const float *__restrict__ x1f = nullptr,
                                             const float *__restrict__ x2f = nullptr) {
  double bt1[C], bt2[C];
  src_beta<C, OTF1>(x1, cp, bt1);
  src_beta<C, false>(x2, cp, bt2);
  int k = b + (lane_id() & (G - 1));
  double vn[U];
  int cn[U];
  if (PIPE) load_slots<U, G>(k, e, col, val, vn, cn);
  while (k < e) {
    if (!PIPE) load_slots<U, G>(k, e, col, val, vn, cn);
    double v[U];
    double xv[U][C];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int idx = k + u * G;
      v[u] = vn[u];
      if (cn[u] < 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) xv[u][c] = 0.0;
      } else if constexpr (F32) {         // FP32 copies of plain vectors
        const float *xf = idx < s ? x1f : x2f;
        const size_t off = (size_t)cn[u] * ld + cp;
#pragma unroll
        for (int c = 0; c < C; ++c) xv[u][c] = (double)xf[off + c];
      } else if (idx < s) {
        src_load<C, OTF1>(x1, (size_t)cn[u] * ld + cp, bt1, xv[u]);
      } else {
        src_load<C, false>(x2, (size_t)cn[u] * ld + cp, bt2, xv[u]);
      }
    }
    const int k0 = k;
    k += U * G;
    if (PIPE) load_slots<U, G>(k, e, col, val, vn, cn);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int idx = k0 + u * G;
      double v1 = idx < s ? v[u] : 0.0;
      double v2 = idx < s ? 0.0 : v[u];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        acc1[c] = tfma(v1, xv[u][c], acc1[c]);
        acc2[c] = tfma(v2, xv[u][c], acc2[c]);
      }
    }
  }
}

// Two sums over one row at once (one wave per row, entries in the lane order
// of csr_row_acc): au += val * xs[j] and av += val * qs[j].  SCALED: the
// gathered entries are multiplied by the preconditioner entry d_j = xs.dinv[j]
// (1 without one); WITHV = false: the second sum is skipped.
template <int C, typename VT, bool SCALED, bool WITHV, int U = (Unroll<C>::U + 1) / 2, bool F32 = false>
__device__ __forceinline__ void csr_row_acc_uv(int b, int e, const int *__restrict__ col,
                                               const VT *__restrict__ val, const Src &rs,
                                               const Src &qs, int ld, int cp, double (&au)[C],
                                               double (&av)[C], const float *__restrict__ rs32 = nullptr,
                                               const float *__restrict__ qs32 = nullptr) {
  int k = b + lane_id();
  while (k < e) {
    double v[U];
    int cc[U];
    load_slots<U, kWave>(k, e, col, val, v, cc);
    double xr[U][C], xq[U][C];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (cc[u] >= 0) {
        const size_t off = (size_t)cc[u] * ld + cp;
        const double d = (SCALED && rs.dinv) ? rs.dinv[cc[u]] : 1.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          if constexpr (F32) {             // FP32 copies (never scaled: iterations k >= 1)
            xr[u][c] = (double)rs32[off + c];
            xq[u][c] = WITHV ? (double)qs32[off + c] : 0.0;
          } else {
            xr[u][c] = SCALED ? d * rs.x[off + c] : rs.x[off + c];
            xq[u][c] = WITHV ? qs.x[off + c] : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c) { xr[u][c] = 0.0; xq[u][c] = 0.0; }
      }
    }
    k += U * kWave;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        au[c] = tfma(v[u], xr[u][c], au[c]);
        if (WITHV) av[c] = tfma(v[u], xq[u][c], av[c]);
      }
  }
}

// out = base + sign * A x  for CSR rows (one wave per row).
// Used for y = K_IG p and for the back-substitution right side b_I - K_IG u_G.
// With OTF and dir != nullptr the kernel also stores the direction it forms
// at its gathers, dir = z + beta pp, for the ndir interface rows (a slice per
// workgroup), so later kernels of the iteration gather it as a plain vector.
template <int C, typename VT, bool OTF>
__global__ void __launch_bounds__(kBlock)
k_csr_rows(int nrows, const int *__restrict__ ptr, const int *__restrict__ col,
           const VT *__restrict__ val, Src x, int ld,
           const double *__restrict__ base, double sign, double *__restrict__ out,
           int ndir = 0, double *__restrict__ dir = nullptr) {
  if (OTF && dir) {
    const int per = (ndir + gridDim.x - 1) / gridDim.x;
    const int j0 = blockIdx.x * per;
    const int n = max(0, min(per, ndir - j0)) * ld;
    for (int e = threadIdx.x; e < n; e += kBlock) {
      const size_t o = (size_t)j0 * ld + e;
      const int c = e % ld;
      dir[o] = fma(x.beta[c], x.pp[o], x.z[o]);
    }
  }
  int row = blockIdx.x * kWavesPerBlock + wave_id();
  if (row >= nrows) return;
  int b = ptr[row], e = ptr[row + 1];
  for (int cp = 0; cp < ld; cp += C) {
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    if (!OTF && x.x32) csr_row_acc<C, VT, OTF, Unroll<C>::U, kWave, false, true>(b, e, col, val, x, ld, cp, acc);
    else csr_row_acc<C, VT, OTF>(b, e, col, val, x, ld, cp, acc);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = wave_sum(acc[c]);
    if (lane_id() == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        size_t o = (size_t)row * ld + cp + c;
        out[o] = (base ? base[o] : 0.0) + sign * acc[c];
      }
    }
  }
}

// Dense symmetric interior blocks, one wave per interior row:
// out_I = base + sign * blockdiag(M_k) y_I.  M_k is K_II^k (residual) or
// (K_II^k)^{-1} (interior solve).  Row i of a symmetric column-major block
// is the contiguous column i.  MT: stored type, AT: accumulation type.
template <int C, typename MT, typename AT>
__global__ void __launch_bounds__(kBlock)
k_dense_rows(int nrows, const MT *__restrict__ blocks, const long long *__restrict__ koff,
             const int *__restrict__ ioff, const int *__restrict__ ni,
             const int *__restrict__ rowsub, const double *__restrict__ y, int ld,
             const double *__restrict__ base, double sign, double *__restrict__ out,
             // optional sparse part (interior residual): out -= K_IG u_G
             const int *__restrict__ sptr, const int *__restrict__ scol,
             const double *__restrict__ sval, const double *__restrict__ sx,
             float *__restrict__ out32 = nullptr) {   // FP32 copy of out (gathered later)
  int r = blockIdx.x * kWavesPerBlock + wave_id();
  if (r >= nrows) return;
  int k = rowsub[r];
  int i0 = ioff[k];
  int n = ni[k];
  const MT *row = blocks + koff[k] + (size_t)(r - i0) * n;
  const double *yb = y + (size_t)i0 * ld;
  for (int cp = 0; cp < ld; cp += C) {
    AT acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (AT)0;
    constexpr int U = Unroll<C>::U;
    for (int j = lane_id(); j < n; j += U * kWave) {
      AT a[U];
      double yv[U][C];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int jj = j + u * kWave;
        bool ok = jj < n;
        a[u] = ok ? (AT)row[jj] : (AT)0;
        const double *yr = yb + (size_t)(ok ? jj : 0) * ld + cp;
#pragma unroll
        for (int c = 0; c < C; ++c) yv[u][c] = ok ? yr[c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = tfma(a[u], (AT)yv[u][c], acc[c]);
    }
    double sacc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) sacc[c] = 0.0;
    if (sptr) {
      Src sxs{sx, nullptr, nullptr, nullptr};
      csr_row_acc<C, double, false>(sptr[r], sptr[r + 1], scol, sval, sxs, ld, cp, sacc);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      acc[c] = wave_sum(acc[c]);
      if (sptr) sacc[c] = wave_sum(sacc[c]);
    }
    if (lane_id() == 0) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        size_t o = (size_t)r * ld + cp + c;
        const double ov = (base ? base[o] : 0.0) + sign * ((double)acc[c] + sacc[c]);
        out[o] = ov;
        if (out32) out32[o] = (float)ov;
      }
    }
  }
}

// Interior solve w = blockdiag(K_II^-1) y for wide batches: one wave takes
// kRB consecutive rows of one subdomain (rb_first[b] = first row of block b;
// blocks never cross subdomains) and shares every y load among them.  Each
// lane visits the same entries in the same order as k_dense_rows and the
// partial sums go through the same butterfly, so every entry is bit-identical
// to the one-row-per-wave kernel.
constexpr int kRB = 4;
template <int C, typename MT, typename AT>
__global__ void __launch_bounds__(kBlock)
k_dense_rows_rb(int nblk, const int *__restrict__ rb_first, const MT *__restrict__ blocks,
                const long long *__restrict__ koff, const int *__restrict__ ioff,
                const int *__restrict__ ni, const int *__restrict__ rowsub,
                const double *__restrict__ y, int ld, double *__restrict__ out,
                float *__restrict__ out32 = nullptr) {
  const int bk = blockIdx.x * kWavesPerBlock + wave_id();
  if (bk >= nblk) return;
  const int r0 = rb_first[bk];
  const int k = rowsub[r0];
  const int i0 = ioff[k], n = ni[k];
  const int nr = min(kRB, i0 + n - r0);
  const MT *rows = blocks + koff[k] + (size_t)(r0 - i0) * n;
  const double *yb = y + (size_t)i0 * ld;
  for (int cp = 0; cp < ld; cp += C) {
    AT acc[kRB][C];
#pragma unroll
    for (int r = 0; r < kRB; ++r)
#pragma unroll
      for (int c = 0; c < C; ++c) acc[r][c] = (AT)0;
#pragma unroll 2
    for (int j = lane_id(); j < n; j += kWave) {
      AT a[kRB];
#pragma unroll
      for (int r = 0; r < kRB; ++r) a[r] = r < nr ? (AT)rows[(size_t)r * n + j] : (AT)0;
      const double *yr = yb + (size_t)j * ld + cp;
      AT yv[C];
#pragma unroll
      for (int c = 0; c < C; ++c) yv[c] = (AT)yr[c];
#pragma unroll
      for (int r = 0; r < kRB; ++r)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[r][c] = tfma(a[r], yv[c], acc[r][c]);
    }
#pragma unroll
    for (int r = 0; r < kRB; ++r) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        AT v = wave_sum(acc[r][c]);
        if (lane_id() == 0 && r < nr) {
          const double ov = 0.0 + 1.0 * ((double)v + 0.0);
          out[(size_t)(r0 + r) * ld + cp + c] = ov;
          if (out32) out32[(size_t)(r0 + r) * ld + cp + c] = (float)ov;
        }
      }
    }
  }
}

// Interface rows of [K_GG | K_GI]: per row, entries [ptr, split) are K_GG
// (columns index p), entries [split, ptr+1) are K_GI (columns index z_I).
//   out = base + c1 * K_GG p + c2 * K_GI z
// A group of G lanes per row (G = 32: two rows per wave), NW waves per
// workgroup: a workgroup covers NW * 64 / G consecutive rows.  With dot != 0
// (the CG operator product q = S p), the row's direction entries p_j are
// stored to pout and the workgroup writes its partial of p^T q (its rows
// summed in order) to red.part2; the last workgroup of each group of
// kPGroup chunks writes the group sum to red.part3.  The group sums are
// reduced by every workgroup of the following update kernel in the same
// fixed order, so no workgroup here waits for the whole grid (one counter for
// the whole grid serialises its same-address atomics over every workgroup).
constexpr int kGRows = 4;                         // waves per workgroup
constexpr int kGLanes = 32;                       // lanes per interface row
constexpr int kGRowsPerWave = kWave / kGLanes;
constexpr int kGChunk = kGRows * kGRowsPerWave;   // rows per workgroup / partial
template <int C> struct GUnroll { static constexpr int U = C == 1 ? 8 : (C <= 4 ? 4 : (C <= 8 ? 2 : 1)); };

template <int C, typename VT, bool OTF, int G = kGLanes, int U = GUnroll<C>::U, bool PIPE = false,
          int NW = kGRows, bool G32 = false>
__device__ __forceinline__ void gamma_rows_body(int nrows, const int *__restrict__ ptr, const int *__restrict__ split,
             const int *__restrict__ col, const VT *__restrict__ val, Src p,
             const double *__restrict__ z, int ld, const double *__restrict__ base, double c1,
             double c2, double *__restrict__ out, int dot, double *__restrict__ pout,
             RedBuf red, ColState st, const double *__restrict__ dinv,
             double *__restrict__ qd, Gather32 g32) {
  constexpr int RPW = kWave / G, CH = NW * RPW;
  // three-launch iteration (qd given): nothing to do once every column stopped
  // (st.flag[1], written by the interior-solve launch just before)
  if (qd && st.flag[1] == 0) return;
  __shared__ double prod[CH * kMaxLd];
  const int wv = wave_id(), lane = lane_id();
  const int jl = wv * RPW + lane / G;          // row within the chunk
  const bool head = (lane & (G - 1)) == 0;
  const int j = blockIdx.x * CH + jl;
  const Src zs{z, nullptr, nullptr, nullptr};
  int b = 0, s = 0, e = 0;
  if (j < nrows) { b = ptr[j]; s = split[j]; e = ptr[j + 1]; }
  for (int cp = 0; cp < ld; cp += C) {
    double a1[C], a2[C], pj[C];
#pragma unroll
    for (int c = 0; c < C; ++c) { a1[c] = 0.0; a2[c] = 0.0; pj[c] = 0.0; }
    if (dot && head && j < nrows) {     // this row's direction entries, loaded early
      double bt[C];
      src_beta<C, OTF>(p, cp, bt);
      src_load<C, OTF>(p, (size_t)j * ld + cp, bt, pj);
    }
    if (j < nrows) {
      if (c1 != 0.0 && c2 != 0.0) {
        if constexpr (G32 && !OTF)
          csr_row_acc2<C, VT, OTF, U, G, PIPE, true>(b, s, e, col, val, p, zs, ld, cp, a1, a2, g32.p, g32.w);
        else
          csr_row_acc2<C, VT, OTF, U, G, PIPE>(b, s, e, col, val, p, zs, ld, cp, a1, a2);
      }
      else if (c1 != 0.0) csr_row_acc<C, VT, OTF, U, G, PIPE>(b, s, col, val, p, ld, cp, a1);
      else if (c2 != 0.0) csr_row_acc<C, VT, false, U, G, PIPE>(s, e, col, val, zs, ld, cp, a2);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      a1[c] = group_sum<G>(a1[c]);
      a2[c] = group_sum<G>(a2[c]);
    }
    if (head) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double q = 0.0;
        if (j < nrows) {
          size_t o = (size_t)j * ld + cp + c;
          q = (base ? base[o] : 0.0) + c1 * a1[c] + c2 * a2[c];
          out[o] = q;
          if (qd) {                         // D^{-1} q for the next K_IG launch
            const double dq = dinv ? dinv[j] * q : q;
            qd[o] = dq;
            if constexpr (G32) {
              if (g32.qd_out) g32.qd_out[o] = (float)dq;
            }
          }
          if (dot) {
            if (pout) pout[o] = pj[c];      // this row of the direction, kept for the update
            q *= pj[c];
          }
        }
        prod[jl * ld + cp + c] = q;
      }
    }
  }
  if (!dot) return;
  __syncthreads();
  for (int c = wv; c < ld; c += NW)
    if (lane == 0) {
      double sum = 0.0;
      for (int r = 0; r < CH; ++r) sum += prod[r * ld + c];
      store_partial(red.part2 + (size_t)blockIdx.x * ld + c, sum);
    }
  // the last workgroup of this chunk group writes the group sum
  const int grp = blockIdx.x / kPGroup;
  const int members = min(kPGroup, (int)gridDim.x - grp * kPGroup);
  __shared__ int lflag;
  unsigned *cnt = red.gcount + (size_t)grp * kCounterStride;
  if (!last_of(cnt, (unsigned)members, &lflag)) return;
  group_sums_store(red.part2, gridDim.x, ld, grp, red.part3, wv, NW);
  __syncthreads();
  if (threadIdx.x == 0) reset_counter(cnt);
}

template <int C, typename VT, bool OTF, int G = kGLanes, int U = GUnroll<C>::U, bool PIPE = false,
          int NW = kGRows, bool G32 = false>
__global__ void __launch_bounds__(NW * kWave)
k_gamma_rows(int nrows, const int *__restrict__ ptr, const int *__restrict__ split,
             const int *__restrict__ col, const VT *__restrict__ val, Src p,
             const double *__restrict__ z, int ld, const double *__restrict__ base, double c1,
             double c2, double *__restrict__ out, int dot, double *__restrict__ pout,
             RedBuf red, ColState st, const double *__restrict__ dinv, double *__restrict__ qd,
             Gather32 g32) {
  gamma_rows_body<C, VT, OTF, G, U, PIPE, NW, G32>(nrows, ptr, split, col, val, p, z, ld, base, c1, c2,
                                                   out, dot, pout, red, st, dinv, qd, g32);
}


// ----------------------------------------------------------- CG updates --
// Chunks of kRowsE interface rows x ld columns; a workgroup handles cpw
// consecutive chunks in one pass (cpw * ld <= 64; cpw is a launch choice:
// every chunk writes the same partials whatever cpw is, so results do not
// depend on it).
// mode 0 (init):   x = 0, r given, z = D^{-1} r, p = 0 (so the first
//                  direction z + 0 * p is z);                 dots: r.z, r.r
// mode 1 (update): a = rz / p^T q from the npq group sums of the interface-row
//                  kernel (every workgroup reduces them in the same order, so
//                  all compute the same a; p^T q <= 0 is a breakdown and
//                  stops the column), then
//                  x += a p, r -= a q, z = D^{-1} r (active);  dots: r.z, r.r
// mode 2 (masked init): columns with mask[c] != 0 restart from the residual
//                  given in q (mode 0 for those columns), the others keep
//                  their state.
// mode 3 (residual replacement; RED = 2 only, after a mode-1 launch of the
//                  same step): the columns that stepped (act_prev and no
//                  breakdown) take the residual given in q, recomputed from x
//                  with more accurate operators, as r, and z = D^{-1} r; x and
//                  p are kept.  The chunk partials of r.z and r.r are those of
//                  the new residual, so the direction launch that follows
//                  forms beta, the convergence test and p from it.
// The last workgroup then updates the column state:
//   init:   rz = r.z, active = (r.r > stop2) for c < nrhs, iters = 0
//   update: iters += 1; converged when r.r <= stop2; beta = r.z / rz_old
// and, when host_nact is given, publishes (number of active columns + 1) to
// host memory (a plain system-coherent store: the host reads only that value).
// E = elements per thread (cpw * kRowsE * ld / kBlock, at least 1).
// RED = 1 (grouped; one chunk per workgroup): the chunk partials of r.z and
// r.r are first summed per group of kPGroup workgroups by the group's last
// workgroup (into red.part2: r.z group sums, then r.r group sums), and the last
// group finishes the column state from the group sums -- the load of the final
// sum spread over the groups instead of one workgroup reducing every chunk of
// every column.
// RED = 2 (split; mode 1 only): the launch ends with the chunk partials (no
// completion count); k_cg_direction_state reduces them, in the tree of RED = 1,
// and finishes the column state.
// Workgroup 0 records the state this step started from (r.z, active) and its
// step length and breakdown marks for it.
template <int E, int RED = 0>
__global__ void __launch_bounds__(kBlock)
k_cg_update(int mode, int nrows, int ld, int nrhs, const double *__restrict__ dinv,
            double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
            double *__restrict__ p, const double *__restrict__ q, RedBuf red, ColState st,
            int use_precond, int *__restrict__ host_nact, int init_p_is_z,
            const int *__restrict__ mask, int npq, int cpw, float *__restrict__ p32,
            const int *__restrict__ run) {
  if (run && *run == 0) return;                       // every column has stopped (see k_tile_rows)
  __shared__ double lds[kRowsE * kMaxLd];
  __shared__ double salpha[kMaxLd];
  __shared__ int sact[kMaxLd];
  __shared__ int lflag;
  const int wv = wave_id(), lane = lane_id();
  const int nchunks = (nrows + kRowsE - 1) / kRowsE;
  const int chunk0 = blockIdx.x * cpw;
  const int nck = min(cpw, nchunks - chunk0);         // chunks of this workgroup
  const int nel = nck * kRowsE * ld;                  // <= E * kBlock
  const int row0 = chunk0 * kRowsE;
  // this thread's elements, loaded before the step length is known (their
  // loads overlap the reduction below)
  double rv[E], qv[E], xv[E], pv[E], dv[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = threadIdx.x + k * kBlock;
    rv[k] = qv[k] = xv[k] = pv[k] = 0.0;
    dv[k] = 1.0;
    if (e < nel) {
      const int lr = e / ld, c = e - lr * ld, j = row0 + lr;
      if (j < nrows) {
        const size_t o = (size_t)j * ld + c;
        rv[k] = r[o];
        if (mode != 0) qv[k] = q[o];                   // mode 2: new residual in q
        if (mode == 1) {
          xv[k] = x[o];
          pv[k] = p[o];
        }
        if (use_precond) dv[k] = dinv[j];
      }
    }
  }
  if (mode == 3) {
    for (int c = threadIdx.x; c < ld; c += kBlock) sact[c] = st.act_prev[c] && !st.brk[c];
    if (blockIdx.x == 0 && threadIdx.x == 0) st.flag[3] = 1;    // read by the direction launch
    __syncthreads();
  }
  if (mode == 1) {
    // wave wv takes the columns c0 .. c0+7 of every group of 32 (the loads of a
    // wave's columns overlap; each column's sum is that of partials_sum)
    constexpr int NC = 8;
    for (int c0 = wv * NC; c0 < ld; c0 += kWavesPerBlock * NC) {
      const int nc = min(NC, ld - c0);
      double pq[NC];
      // written by the last launch; one batch of loads (few group sums), which
      // keeps the registers of this phase low while the element loads are in flight
      partials_sum_cols<NC, false, 1>(red.part3, npq, ld, c0, nc, pq);
      if (lane < nc) {
        const int c = c0 + lane;
        double pqc = pq[0];
#pragma unroll
        for (int u = 1; u < NC; ++u) if (lane == u) pqc = pq[u];
        int act = st.active[c];
        double a = 0.0;
        if (act) {
          if (!(pqc > 0.0)) act = 0;
          else a = st.rz[c] / pqc;
        }
        salpha[c] = a;
        sact[c] = act;
        if (RED == 2 && blockIdx.x == 0) {
          st.rz_prev[c] = st.rz[c];
          st.act_prev[c] = st.active[c];
          st.brk[c] = st.active[c] && !act;
          st.alpha[c] = a;
        }
      }
    }
    __syncthreads();
  }
  // element-wise update; products r*z to LDS, r*r kept in registers.  The new
  // values stay in registers until this workgroup's partials are published
  // (flush below): the completion wait before the count then covers only the
  // partial stores, not the bulk of the vector stores.
  double rzv[E], rrv[E], xn[E], rn[E], zn[E], pn[E];
  int wm[E];                                          // 1: x, 2: r, 4: z, 8: p
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = threadIdx.x + k * kBlock;
    rzv[k] = rrv[k] = 0.0;
    wm[k] = 0;
    xn[k] = rn[k] = zn[k] = pn[k] = 0.0;
    if (e < nel) {
      const int lr = e / ld, c = e - lr * ld;
      const int j = row0 + lr;
      double rz = 0.0;
      if (j < nrows) {
        const size_t o = (size_t)j * ld + c;
        const bool init = mode == 0 || (mode == 2 && mask[c]);
        const bool act = init ? true : ((mode == 1 || mode == 3) && sact[c] != 0);
        const bool repl = (mode == 2 && init) || (mode == 3 && act);
        double rr_ = repl ? qv[k] : rv[k];
        if (repl) wm[k] |= 2;
        if (mode == 1 && act) {
          const double a = salpha[c];
          xn[k] = fma(a, pv[k], xv[k]);
          rr_ = fma(-a, qv[k], rr_);
          wm[k] |= 3;
        }
        if (init) {
          xn[k] = 0.0;
          wm[k] |= 1;
        }
        rn[k] = rr_;
        double zv = use_precond ? dv[k] * rr_ : rr_;
        if (act) wm[k] |= 4;
        else zv = z[o];
        zn[k] = zv;
        if (init) {                                 // direction z, or none yet (beta = 0)
          pn[k] = init_p_is_z ? zv : 0.0;
          wm[k] |= 8;
        }
        rz = rr_ * zv;
        rrv[k] = rr_ * rr_;
      }
      rzv[k] = rz;
      if constexpr (E < 4) lds[e] = rz;
    }
  }
  auto flush = [&]() {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      if (!wm[k]) continue;
      const int e = threadIdx.x + k * kBlock;
      const int lr = e / ld, c = e - lr * ld;
      const size_t o = (size_t)(row0 + lr) * ld + c;
      if (wm[k] & 1) x[o] = xn[k];
      if (wm[k] & 2) r[o] = rn[k];
      if (wm[k] & 4) z[o] = zn[k];
      if (wm[k] & 8) {
        p[o] = pn[k];
        if (p32) p32[o] = (float)pn[k];
      }
    }
  };
  if constexpr (E >= 4) {                             // (one chunk, ld = 4 E)
    chunk64_sums2<E>(rzv, rrv, lds, red.part0 + (size_t)chunk0 * ld, red.part1 + (size_t)chunk0 * ld);
  } else {
    __syncthreads();
    for (int t = wv; t < nck * ld; t += kWavesPerBlock) {
      const int k = t / ld, c = t - k * ld;
      double sm = chunk64_sum(lds + (size_t)k * kRowsE * ld, ld, c);
      if (lane == 0) __hip_atomic_store(red.part0 + (size_t)(chunk0 + k) * ld + c, sm, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  #pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e < nel) lds[e] = rrv[k];
    }
    __syncthreads();
    for (int t = wv; t < nck * ld; t += kWavesPerBlock) {
      const int k = t / ld, c = t - k * ld;
      double sm = chunk64_sum(lds + (size_t)k * kRowsE * ld, ld, c);
      if (lane == 0) __hip_atomic_store(red.part1 + (size_t)(chunk0 + k) * ld + c, sm, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if constexpr (RED == 2) {                           // the direction launch reduces them
    flush();
    return;
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // both partial stores complete before the count
  const double *fin0 = red.part0, *fin1 = red.part1;
  int nfin = nchunks;
  if constexpr (RED == 1) {
    const int ngrp = ((int)gridDim.x + kPGroup - 1) / kPGroup;
    const int grp = blockIdx.x / kPGroup;
    const int members = min(kPGroup, (int)gridDim.x - grp * kPGroup);
    unsigned *cnt = red.gcount + (size_t)grp * kCounterStride;
    const bool last = last_of(cnt, (unsigned)members, &lflag);
    flush();
    if (!last) return;
    double *gs0 = red.part2, *gs1 = red.part2 + (size_t)ngrp * ld;
    group_sums_store(red.part0, nchunks, ld, grp, gs0, wv, kWavesPerBlock);
    group_sums_store(red.part1, nchunks, ld, grp, gs1, wv, kWavesPerBlock);
    __syncthreads();
    if (threadIdx.x == 0) reset_counter(cnt);
    if (!last_of(&red.counter[1], (unsigned)ngrp, &lflag)) return;
    fin0 = gs0;
    fin1 = gs1;
    nfin = ngrp;
  } else {
    const bool last = last_block(&red.counter[1], &lflag);
    flush();
    if (!last) return;
  }
  constexpr int NC2 = 4;
  for (int c0 = wv * NC2; c0 < ld; c0 += kWavesPerBlock * NC2) {
    const int nc = min(NC2, ld - c0);
    double rzv[NC2], rrv2[NC2];
    partials_sum2_cols<NC2>(fin0, fin1, nfin, ld, c0, nc, rzv, rrv2);
    // lane u < nc finishes column c0 + u
    double rz = rzv[0], rr = rrv2[0];
#pragma unroll
    for (int u = 1; u < NC2; ++u)
      if (lane == u) { rz = rzv[u]; rr = rrv2[u]; }
    if (lane < nc) {
      const int c = c0 + lane;
      int active = st.active[c];
      const double rzo = st.rz[c];
      const int mk = mode == 2 ? mask[c] : 0;
      const double s2 = st.stop2[c];
      const int it0 = st.iters[c];
      if (mode == 0 || (mode == 2 && mk)) {
        st.rz[c] = rz;
        st.iters[c] = 0;
        st.beta[c] = 0.0;
        st.ref2[c] = rr;
        active = ((mode == 2 || c < nrhs) && rr > s2) ? 1 : 0;
      } else if (mode == 1) {
        st.alpha[c] = salpha[c];
        if (active && !sact[c]) {           // breakdown: p^T q <= 0
          active = 0;
          st.flag[0] = 1;
        } else if (sact[c]) {
          st.iters[c] = it0 + 1;
          st.beta[c] = rz / rzo;
          st.rz[c] = rz;
          if (rr <= s2) active = 0;
        }
      }
      st.active[c] = active;
      sact[c] = active;
      if (mode != 2 || mk) st.nrm2[c] = rr;
    }
  }
  __syncthreads();
  if (wv == 0) {
    int na = lane < ld ? sact[lane] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) na += __shfl_xor(na, o, kWave);
    if (lane == 0) {
      if (mode == 0) {                   // a new solve starts without breakdown or replacement
        st.flag[0] = 0;
        st.flag[2] = 0;
        st.flag[3] = 0;
      }
      if (st.flag[0]) na = 0;            // breakdown ends the loop
      st.flag[1] = na > 0 ? 1 : 0;       // loop decision for the persistent launch
      if (host_nact) __hip_atomic_store(host_nact, na + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      reset_counter(&red.counter[1]);
    }
  }
}

// ------------------------------------------ three-launch CG iteration --
// Preconditioned CG on S with one launch fewer per iteration and no
// completion counters in the update.  With p_k = z_k + beta_{k-1} p_{k-1},
//   K_IG p_k = K_IG z_k + beta_{k-1} K_IG p_{k-1},
// so w_k = K_II^{-1} K_IG p_k = K_II^{-1} K_IG z_k + beta_{k-1} w_{k-1}, and with
// z_k = z_{k-1} - alpha_{k-1} D^{-1} q_{k-1} (both stored; the interface-row kernel
// writes D^{-1} q with q),
//   K_IG z_k = K_IG z_{k-1} - alpha_{k-1} K_IG D^{-1} q_{k-1},
// two row sums that need no step length until the row is complete.  (The
// slices compute z_k = D^{-1} r_k from the residual; the two agree up to
// rounding.)  z alternates between two buffers like r.  Modes 0 and 1 only.
// Iteration k is then
//   K1 k_cg_kig:   y = K_IG z_k (the two sums, combined with alpha_{k-1});
//                  the update of 64-row interface slices: x_k = x_{k-1} +
//                  alpha p_{k-1}, r_k = r_{k-1} - alpha q_{k-1}, z_k = D^{-1} r_k and
//                  chunk partials of r_k.z_k and r_k.r_k;
//   K2 k_cg_dense: w_k = K_II^{-1} y + beta_{k-1} w_{k-1}, p_k = z_k + beta_{k-1} p_{k-1}
//                  for 64-row slices; one workgroup writes the column state of
//                  iteration k (convergence r_k.r_k <= stop2, iteration count,
//                  host flag);
//   K3 k_gamma_rows: q_k = K_GG p_k - K_GI w_k and the p_k.q_k partials.
// alpha_{k-1} = r_{k-1}.z_{k-1} / p_{k-1}.q_{k-1} (from the interface-row group sums)
// and beta_{k-1} = r_k.z_k / r_{k-1}.z_{k-1} (from K1's chunk partials) are reduced
// by a fifth wave of every workgroup while the other four do row work.
// Workgroups are dispatched in index order, so the ones with the longest
// chains come first: K2's workgroup 0 writes the column state, then one
// workgroup per 64-row interface slice (nsl = ceil(nG / 64), plus 1 in K2),
// then the row workgroups, four rows each (one per wave).  Iteration 0 starts the columns (mode 0: all, mode 2: those
// with mask[c]): no step, x = 0, beta = 0, so p_0 = z_0 and w_0 = K_II^{-1} K_IG z_0.
// The residual alternates between two buffers (K1 gathers r_{k-1} while it
// writes r_k); the column state of iteration k lives in slot k & 1.  Per
// column every reduction runs the same tree for every batch width.
struct CgVec {
  const double *dinv;   // 1 / diag(S), nullptr: no preconditioner
  double *x;            // iterate
  const double *r_old;  // r_{k-1} (iteration 0: the initial residual)
  double *r_new;        // r_k
  const double *z_old;  // z_{k-1}
  double *z;            // z_k
  double *p;            // p_{k-1} before K2, p_k after
  const double *q;      // S p_{k-1}
  const double *qd;     // D^{-1} S p_{k-1} (written with q by the interface-row kernel)
};


__device__ __forceinline__ bool cg_starts(int mode, const int *mask, int c) {
  return mode == 0 || (mode == 2 && mask[c] != 0);
}

// Lane part of partials_sum (items lane, lane + 64, ... added in increasing
// order, the same sum) for partials written by an earlier launch, with
// ordinary cacheable loads and few registers.
__device__ __forceinline__ double prev_partials_lane(const double *part, int P, int ld, int c) {
  double s = 0.0;
#pragma unroll 2
  for (int i = lane_id(); i < P; i += kWave) s += part[i * ld + c];
  return s;
}

// Step length of column c from loaded inputs (K1): writes salpha / supd.
__device__ __forceinline__ void cg_k1_column(int mode, const int *mask, int c, int act0, double rz0,
                                             double pq_lane, ColState st, double *salpha, int *supd) {
  const double pq = wave_sum(pq_lane);
  const int act = cg_starts(mode, mask, c) ? 0 : act0;
  double a = 0.0;
  int up = 0, brk = 0;
  if (act) {
    if (pq > 0.0) {
      a = rz0 / pq;
      up = 1;
    } else {
      brk = 1;              // p^T S p <= 0: the column stops (recorded by K2)
    }
  }
  if (lane_id() == 0) {
    salpha[c] = a;
    supd[c] = up;
    if (blockIdx.x == 0) st.bd[c] = brk;
  }
}

// K1.  Workgroup g < nsl updates interface rows 64g .. 64g+63; the others
// take four interior rows each.  Wave w reduces the step length of columns
// w, w+4, ...; the loads of its first column are issued before its row work.
// E = elements per thread of a slice (64 ld / 256).
template <int C, int E, typename VT, bool G32 = false>
__global__ void __launch_bounds__(kBlock)
k_cg_kig(int mode, int par, int nrows, int nsl, const int *__restrict__ ptr,
         const int *__restrict__ col, const VT *__restrict__ val, int nG, int ld, CgVec v,
         double *__restrict__ y, RedBuf red, ColState st, const int *__restrict__ mask, int npq,
         Gather32 g32) {
  // every column stopped at the previous iteration (st.flag[1], written by its
  // K2): nothing to update or apply (an iteration launched ahead of the host's
  // convergence check)
  if (mode == 1 && st.flag[1] == 0) return;
  __shared__ double salpha[kMaxLd];
  __shared__ int supd[kMaxLd];
  __shared__ double lds[kRowsE * 4 * E];
  const int wv = wave_id(), lane = lane_id();
  const bool rowblk = (int)blockIdx.x >= nsl;
  const int prev = (par ^ 1) * kMaxLd;
  // first column's inputs, loaded before the row work (at most 64 group
  // sums: one value per lane, the lane part of prev_partials_lane)
  int act0 = 0;
  double rz0 = 0.0, pq1 = 0.0;
  const bool few = npq <= kWave;
  if (wv < ld) {
    act0 = st.act2[prev + wv];
    rz0 = st.rz2[prev + wv];
    if (few) pq1 = 0.0 + (lane < npq ? red.part3[(size_t)lane * ld + wv] : 0.0);
  }
  auto pq_lane0 = [&]() { return few ? pq1 : prev_partials_lane(red.part3, npq, ld, wv); };
  if (rowblk) {
    // u = K_IG z_{k-1} and v = K_IG D^{-1} q_{k-1} for this wave's row,
    // y = u - alpha v once alpha is known (iteration 0: u = K_IG D^{-1} r_0)
    const int row = ((int)blockIdx.x - nsl) * kWavesPerBlock + wv;
    const Src rs{v.r_old, nullptr, nullptr, nullptr, nullptr, v.dinv, nullptr};
    const Src zs{v.z_old, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const Src qs{v.qd, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double au[C], av[C];
    int b = 0, e = 0;
    if (row < nrows) {
      b = ptr[row];
      e = ptr[row + 1];
    }
    bool first = true;
    for (int cp = 0; cp < ld; cp += C) {
#pragma unroll
      for (int c = 0; c < C; ++c) { au[c] = 0.0; av[c] = 0.0; }
      if (row < nrows) {
        if (mode == 0) csr_row_acc_uv<C, VT, true, false>(b, e, col, val, rs, rs, ld, cp, au, av);
        else if constexpr (G32)
          csr_row_acc_uv<C, VT, false, true, (Unroll<C>::U + 1) / 2, true>(b, e, col, val, zs, qs, ld, cp, au,
                                                                          av, g32.z_old, g32.qd);
        else csr_row_acc_uv<C, VT, false, true>(b, e, col, val, zs, qs, ld, cp, au, av);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) {
        au[c] = wave_sum(au[c]);
        av[c] = wave_sum(av[c]);
      }
      if (first) {
        if (wv < ld) cg_k1_column(mode, mask, wv, act0, rz0, pq_lane0(), st, salpha, supd);
        if constexpr (C > kWavesPerBlock)      // (below 16 columns ld == C)
          for (int c = wv + kWavesPerBlock; c < ld; c += kWavesPerBlock)
            cg_k1_column(mode, mask, c, st.act2[prev + c], st.rz2[prev + c],
                         prev_partials_lane(red.part3, npq, ld, c), st, salpha, supd);
        __syncthreads();
        first = false;
      }
      if (row < nrows && lane == 0)
#pragma unroll
        for (int c = 0; c < C; ++c)
          y[(size_t)row * ld + cp + c] = supd[cp + c] ? fma(-salpha[cp + c], av[c], au[c]) : au[c];
    }
    return;
  }
  // slice workgroup: the update of interface rows 64 g .. 64 g + 63
  const int g = blockIdx.x;
  const int row0 = g * kRowsE;
  const int nel = kRowsE * ld;
  // operands loaded before the step length is known (narrow batches; wide
  // ones load them where they are used)
  constexpr int EP = E <= 2 ? E : 1;
  double ro[EP], qv[EP], xv[EP], pv[EP], dv[EP];
#pragma unroll
  for (int k = 0; k < EP; ++k) {
    const int e = threadIdx.x + k * kBlock;
    const int lr = e / ld, c = e - lr * ld, j = row0 + lr;
    ro[k] = qv[k] = xv[k] = pv[k] = 0.0;
    dv[k] = 1.0;
    if (E <= 2 && e < nel && j < nG) {
      const size_t o = (size_t)j * ld + c;
      ro[k] = v.r_old[o];
      qv[k] = v.q[o];
      xv[k] = v.x[o];
      pv[k] = v.p[o];
      if (v.dinv) dv[k] = v.dinv[j];
    }
  }
  if (wv < ld) cg_k1_column(mode, mask, wv, act0, rz0, pq_lane0(), st, salpha, supd);
  if constexpr (C > kWavesPerBlock)
    for (int c = wv + kWavesPerBlock; c < ld; c += kWavesPerBlock)
      cg_k1_column(mode, mask, c, st.act2[prev + c], st.rz2[prev + c],
                   prev_partials_lane(red.part3, npq, ld, c), st, salpha, supd);
  __syncthreads();
  double rrv[E];
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = threadIdx.x + k * kBlock;
    rrv[k] = 0.0;
    if (e < nel) {
      const int lr = e / ld, c = e - lr * ld, j = row0 + lr;
      double rz = 0.0;
      if (j < nG) {
        const size_t o = (size_t)j * ld + c;
        const int kp = E <= 2 ? k : 0;
        const double r0 = E <= 2 ? ro[kp] : v.r_old[o];
        double rn = r0;
        if (supd[c]) {
          const double a = salpha[c];
          v.x[o] = fma(a, E <= 2 ? pv[kp] : v.p[o], E <= 2 ? xv[kp] : v.x[o]);
          rn = fma(-a, E <= 2 ? qv[kp] : v.q[o], r0);
        } else if (cg_starts(mode, mask, c)) {
          v.x[o] = 0.0;
        }
        const double d = E <= 2 ? dv[kp] : (v.dinv ? v.dinv[j] : 1.0);
        const double zv = v.dinv ? d * rn : rn;
        v.r_new[o] = rn;
        v.z[o] = zv;
        if constexpr (G32) g32.z[o] = (float)zv;
        rz = rn * zv;
        rrv[k] = rn * rn;
      }
      lds[e] = rz;
    }
  }
  __syncthreads();
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    const double sm = chunk64_sum(lds, ld, c);
    if (lane == 0) red.part0[(size_t)g * ld + c] = sm;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = threadIdx.x + k * kBlock;
    if (e < nel) lds[e] = rrv[k];
  }
  __syncthreads();
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    const double sm = chunk64_sum(lds, ld, c);
    if (lane == 0) red.part1[(size_t)g * ld + c] = sm;
  }
}

// Inputs of K2's column scalars for column c (loads only).
// Inputs of K2's column scalars for column c (rzl, rrl: lane parts of the
// partial sums, or NaN when not loaded yet).
struct CgK2In {
  int act0, bd0, it0;
  double rz0, s2, rzl, rrl;
};
__device__ __forceinline__ CgK2In cg_k2_load(int par, int ld, RedBuf red, ColState st, int nch, bool leader,
                                             int c) {
  const int prev = (par ^ 1) * kMaxLd;
  CgK2In in;
  in.act0 = st.act2[prev + c];
  in.bd0 = st.bd[c];
  in.rz0 = st.rz2[prev + c];
  in.rzl = prev_partials_lane(red.part0, nch, ld, c);
  in.rrl = 0.0;
  in.it0 = 0;
  in.s2 = 0.0;
  if (leader) {
    in.rrl = prev_partials_lane(red.part1, nch, ld, c);
    in.it0 = st.iters[c];
    in.s2 = st.stop2[c];
  }
  return in;
}

// beta of column c into sbeta / sinit; in the state workgroup (leader) also
// the column state of iteration k (scnt = new active flag).
__device__ __forceinline__ void cg_k2_column(int mode, int par, int nrhs, const int *mask, int c,
                                             const CgK2In &in, bool leader, ColState st, RedBuf red,
                                             int nch, int ld, double *sbeta, int *sinit, int *scnt,
                                             int *sbk) {
  const double rz = wave_sum(in.rzl);
  const double rr = leader ? wave_sum(in.rrl) : 0.0;
  if (lane_id() != 0) return;
  const int cur = par * kMaxLd;
  const bool init = cg_starts(mode, mask, c);
  const int act = init ? 0 : in.act0;
  const bool brk = act && in.bd0 != 0;
  sbeta[c] = (act && !brk) ? rz / in.rz0 : 0.0;
  sinit[c] = init ? 1 : 0;
  if (!leader) return;
  int active;
  sbk[c] = (act && brk) ? 1 : 0;
  if (init) {
    st.rz2[cur + c] = rz;
    st.iters[c] = 0;
    active = ((mode == 2 || c < nrhs) && rr > in.s2) ? 1 : 0;
    st.nrm2[c] = rr;
  } else {
    active = act;
    st.rz2[cur + c] = (act && !brk) ? rz : in.rz0;
    if (act && brk) {
      active = 0;
      st.flag[0] = 1;
    } else if (act) {
      st.iters[c] = in.it0 + 1;
      if (rr <= in.s2) active = 0;
    }
    if (mode != 2) st.nrm2[c] = rr;
  }
  st.act2[cur + c] = active;
  st.active[c] = active;
  scnt[c] = active;
}

// All column scalars of K2 (wave w: columns w, w+4, ...; the first one's
// inputs passed in when have0), then a barrier; the state workgroup then
// publishes the number of active columns (+1) to the host.
__device__ __forceinline__ void cg_k2_scalars(int mode, int par, int ld, int nrhs, const int *mask, RedBuf red,
                                              ColState st, int nch, bool leader, bool have0, const CgK2In &in0,
                                              int flag0, int *__restrict__ host_nact, double *sbeta,
                                              int *sinit, int *scnt, int *sbk) {
  const int wv = wave_id();
  if (wv < ld)
    cg_k2_column(mode, par, nrhs, mask, wv, have0 ? in0 : cg_k2_load(par, ld, red, st, nch, leader, wv), leader,
                 st, red, nch, ld, sbeta, sinit, scnt, sbk);
  for (int c = wv + kWavesPerBlock; c < ld; c += kWavesPerBlock)
    cg_k2_column(mode, par, nrhs, mask, c, cg_k2_load(par, ld, red, st, nch, leader, c), leader, st, red, nch,
                 ld, sbeta, sinit, scnt, sbk);
  __syncthreads();
  if (leader && wv == 0) {
    const int lane = lane_id();
    int na = lane < ld ? scnt[lane] : 0;
    int nb = lane < ld ? sbk[lane] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      na += __shfl_xor(na, o, kWave);
      nb += __shfl_xor(nb, o, kWave);
    }
    if (lane == 0) {
      if (mode == 0) st.flag[0] = 0;                    // a new solve starts without breakdown
      if ((mode != 0 && flag0) || nb) na = 0;           // breakdown ends the loop
      st.flag[1] = na > 0 ? 1 : 0;
      if (host_nact) __hip_atomic_store(host_nact, na + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// K2 direction slice of workgroup 1 + g: p = z + beta p (started columns
// p = z) for interface rows 64g .. 64g+63; the first element per thread is
// loaded before the scalars are known.
__device__ __forceinline__ void cg_k2_slice_pre(int nG, int ld, const double *__restrict__ z,
                                                const double *__restrict__ p, double &z0, double &p0) {
  const int e = threadIdx.x, lr = e / ld, j = ((int)blockIdx.x - 1) * kRowsE + lr;
  z0 = p0 = 0.0;
  if (e < kRowsE * ld && j < nG) {
    z0 = z[(size_t)j * ld + (e - lr * ld)];
    p0 = p[(size_t)j * ld + (e - lr * ld)];
  }
}
template <bool G32>
__device__ __forceinline__ void cg_k2_slice(int nG, int ld, const double *__restrict__ z,
                                            double *__restrict__ p, const double *sbeta,
                                            const int *sinit, double z0, double p0,
                                            float *__restrict__ p32) {
  const int row0 = ((int)blockIdx.x - 1) * kRowsE;
  for (int e = threadIdx.x; e < kRowsE * ld; e += kBlock) {
    const int lr = e / ld, c = e - lr * ld, j = row0 + lr;
    if (j >= nG) break;
    const size_t o = (size_t)j * ld + c;
    const bool first = e == (int)threadIdx.x;
    const double zv = first ? z0 : z[o];
    const double pv = first ? p0 : p[o];
    const double pn = sinit[c] ? zv : fma(sbeta[c], pv, zv);
    p[o] = pn;
    if constexpr (G32) p32[o] = (float)pn;
  }
}

// K2: workgroup 0 writes the column state, workgroups 1 .. nsl-1 update the
// direction slices, the others take interior rows: one row per wave (row
// arithmetic of k_dense_rows), w = result + beta w_prev.
template <int C, typename MT, typename AT, bool G32 = false>
__global__ void __launch_bounds__(kBlock)
k_cg_dense(int mode, int par, int nrows, int nsl, const MT *__restrict__ blocks,
           const long long *__restrict__ koff, const int *__restrict__ ioff, const int *__restrict__ ni,
           const int *__restrict__ rowsub, const double *__restrict__ y, int ld, double *__restrict__ w,
           int nG, int nrhs, const double *__restrict__ z, double *__restrict__ p, RedBuf red,
           ColState st, const int *__restrict__ mask, int *__restrict__ host_nact, Gather32 g32) {
  if (mode == 1 && st.flag[1] == 0) {       // every column stopped (see k_cg_kig)
    if (blockIdx.x == 0 && threadIdx.x == 0 && host_nact)
      __hip_atomic_store(host_nact, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  __shared__ double sbeta[kMaxLd];
  __shared__ int sinit[kMaxLd];
  __shared__ int scnt[kMaxLd];
  __shared__ int sbk[kMaxLd];
  __shared__ double sp[C][kWavesPerBlock][kWave];
  const int wv = wave_id(), lane = lane_id();
  const int nch = (nG + kRowsE - 1) / kRowsE;
  const bool leader = blockIdx.x == 0;
  const bool rowblk = (int)blockIdx.x >= nsl;
  if (!rowblk) {
    const int flag0 = leader ? st.flag[0] : 0;
    double z0 = 0.0, p0 = 0.0;
    if (!leader) cg_k2_slice_pre(nG, ld, z, p, z0, p0);
    cg_k2_scalars(mode, par, ld, nrhs, mask, red, st, nch, leader, false, CgK2In{}, flag0, host_nact, sbeta,
                  sinit, scnt, sbk);
    if (!leader) cg_k2_slice<G32>(nG, ld, z, p, sbeta, sinit, z0, p0, g32.p);
    return;
  }
  // (launched with C == ld <= 4: one pass covers every column)
  // Column scalar inputs loaded before the row work: the scalars of column
  // c < ld, and, with nch <= 256, wave w's part of the r.z partials (item
  // 64 w + lane of every column; combined through LDS afterwards in the order
  // of prev_partials_lane).
  const bool early = nch <= kWavesPerBlock * kWave;
  double pz[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int i = wv * kWave + lane;
    pz[c] = (early && i < nch) ? red.part0[(size_t)i * ld + c] : 0.0;
  }
  const int r = ((int)blockIdx.x - nsl) * kWavesPerBlock + wv;
  double t = 0.0, wp = 0.0;
  bool have = false;
  if (r < nrows) {
    if (lane < ld) wp = w[(size_t)r * ld + lane];     // w_prev, loaded early
    const int k = rowsub[r];
    const int i0 = ioff[k];
    const int n = ni[k];
    const MT *row = blocks + koff[k] + (size_t)(r - i0) * n;
    const double *yb = y + (size_t)i0 * ld;
    AT acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (AT)0;
    constexpr int U = Unroll<C>::U;
    for (int j = lane; j < n; j += U * kWave) {
      AT a[U];
      double yv[U][C];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int jj = j + u * kWave;
        bool ok = jj < n;
        a[u] = ok ? (AT)row[jj] : (AT)0;
        const double *yr = yb + (size_t)(ok ? jj : 0) * ld;
#pragma unroll
        for (int c = 0; c < C; ++c) yv[u][c] = ok ? yr[c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = tfma(a[u], (AT)yv[u][c], acc[c]);
    }
    // lane c keeps column c's result
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double sv = (double)wave_sum(acc[c]);
      if (lane == c) t = sv;
    }
    have = true;
  }
  CgK2In in0{};
  if (early) {
#pragma unroll
    for (int c = 0; c < C; ++c) sp[c][wv][lane] = pz[c];
    __syncthreads();
    if (wv < ld) {
      const int prev = (par ^ 1) * kMaxLd;
      in0.act0 = st.act2[prev + wv];
      in0.bd0 = st.bd[wv];
      in0.rz0 = st.rz2[prev + wv];
      in0.rzl = 0.0;
#pragma unroll
      for (int bw = 0; bw < kWavesPerBlock; ++bw) in0.rzl += sp[wv][bw][lane];
      in0.rrl = 0.0;
      in0.it0 = 0;
      in0.s2 = 0.0;
    }
  }
  cg_k2_scalars(mode, par, ld, nrhs, mask, red, st, nch, false, early, in0, 0, nullptr, sbeta, sinit, scnt, sbk);
  if (have && lane < ld) {
    const int c = lane;
    const double wn = sinit[c] ? t : fma(sbeta[c], wp, t);
    w[(size_t)r * ld + c] = wn;
    if constexpr (G32) g32.w[(size_t)r * ld + c] = (float)wn;
  }
}

// K2 for wide batches (ld >= 8): kRB rows per wave (row arithmetic of
// k_dense_rows_rb), results parked in LDS until beta is known.
template <int C, typename MT, typename AT, bool G32 = false>
__global__ void __launch_bounds__(kBlock)
k_cg_dense_rb(int mode, int par, int nblk, int nsl, const int *__restrict__ rb_first,
              const MT *__restrict__ blocks, const long long *__restrict__ koff,
              const int *__restrict__ ioff, const int *__restrict__ ni, const int *__restrict__ rowsub,
              const double *__restrict__ y, int ld, double *__restrict__ w, int nG, int nrhs,
              const double *__restrict__ z, double *__restrict__ p, RedBuf red, ColState st,
              const int *__restrict__ mask, int *__restrict__ host_nact, Gather32 g32) {
  if (mode == 1 && st.flag[1] == 0) {       // every column stopped (see k_cg_kig)
    if (blockIdx.x == 0 && threadIdx.x == 0 && host_nact)
      __hip_atomic_store(host_nact, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  __shared__ double sbeta[kMaxLd];
  __shared__ int sinit[kMaxLd];
  __shared__ int scnt[kMaxLd];
  __shared__ int sbk[kMaxLd];
  __shared__ double st_[kWavesPerBlock][kRB][kMaxLd];
  const int wv = wave_id(), lane = lane_id();
  const int nch = (nG + kRowsE - 1) / kRowsE;
  const bool leader = blockIdx.x == 0;
  const bool rowblk = (int)blockIdx.x >= nsl;
  if (!rowblk) {
    const int flag0 = leader ? st.flag[0] : 0;
    double z0 = 0.0, p0 = 0.0;
    if (!leader) cg_k2_slice_pre(nG, ld, z, p, z0, p0);
    cg_k2_scalars(mode, par, ld, nrhs, mask, red, st, nch, leader, false, CgK2In{}, flag0, host_nact, sbeta,
                  sinit, scnt, sbk);
    if (!leader) cg_k2_slice<G32>(nG, ld, z, p, sbeta, sinit, z0, p0, g32.p);
    return;
  }
  const int bk = ((int)blockIdx.x - nsl) * kWavesPerBlock + wv;
  int r0 = 0, nr = 0;
  if (bk < nblk) {
    r0 = rb_first[bk];
    const int k = rowsub[r0];
    const int i0 = ioff[k], n = ni[k];
    nr = min(kRB, i0 + n - r0);
    const MT *rows = blocks + koff[k] + (size_t)(r0 - i0) * n;
    const double *yb = y + (size_t)i0 * ld;
    for (int cp = 0; cp < ld; cp += C) {
      AT acc[kRB][C];
#pragma unroll
      for (int rr = 0; rr < kRB; ++rr)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[rr][c] = (AT)0;
#pragma unroll 2
      for (int j = lane; j < n; j += kWave) {
        AT a[kRB];
#pragma unroll
        for (int rr = 0; rr < kRB; ++rr) a[rr] = rr < nr ? (AT)rows[(size_t)rr * n + j] : (AT)0;
        const double *yr = yb + (size_t)j * ld + cp;
        AT yv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) yv[c] = (AT)yr[c];
#pragma unroll
        for (int rr = 0; rr < kRB; ++rr)
#pragma unroll
          for (int c = 0; c < C; ++c) acc[rr][c] = tfma(a[rr], yv[c], acc[rr][c]);
      }
#pragma unroll
      for (int rr = 0; rr < kRB; ++rr)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          AT sv = wave_sum(acc[rr][c]);
          if (lane == 0) st_[wv][rr][cp + c] = (double)sv;
        }
    }
  }
  cg_k2_scalars(mode, par, ld, nrhs, mask, red, st, nch, false, false, CgK2In{}, 0, nullptr, sbeta, sinit, scnt,
                sbk);
  for (int rr = 0; rr < nr; ++rr)
    for (int c = lane; c < ld; c += kWave) {
      const size_t o = (size_t)(r0 + rr) * ld + c;
      const double wn = sinit[c] ? st_[wv][rr][c] : fma(sbeta[c], w[o], st_[wv][rr][c]);
      w[o] = wn;
      if constexpr (G32) g32.w[o] = (float)wn;
    }
}

// stop2[c] = f^2 * v[c]  (v: squared norms)
__global__ void k_set_stop(int ld, double f2, const double *__restrict__ v, ColState st) {
  int c = threadIdx.x;
  if (c < ld) st.stop2[c] = f2 * v[c];
}

// p = z + beta p for the active columns (when the direction is kept in memory
// instead of being formed where it is gathered).
__global__ void __launch_bounds__(kBlock)
k_cg_direction(int nrows, int ld, const double *__restrict__ z, double *__restrict__ p,
               ColState st, float *__restrict__ p32 = nullptr) {
  size_t n = (size_t)nrows * ld;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBlock) {
    int c = (int)(e % ld);
    if (st.active[c]) {
      const double pn = fma(st.beta[c], p[e], z[e]);
      p[e] = pn;
      if (p32) p32[e] = (float)pn;      // copy gathered by the FP32-data products
    }
  }
}

// End of a CG step after the split update (k_cg_update<E, 2>).  The column
// sums of r.z and r.r are formed from the nch chunk partials of the update in
// one fixed order -- group sums over kPGroup consecutive chunks by the tree of
// chunk_group_sum (one thread per column, dot and group, the butterfly's pairs
// added in registers), then the groups in order -- which gives the bits of the
// grouped update's two levels.  Workgroup b >= 1 updates the direction
// p = z + beta p of the still iterating columns for column block (b - 1) % ncb
// (kDirCols columns, or ld when narrower) over its share of the rows, and
// reduces the sums of that block only; workgroup 0 reduces every column and
// writes the column state (from the sums and the state the step started from:
// rz_prev, act_prev, brk, recorded by the update's workgroup 0; the state is
// read by no other workgroup of this launch), and publishes (active columns +
// 1) to host_nact; it updates no rows, so its longer reduction runs beside
// the others' row work.  ld: a power of two from 8 to kMaxLd; the grid 1 plus
// a multiple of ld / min(ld, kDirCols).  run: as in k_tile_rows; it is st.flag + 1,
// which workgroup 0 of this launch rewrites.  A workgroup that reads the new
// value 0 has no active column to update either, so either value gives the
// same result.
constexpr int kDirCols = 16;       // 128-byte row segments
constexpr int kDirBlock = 512;
constexpr int kDirE = 12;          // direction elements per thread held across the reduction

// tot[t * kMaxLd + c] = sum of dot t (0: r.z, 1: r.r) of column c, c0 <= c < c0 + nc
// (2 nc dividing kDirBlock); gsum: kDirBlock doubles of LDS.
__device__ __forceinline__ void direction_sums(const RedBuf &red, int ld, int nch, int c0, int nc, double *gsum,
                                               double *tot) {
  const int pairs = 2 * nc, gpp = kDirBlock / pairs;
  const int ngrp = (nch + kPGroup - 1) / kPGroup;
  const int q = threadIdx.x % pairs, gi = threadIdx.x / pairs;
  const int t = q / nc, c = c0 + (q - t * nc);
  const double *src = (t ? red.part1 : red.part0) + c;
  double acc = 0.0;                             // (threads q < pairs: the running sum)
  for (int g0 = 0; g0 < ngrp; g0 += gpp) {
    const int g = g0 + gi;
    double s = 0.0;
    if (g < ngrp) {
      double u[kPGroup];
#pragma unroll
      for (int m = 0; m < kPGroup; ++m) {
        const int ch = g * kPGroup + m;
        u[m] = ch < nch ? src[(size_t)ch * ld] : 0.0;
      }
#pragma unroll
      for (int h = kPGroup / 2; h >= 1; h /= 2)
#pragma unroll
        for (int m = 0; m < h; ++m) u[m] += u[m + h];
      s = u[0];
    }
    __syncthreads();                            // the last pass's sums are consumed
    gsum[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < pairs)
      for (int i = 0; i < gpp && g0 + i < ngrp; ++i) acc += gsum[i * pairs + threadIdx.x];
  }
  if (threadIdx.x < pairs) tot[t * kMaxLd + c] = acc;
  __syncthreads();
}

__global__ void __launch_bounds__(kDirBlock)
k_cg_direction_state(int nrows, int ld, const double *__restrict__ z, double *__restrict__ p, RedBuf red,
                     ColState st, int nch, int *__restrict__ host_nact, float *__restrict__ p32,
                     const int *__restrict__ run, double drop2) {
  if (run && *run == 0) {              // every column had stopped: nothing changes, report none active
    if (blockIdx.x == 0 && threadIdx.x == 0 && host_nact)
      __hip_atomic_store(host_nact, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  __shared__ double gsum[kDirBlock];
  __shared__ double tot[2 * kMaxLd];
  __shared__ double sbeta[kMaxLd];
  __shared__ int sact[kMaxLd];
  __shared__ int sdue[kMaxLd];
  const int cw = min(ld, kDirCols), ncb = ld / cw;
  // workgroup 0: every column's sums and state, no direction rows; workgroup
  // b >= 1: column block (b - 1) % ncb over row share (b - 1) / ncb
  const bool all = blockIdx.x == 0;
  const int wb = all ? 0 : (int)blockIdx.x - 1;
  const int cb = wb % ncb, rr = wb / ncb, nrr = ((int)gridDim.x - 1) / ncb;
  const int c0 = all ? 0 : cb * cw, nc = all ? ld : cw;
  // rows [j0, j1) of column block cb; the first kDirE elements per thread are
  // loaded before the sums, so that their loads overlap the reduction
  const int per = (nrows + nrr - 1) / nrr;
  const int j0 = min(nrows, rr * per), j1 = min(nrows, j0 + per);
  const int n = all ? 0 : (j1 - j0) * cw;
  auto offset = [&](int i) {
    const int jr = i / cw;
    return (size_t)(j0 + jr) * ld + cb * cw + (i - jr * cw);
  };
  double zv[kDirE], pv[kDirE];
#pragma unroll
  for (int k = 0; k < kDirE; ++k) {
    const int i = threadIdx.x + k * kDirBlock;
    zv[k] = pv[k] = 0.0;
    if (i < n) {
      const size_t e = offset(i);
      zv[k] = z[e];
      pv[k] = p[e];
    }
  }
  direction_sums(red, ld, nch, c0, nc, gsum, tot);
  if (threadIdx.x < nc) {
    const int c = c0 + threadIdx.x;
    const double rz = tot[c], rr2 = tot[kMaxLd + c];
    const int act0 = st.act_prev[c], brk = st.brk[c];
    int act = 0;
    double beta = 0.0;
    if (act0 && !brk) {
      beta = rz / st.rz_prev[c];
      act = rr2 > st.stop2[c] ? 1 : 0;
    }
    if (all) {
      if (act0 && brk) st.flag[0] = 1;            // breakdown: p^T q <= 0
      if (act0 && !brk) {
        st.iters[c] += 1;
        st.beta[c] = beta;
        st.rz[c] = rz;
      }
      // residual replacement: the reference norm after one, and whether the
      // column is due for the next.  A replaced residual no smaller than the
      // one replaced before means the directions make no progress on the
      // true residual (operators too inaccurate for the system): the column
      // stops, and the FP64 check of its residual decides what follows.
      double ref = st.ref2[c];
      if (st.flag[3] && act0 && !brk) {     // replaced in this step
        if (!(rr2 < ref)) act = 0;
        ref = rr2;
        st.ref2[c] = ref;
      }
      sdue[c] = (act && rr2 < drop2 * ref) ? 1 : 0;
      st.active[c] = act;
      st.nrm2[c] = rr2;
    }
    sbeta[c] = beta;
    sact[c] = act;
  }
  __syncthreads();
  if (all && threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    int na = lane < ld ? sact[lane] : 0;
    int nd = lane < ld ? sdue[lane] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      na += __shfl_xor(na, o, kWave);
      nd += __shfl_xor(nd, o, kWave);
    }
    if (lane == 0) {
      if (st.flag[0]) na = 0;            // breakdown ends the loop
      st.flag[1] = na > 0 ? 1 : 0;
      st.flag[2] = (na > 0 && nd > 0) ? 1 : 0;
      st.flag[3] = 0;
      if (host_nact) __hip_atomic_store(host_nact, na + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
#pragma unroll
  for (int k = 0; k < kDirE; ++k) {
    const int i = threadIdx.x + k * kDirBlock;
    const int c = cb * cw + (i & (cw - 1));
    if (i < n && sact[c]) {
      const size_t e = offset(i);
      const double pn = fma(sbeta[c], pv[k], zv[k]);
      p[e] = pn;
      if (p32) p32[e] = (float)pn;
    }
  }
  for (int i = threadIdx.x + kDirE * kDirBlock; i < n; i += kDirBlock) {
    const int c = cb * cw + (i & (cw - 1));
    if (sact[c]) {
      const size_t e = offset(i);
      const double pn = fma(sbeta[c], p[e], z[e]);
      p[e] = pn;
      if (p32) p32[e] = (float)pn;
    }
  }
}

// ------------------------------------------------------- vector helpers --
// out[i*ld + c] = b[c*ldb + map[i]] for c < nrhs, 0 for padded columns.
__global__ void k_gather(int n, const int *__restrict__ map, const double *__restrict__ b,
                         int ldb, int nrhs, int ld, double *__restrict__ out) {
  size_t total = (size_t)n * ld;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / ld), c = (int)(e % ld);
    out[e] = c < nrhs ? b[(size_t)c * ldb + map[i]] : 0.0;
  }
}

// u[c*ldu + map[i]] = in[i*ld + c] for c < nrhs.
__global__ void k_scatter(int n, const int *__restrict__ map, const double *__restrict__ in,
                          int ld, int nrhs, double *__restrict__ u, int ldu) {
  size_t total = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e / n), i = (int)(e % n);
    u[(size_t)c * ldu + map[i]] = in[(size_t)i * ld + c];
  }
}

// y[e] += x[e] for the columns whose mask is set (refinement correction).
__global__ void k_axpy_masked(size_t n, int ld, const double *__restrict__ x,
                              double *__restrict__ y, const int *__restrict__ mask) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e % ld);
    if (mask[c]) y[e] += x[e];
  }
}

// Fixed-tree column norms: the last workgroup adds sum_rows v^2 into acc[c]
// (acc zeroed by the host when starting a new norm).
__global__ void __launch_bounds__(kBlock)
k_colnorm2(int nrows, int ld, const double *__restrict__ v, RedBuf red, double *acc) {
  __shared__ double lds[kRowsE * kMaxLd];
  __shared__ int lflag;
  const int row0 = blockIdx.x * kRowsE;
  const int wv = wave_id(), lane = lane_id();
  for (int e = threadIdx.x; e < kRowsE * ld; e += kBlock) {
    int lr = e / ld, c = e - lr * ld;
    int j = row0 + lr;
    double t = 0.0;
    if (j < nrows) { double a = v[(size_t)j * ld + c]; t = a * a; }
    lds[lr * ld + c] = t;
  }
  __syncthreads();
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    double s = chunk64_sum(lds, ld, c);
    if (lane == 0) store_partial(red.part0 + (size_t)blockIdx.x * ld + c, s);
  }
  if (!last_block(&red.counter[2], &lflag)) return;
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    double s = partials_sum(red.part0, gridDim.x, ld, c);
    if (lane == 0) acc[c] += s;
  }
  __syncthreads();
  if (threadIdx.x == 0) reset_counter(&red.counter[2]);
}

// out[c] = squared 2-norm of column c of the stacked vector [vI; vG]
// (nI + nG rows in the DD layout): 64-row chunk partials by the wave
// butterfly, summed in order by the last workgroup.  With stop2 != nullptr
// also stop2[c] = f2 * out[c] (CG stopping thresholds).
__global__ void __launch_bounds__(kBlock)
k_norm2(int nI, int nG, int ld, const double *__restrict__ vI, const double *__restrict__ vG,
        RedBuf red, double *__restrict__ out, double f2, double *__restrict__ stop2) {
  __shared__ double lds[kRowsE * kMaxLd];
  __shared__ int lflag;
  const int n = nI + nG;
  const int row0 = blockIdx.x * kRowsE;
  const int wv = wave_id(), lane = lane_id();
  for (int e = threadIdx.x; e < kRowsE * ld; e += kBlock) {
    int lr = e / ld, c = e - lr * ld;
    int j = row0 + lr;
    double t = 0.0;
    if (j < n) {
      double a = j < nI ? vI[(size_t)j * ld + c] : vG[(size_t)(j - nI) * ld + c];
      t = a * a;
    }
    lds[lr * ld + c] = t;
  }
  __syncthreads();
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    double sm = chunk64_sum(lds, ld, c);
    if (lane == 0) store_partial(red.part0 + (size_t)blockIdx.x * ld + c, sm);
  }
  if (!last_block(&red.counter[2], &lflag)) return;
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    double sm = partials_sum(red.part0, gridDim.x, ld, c);
    if (lane == 0) {
      out[c] = sm;
      if (stop2) stop2[c] = f2 * sm;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) reset_counter(&red.counter[2]);
}

// Right-hand sides into the DD layout, both parts in one launch: row i < nI
// of the stacked output is b[imap[i]], row nI + k is b[gmap[k]]; columns
// c >= nrhs of the ld-wide layout are zero.
__global__ void k_gather2(int nI, int nG, const int *__restrict__ imap, const int *__restrict__ gmap,
                          const double *__restrict__ b, int ldb, int nrhs, int ld,
                          double *__restrict__ outI, double *__restrict__ outG) {
  size_t total = (size_t)(nI + nG) * ld;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / ld), c = (int)(e % ld);
    bool in = i < nI;
    int g = in ? imap[i] : gmap[i - nI];
    double v = c < nrhs ? b[(size_t)c * ldb + g] : 0.0;
    if (in) outI[e] = v;
    else outG[e - (size_t)nI * ld] = v;
  }
}

// Solution out of the DD layout, both parts in one launch.
__global__ void k_scatter2(int nI, int nG, const int *__restrict__ imap, const int *__restrict__ gmap,
                           const double *__restrict__ inI, const double *__restrict__ inG, int ld,
                           int nrhs, double *__restrict__ u, int ldu) {
  const int n = nI + nG;
  size_t total = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e / n), i = (int)(e % n);
    if (i < nI) u[(size_t)c * ldu + imap[i]] = inI[(size_t)i * ld + c];
    else u[(size_t)c * ldu + gmap[i - nI]] = inG[(size_t)(i - nI) * ld + c];
  }
}

// y += x on the columns with mask[c] != 0, both parts in one launch.
// Undo of the last correction of the masked columns: y -= x, or y = 0 when
// the correction was the whole iterate (zero != 0).
__global__ void k_undo2_masked(size_t nIe, size_t nGe, int ld, const double *__restrict__ xI,
                               const double *__restrict__ xG, double *__restrict__ yI,
                               double *__restrict__ yG, const int *__restrict__ mask, int zero) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nIe + nGe;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e % ld);
    if (!mask[c]) continue;
    if (e < nIe) yI[e] = zero ? 0.0 : yI[e] - xI[e];
    else yG[e - nIe] = zero ? 0.0 : yG[e - nIe] - xG[e - nIe];
  }
}

__global__ void k_axpy2_masked(size_t nIe, size_t nGe, int ld, const double *__restrict__ xI,
                               const double *__restrict__ xG, double *__restrict__ yI,
                               double *__restrict__ yG, const int *__restrict__ mask) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nIe + nGe;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e % ld);
    if (!mask[c]) continue;
    if (e < nIe) yI[e] += xI[e];
    else yG[e - nIe] += xG[e - nIe];
  }
}

// Deterministic synthetic right-hand sides for the autotuner: entry (i, c) of
// an n x nrhs column-major block, uniform in [-1, 1) from a 64-bit mix of
// (seed, c, i) (SplitMix64 finaliser).
__global__ void k_fill_rhs(int n, int nrhs, int ld, unsigned long long seed, double *__restrict__ b) {
  size_t total = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e / n), i = (int)(e % n);
    unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (1ull + (unsigned long long)c * n + i);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    b[(size_t)c * ld + i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

// Column moves for continuous batching (column-major user blocks, DD-layout
// slots): dst[i*ld + slot[j]] = src[j*lds + map[i]]  (gather),
// dst[j*ldd + map[i]] = src[i*ld + slot[j]]           (scatter).
__global__ void k_gather_cols(int n, const int *__restrict__ map, const double *__restrict__ src,
                              int lds, int ncol, const int *__restrict__ slot, int ld,
                              double *__restrict__ dst) {
  size_t total = (size_t)n * ncol;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int j = (int)(e / n), i = (int)(e % n);
    dst[(size_t)i * ld + slot[j]] = src[(size_t)j * lds + map[i]];
  }
}

__global__ void k_scatter_cols(int n, const int *__restrict__ map, const double *__restrict__ src,
                               int ld, int ncol, const int *__restrict__ slot,
                               double *__restrict__ dst, int ldd) {
  size_t total = (size_t)n * ncol;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int j = (int)(e / n), i = (int)(e % n);
    dst[(size_t)j * ldd + map[i]] = src[(size_t)i * ld + slot[j]];
  }
}

// y[:, c] = a * y[:, c] + x[:, c] for the masked columns (a = 0: copy, x = null: scale)
__global__ void k_cols_update(size_t n, int ld, double a, const double *__restrict__ x,
                              double *__restrict__ y, const int *__restrict__ mask) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    int c = (int)(e % ld);
    if (mask[c]) y[e] = a * y[e] + (x ? x[e] : 0.0);
  }
}

// Move a DD-layout block from column stride lo to column stride ln (ln, lo
// powers of two; columns >= min(lo, ln) of the destination are zeroed).
__global__ void k_relayout(int n, int lo, int ln, const double *__restrict__ src,
                           double *__restrict__ dst) {
  size_t total = (size_t)n * ln;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int i = (int)(e / ln), c = (int)(e % ln);
    dst[e] = c < lo ? src[(size_t)i * lo + c] : 0.0;
  }
}

// ------------------------------------------------------------- factor --
// Batched dense Cholesky, one workgroup per subdomain, in place on the
// column-major block (lower triangle), right-looking with 16-wide panels:
//   1. factor the 16x16 diagonal block (one wave, LDS),
//   2. panel solve L21 = A21 L11^{-T} (one thread per row),
//   3. trailing update A22 -= L21 L21^T on 16x16 tiles with MFMA
//      (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32) or vector FMA.
// status[k] receives 1 + the column of the first non-positive pivot.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma16x16x4(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef dbl4 type; };
template <> struct Vec4<float> { typedef flt4 type; };
// Row of accumulator register r held by lane group g = lane/16 (column lane%16).
// A and B operands: lane l holds A[l%16][l/16] and B[l/16][l%16] for both.
// Output: f32 16x16x4 keeps four consecutive rows per lane group,
// f64 16x16x4 interleaves them (rows g, g+4, g+8, g+12), as measured on gfx950.
__device__ __forceinline__ int acc_row(double, int g, int r) { return g + 4 * r; }
__device__ __forceinline__ int acc_row(float, int g, int r) { return 4 * g + r; }

constexpr int kNB = 16;

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_potrf(T *__restrict__ blocks, const long long *__restrict__ koff, const int *__restrict__ ni,
        int *__restrict__ status, int use_mfma) {
  __shared__ T D[kNB][kNB + 1];
  const int k = blockIdx.x;
  const int n = ni[k];
  T *A = blocks + koff[k];
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  int fail = 0;
  for (int k0 = 0; k0 < n; k0 += kNB) {
    const int kb = min(kNB, n - k0);
    // 1. diagonal block
    for (int e = tid; e < kNB * kNB; e += kBlock) {
      int i = e % kNB, j = e / kNB;
      D[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + j) * n + k0 + i] : T(0);
    }
    __syncthreads();
    if (wv == 0) {
      for (int j = 0; j < kb; ++j) {
        T d = D[j][j];
        if (!(d > T(0))) {
          if (lane == 0 && fail == 0) fail = k0 + j + 1;
          d = T(1);
        }
        T piv = sqrt(d);
        if (lane == 0) D[j][j] = piv;
        if (lane > j && lane < kb) D[lane][j] = D[lane][j] / piv;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        // rank-1 update of the remaining lower part of the block
        for (int e = lane; e < kNB * kNB; e += kWave) {
          int i = e % kNB, l = e / kNB;
          if (l > j && i >= l && i < kb) D[i][l] -= D[i][j] * D[l][j];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    for (int e = tid; e < kNB * kNB; e += kBlock) {
      int i = e % kNB, j = e / kNB;
      if (i < kb && j < kb && i >= j) A[(size_t)(k0 + j) * n + k0 + i] = D[i][j];
    }
    // 2. panel: rows below the block
    for (int i = k0 + kb + tid; i < n; i += kBlock) {
      T xr[kNB];
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (j < kb) {
          T a = A[(size_t)(k0 + j) * n + i];
          for (int q = 0; q < j; ++q) a -= xr[q] * D[j][q];
          xr[j] = a / D[j][j];
        }
      }
#pragma unroll
      for (int j = 0; j < kNB; ++j)
        if (j < kb) A[(size_t)(k0 + j) * n + i] = xr[j];
    }
    __threadfence_block();
    __syncthreads();
    // 3. trailing update on 16x16 tiles of the lower triangle
    const int t0 = k0 + kb;
    const int m = n - t0;
    if (m > 0) {
      const int T16 = (m + 15) / 16;
      const int ntiles = T16 * (T16 + 1) / 2;
      for (int t = wv; t < ntiles; t += kWavesPerBlock) {
        // tile (ti, tj), tj <= ti, enumerated row by row
        int ti = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
        while (ti * (ti + 1) / 2 > t) --ti;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        int tj = t - ti * (ti + 1) / 2;
        int i0 = t0 + 16 * ti, j0 = t0 + 16 * tj;
        int ci = lane % 16, rq = lane / 16;           // fragment coordinates
        typename Vec4<T>::type acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int i = i0 + acc_row(T(0), rq, r), j = j0 + ci;
          acc[r] = (i < n && j < n) ? A[(size_t)j * n + i] : T(0);
        }
        if (use_mfma) {
#pragma unroll
          for (int kk = 0; kk < kNB; kk += 4) {
            int q = kk + rq;
            int ia = i0 + ci, jb = j0 + ci;
            T a = (q < kb && ia < n) ? -A[(size_t)(k0 + q) * n + ia] : T(0);
            T b = (q < kb && jb < n) ? A[(size_t)(k0 + q) * n + jb] : T(0);
            acc = mfma16x16x4(a, b, acc);
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            int i = i0 + acc_row(T(0), rq, r), j = j0 + ci;
            if (i < n && j < n) {
              T s = acc[r];
              for (int q = 0; q < kb; ++q)
                s -= A[(size_t)(k0 + q) * n + i] * A[(size_t)(k0 + q) * n + j];
              acc[r] = s;
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int i = i0 + acc_row(T(0), rq, r), j = j0 + ci;
          if (i < n && j < n && i >= j) A[(size_t)j * n + i] = acc[r];
        }
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  if (wv == 0 && lane == 0) status[k] = fail;
}

// Blocked triangular solves with the factor of one subdomain, applied to an
// n x ncol block B (element (i,t) at B[i*rs + t*cs]), in place:
//   forward  L X = B, then backward  L^T Y = X   (Y = K_II^{-1} B).
// 16-row blocks: the diagonal triangle is solved per column by one thread,
// the rows beyond it are updated in parallel.
template <typename LT, typename BT, typename AT>
__device__ void trsm_llt(const LT *__restrict__ L, int n, BT *B, int rs, int cs, int ncol) {
  // forward
  for (int jb = 0; jb < n; jb += kNB) {
    int nb = min(kNB, n - jb);
    for (int t = threadIdx.x; t < ncol; t += kBlock) {
      for (int r = 0; r < nb; ++r) {
        int i = jb + r;
        AT s = (AT)B[(size_t)i * rs + (size_t)t * cs];
        for (int q = 0; q < r; ++q)
          s -= (AT)L[(size_t)(jb + q) * n + i] * (AT)B[(size_t)(jb + q) * rs + (size_t)t * cs];
        B[(size_t)i * rs + (size_t)t * cs] = (BT)(s / (AT)L[(size_t)i * n + i]);
      }
    }
    __threadfence_block();
    __syncthreads();
    int rem = n - (jb + nb);
    for (int e = threadIdx.x; e < rem * ncol; e += kBlock) {
      int i = jb + nb + e / ncol, t = e % ncol;
      AT s = (AT)B[(size_t)i * rs + (size_t)t * cs];
      for (int q = 0; q < nb; ++q)
        s -= (AT)L[(size_t)(jb + q) * n + i] * (AT)B[(size_t)(jb + q) * rs + (size_t)t * cs];
      B[(size_t)i * rs + (size_t)t * cs] = (BT)s;
    }
    __threadfence_block();
    __syncthreads();
  }
  // backward
  int last = ((n - 1) / kNB) * kNB;
  for (int jb = last; jb >= 0; jb -= kNB) {
    int nb = min(kNB, n - jb);
    for (int t = threadIdx.x; t < ncol; t += kBlock) {
      for (int r = nb - 1; r >= 0; --r) {
        int i = jb + r;
        AT s = (AT)B[(size_t)i * rs + (size_t)t * cs];
        for (int q = r + 1; q < nb; ++q)
          s -= (AT)L[(size_t)i * n + jb + q] * (AT)B[(size_t)(jb + q) * rs + (size_t)t * cs];
        B[(size_t)i * rs + (size_t)t * cs] = (BT)(s / (AT)L[(size_t)i * n + i]);
      }
    }
    __threadfence_block();
    __syncthreads();
    for (int e = threadIdx.x; e < jb * ncol; e += kBlock) {
      int i = e / ncol, t = e % ncol;
      AT s = (AT)B[(size_t)i * rs + (size_t)t * cs];
      const LT *Lc = L + (size_t)i * n + jb;   // L[jb+q][i], q < nb: contiguous
      for (int q = 0; q < nb; ++q) s -= (AT)Lc[q] * (AT)B[(size_t)(jb + q) * rs + (size_t)t * cs];
      B[(size_t)i * rs + (size_t)t * cs] = (BT)s;
    }
    __threadfence_block();
    __syncthreads();
  }
}

// The same factorisation split into two launches per 16-wide panel so the
// trailing updates of all subdomains spread over the whole GPU (one
// workgroup per subdomain leaves most CUs idle).  Same arithmetic as k_potrf
// step for step, so the factor is bit-identical.
// Panel k0 = 16 * J: factor the diagonal block and solve the rows below it.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_potrf_panel(T *__restrict__ blocks, const long long *__restrict__ koff,
              const int *__restrict__ ni, int *__restrict__ status, int J) {
  __shared__ T D[kNB][kNB + 1];
  const int k = blockIdx.x;
  const int n = ni[k];
  const int k0 = kNB * J;
  if (k0 >= n) return;
  T *A = blocks + koff[k];
  const int tid = threadIdx.x, lane = lane_id(), wv = wave_id();
  const int kb = min(kNB, n - k0);
  int fail = 0;
  for (int e = tid; e < kNB * kNB; e += kBlock) {
    int i = e % kNB, j = e / kNB;
    D[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + j) * n + k0 + i] : T(0);
  }
  __syncthreads();
  if (wv == 0) {
    for (int j = 0; j < kb; ++j) {
      T d = D[j][j];
      if (!(d > T(0))) {
        if (lane == 0 && fail == 0) fail = k0 + j + 1;
        d = T(1);
      }
      T piv = sqrt(d);
      if (lane == 0) D[j][j] = piv;
      if (lane > j && lane < kb) D[lane][j] = D[lane][j] / piv;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (int e = lane; e < kNB * kNB; e += kWave) {
        int i = e % kNB, l = e / kNB;
        if (l > j && i >= l && i < kb) D[i][l] -= D[i][j] * D[l][j];
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0 && fail && status[k] == 0) status[k] = fail;
  }
  __syncthreads();
  for (int e = tid; e < kNB * kNB; e += kBlock) {
    int i = e % kNB, j = e / kNB;
    if (i < kb && j < kb && i >= j) A[(size_t)(k0 + j) * n + k0 + i] = D[i][j];
  }
  for (int i = k0 + kb + tid; i < n; i += kBlock) {
    T xr[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
      if (j < kb) {
        T a = A[(size_t)(k0 + j) * n + i];
        for (int q = 0; q < j; ++q) a -= xr[q] * D[j][q];
        xr[j] = a / D[j][j];
      }
    }
#pragma unroll
    for (int j = 0; j < kNB; ++j)
      if (j < kb) A[(size_t)(k0 + j) * n + i] = xr[j];
  }
}

// The whole factorisation (the Cholesky factors K_II^k = L_k L_k^T of eq.
// splittingBlockCholesky) in one launch, left-looking by 16-wide block
// columns: one workgroup per (subdomain k, block column J) computes
//   A[J:, J] -= sum_{Q < J} L[J:, Q] L[J, Q]^T,   L[J][J] = chol(A[J][J]),
//   L[I][J] = A[I][J] L[J][J]^{-T}  (I > J),
// the last step as the MFMA product L[I][J]^T = L[J][J]^{-1} A[I][J]^T with the
// inverted diagonal block (which is also X[J][J] of X = L^{-1}, written to Xd
// when given, row-major).  Wave w keeps its row tiles I = J + w + 4m,
// m < OWN, in accumulator registers across the whole sum.
//
// Workgroups take tickets t = J * n_sub + k in the order they start, so a
// workgroup only ever waits for block columns of smaller tickets, which have
// already started: the waits cannot deadlock whatever the residency.  A
// finished block column is written with device-coherent stores, waited for
// (vmcnt 0) and published in done[k * ntmax + J]; its tile (J+1, J) is
// published first in done[(n_sub + k) * ntmax + J], which is all the next
// column's diagonal tile needs, so that column factors its diagonal block
// while this one is still storing the rest.  Readers poll the flags with
// device-coherent loads (64 flags per poll) and read the columns the same way,
// so no cache write-back or invalidate is involved.  Every poll is bounded:
// after `spin` sleeps (kFlowSpin unless the host sets a smaller limit) the wave
// raises *timeout and stops waiting, so the launch always drains (the factor
// is then garbage and the host reports it).
// A non-positive pivot raises status[k] = column + 1 unless a smaller column
// of the same subdomain already did: the status store of column J settles
// before J's early flag, which column J+1 waits for before its own pivots.
constexpr int kFlowSpin = 1 << 18;
// Value of v in lane l (l uniform) as a wave-uniform scalar.
__device__ __forceinline__ double bcast_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float bcast_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <typename T>
__device__ __forceinline__ T load_coherent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_coherent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T, int OWN>
__global__ void __launch_bounds__(kBlock)
k_potrf_flow(T *__restrict__ blocks, const long long *__restrict__ koff, const int *__restrict__ ni,
             int n_sub, int ntmax, int *__restrict__ status, unsigned *__restrict__ ticket,
             int *__restrict__ done, int *__restrict__ timeout, T *__restrict__ Xd, int spin) {
  typedef typename Vec4<T>::type V4;
  __shared__ int s_ticket;
  __shared__ T D[16][17];                    // diagonal block, then its factor
  __shared__ T Di[16][17];                   // inverse of the factor's diagonal block
  __shared__ T S[kWavesPerBlock][16][17];    // per-wave tile transpose
  if (threadIdx.x == 0) s_ticket = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int k = s_ticket % n_sub, J = s_ticket / n_sub;
  const int n = ni[k], nt = (n + 15) / 16;
  if (J >= nt) return;
  T *A = blocks + koff[k];                   // column-major: A[i][j] at j * n + i
  int *dk = done + (size_t)k * ntmax;                       // column finished
  int *ek = done + (size_t)(n_sub + k) * ntmax;             // its first tile below the diagonal stored
  const int lane = lane_id(), c = lane % 16, g = lane / 16, w = wave_id();
  const int cj = 16 * J + c;
  V4 acc[OWN];
#pragma unroll
  for (int m = 0; m < OWN; ++m) {
    const int I = J + w + 4 * m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + acc_row(T(0), g, r);
      acc[m][r] = (I < nt && row < n && cj < n) ? A[(size_t)cj * n + row] : T(0);
    }
  }
  // wait until block column Q is finished (flags polled 64 at a time), bounded
  int avail = 0;                             // block columns known finished
  bool waited_out = false;
  auto wait_done = [&](int Q) {
    if (Q < avail) return;
    unsigned long long fin = 0;
    for (int it = 0;; ++it) {
      const int f = (Q + lane < J) ? load_coherent(dk + Q + lane) : 0;
      fin = __ballot(f != 0);
      if ((fin & 1ull) || waited_out) break;
      if (it >= spin) {
        waited_out = true;
        if (lane == 0) store_coherent(timeout, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    avail = waited_out ? J : Q + (~fin == 0ull ? 64 : __builtin_ctzll(~fin));
  };
  // subtract L[I][Q] L[J][Q]^T from the row tiles m0 <= m < m1 of this wave
  auto update = [&](int Q, int m0, int m1) {
    const T *col = A + (size_t)(16 * Q + 4 * g) * n;
    T b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = cj < n ? load_coherent(col + (size_t)t * n + cj) : T(0);
#pragma unroll
    for (int m = 0; m < OWN; ++m) {
      const int I = J + w + 4 * m;
      if (m >= m0 && m < m1 && I < nt) {
        const int row = 16 * I + c;
        T a[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = row < n ? -load_coherent(col + (size_t)t * n + row) : T(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[m] = mfma16x16x4(a[t], b[t], acc[m]);
      }
    }
  };
  for (int Q = 0; Q + 1 < J; ++Q) {
    wait_done(Q);
    update(Q, 0, OWN);
  }
  if (J > 0 && w == 0) {
    // the diagonal tile needs only tile (J, J-1) of the last column, which its
    // owner publishes (early flag) before the rest of that column
    for (int it = 0;; ++it) {
      if (waited_out || load_coherent(ek + J - 1) != 0) break;
      if (it >= spin) {
        waited_out = true;
        if (lane == 0) store_coherent(timeout, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    update(J - 1, 0, 1);
  }
  const int kb = min(16, n - 16 * J);
  if (w == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) D[acc_row(T(0), g, r)][c] = acc[0][r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // Cholesky of the diagonal block in registers: lane l < 16 holds row l;
    // step j broadcasts the pivot and column j lane by lane (v_readlane).  Entries right of
    // the diagonal become garbage and are never read.
    T a[16], rd[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = D[lane % 16][q];
    int fail = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      rd[j] = T(1);                          // identity past the block's end
      if (j < kb) {
        T d = bcast_lane(a[j], j);
        if (!(d > T(0))) {
          if (fail == 0) fail = 16 * J + j + 1;
          d = T(1);
        }
        const T piv = sqrt(d);
        rd[j] = T(1) / piv;
        if (lane == j) a[j] = piv;
        else if (lane > j) a[j] *= rd[j];
#pragma unroll
        for (int m = j + 1; m < 16; ++m) {
          const T lmj = bcast_lane(a[j], m);
          if (lane > j) a[m] -= a[j] * lmj;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    if (lane < 16) {
#pragma unroll
      for (int q = 0; q < 16; ++q) D[lane][q] = q < lane ? a[q] : (q == lane && lane < kb ? a[q] : T(0));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // column `lane` of the inverse by forward substitution (reciprocal pivots)
    T y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      T v = T(i == lane ? 1 : 0);
#pragma unroll
      for (int q = 0; q < i; ++q) v -= D[i][q] * y[q];
      y[i] = v * rd[i];
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) Di[i][lane] = y[i];
    }
    if (fail && lane == 0 && load_coherent(status + k) == 0) store_coherent(status + k, fail);
    for (int e = lane; e < 256; e += kWave) {
      const int i = e % 16, j = e / 16;
      if (i < kb && j < kb && i >= j) store_coherent(A + (size_t)(16 * J + j) * n + 16 * J + i, D[i][j]);
    }
  }
  if (J > 0) {                               // the rest of the last column's update
    wait_done(J - 1);
    update(J - 1, w == 0 ? 1 : 0, OWN);
  }
  if (w == 0) __builtin_amdgcn_s_waitcnt(0x0F70);   // the status store settles before the early flag
  __syncthreads();
  if (Xd && w == 0) {
    T *Xk = Xd + koff[k];
    for (int e = lane; e < 256; e += kWave) {
      const int i = e / 16, j = e % 16;
      if (i < kb && j < kb) Xk[(size_t)(16 * J + i) * n + 16 * J + j] = Di[i][j];
    }
  }
  T da[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) da[t] = Di[c][4 * g + t];
#pragma unroll
  for (int m = 0; m < OWN; ++m) {
    const int I = J + w + 4 * m;
    if (I > J && I < nt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) S[w][acc_row(T(0), g, r)][c] = acc[m][r];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      T bt[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bt[t] = S[w][c][4 * g + t];
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      V4 z;
#pragma unroll
      for (int r = 0; r < 4; ++r) z[r] = T(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) z = mfma16x16x4(da[t], bt[t], z);
      const int row = 16 * I + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int colj = 16 * J + acc_row(T(0), g, r);
        if (row < n && colj < n) store_coherent(A + (size_t)colj * n + row, z[r]);
      }
      if (w == 1 && m == 0) {                // tile (J+1, J): early flag of this column
        __builtin_amdgcn_s_waitcnt(0x0F70);
        if (lane == 0) store_coherent(ek + J, 1);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);        // vmcnt(0): this thread's stores are done
  __syncthreads();
  if (threadIdx.x == 0) store_coherent(dk + J, 1);
}

// Trailing update of panel J: A22 -= L21 L21^T on the 16x16 lower tiles of
// every subdomain; grid (tile chunks, subdomains), one wave per tile.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_potrf_update(T *__restrict__ blocks, const long long *__restrict__ koff,
               const int *__restrict__ ni, int J, int use_mfma) {
  const int k = blockIdx.y;
  const int n = ni[k];
  const int k0 = kNB * J;
  const int kb = min(kNB, n - k0);
  const int t0 = k0 + kb;
  const int m = n - t0;
  if (kb <= 0 || m <= 0) return;
  const int T16 = (m + 15) / 16;
  const int ntiles = T16 * (T16 + 1) / 2;
  const int t = blockIdx.x * kWavesPerBlock + wave_id();
  if (t >= ntiles) return;
  T *A = blocks + koff[k];
  const int lane = lane_id();
  int ti = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while (ti * (ti + 1) / 2 > t) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  int tj = t - ti * (ti + 1) / 2;
  int i0 = t0 + 16 * ti, j0 = t0 + 16 * tj;
  int ci = lane % 16, rq = lane / 16;
  typename Vec4<T>::type acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int i = i0 + acc_row(T(0), rq, r), j = j0 + ci;
    acc[r] = (i < n && j < n) ? A[(size_t)j * n + i] : T(0);
  }
  if (use_mfma) {
#pragma unroll
    for (int kk = 0; kk < kNB; kk += 4) {
      int q = kk + rq;
      int ia = i0 + ci, jb = j0 + ci;
      T a = (q < kb && ia < n) ? -A[(size_t)(k0 + q) * n + ia] : T(0);
      T b = (q < kb && jb < n) ? A[(size_t)(k0 + q) * n + jb] : T(0);
      acc = mfma16x16x4(a, b, acc);
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i = i0 + acc_row(T(0), rq, r), j = j0 + ci;
      if (i < n && j < n) {
        T sv = acc[r];
        for (int q = 0; q < kb; ++q)
          sv -= A[(size_t)(k0 + q) * n + i] * A[(size_t)(k0 + q) * n + j];
        acc[r] = sv;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int i = i0 + acc_row(T(0), rq, r), j = j0 + ci;
    if (i < n && j < n && i >= j) A[(size_t)j * n + i] = acc[r];
  }
}

// ------------------------------------------------ explicit inverse on MFMA --
// K_II^{-1} = L^{-T} L^{-1} in two steps, both on the matrix cores:
//   1. X = L^{-1} (lower triangular, stored row-major: X[r][c] at r*n + c),
//      one wave per (subdomain, 16-column tile C), block forward substitution
//        X_RC = L_RR^{-1} (delta_RC I - sum_{C <= Q < R} L_RQ X_QC),
//      the sum on MFMA 16x16x4 (q in steps of 4, increasing), the 16x16
//      triangular solve with L_RR in LDS;
//   2. K_II^{-1} = X^T X, one wave per 16x16 output tile (I >= J):
//        (X^T X)_ij = sum_{r >= 16 I} X[r][i] X[r][j]   (r in steps of 4),
//      written to both halves of the symmetric block (row i = column i).
// Operand layout of v_mfma_{f64,f32}_16x16x4: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; accumulator register r of lane l is row acc_row(g, r) of
// column l%16, g = l/16.
template <typename T>
__global__ void __launch_bounds__(kWave)
k_trtri(const T *__restrict__ L, T *__restrict__ X, const long long *__restrict__ koff,
        const int *__restrict__ ni) {
  const int k = blockIdx.x, C = blockIdx.y;
  const int n = ni[k];
  const int nt = (n + 15) / 16;
  if (C >= nt) return;
  const T *Lk = L + koff[k];          // column-major: L[i][j] at j*n + i
  T *Xk = X + koff[k];                // row-major
  __shared__ T S[16][17];             // right-hand side, then solution, of one block row
  __shared__ T D[16][17];             // diagonal block L_RR
  const int lane = threadIdx.x, ci = lane % 16, g = lane / 16;
  const int c0 = 16 * C;
  const int jc = c0 + ci;             // this lane's column of the tile
  // rows above the tile's diagonal block are zero
  for (int e = lane; e < c0 * 16; e += kWave) {
    const int r = e / 16, j = c0 + e % 16;
    if (j < n) Xk[(size_t)r * n + j] = T(0);
  }
  for (int R = C; R < nt; ++R) {
    const int r0 = 16 * R;
    // diagonal block of L into LDS (zero outside the matrix)
    for (int e = lane; e < 256; e += kWave) {
      const int i = e % 16, j = e / 16;
      D[i][j] = (r0 + i < n && r0 + j < n) ? Lk[(size_t)(r0 + j) * n + r0 + i] : T(0);
    }
    typename Vec4<T>::type acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = T(0);
    // acc = - sum_{c0 <= q < r0} L[r0+i][q] X[q][c0+j]
    const int ia = r0 + ci;
    for (int q0 = c0; q0 < r0; q0 += 4) {
      const int q = q0 + g;
      const T a = ia < n ? -Lk[(size_t)q * n + ia] : T(0);
      const T b = jc < n ? Xk[(size_t)q * n + jc] : T(0);
      acc = mfma16x16x4(a, b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = acc_row(T(0), g, r);
      T v = acc[r];
      if (R == C && i == ci) v += T(1);
      S[i][ci] = v;
    }
    __syncthreads();
    // forward substitution L_RR Y = S, the 16 columns in parallel
    if (lane < 16) {
      for (int i = 0; i < 16 && r0 + i < n; ++i) {
        T sv = S[i][lane];
        for (int q = 0; q < i; ++q) sv -= D[i][q] * S[q][lane];
        S[i][lane] = sv / D[i][i];
      }
    }
    __syncthreads();
    for (int e = lane; e < 256; e += kWave) {
      const int i = e / 16, j = e % 16;
      const int r = r0 + i, cc = c0 + j;
      if (r < n && cc < n) Xk[(size_t)r * n + cc] = r >= cc ? S[i][j] : T(0);
    }
    __threadfence_block();      // the stored rows feed the next block rows of this wave
    __syncthreads();
  }
}

// X = L^{-1} (for the explicit K_II^{-1} = X^T X applied in every interior
// solve, eq. splittingBlockCholesky) in two launches (the one-wave-per-block-
// column k_trtri above is the fallback when a block column does not fit in LDS).
//
// First the inverse of every diagonal 16x16 block, X[R][R] = L[R][R]^{-1}, one
// wave per (subdomain, block R), strict upper part zero.
template <typename T>
__global__ void __launch_bounds__(kWave)
k_trtri_diag(const T *__restrict__ L, T *__restrict__ X, const long long *__restrict__ koff,
             const int *__restrict__ ni) {
  const int k = blockIdx.x, R = blockIdx.y;
  const int n = ni[k], nt = (n + 15) / 16;
  if (R >= nt) return;
  const T *Lk = L + koff[k];          // column-major
  T *Xk = X + koff[k];                // row-major
  __shared__ T D[16][17];
  __shared__ T Y[16][17];
  const int r0 = 16 * R, m = min(16, n - r0), lane = threadIdx.x;
  for (int e = lane; e < 256; e += kWave) {
    const int i = e % 16, j = e / 16;
    D[i][j] = (i < m && j < m) ? Lk[(size_t)(r0 + j) * n + r0 + i] : T(i == j ? 1 : 0);
  }
  __syncthreads();
  if (lane < 16) {
    const int j = lane;               // column j of the inverse by forward substitution
    for (int i = 0; i < 16; ++i) {
      T v = T(i == j ? 1 : 0);
      for (int q = j; q < i; ++q) v -= D[i][q] * Y[q][j];
      Y[i][j] = i < j ? T(0) : v / D[i][i];
    }
  }
  __syncthreads();
  for (int e = lane; e < 256; e += kWave) {
    const int i = e / 16, j = e % 16;
    if (i < m && j < m) Xk[(size_t)(r0 + i) * n + r0 + j] = Y[i][j];
  }
}

// Then the blocks below the diagonal, one workgroup of four waves per
// (subdomain, block column C):
//   X[R][C] = -X[R][R] * sum_{C <= Q < R} L[R][Q] X[Q][C],   R = C+1, C+2, ...
// The column's finished blocks stay in LDS (dynamic, tiles_max * 256 + 2048
// elements), each in the B-operand order of the 16x16x4 product (element (i, j)
// at ((i / 4) * 16 + j) * 4 + i % 4, so lane 16 g + c reads its four k-steps as
// one vector).  Block Q's products belong to wave (Q - C) % 4, which is also
// the wave that finishes block Q: it alone reads the block back, so one barrier
// per block row (before the four partial sums are combined) is enough.  The
// partial sums alternate between two LDS buffers by block-row parity.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_trtri_panel(const T *__restrict__ L, T *__restrict__ X, const long long *__restrict__ koff,
              const int *__restrict__ ni) {
  typedef typename Vec4<T>::type V4;
  extern __shared__ double trtri_lds[];
  T *Yp = reinterpret_cast<T *>(trtri_lds);          // [2][4 waves][16 x 16] partial sums
  T *P = Yp + 2 * kWavesPerBlock * 256;              // finished blocks of the column
  const int k = blockIdx.x, C = blockIdx.y;
  const int n = ni[k], nt = (n + 15) / 16;
  if (C >= nt - 1) return;
  const T *Lk = L + koff[k];          // column-major
  T *Xk = X + koff[k];                // row-major
  const int lane = lane_id(), c = lane % 16, g = lane / 16, w = wave_id();
  const int c0 = 16 * C;
  for (int e = threadIdx.x; e < 256; e += kBlock) {      // block C is full (C < nt - 1)
    const int i = e / 16, j = e % 16;
    P[((i / 4) * 16 + j) * 4 + i % 4] = Xk[(size_t)(c0 + i) * n + c0 + j];
  }
  __syncthreads();
  for (int R = C + 1; R < nt; ++R) {
    const int r0 = 16 * R, row = r0 + c;
    const bool rv = row < n;
    const bool owner = w == (R - C) % kWavesPerBlock;
    T dA[4];
    if (owner) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = r0 + 4 * g + t;
        dA[t] = (rv && col < n) ? Xk[(size_t)row * n + col] : T(0);
      }
    }
    V4 acc0, acc1;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc0[r] = acc1[r] = T(0);
    int Q = C + w;
    for (; Q + kWavesPerBlock < R; Q += 2 * kWavesPerBlock) {
      const T *l0 = Lk + (size_t)(16 * Q + 4 * g) * n + row;
      const T *l1 = l0 + (size_t)16 * kWavesPerBlock * n;
      T a[8];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = rv ? l0[(size_t)t * n] : T(0);
        a[4 + t] = rv ? l1[(size_t)t * n] : T(0);
      }
      const V4 b0 = *reinterpret_cast<const V4 *>(P + (Q - C) * 256 + 4 * lane);
      const V4 b1 = *reinterpret_cast<const V4 *>(P + (Q + kWavesPerBlock - C) * 256 + 4 * lane);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc0 = mfma16x16x4(a[t], b0[t], acc0);
        acc1 = mfma16x16x4(a[4 + t], b1[t], acc1);
      }
    }
    if (Q < R) {
      const T *l0 = Lk + (size_t)(16 * Q + 4 * g) * n + row;
      T a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = rv ? l0[(size_t)t * n] : T(0);
      const V4 b0 = *reinterpret_cast<const V4 *>(P + (Q - C) * 256 + 4 * lane);
#pragma unroll
      for (int t = 0; t < 4; ++t) acc0 = mfma16x16x4(a[t], b0[t], acc0);
    }
    T *yw = Yp + (R & 1) * (kWavesPerBlock * 256) + w * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) yw[acc_row(T(0), g, r) * 16 + c] = acc0[r] + acc1[r];
    __syncthreads();
    if (owner) {
      const T *y = Yp + (R & 1) * (kWavesPerBlock * 256);
      V4 z;
#pragma unroll
      for (int r = 0; r < 4; ++r) z[r] = T(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int o = (4 * g + t) * 16 + c;
        const T b = (y[o] + y[256 + o]) + (y[512 + o] + y[768 + o]);
        z = mfma16x16x4(dA[t], b, z);
      }
      T *pr = P + (R - C) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = acc_row(T(0), g, r);
        const T v = -z[r];
        pr[((i / 4) * 16 + c) * 4 + i % 4] = v;
        if (r0 + i < n) Xk[(size_t)(r0 + i) * n + c0 + c] = v;
      }
    }
  }
}
static_assert(kWavesPerBlock == 4, "k_trtri_panel combines four partial sums");

// tiles[t] = (subdomain, I << 16 | J) for the output tiles I >= J of every block.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_gram(const T *__restrict__ X, T *__restrict__ Kinv, const long long *__restrict__ koff,
       const int *__restrict__ ni, const int2 *__restrict__ tiles, int ntiles) {
  const int t = blockIdx.x * kWavesPerBlock + wave_id();
  if (t >= ntiles) return;
  const int k = tiles[t].x;
  const int I = tiles[t].y >> 16, J = tiles[t].y & 0xffff;
  const int n = ni[k];
  const T *Xk = X + koff[k];
  T *Kk = Kinv + koff[k];
  const int lane = lane_id(), ci = lane % 16, g = lane / 16;
  const int ia = 16 * I + ci, jb = 16 * J + ci;
  // four independent accumulators over rows r0, r0 + 4, r0 + 8, r0 + 12 (the
  // loads of 16 rows go out together), summed in a fixed order at the end
  typename Vec4<T>::type acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[u][r] = T(0);
  for (int r0 = 16 * I; r0 < n; r0 += 16) {
    T a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 4 * u + g;
      a[u] = (r < n && ia < n) ? Xk[(size_t)r * n + ia] : T(0);
      b[u] = (r < n && jb < n) ? Xk[(size_t)r * n + jb] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = mfma16x16x4(a[u], b[u], acc[u]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const T v = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
    const int i = 16 * I + acc_row(T(0), g, r), j = 16 * J + ci;
    if (i < n && j < n && (I > J || i >= j)) {
      Kk[(size_t)j * n + i] = v;
      Kk[(size_t)i * n + j] = v;
    }
  }
}

// K_II^{-1} from the factor, 16 columns of the identity per workgroup:
// grid (n_sub, column chunks).
constexpr int kInvCols = 16;
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_inverse(const T *__restrict__ L, T *__restrict__ Kinv, const long long *__restrict__ koff,
          const int *__restrict__ ni) {
  const int k = blockIdx.x;
  const int n = ni[k];
  const int c0 = blockIdx.y * kInvCols;
  if (c0 >= n) return;
  const int ncol = min(kInvCols, n - c0);
  T *B = Kinv + koff[k] + (size_t)c0 * n;   // columns c0.. of the column-major block
  for (int e = threadIdx.x; e < n * ncol; e += kBlock) {
    int i = e % n, t = e / n;
    B[(size_t)t * n + i] = (i == c0 + t) ? T(1) : T(0);
  }
  __threadfence_block();
  __syncthreads();
  trsm_llt<T, T, T>(L + koff[k], n, B, 1, n, ncol);
}

// Make every block exactly symmetric: M = (M + M^T) / 2.
template <typename T>
__global__ void k_symmetrize(T *__restrict__ M, const long long *__restrict__ koff,
                             const int *__restrict__ ni) {
  const int k = blockIdx.x;
  const int n = ni[k];
  T *A = M + koff[k];
  for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < n * n; e += gridDim.y * blockDim.x) {
    int i = e % n, j = e / n;
    if (i > j) {
      T a = A[(size_t)j * n + i], b = A[(size_t)i * n + j];
      T m = (a + b) * T(0.5);
      A[(size_t)j * n + i] = m;
      A[(size_t)i * n + j] = m;
    }
  }
}

// Per-iteration interior solves by triangular sweeps (variant TRSM):
// z_I^k = L_k^{-T} L_k^{-1} y_I^k for all columns; grid (n_sub, ld / ncolw).
template <typename T, typename AT>
__global__ void __launch_bounds__(kBlock)
k_trsm_apply(const T *__restrict__ L, const long long *__restrict__ koff,
             const int *__restrict__ ioff, const int *__restrict__ ni,
             const double *__restrict__ y, double *__restrict__ z, int ld, int ncolw) {
  const int k = blockIdx.x;
  const int n = ni[k];
  const int c0 = blockIdx.y * ncolw;
  const size_t base = (size_t)ioff[k] * ld + c0;
  for (int e = threadIdx.x; e < n * ncolw; e += kBlock) {
    int i = e / ncolw, t = e % ncolw;
    z[base + (size_t)i * ld + t] = y[base + (size_t)i * ld + t];
  }
  __threadfence_block();
  __syncthreads();
  trsm_llt<T, double, AT>(L + koff[k], n, z + base, ld, 1, ncolw);
}

// Exact diagonal of S (Jacobi preconditioner), one wave per interface row j:
//   d_j = (K_GG)_jj - sum_{a,b in row j of K_GI, same subdomain} v_a v_b (K_II^k)^{-1}_{ab}
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_schur_diag(int nrows, const int *__restrict__ ptr, const int *__restrict__ split,
             const int *__restrict__ col, const double *__restrict__ val,
             const T *__restrict__ Kinv, const long long *__restrict__ koff,
             const int *__restrict__ ioff, const int *__restrict__ ni,
             const int *__restrict__ rowsub, double *__restrict__ diag,
             double *__restrict__ dinv, int *__restrict__ bad) {
  int j = blockIdx.x * kWavesPerBlock + wave_id();
  if (j >= nrows) return;
  int b = ptr[j], s = split[j], e = ptr[j + 1];
  double kjj = 0.0;
  for (int a = b + lane_id(); a < s; a += kWave)
    if (col[a] == j) kjj += val[a];
  kjj = wave_sum(kjj);
  double acc = 0.0;
  for (int a = s + lane_id(); a < e; a += kWave) {
    int ia = col[a];
    int k = rowsub[ia];
    int n = ni[k];
    const T *row = Kinv + koff[k] + (size_t)(ia - ioff[k]) * n;
    double t = 0.0;
    for (int b2 = s; b2 < e; ++b2) {
      int ib = col[b2];
      if (rowsub[ib] == k) t += (double)row[ib - ioff[k]] * val[b2];
    }
    acc += val[a] * t;
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) {
    double d = kjj - acc;
    diag[j] = d;
    if (!(d > 0.0)) { *bad = j + 1; d = 1.0; }
    dinv[j] = 1.0 / d;
  }
}

// The same diagonal (of S_k in eq. subSchurComplement, summed over the
// subdomains) on the matrix cores.  With X_k = L_k^{-1} (K_II^k = L_k L_k^T),
//   (K_GI^k (K_II^k)^{-1} K_IG^k)_jj = || X_k K_IG^k e_j ||^2,
// so each subdomain contributes the column sums of squares of W_k = X_k K_IG^k.
//
// K_IG^k is packed densely into 16-column strips of 16x16 tiles, each tile in
// the f64 16x16x4 B-operand order: element (row 16K + 4g + t, column 16J + c)
// of strip J sits at ((J * nt + K) * 256) + (16 g + c) * 4 + t, so lane
// l = 16 g + c reads its four k-steps of a tile as one 32-byte vector.
__global__ void k_pack_strips(long long n, const double *__restrict__ val,
                              const long long *__restrict__ pos, double *__restrict__ packed) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < n;
       a += (long long)gridDim.x * blockDim.x)
    atomicAdd(packed + pos[a], val[a]);      // repeated (row, column) entries add up
}

// One workgroup per strip item (k, J, K_first, K_last), the first and last row
// tiles of strip J that hold nonzeros (k < 0: padding, nothing to do).  W's row tiles I < K_first are zero;
// row tile I >= K_first sums X[I][K] V[K][J] over K_first <= K <= min(I, K_last)
// (X is lower triangular).  The row tiles go round-robin to the waves; each
// lane adds the squares of its accumulator rows, the lanes of one column and
// then the waves are combined in a fixed order, so dloc[goff[k] + 16 J + c]
// (column 16 J + c of subdomain k's local interface) has the same bits on
// every run.  X in the factor's precision, W in FP64.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_schur_wsq(const T *__restrict__ X, const double *__restrict__ packed,
            const long long *__restrict__ koff, const long long *__restrict__ voff,
            const int *__restrict__ ni, const int *__restrict__ goff, const int4 *__restrict__ items,
            double *__restrict__ dloc) {
  __shared__ double part[kWavesPerBlock][16];
  const int4 it = items[blockIdx.x];
  if (it.x < 0) return;                      // padding of the XCD-interleaved item list
  const int k = it.x, J = it.y, kf = it.z, kl = it.w;
  const int n = ni[k], nt = (n + 15) / 16;
  const int lane = lane_id(), c = lane % 16, g = lane / 16, w = wave_id();
  const T *Xk = X + koff[k];
  const double *V = packed + voff[k] + (size_t)J * nt * 256 + 4 * lane;
  double ssq = 0.0;
  for (int I = kf + w; I < nt; I += kWavesPerBlock) {
    const int row = 16 * I + c;
    const T *xr = Xk + (size_t)(row < n ? row : 0) * n;
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    const int ke = I < kl ? I : kl;
    int K = kf;
    for (; K + 1 <= ke; K += 2) {            // two row tiles per step: their loads go out together
      const int q = 16 * K + 4 * g;
      const dbl4 b0 = *reinterpret_cast<const dbl4 *>(V + (size_t)K * 256);
      const dbl4 b1 = *reinterpret_cast<const dbl4 *>(V + (size_t)(K + 1) * 256);
      double a[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int qt = q + (t < 4 ? t : 12 + t);
        a[t] = (row < n && qt < n) ? (double)xr[qt] : 0.0;
      }
      acc0 = mfma16x16x4(a[0], b0[0], acc0);
      acc1 = mfma16x16x4(a[1], b0[1], acc1);
      acc0 = mfma16x16x4(a[2], b0[2], acc0);
      acc1 = mfma16x16x4(a[3], b0[3], acc1);
      acc0 = mfma16x16x4(a[4], b1[0], acc0);
      acc1 = mfma16x16x4(a[5], b1[1], acc1);
      acc0 = mfma16x16x4(a[6], b1[2], acc0);
      acc1 = mfma16x16x4(a[7], b1[3], acc1);
    }
    if (K <= ke) {
      const int q = 16 * K + 4 * g;
      const dbl4 b = *reinterpret_cast<const dbl4 *>(V + (size_t)K * 256);
      double a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = (row < n && q + t < n) ? (double)xr[q + t] : 0.0;
      acc0 = mfma16x16x4(a[0], b[0], acc0);
      acc1 = mfma16x16x4(a[1], b[1], acc1);
      acc0 = mfma16x16x4(a[2], b[2], acc0);
      acc1 = mfma16x16x4(a[3], b[3], acc1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double v = acc0[r] + acc1[r];
      ssq += v * v;
    }
  }
  ssq += __shfl_xor(ssq, 16, kWave);
  ssq += __shfl_xor(ssq, 32, kWave);
  if (g == 0) part[w][c] = ssq;
  __syncthreads();
  if (threadIdx.x < 16) {
    const int t = threadIdx.x, jl = 16 * J + t;
    if (jl < goff[k + 1] - goff[k]) dloc[goff[k] + jl] = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
  }
}
static_assert(kWavesPerBlock == 4, "k_schur_wsq combines four waves");

// d_j = (K_GG)_jj - sum over the subdomains k next to interface dof j (in
// subdomain order) of their contributions dloc[dent[e]], dptr[j] <= e < dptr[j+1].
__global__ void k_schur_diag_sum(int nrows, const double *__restrict__ kgg_diag,
                                 const int *__restrict__ dptr, const int *__restrict__ dent,
                                 const double *__restrict__ dloc, double *__restrict__ diag,
                                 double *__restrict__ dinv, int *__restrict__ bad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  double s = 0.0;
  for (int e = dptr[j]; e < dptr[j + 1]; ++e) s += dloc[dent[e]];
  double d = kgg_diag[j] - s;
  diag[j] = d;
  if (!(d > 0.0)) { *bad = j + 1; d = 1.0; }
  dinv[j] = 1.0 / d;
}

// FP64 -> FP32 copy (mixed-precision operators).
__global__ void k_to_f32(size_t n, const double *__restrict__ a, float *__restrict__ b) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    b[e] = (float)a[e];
}

template <typename T>
__global__ void k_copy(size_t n, const T *__restrict__ a, T *__restrict__ b) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

}  // namespace dd
