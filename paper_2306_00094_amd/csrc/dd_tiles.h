// Wide-batch operator products on the matrix cores (gfx950).
//
// With 8 or more right-hand sides the CSR row products of the CG iteration are
// bound by their vector gathers: every nonzero fetches a whole ld-wide slice
// of the vector it multiplies, so at 32 columns the gathers move about 30
// times the bytes of the matrix.  Here the coupling matrices are stored as
// dense units of 16 rows x 8 columns (block CSR over blocks of 16 or 32 rows
// and 8 columns: two k-steps of the 16x16x4 matrix instructions) and every
// unit is applied to an 8-row slice of the multiplied vector by
// v_mfma_f64_16x16x4f64: a slice is then fetched once per unit instead of
// once per nonzero, and the matrix bytes stream once per iteration.  (Units 8
// columns wide leave fewer stored zeros than 16x16 tiles on nonlocal
// operators: on the peridynamic interface rows 54 % of the values are
// nonzero against 47 %.)
//
// The interior solves w = K_II^-1 y, a dense product per subdomain, use the
// same instruction on 16x16 tiles of the explicit inverse (FP64), or
// v_mfma_f32_16x16x4f32 with FP32 accumulation in the mixed path.
//
// Operator of the CG iteration these kernels serve: S p summed over
// subdomains (eq. subSchurComplement, summed as in eq. SchurComplement),
// y = K_IG p, w = K_II^-1 y, q = K_GG p - K_GI w.
//
// Per output column the arithmetic depends only on that column (the matrix
// instructions compute each output element from its own row and column), so
// a column's result does not depend on the batch width among the widths this
// path serves; it differs in rounding from the CSR kernels of narrow batches.
#pragma once
#include <type_traits>

#include "dd_kernels.h"

namespace dd {

constexpr int kT = 16;   // tile edge

// Tile storage: 256 values per tile; lane l of the wave holds
// T[l % 16][4 s + l / 16], the A operand of step s (s = 0..3) of the 16x16x4
// instruction.  FP64 tiles keep steps 0-1 of lane l at 2l, 2l+1 and steps 2-3
// at 128 + 2l, 128 + 2l + 1, so that each of a wave's two 16-byte loads reads
// 1 KB contiguous (whole cache lines); FP32 tiles keep the four steps of lane
// l at 4l .. 4l+3, one 16-byte load per lane.
template <typename T> struct TileLayout;
template <> struct TileLayout<double> {
  static __host__ __device__ constexpr int pos(int l, int s) { return (s >> 1) * 128 + 2 * l + (s & 1); }
  static __host__ __device__ constexpr int lane(int p) { return (p & 127) >> 1; }
  static __host__ __device__ constexpr int step(int p) { return ((p >> 7) << 1) | (p & 1); }
};
template <> struct TileLayout<float> {
  static __host__ __device__ constexpr int pos(int l, int s) { return 4 * l + s; }
  static __host__ __device__ constexpr int lane(int p) { return p >> 2; }
  static __host__ __device__ constexpr int step(int p) { return p & 3; }
};

// Coupling units: 16 rows x kTU = 8 columns, kUV = 128 values; lane l holds
// U[l % 16][4 s + l / 16], the A operand of step s (s = 0, 1), at 2 l + s (one
// 16-byte load per lane in FP64).
constexpr int kTU = 8, kUV = kT * kTU;
struct UnitLayout {
  static __host__ __device__ constexpr int pos(int l, int s) { return 2 * l + s; }
};

// A operand of a streamed FP64 coupling unit (nontemporal loads).
__device__ __forceinline__ void unit_a(const double *unit, int lane, double (&a)[2]) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 u = __builtin_nontemporal_load((const v2 *)(unit + 2 * lane));
  a[0] = u[0];
  a[1] = u[1];
}

// FP32 copies (mixed path) interleave the RB units of an entry per lane --
// lane l holds slice h, step s at RB (2 l) + 2 h + s -- so that a lane loads
// its operands of a two-slice entry with one 16-byte load, as the FP64 units
// do per slice.
template <int RB>
__device__ __forceinline__ void entry_a32(const float *entry, int lane, float (&a)[RB][2]) {
  typedef float vt __attribute__((ext_vector_type(2 * RB)));
  const vt u = __builtin_nontemporal_load((const vt *)(entry + 2 * RB * lane));
#pragma unroll
  for (int h = 0; h < RB; ++h) {
    a[h][0] = u[2 * h];
    a[h][1] = u[2 * h + 1];
  }
}

// FP64 units (entries of RB units, UnitLayout each) -> the interleaved FP32
// copies read by entry_a32.
__global__ void k_units_to_f32(size_t nent, int RB, const double *__restrict__ in, float *__restrict__ out) {
  const size_t per = (size_t)RB * kUV;
  for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < nent * per;
       o += (size_t)gridDim.x * blockDim.x) {
    const size_t t = o / per;
    const int r = (int)(o - t * per);
    const int l = r / (2 * RB), h = (r >> 1) % RB, st = r & 1;
    out[o] = (float)in[(t * RB + h) * kUV + UnitLayout::pos(l, st)];
  }
}

// Columns of the vector slices: with NCB column blocks of 16 (ld = 16 NCB for
// NCB >= 2) lane l holds the NCB consecutive columns NCB (l % 16) + q, q < NCB,
// of each row it reads, so that one 16- or 32-byte load brings all of them
// (the q-th matrix instruction then computes the columns NCB j + q, j < 16).
// For NCB = 1 lane l holds column l % 16; at ld = 8 the lanes of columns
// 8..15 read columns 0..7 again (their products land in output columns that
// are not stored).
template <int NCB>
__device__ __forceinline__ int slice_col0(int l16, int ld) {
  return NCB == 1 ? (l16 & (ld - 1)) : NCB * l16;
}
template <int NCB>
__device__ __forceinline__ void slice_row(const double *__restrict__ p, double (&v)[NCB]) {
  if constexpr (NCB == 1) {
    v[0] = p[0];
  } else {
    typedef double vt __attribute__((ext_vector_type(NCB)));
    const vt w = *(const vt *)p;
#pragma unroll
    for (int q = 0; q < NCB; ++q) v[q] = w[q];
  }
}
template <int NCB>
__device__ __forceinline__ void slice_row(const float *__restrict__ p, float (&v)[NCB]) {
  if constexpr (NCB == 1) {
    v[0] = p[0];
  } else {
    typedef float vt __attribute__((ext_vector_type(NCB)));
    const vt w = *(const vt *)p;
#pragma unroll
    for (int q = 0; q < NCB; ++q) v[q] = w[q];
  }
}

// One 8-row slice of x (rows cb*8 .. cb*8+7, DD layout with leading
// dimension ld) in the B-operand order: lane l takes row cb*8 + 4 s + l/16 for
// step s, its columns as above.  Rows past the last row n - 1 read row n - 1
// (the unit entries they meet are zero).  The loads are unconditional, so the
// compiler can count them when it waits for a buffer.
template <int NCB>
__device__ __forceinline__ void load_slice(const double *__restrict__ x, int n, int ld, int cb,
                                           double (&xv)[2][NCB]) {
  const int lane = lane_id(), g = lane >> 4, l16 = lane & 15;
  const double *p = x + slice_col0<NCB>(l16, ld);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int row = min(cb * kTU + 4 * s + g, n - 1);
    slice_row<NCB>(p + (size_t)row * ld, xv[s]);
  }
}
// (FP32 copy of the vector: the same slices, half the bytes)
template <int NCB>
__device__ __forceinline__ void load_slice(const float *__restrict__ x, int n, int ld, int cb,
                                           float (&xv)[2][NCB]) {
  const int lane = lane_id(), g = lane >> 4, l16 = lane & 15;
  const float *p = x + slice_col0<NCB>(l16, ld);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int row = min(cb * kTU + 4 * s + g, n - 1);
    slice_row<NCB>(p + (size_t)row * ld, xv[s]);
  }
}

// acc[h][q] += U_h * X over the entries t0, t0 + st, t0 + 2 st, ... (< t1) of
// one row block, in that order (t0, t1, st uniform over the wave); entry t holds
// the RB units U_h (16-row slice h of the block) at tval + (t RB + h) kUV, all
// multiplying the same 8-row slice of x, which is loaded once.  The entries'
// column blocks are fetched 64 at a time, one per lane, and broadcast by
// readlane; D register buffers hold the operands of the next D entries while an
// entry's instructions run (the last loads of a wave repeat its last entry and
// are not used).  Scheduling barriers keep every group of loads in program
// order, so that the instructions of one buffer wait only for that buffer's
// loads, the other buffers' staying in flight.
template <int NCB, int D, int RB>
__device__ __forceinline__ void tile_row_acc(int t0, int t1, int st, const int *__restrict__ tcol,
                                             const double *__restrict__ tval, const double *__restrict__ x,
                                             int n, int ld, double sgn, dbl4 (&acc)[RB][NCB]) {
  const int cnt = t0 < t1 ? (t1 - t0 + st - 1) / st : 0;
  const int lane = lane_id();
  for (int base = 0; base < cnt; base += kWave) {
    const int nb = min(kWave, cnt - base);
    const int mycol = lane < nb ? tcol[t0 + (base + lane) * st] : 0;
    const double *tv = tval + (size_t)(t0 + base * st) * RB * kUV;
    const size_t tstride = (size_t)st * RB * kUV;
    double a[D][RB][2], xs[D][2][NCB];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int jd = min(d, nb - 1);
#pragma unroll
      for (int h = 0; h < RB; ++h) unit_a(tv + jd * tstride + h * kUV, lane, a[d][h]);
      load_slice<NCB>(x, n, ld, __builtin_amdgcn_readlane(mycol, jd), xs[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int j = 0; j < nb; j += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (j + d < nb) {
#pragma unroll
          for (int s = 0; s < 2; ++s)              // sgn = +-1: exact
#pragma unroll
            for (int q = 0; q < NCB; ++q) xs[d][s][q] *= sgn;
#pragma unroll
          for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int h = 0; h < RB; ++h)
#pragma unroll
              for (int q = 0; q < NCB; ++q) acc[h][q] = mfma16x16x4(a[d][h][s], xs[d][s][q], acc[h][q]);
        }
        __builtin_amdgcn_sched_barrier(0);
        const int jn = min(j + d + D, nb - 1);
#pragma unroll
        for (int h = 0; h < RB; ++h) unit_a(tv + jn * tstride + h * kUV, lane, a[d][h]);
        load_slice<NCB>(x, n, ld, __builtin_amdgcn_readlane(mycol, jn), xs[d]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// tile_row_acc for FP32 units (mixed path, entries interleaved as read by
// entry_a32) on v_mfma_f32_16x16x4f32: the slice is rounded to FP32, the two
// steps of an entry accumulate its 8 products per output element in FP32, and
// each entry's sums are added to the FP64 accumulators, so FP32 rounding
// enters only within one entry.  The accumulators hold rows in the FP32
// instruction's order (row 4 (l / 16) + r of lane l, register r).
template <int NCB, int D, int RB, typename XT>
__device__ __forceinline__ void tile_row_acc_f32(int t0, int t1, int st, const int *__restrict__ tcol,
                                                 const float *__restrict__ tval, const XT *__restrict__ x,
                                                 int n, int ld, double sgn, dbl4 (&acc)[RB][NCB]) {
  const int cnt = t0 < t1 ? (t1 - t0 + st - 1) / st : 0;
  const int lane = lane_id();
  const float fs = (float)sgn;
  for (int base = 0; base < cnt; base += kWave) {
    const int nb = min(kWave, cnt - base);
    const int mycol = lane < nb ? tcol[t0 + (base + lane) * st] : 0;
    const float *tv = tval + (size_t)(t0 + base * st) * RB * kUV;
    const size_t tstride = (size_t)st * RB * kUV;
    float a[D][RB][2];
    XT xs[D][2][NCB];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int jd = min(d, nb - 1);
      entry_a32<RB>(tv + jd * tstride, lane, a[d]);
      load_slice<NCB>(x, n, ld, __builtin_amdgcn_readlane(mycol, jd), xs[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int j = 0; j < nb; j += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (j + d < nb) {
          flt4 c32[RB][NCB];
#pragma unroll
          for (int h = 0; h < RB; ++h)
#pragma unroll
            for (int q = 0; q < NCB; ++q)
#pragma unroll
              for (int r = 0; r < 4; ++r) c32[h][q][r] = 0.0f;
#pragma unroll
          for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int q = 0; q < NCB; ++q) {
              const float xf = fs * (float)xs[d][s][q];        // sgn = +-1: exact
#pragma unroll
              for (int h = 0; h < RB; ++h) c32[h][q] = mfma16x16x4(a[d][h][s], xf, c32[h][q]);
            }
#pragma unroll
          for (int h = 0; h < RB; ++h)
#pragma unroll
            for (int q = 0; q < NCB; ++q)
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[h][q][r] += (double)c32[h][q][r];
        }
        __builtin_amdgcn_sched_barrier(0);
        const int jn = min(j + d + D, nb - 1);
        entry_a32<RB>(tv + jn * tstride, lane, a[d]);
        load_slice<NCB>(x, n, ld, __builtin_amdgcn_readlane(mycol, jn), xs[d]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// Row of a 16-row slice held in accumulator register r of lane group g: the
// FP64 instruction's order (g + 4 r) or the FP32 one's (4 g + r).
template <typename VT>
__device__ __forceinline__ int acc_row(int g, int r) {
  return std::is_same<VT, float>::value ? 4 * g + r : g + 4 * r;
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch; each XCD has its own
// L2).  Workgroup b takes item xcd_item(b, n) so that every XCD works through
// one contiguous eighth of the items: neighbouring row blocks, which multiply
// mostly the same vector slices, then share one L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, i = b / kXcd, q = n / kXcd, r = n % kXcd;
  return x * q + min(x, r) + i;
}

// Wave index as a uniform (scalar) value.
__device__ __forceinline__ int wave_uniform() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Waves per 16-row block: the block's tiles are dealt to them in turn and their
// partial products summed in wave order through LDS.
constexpr int kTW = 4;

// One workgroup per block of 16 rows of a tiled matrix:
//   out = base + sum over waves w of (c1 * (entries [ptr, split) of wave w applied to x1)
//                                     + c2 * (entries [split, ptr+1) of wave w applied to x2))
// (split == nullptr: one part, entries [ptr, ptr+1) applied to x1; base may be
// nullptr; a part whose coefficient is 0 is skipped) for the RB x 16 rows of
// one row block.  x1 has n1 rows, x2 n2 rows, out nrows rows; all three DD
// layout with leading dimension ld.  Wave w takes entries b + w, b + w + kTW,
// ...; the wave sums are added in wave order.  With DOT the workgroup also
// writes x1^T out over its rows (rows in order) per column to red.part2, and
// the last of every kPGroup consecutive workgroups the group sum to red.part3,
// which the update kernel reduces (the step length of the CG iteration, from
// p^T S p).  run (may be nullptr): the CG loop's flag of columns still
// iterating; when it reads 0 the launch does nothing (the loop's host runs a
// few iterations ahead of the device).  x1f, x2f (FP32 units only; may be
// nullptr): FP32 copies of x1, x2 whose slices the products load instead.
template <typename VT, int NCB, bool DOT, int D, int RB>
__global__ void __launch_bounds__(kTW * kWave)
k_tile_rows(int nrb, int nrows, const int *__restrict__ ptr, const int *__restrict__ split,
            const int *__restrict__ tcol, const VT *__restrict__ tval, const double *__restrict__ x1,
            int n1, const double *__restrict__ x2, int n2, int ld, const double *__restrict__ base,
            double c1, double c2, double *__restrict__ out, RedBuf red, const int *__restrict__ run,
            const float *__restrict__ x1f, const float *__restrict__ x2f) {
  if (run && *run == 0) return;                  // every column of the CG loop has stopped
  constexpr int H = RB * kT;                     // rows of a block
  const int wv = wave_uniform(), lane = lane_id(), g = lane >> 4, l16 = lane & 15;
  const int rb = xcd_item(blockIdx.x, nrb);
  // one accumulator: with both parts, the second part's products enter the
  // same sums with x2 negated when c2 = -c1 (exact), and the total is scaled by
  // c1; a lone part is scaled by its own coefficient.  Only c2 = +-c1 is
  // served with both parts.
  dbl4 acc[RB][NCB];
#pragma unroll
  for (int h = 0; h < RB; ++h)
#pragma unroll
    for (int q = 0; q < NCB; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[h][q][r] = 0.0;
  const int b = ptr[rb], e = ptr[rb + 1], s = split ? split[rb] : e;
  const double sg2 = (c1 != 0.0 && c2 == -c1) ? -1.0 : 1.0;
  const int nel = H * ld;
  constexpr int NF = kMaxLd * H / (kTW * kWave);
  // this thread's output elements; with DOT, their x1 values are loaded now, so
  // that the loads are done when the block's sums are (the dot product then
  // costs no memory round trip after the product)
  double xd[NF];
#pragma unroll
  for (int u = 0; u < NF; ++u) {
    const int el = threadIdx.x + u * kTW * kWave;
    const int lr = el / ld, row = rb * H + lr;
    xd[u] = (DOT && el < nel && row < nrows) ? x1[(size_t)row * ld + (el - lr * ld)] : 0.0;
  }
  if constexpr (std::is_same<VT, float>::value) {
    // (x1f, x2f: FP32 copies of x1, x2 -- the products round the slices to
    // FP32 anyway, so the sums are the same bit for bit, from half the bytes)
    if (c1 != 0.0) {
      if (x1f) tile_row_acc_f32<NCB, D, RB>(b + wv, s, kTW, tcol, tval, x1f, n1, ld, 1.0, acc);
      else tile_row_acc_f32<NCB, D, RB>(b + wv, s, kTW, tcol, tval, x1, n1, ld, 1.0, acc);
    }
    if (split && c2 != 0.0) {
      if (x2f) tile_row_acc_f32<NCB, D, RB>(s + wv, e, kTW, tcol, tval, x2f, n2, ld, sg2, acc);
      else tile_row_acc_f32<NCB, D, RB>(s + wv, e, kTW, tcol, tval, x2, n2, ld, sg2, acc);
    }
  } else {
    if (c1 != 0.0) tile_row_acc<NCB, D, RB>(b + wv, s, kTW, tcol, tval, x1, n1, ld, 1.0, acc);
    if (split && c2 != 0.0) tile_row_acc<NCB, D, RB>(s + wv, e, kTW, tcol, tval, x2, n2, ld, sg2, acc);
  }
  const double cf = c1 != 0.0 ? c1 : c2;
  __shared__ double part[kTW * H * kT * NCB];    // ld <= 16 NCB
#pragma unroll
  for (int h = 0; h < RB; ++h)
#pragma unroll
    for (int q = 0; q < NCB; ++q) {
      const int col = NCB * l16 + q;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = h * kT + acc_row<VT>(g, r);   // row of the block held in register r
        if (col < ld) part[(wv * H + lr) * ld + col] = cf * acc[h][q][r];
      }
    }
  __syncthreads();
  double fin[NF], vo[NF];
#pragma unroll
  for (int u = 0; u < NF; ++u) {
    const int el = threadIdx.x + u * kTW * kWave;
    fin[u] = vo[u] = 0.0;
    if (el < nel) {
      const int lr = el / ld, col = el - lr * ld, row = rb * H + lr;
      double v = part[el];
#pragma unroll
      for (int w = 1; w < kTW; ++w) v += part[w * nel + el];
      if (row < nrows) {
        const size_t o = (size_t)row * ld + col;
        v += base ? base[o] : 0.0;
        vo[u] = v;
        if (DOT) fin[u] = v * xd[u];
        else out[o] = v;
      }
    }
  }
  if (!DOT) return;
  // (the output is stored after this workgroup has counted itself done: the
  // completion wait before the count then covers the partial only)
  auto store_out = [&]() {
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int el = threadIdx.x + u * kTW * kWave;
      const int lr = el / ld, row = rb * H + lr;
      if (el < nel && row < nrows) out[(size_t)row * ld + (el - lr * ld)] = vo[u];
    }
  };
  __syncthreads();                               // every wave read its part: reuse it
#pragma unroll
  for (int u = 0; u < NF; ++u) {
    const int el = threadIdx.x + u * kTW * kWave;
    if (el < nel) part[el] = fin[u];
  }
  __syncthreads();
  if ((int)threadIdx.x < ld) {
    const int c = threadIdx.x;
    double sm = 0.0;
    for (int lr = 0; lr < H; ++lr) sm += part[lr * ld + c];
    store_partial(red.part2 + (size_t)rb * ld + c, sm);
  }
  const int grp = rb / kPGroup;
  const int members = min(kPGroup, (int)gridDim.x - grp * kPGroup);
  __shared__ int lflag;
  unsigned *cnt = red.gcount + (size_t)grp * kCounterStride;
  const bool last = last_of(cnt, (unsigned)members, &lflag);
  store_out();
  if (!last) return;
  // (read by the next launch: no completion wait)
  group_sums_store(red.part2, gridDim.x, ld, grp, red.part3, wv, kTW, false);
  __syncthreads();
  if (threadIdx.x == 0) reset_counter(cnt);
}

// Interior solve w = base + sign * K_II^-1 y on the matrix cores (or, with the
// blocks K_II themselves, the interior part of a residual): one workgroup per
// work item (subdomain k, 16-row tile I of its block; items[b] is the item of
// workgroup b, arranged by the host so that all items of a subdomain run on one
// XCD, and k = -1 pads).  The blocks are packed
// by k_pack_tiles into 16x16 tiles in the A-operand order, block row I of
// subdomain k at toff[k] + I * nt_k * 256 (nt_k = ceil(n_k / 16) tiles per
// row, zero padded).  Wave w applies the tiles J = w, w + kTW, ... to the
// 16-row slices of y; the wave sums are added in wave order.  FP64 blocks:
// v_mfma_f64_16x16x4f64; FP32 blocks (mixed path): v_mfma_f32_16x16x4f32 with
// FP32 operands and accumulation, the wave sums added in FP64.
template <typename MT> struct DenseAcc;
template <> struct DenseAcc<double> {
  typedef dbl4 acc_t;
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <> struct DenseAcc<float> {
  typedef flt4 acc_t;
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

// A operand of a packed interior-block tile (layout of TileLayout<MT>).
template <typename MT> struct TileAT;
template <> struct TileAT<double> {
  typedef double v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ void load(const double *tile, int lane, double (&a)[4]) {
    const v2 u = *(const v2 *)(tile + 2 * lane);
    const v2 v = *(const v2 *)(tile + 128 + 2 * lane);
    a[0] = u[0]; a[1] = u[1]; a[2] = v[0]; a[3] = v[1];
  }
};
template <> struct TileAT<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void load(const float *tile, int lane, float (&a)[4]) {
    const v4 v = *(const v4 *)(tile + 4 * lane);
    a[0] = v[0]; a[1] = v[1]; a[2] = v[2]; a[3] = v[3];
  }
};

template <typename MT, int NCB>
__global__ void __launch_bounds__(kTW * kWave)
k_dense_tiles(int nall, const int2 *__restrict__ items, const MT *__restrict__ packed,
              const long long *__restrict__ toff, const int *__restrict__ ioff,
              const int *__restrict__ ni, const double *__restrict__ y, int ld,
              const double *__restrict__ base, double sign, double *__restrict__ w,
              const int *__restrict__ run, float *__restrict__ w32) {
  if (run && *run == 0) return;                  // every column of the CG loop has stopped
  const int wv = wave_uniform(), lane = lane_id(), g = lane >> 4, l16 = lane & 15;
  const int2 item = items[blockIdx.x];
  if (item.x < 0) return;                        // padding of a short XCD list
  const int k = item.x, r0 = item.y * kT;
  const int n = ni[k], i0 = ioff[k];
  const int nt = (n + kT - 1) / kT;
  const MT *A = packed + toff[k] + (size_t)item.y * nt * 256;
  // y rows past the block (the next subdomain's, or the last row repeated at
  // the end of y) meet the zero padding of the packed tiles
  const double *yb = y + slice_col0<NCB>(l16, ld);
  typedef typename DenseAcc<MT>::acc_t acc_t;
  acc_t acc[NCB];
#pragma unroll
  for (int q = 0; q < NCB; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[q][r] = (MT)0;
  auto load = [&](int J, MT (&a)[4], MT (&b)[4][NCB]) {
    TileAT<MT>::load(A + (size_t)J * 256, lane, a);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double v[NCB];
      slice_row<NCB>(yb + (size_t)min(i0 + J * kT + 4 * s + g, nall - 1) * ld, v);
#pragma unroll
      for (int q = 0; q < NCB; ++q) b[s][q] = (MT)v[q];
    }
  };
  auto mma = [&](const MT (&a)[4], const MT (&b)[4][NCB]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < NCB; ++q) acc[q] = mfma16x16x4(a[s], b[s][q], acc[q]);
  };
  // tiles J = wv, wv + kTW, ...: two register buffers in flight, each group of
  // loads kept in program order (see tile_row_acc)
  const int cnt = wv < nt ? (nt - wv + kTW - 1) / kTW : 0;
  if (cnt > 0) {
    MT a0[4], b0[4][NCB], a1[4], b1[4][NCB];
    load(wv, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    load(wv + kTW * min(1, cnt - 1), a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    for (int j = 0; j < cnt; j += 2) {
      mma(a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      load(wv + kTW * min(j + 2, cnt - 1), a0, b0);
      __builtin_amdgcn_sched_barrier(0);
      if (j + 1 < cnt) mma(a1, b1);
      __builtin_amdgcn_sched_barrier(0);
      load(wv + kTW * min(j + 3, cnt - 1), a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __shared__ double part[kTW * kT * kT * NCB];   // ld <= 16 NCB
#pragma unroll
  for (int q = 0; q < NCB; ++q) {
    const int c = NCB * l16 + q;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (c < ld) part[(wv * kT + DenseAcc<MT>::row(g, r)) * ld + c] = (double)acc[q][r];
  }
  __syncthreads();
  const int nel = kT * ld;
  for (int el = threadIdx.x; el < nel; el += kTW * kWave) {
    const int lr = el / ld, c = el - lr * ld, row = r0 + lr;
    if (row < n) {
      double v = part[el];
#pragma unroll
      for (int u = 1; u < kTW; ++u) v += part[u * nel + el];
      const size_t o = (size_t)(i0 + row) * ld + c;
      const double wv2 = (base ? base[o] : 0.0) + sign * v;
      w[o] = wv2;
      if (w32) w32[o] = (float)wv2;          // FP32 copy for the FP32 unit products
    }
  }
}

// Packs column-major dense blocks (n_k x n_k at koff[k]) into the tile order
// of k_dense_tiles: tile (I, J) of block k at toff[k] + (I * nt + J) * 256,
// lane l holding B[16 I + l % 16][16 J + 4 s + l / 16] at position
// TileLayout<T>::pos(l, s).
template <typename T>
__global__ void k_pack_tiles(int nsub, const T *__restrict__ blocks, const long long *__restrict__ koff,
                             const long long *__restrict__ toff, const int *__restrict__ ni,
                             T *__restrict__ packed) {
  const int k = blockIdx.y;
  if (k >= nsub) return;
  const int n = ni[k], nt = (n + kT - 1) / kT;
  const long long tot = (long long)nt * nt * 256;
  const T *B = blocks + koff[k];
  T *P = packed + toff[k];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / 256), pos = (int)(e % 256);
    const int I = t / nt, J = t % nt, l = TileLayout<T>::lane(pos), s = TileLayout<T>::step(pos);
    const int i = I * kT + (l & 15), j = J * kT + 4 * s + (l >> 4);
    P[e] = (i < n && j < n) ? B[(size_t)j * n + i] : (T)0;
  }
}

}  // namespace dd
