// Persistent cooperative CG kernel: the whole interface CG loop in one
// launch.  Every iteration runs four phases over all resident waves,
// separated by grid barriers:
//   A  y = K_IG p                (interior rows, p = z + beta p_prev on the fly)
//   B  w = K_II^{-1} y           (interior rows)
//   C  q = K_GG p - K_GI w       (interface rows; 16-row chunk partials of p.q)
//      -> barrier leader: alpha = rz / p.q
//   D  x += alpha p, r -= alpha q, z = D^{-1} r  (64-row chunk partials of r.z, r.r)
//      -> barrier leader: beta, convergence, loop decision
// The per-row and per-chunk arithmetic is the same as in the one-kernel-per-
// phase path, so both launch modes give bit-identical results.
//
// Memory visibility across workgroups (and XCDs, whose L2 caches are not
// coherent with each other): values produced in a phase are written with
// device-coherent stores and each writer waits for its stores before the
// barrier; after a barrier each workgroup invalidates its non-coherent cache
// lines (agent-scope acquire) before reading.  Loop state is read with
// device-coherent vector loads, never through the scalar cache.
//
// Barrier safety: every wait is bounded.  A workgroup that spins past the
// limit raises the shared abort flag; every other workgroup then leaves at
// its next barrier, so the grid always drains.
#pragma once
#include "dd_kernels.h"

namespace dd {

constexpr int kPBlock = 16 * kWave;   // 16 waves per workgroup
// Narrower unroll than the per-phase kernels: the fused kernel holds the
// registers of all phases and must fit 16 waves per workgroup.
template <int C> struct PUnroll { static constexpr int U = C == 1 ? 4 : (C <= 4 ? 2 : 1); };

__device__ __forceinline__ void store_coh(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coh(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_coh(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_coh(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

struct GridBar {
  unsigned *count;     // arrivals at the current barrier
  unsigned *gen;       // barrier generation
  unsigned *abort;     // set when a wait exceeded the limit
  long long spin_limit;
};

// Grid barrier.  The last workgroup to arrive runs leader() (with all its
// threads) before releasing the others.  Returns false if the grid aborted.
template <typename F>
__device__ __forceinline__ bool grid_barrier(const GridBar &b, int *s_role, F leader) {
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned g = __hip_atomic_load(b.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned prev = __hip_atomic_fetch_add(b.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int role = 0;
    if (__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      role = -1;
    } else if (prev == gridDim.x - 1) {
      role = 1;
    } else {
      long long n = 0;
      while (__hip_atomic_load(b.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { role = -1; break; }
        if (++n > b.spin_limit) {
          __hip_atomic_store(b.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          role = -1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_role = role;
  }
  __syncthreads();
  const int role = *s_role;
  if (role == 1) {
    leader();
    wait_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(b.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      wait_stores();
      __hip_atomic_fetch_add(b.gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
  return role >= 0;
}

template <typename VT, typename MT>
struct PArgs {
  int NI, nG, ld, nrhs, max_it, use_precond;
  // K_IG (interior rows, interface columns)
  const int *ig_ptr, *ig_col;
  const VT *ig_val;
  // interior inverse blocks
  const MT *kinv;
  const long long *koff;
  const int *ioff, *ni, *rowsub;
  // interface rows [K_GG | K_GI]
  const int *g_ptr, *g_split, *g_col;
  const VT *g_val;
  const double *dinv;
  // vectors (DD layout)
  double *x, *r, *z, *pA, *pB, *q, *y, *w;
  RedBuf red;
  ColState st;
  int *go;             // loop decision (1 = iterate), written by leaders
  GridBar bar;
};

template <int C, typename VT, typename MT, typename AT>
__global__ void __launch_bounds__(kPBlock)
k_pcg_persistent(PArgs<VT, MT> a) {
  __shared__ double lds[kRowsE * kMaxLd];
  __shared__ double sbeta[kMaxLd];
  __shared__ double salpha[kMaxLd];
  __shared__ int sact[kMaxLd];
  __shared__ int s_role;
  __shared__ int s_na;
  constexpr int WPB = kPBlock / kWave;
  const int wv = wave_id(), lane = lane_id();
  const int gw = blockIdx.x * WPB + wv, nw = gridDim.x * WPB;
  const int ld = a.ld;
  const int PC = (a.nG + kGChunk - 1) / kGChunk;   // interface chunks of phase C
  const int PD = (a.nG + kRowsE - 1) / kRowsE;     // interface chunks of phase D
  double *pA = a.pA, *pB = a.pB;
  int it = 0;
  while (load_coh(a.go)) {
    ++it;
    for (int c = threadIdx.x; c < ld; c += kPBlock) sbeta[c] = load_coh(a.st.beta + c);
    __syncthreads();
    const Src P{nullptr, a.z, pA, sbeta};
    // ---- A: y = K_IG p
    for (int row = gw; row < a.NI; row += nw) {
      int b = a.ig_ptr[row], e = a.ig_ptr[row + 1];
      for (int cp = 0; cp < ld; cp += C) {
        double acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = 0.0;
        csr_row_acc<C, VT, true, PUnroll<C>::U>(b, e, a.ig_col, a.ig_val, P, ld, cp, acc);
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = wave_sum(acc[c]);
        if (lane == 0)
#pragma unroll
          for (int c = 0; c < C; ++c) store_coh(a.y + (size_t)row * ld + cp + c, acc[c]);
      }
    }
    if (!grid_barrier(a.bar, &s_role, [] {})) return;
    // ---- B: w = K_II^{-1} y (same row arithmetic as k_dense_rows)
    for (int r = gw; r < a.NI; r += nw) {
      int k = a.rowsub[r];
      int i0 = a.ioff[k];
      int n = a.ni[k];
      const MT *rowp = a.kinv + a.koff[k] + (size_t)(r - i0) * n;
      const double *yb = a.y + (size_t)i0 * ld;
      for (int cp = 0; cp < ld; cp += C) {
        AT acc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = (AT)0;
        constexpr int U = PUnroll<C>::U;
        for (int j = lane; j < n; j += U * kWave) {
          AT av[U];
          double yv[U][C];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            int jj = j + u * kWave;
            bool ok = jj < n;
            av[u] = ok ? (AT)rowp[jj] : (AT)0;
            const double *yr = yb + (size_t)(ok ? jj : 0) * ld + cp;
#pragma unroll
            for (int c = 0; c < C; ++c) yv[u][c] = ok ? yr[c] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c] = tfma(av[u], (AT)yv[u][c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = wave_sum(acc[c]);
        if (lane == 0)
#pragma unroll
          for (int c = 0; c < C; ++c) store_coh(a.w + (size_t)r * ld + cp + c, (double)acc[c]);
      }
    }
    if (!grid_barrier(a.bar, &s_role, [] {})) return;
    // ---- C: q = K_GG p - K_GI w, store this row's direction, chunk partials of p.q
    //      (same row arithmetic, chunks and reduction tree as k_gamma_rows; a
    //      workgroup handles CPB chunks of kGChunk rows at a time)
    const Src ws{a.w, nullptr, nullptr, nullptr};
    constexpr int CPB = WPB / kGRows;
    const int NSC = (PC + CPB - 1) / CPB;
    for (int sc = blockIdx.x; sc < NSC; sc += gridDim.x) {
      const int sub = wv / kGRows;
      const int ch = sc * CPB + sub;
      const int jl = (wv % kGRows) * kGRowsPerWave + lane / kGLanes;
      const bool head = (lane & (kGLanes - 1)) == 0;
      const int j = ch * kGChunk + jl;
      for (int cp = 0; cp < ld; cp += C) {
        double a1[C], a2[C];
#pragma unroll
        for (int c = 0; c < C; ++c) { a1[c] = 0.0; a2[c] = 0.0; }
        if (j < a.nG) {
          int b = a.g_ptr[j], s = a.g_split[j], e = a.g_ptr[j + 1];
          csr_row_acc2<C, VT, true, PUnroll<C>::U, kGLanes>(b, s, e, a.g_col, a.g_val, P, ws, ld, cp,
                                                            a1, a2);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          a1[c] = group_sum<kGLanes>(a1[c]);
          a2[c] = group_sum<kGLanes>(a2[c]);
        }
        if (head) {
#pragma unroll
          for (int c = 0; c < C; ++c) {
            double prod = 0.0;
            if (j < a.nG) {
              size_t o = (size_t)j * ld + cp + c;
              double pj = fma(sbeta[cp + c], load_coh(pA + o), load_coh(a.z + o));
              double qv = a1[c] - a2[c];
              store_coh(a.q + o, qv);
              store_coh(pB + o, pj);
              prod = qv * pj;
            }
            lds[(sub * kGChunk + jl) * ld + cp + c] = prod;
          }
        }
      }
      __syncthreads();
      for (int t = wv; t < CPB * ld; t += WPB) {
        const int sub2 = t / ld, c = t - sub2 * ld;
        const int ch2 = sc * CPB + sub2;
        if (lane == 0 && ch2 < PC) {
          double s = 0.0;
          for (int rr = 0; rr < kGChunk; ++rr) s += lds[(sub2 * kGChunk + rr) * ld + c];
          store_partial(a.red.part2 + (size_t)ch2 * ld + c, s);
        }
      }
      __syncthreads();
    }
    const int G2 = (PC + kPGroup - 1) / kPGroup;
    bool ok = grid_barrier(a.bar, &s_role, [&] {
      for (int t = wv; t < G2 * ld; t += WPB) {
        const int g = t / ld, c = t - g * ld;
        double v = chunk_group_sum(a.red.part2, PC, ld, c, g);
        if (lane == 0) store_partial(a.red.part3 + (size_t)g * ld + c, v);
      }
      __syncthreads();
      for (int c = wv; c < ld; c += WPB) {
        double pq = partials_sum(a.red.part3, G2, ld, c);
        if (lane == 0) {
          double al = 0.0;
          if (load_coh(a.st.active + c)) {
            if (!(pq > 0.0)) {
              store_coh(a.st.flag, 1);
              store_coh(a.st.active + c, 0);
            } else {
              al = load_coh(a.st.rz + c) / pq;
            }
          }
          store_coh(a.st.alpha + c, al);
        }
      }
    });
    if (!ok) return;
    // ---- D: updates and chunk partials of r.z and r.r (as k_cg_update, mode 1)
    for (int c = threadIdx.x; c < ld; c += kPBlock) {
      salpha[c] = load_coh(a.st.alpha + c);
      sact[c] = load_coh(a.st.active + c);
    }
    __syncthreads();
    for (int ch = blockIdx.x; ch < PD; ch += gridDim.x) {
      const int row0 = ch * kRowsE;
      for (int e = threadIdx.x; e < kRowsE * ld; e += kPBlock) {
        int lr = e / ld, c = e - lr * ld;
        int j = row0 + lr;
        double rz = 0.0;
        if (j < a.nG) {
          size_t o = (size_t)j * ld + c;
          double rv = load_coh(a.r + o);
          bool act = sact[c] != 0;
          double zv;
          if (act) {
            double al = salpha[c];
            store_coh(a.x + o, fma(al, load_coh(pB + o), load_coh(a.x + o)));
            rv = fma(-al, load_coh(a.q + o), rv);
            store_coh(a.r + o, rv);
            zv = a.use_precond ? a.dinv[j] * rv : rv;
            store_coh(a.z + o, zv);
          } else {
            zv = load_coh(a.z + o);
          }
          rz = rv * zv;
        }
        lds[lr * ld + c] = rz;
      }
      __syncthreads();
      for (int c = wv; c < ld; c += WPB) {
        double s = chunk64_sum(lds, ld, c);
        if (lane == 0) store_partial(a.red.part0 + (size_t)ch * ld + c, s);
      }
      __syncthreads();
      for (int e = threadIdx.x; e < kRowsE * ld; e += kPBlock) {
        int lr = e / ld, c = e - lr * ld;
        int j = row0 + lr;
        double rr = 0.0;
        if (j < a.nG) { double rv = load_coh(a.r + (size_t)j * ld + c); rr = rv * rv; }
        lds[lr * ld + c] = rr;
      }
      __syncthreads();
      for (int c = wv; c < ld; c += WPB) {
        double s = chunk64_sum(lds, ld, c);
        if (lane == 0) store_partial(a.red.part1 + (size_t)ch * ld + c, s);
      }
      __syncthreads();
    }
    ok = grid_barrier(a.bar, &s_role, [&] {
      if (threadIdx.x == 0) s_na = 0;
      __syncthreads();
      for (int c = wv; c < ld; c += WPB) {
        double rz, rr;
        partials_sum2(a.red.part0, a.red.part1, PD, ld, c, rz, rr);
        if (lane == 0) {
          int act = load_coh(a.st.active + c);
          if (act) {
            store_coh(a.st.iters + c, load_coh(a.st.iters + c) + 1);
            store_coh(a.st.beta + c, rz / load_coh(a.st.rz + c));
            store_coh(a.st.rz + c, rz);
            if (rr <= load_coh(a.st.stop2 + c)) act = 0;
            store_coh(a.st.active + c, act);
          }
          store_coh(a.st.nrm2 + c, rr);
          if (act) atomicAdd(&s_na, 1);
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int go = (s_na > 0 && !load_coh(a.st.flag) && it < a.max_it) ? 1 : 0;
        store_coh(a.go, go);
      }
    });
    if (!ok) return;
    double *t = pA;
    pA = pB;
    pB = t;
  }
}

}  // namespace dd
