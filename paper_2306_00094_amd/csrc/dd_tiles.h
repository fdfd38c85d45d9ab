// Wide-batch operator products on the matrix cores (gfx950).
//
// With 8 or more right-hand sides the CSR row products of the CG iteration are
// bound by their vector gathers: every nonzero fetches a whole ld-wide slice
// of the vector it multiplies, so at 32 columns the gathers move about 30
// times the bytes of the matrix.  Here the coupling matrices are stored as
// dense 16x16 tiles (block CSR over 16-row blocks) and every tile is applied
// to a 16-row slice of the multiplied vector by v_mfma_f64_16x16x4f64: a
// slice is then fetched once per tile instead of once per nonzero, and the
// matrix bytes stream once per iteration.
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
#include "dd_kernels.h"

namespace dd {

constexpr int kT = 16;   // tile edge

// Tile storage: 256 values per tile, lane l of the wave holding
// T[l % 16][4 s + l / 16] at position 4 l + s (s = 0..3), i.e. the A operand
// of step s of the 16x16x4 instruction; one 32-byte (FP64) or 16-byte (FP32)
// load per lane brings a lane's four steps.
template <typename VT> struct TileA;
template <> struct TileA<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void load(const double *p, double (&a)[4]) {
    const v4 v = __builtin_nontemporal_load((const v4 *)p);
    a[0] = v[0]; a[1] = v[1]; a[2] = v[2]; a[3] = v[3];
  }
};
template <> struct TileA<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ void load(const float *p, double (&a)[4]) {
    const v4 v = __builtin_nontemporal_load((const v4 *)p);
    a[0] = v[0]; a[1] = v[1]; a[2] = v[2]; a[3] = v[3];
  }
};

// One 16-row slice of x (rows cb*16 .. cb*16+15, DD layout with leading
// dimension ld) in the B-operand order: lane l takes row cb*16 + 4 s + l/16 and
// column q*16 + l%16 for step s and column block q.  Rows >= n and columns >=
// ld read as zero.
template <int NCB>
__device__ __forceinline__ void load_slice(const double *__restrict__ x, int n, int ld, int cb,
                                           double (&xv)[4][NCB]) {
  const int lane = lane_id(), g = lane >> 4, l16 = lane & 15;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int row = cb * kT + 4 * s + g;
#pragma unroll
    for (int q = 0; q < NCB; ++q) {
      const int col = q * kT + l16;
      xv[s][q] = (row < n && col < ld) ? x[(size_t)row * ld + col] : 0.0;
    }
  }
}

// acc[q] += T * X over the tiles [t0, t1) of one row block.  The next tile's
// operands are loaded while the current tile's instructions run.
template <typename VT, int NCB>
__device__ __forceinline__ void tile_row_acc(int t0, int t1, const int *__restrict__ tcol,
                                             const VT *__restrict__ tval, const double *__restrict__ x,
                                             int n, int ld, dbl4 (&acc)[NCB]) {
  if (t0 >= t1) return;
  const int lane = lane_id();
  double a[4], xv[4][NCB];
  TileA<VT>::load(tval + (size_t)t0 * 256 + 4 * lane, a);
  load_slice<NCB>(x, n, ld, tcol[t0], xv);
  for (int t = t0; t < t1; ++t) {
    double an[4], xn[4][NCB];
    const bool more = t + 1 < t1;
    if (more) {
      TileA<VT>::load(tval + (size_t)(t + 1) * 256 + 4 * lane, an);
      load_slice<NCB>(x, n, ld, tcol[t + 1], xn);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < NCB; ++q) acc[q] = mfma16x16x4(a[s], xv[s][q], acc[q]);
    if (more) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a[s] = an[s];
#pragma unroll
        for (int q = 0; q < NCB; ++q) xv[s][q] = xn[s][q];
      }
    }
  }
}

// Row blocks of a tiled matrix, one wave per block of 16 rows, four per
// workgroup:
//   out = base + c1 * (tiles [ptr, split) applied to x1) + c2 * (tiles [split, ptr+1) applied to x2)
// (split == nullptr: one part, tiles [ptr, ptr+1) applied to x1; base may be
// nullptr; a part whose coefficient is 0 is skipped).  x1 has n1
// rows, x2 n2 rows, out nrows rows; all three DD layout with leading dimension ld.
// With DOT the workgroup also writes its partial of x1^T out per column (its
// 64 rows summed by one fixed butterfly) to red.part2, and the last of every
// kPGroup consecutive workgroups the group sum to red.part3, which the update
// kernel reduces (the step length of the CG iteration, p^T S p).
template <typename VT, int NCB, bool DOT>
__global__ void __launch_bounds__(kBlock)
k_tile_rows(int nrb, int nrows, const int *__restrict__ ptr, const int *__restrict__ split,
            const int *__restrict__ tcol, const VT *__restrict__ tval, const double *__restrict__ x1,
            int n1, const double *__restrict__ x2, int n2, int ld, const double *__restrict__ base,
            double c1, double c2, double *__restrict__ out, RedBuf red) {
  const int wv = wave_id(), lane = lane_id(), g = lane >> 4, l16 = lane & 15;
  const int rb = blockIdx.x * kWavesPerBlock + wv;
  dbl4 acc1[NCB], acc2[NCB];
#pragma unroll
  for (int q = 0; q < NCB; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc1[q][r] = acc2[q][r] = 0.0;
  if (rb < nrb) {
    const int b = ptr[rb], e = ptr[rb + 1], s = split ? split[rb] : e;
    if (c1 != 0.0) tile_row_acc<VT, NCB>(b, s, tcol, tval, x1, n1, ld, acc1);
    if (split && c2 != 0.0) tile_row_acc<VT, NCB>(s, e, tcol, tval, x2, n2, ld, acc2);
  }
  __shared__ double prod[kWavesPerBlock * kT * kMaxLd];
#pragma unroll
  for (int q = 0; q < NCB; ++q) {
    const int col = q * kT + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = g + 4 * r;                  // row of the tile held in register r
      const int row = rb * kT + lr;
      double v = 0.0;
      if (rb < nrb && row < nrows && col < ld) {
        const size_t o = (size_t)row * ld + col;
        v = (base ? base[o] : 0.0) + c1 * acc1[q][r] + c2 * acc2[q][r];
        out[o] = v;
        if (DOT) v *= x1[(size_t)row * ld + col];
      } else {
        v = 0.0;
      }
      if (DOT && col < ld) prod[(wv * kT + lr) * ld + col] = v;
    }
  }
  if (!DOT) return;
  __syncthreads();
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    const double sm = chunk64_sum(prod, ld, c);
    if (lane == 0) store_partial(red.part2 + (size_t)blockIdx.x * ld + c, sm);
  }
  const int grp = blockIdx.x / kPGroup;
  const int members = min(kPGroup, (int)gridDim.x - grp * kPGroup);
  __shared__ int lflag;
  unsigned *cnt = red.gcount + (size_t)grp * kCounterStride;
  if (!last_of(cnt, (unsigned)members, &lflag)) return;
  for (int c = wv; c < ld; c += kWavesPerBlock) {
    const double gs = chunk_group_sum(red.part2, gridDim.x, ld, c, grp);
    if (lane == 0) store_partial(red.part3 + (size_t)grp * ld + c, gs);
  }
  __syncthreads();
  if (threadIdx.x == 0) reset_counter(cnt);
}

// Interior solve w = base + sign * K_II^-1 y on the matrix cores (or, with the
// blocks K_II themselves, the interior part of a residual): one wave per work item
// (subdomain k, 16-row tile I of its block), the tiles of block row I of the
// explicit inverse (column-major n x n at koff[k]) applied to y in column
// order.  FP64 blocks: v_mfma_f64_16x16x4f64; FP32 blocks (mixed path):
// v_mfma_f32_16x16x4f32 with FP32 operands and accumulation.
template <typename MT> struct DenseAcc;
template <> struct DenseAcc<double> {
  typedef dbl4 acc_t;
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <> struct DenseAcc<float> {
  typedef flt4 acc_t;
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

template <typename MT, int NCB>
__global__ void __launch_bounds__(kBlock)
k_dense_tiles(int nitems, const int2 *__restrict__ items, const MT *__restrict__ blocks,
              const long long *__restrict__ koff, const int *__restrict__ ioff,
              const int *__restrict__ ni, const double *__restrict__ y, int ld,
              const double *__restrict__ base, double sign, double *__restrict__ w) {
  const int it = blockIdx.x * kWavesPerBlock + wave_id();
  if (it >= nitems) return;
  const int lane = lane_id(), g = lane >> 4, l16 = lane & 15;
  const int2 item = items[it];
  const int k = item.x, r0 = item.y * kT;
  const int n = ni[k], i0 = ioff[k];
  const MT *A = blocks + koff[k];
  const double *yb = y + (size_t)i0 * ld;
  typedef typename DenseAcc<MT>::acc_t acc_t;
  acc_t acc[NCB];
#pragma unroll
  for (int q = 0; q < NCB; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[q][r] = (MT)0;
  const int ar = r0 + l16;                         // row of the A operand this lane loads
  const int nt = (n + kT - 1) / kT;
  for (int J = 0; J < nt; ++J) {
    MT a[4], b[4][NCB];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = J * kT + 4 * s + g;            // column of A = row of y
      a[s] = (ar < n && col < n) ? A[(size_t)col * n + ar] : (MT)0;
#pragma unroll
      for (int q = 0; q < NCB; ++q) {
        const int c = q * kT + l16;
        b[s][q] = (col < n && c < ld) ? (MT)yb[(size_t)col * ld + c] : (MT)0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < NCB; ++q) acc[q] = mfma16x16x4(a[s], b[s][q], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < NCB; ++q) {
    const int c = q * kT + l16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + DenseAcc<MT>::row(g, r);
      if (row < n && c < ld) {
        const size_t o = (size_t)(i0 + row) * ld + c;
        w[o] = (base ? base[o] : 0.0) + sign * (double)acc[q][r];
      }
    }
  }
}

}  // namespace dd
