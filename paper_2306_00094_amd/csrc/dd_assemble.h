// Nonlocal P1 stiffness assembly on the GPU (2D structured right-triangle
// meshes): the step that produces the matrix the substructuring solver takes.
//
// Bilinear form of the weak problem (eq. bil1):
//   A(u, v) = int int (u(y) - u(x)) (v(y) - v(x)) gamma(x, y) dy dx
// over the domain and its interaction collar, with the truncated kernels of
// eqs. constantkernel (constant), fractionalkernel (|x - y|^-(2+2s)) and
// peridynamics (the 2x2 bond tensor (x-y)(x-y)^T / |x-y|^3), all restricted
// to the interaction ball.  For nodal functions psi and an ordered element
// pair (E, F), x in E and y in F, d_n(x, y) = psi_n(y) - psi_n(x) and the pair
// adds int_E int_F d_m d_n gamma to entry (m, n).  The pair (F, E) adds the
// same (swapping x and y flips both d's), so the row of node m sums, over the
// elements E holding m and every partner F, (2 - [m is a vertex of F]) times
// the integral over (E, F).
//
// Ball truncation per element pair: E and F interact when their barycentres
// lie within delta (the barycentre approximation of the interaction ball,
// section on approximate interaction balls; per pair, so the matrix stays
// symmetric).  Each triangle integral uses the 7-point degree-5 rule
// (Radon; Strang & Fix); under the fractional kernel, pairs that share a
// vertex use the mean of the (7-point, 6-point) and (6-point, 7-point)
// product rules (6-point degree-4 rule of Dunavant 1985), so that no two
// quadrature points coincide.
//
// Output layout (one dense window per free node m = (a, b), row index
// (b - c - 1)(n - 1) + (a - c - 1)): entry for node (a + da, b + db),
// |da|, |db| <= R, at (db + R)(2R + 1) + (da + R); for the peridynamic kernel
// each entry is a 2x2 block stored [row component][window][column component].
//
// One workgroup per row.  The partner triangles F of the search squares of
// the elements E holding the row's node are spread over the threads in a
// fixed stride; each thread integrates its pair into registers.  Every sum
// has a fixed order, so the windows are the same bits from run to run:
//  - each wave accumulates into its own copy of the window in LDS.  In one
//    step of a wave its lanes hold consecutive triangles of at most two
//    squares; within one square and one triangle type (lower right / upper
//    left) the cells differ, and so does the node at any given vertex index.
//    The shares of F's vertices outside E are added in twelve steps (square,
//    type, vertex index) without two lanes touching one entry;
//  - the shares of E's three vertices, which every pair of E touches, are
//    summed per thread (one register set for even, one for odd elements),
//    then over the wave by a fixed butterfly once the wave has passed E;
//  - the copies are added in wave order when the window is stored.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace dd {

constexpr int kAsmBlock = 256;
constexpr int kKerConst = 0, kKerFrac = 1, kKerPD = 2;

constexpr int kAsmMaxW = 128;   // widest window (2R + 1) a launch takes

struct AsmProblem {
  int n, c, N;         // cells per side, collar cells, N = n + 2c
  int R, W, R1;        // window half width, 2R + 1, partner search radius in cells
  int kernel;
  double h, phi, s;
  long long thr;       // barycentre test: squared distance in (h/3)^2 units <= thr
  // Nodes a row can reach: (da, db) with da^2 + db^2 <= rr (node units).  In
  // LDS the window keeps only those, row db + R from disk[db + R] - L(db) to
  // disk[db + R] + L(db), L(db) the largest |da| in the row (asm_disk).
  long long rr;
  int WC;              // nodes kept
  int disk[kAsmMaxW];
};

// The reachable disk of the window (host).  A partner F of an element E
// holding the node m passes the barycentre test when its barycentre is
// within delta of E's; a vertex of a right triangle with legs h lies within
// sqrt(5)/3 h of the barycentre, so every vertex of F is within
// delta + 2 sqrt(5)/3 h < delta + 1.5 h of m.
inline void asm_disk(AsmProblem &P, double delta) {
  const double rho = delta / P.h + 1.5;
  P.rr = (long long)std::ceil(rho * rho);
  int acc = 0;
  for (int db = -P.R; db <= P.R; ++db) {
    P.disk[db + P.R] = acc;                // (a row out of reach keeps no node)
    if ((long long)db * db > P.rr) continue;
    int L = 0;
    while (L < P.R && (long long)(L + 1) * (L + 1) + (long long)db * db <= P.rr) ++L;
    P.disk[db + P.R] = acc + L;
    acc += 2 * L + 1;
  }
  P.WC = acc;
}

// Quadrature rules on the reference triangle: barycentric points and weights
// (summing to 1), {l0, l1, l2, w} per point; rows 0-6 the 7-point rule,
// rows 7-12 the 6-point rule.  Filled from the host (asm_rule_table) before
// each launch; read with uniform indices (scalar loads).
__constant__ double c_asm_rule[13][4];

inline void asm_rule_table(double t[13][4]) {
  // 7 points, degree 5: centroid and two 3-point orbits (a, a, b)
  const double q15 = std::sqrt(15.0);
  const double oa[2] = {(6.0 - q15) / 21.0, (6.0 + q15) / 21.0};
  const double ob[2] = {(9.0 + 2.0 * q15) / 21.0, (9.0 - 2.0 * q15) / 21.0};
  const double ow[2] = {(155.0 - q15) / 1200.0, (155.0 + q15) / 1200.0};
  t[0][0] = t[0][1] = t[0][2] = 1.0 / 3.0;
  t[0][3] = 9.0 / 40.0;
  for (int o = 0; o < 2; ++o)
    for (int k = 0; k < 3; ++k) {
      const int q = 1 + 3 * o + k;
      for (int j = 0; j < 3; ++j) t[q][j] = ((j + k) % 3 == 2) ? ob[o] : oa[o];
      t[q][3] = ow[o];
    }
  // 6 points, degree 4: two 3-point orbits (c, c, 1 - 2c)
  const double cc[2] = {0.445948490915965, 0.091576213509771};
  const double cw[2] = {0.223381589678011, 0.109951743655322};
  for (int o = 0; o < 2; ++o)
    for (int k = 0; k < 3; ++k) {
      const int q = 7 + 3 * o + k;
      for (int j = 0; j < 3; ++j) t[q][j] = ((j + k) % 3 == 2) ? 1.0 - 2.0 * cc[o] : cc[o];
      t[q][3] = cw[o];
    }
}

// Barycentric coordinate k (0..2; -1: the vertex is not in the triangle) of
// a point with coordinates l0, l1, l2 (per-lane index, uniform values).
__device__ __forceinline__ double asm_sel(int k, double l0, double l1, double l2) {
  return k == 0 ? l0 : (k == 1 ? l1 : (k == 2 ? l2 : 0.0));
}

// Vertex grid coordinates of triangle t (0: lower right, 1: upper left) of
// cell (a, b).
__device__ __forceinline__ void asm_tri(int a, int b, int t, int va[3], int vb[3]) {
  va[0] = a;
  vb[0] = b;
  va[1] = a + 1;
  vb[1] = b + t;
  va[2] = a + 1 - t;
  vb[2] = b + 1;
}

// Integral of the ordered pair (E, F) with rule QE (first point of its
// rows in c_asm_rule; NE points) on E and QF (NF points) on F, times `scale`,
// for the row of node m (vertex mE of E, vertex mF of F or -1): acc[u]
// (scalar) or acc[4u .. 4u+3] (2x2 block) for union vertex u < nu.  Union
// vertices 0-2 are E's own (vertex u of E); inF[u] is u's index in F or -1.
// The rule values are uniform (scalar operands).  F's points are the outer
// loop, so the per-lane choice of F's coordinates happens once per point of
// F; E's coordinates need no choice (vertex u of E is coordinate u) except
// for the row's node, chosen once per point of E.
template <int KER, int QE, int NE, int QF, int NF>
__device__ __forceinline__ void asm_pair(const AsmProblem &P, const double Ex[3], const double Ey[3],
                                         const double Fx[3], const double Fy[3], int mE, int mF, int nu,
                                         const int *inF, double scale, double *acc) {
  const double area = 0.5 * P.h * P.h;
  const double cst = area * area * scale * P.phi;
  double bm[NE];                         // the row node's coordinate at E's points
#pragma unroll
  for (int q = 0; q < NE; ++q)
    bm[q] = asm_sel(mE, c_asm_rule[QE + q][0], c_asm_rule[QE + q][1], c_asm_rule[QE + q][2]);
#pragma unroll 1
  for (int p = 0; p < NF; ++p) {
    const double ly0 = c_asm_rule[QF + p][0], ly1 = c_asm_rule[QF + p][1], ly2 = c_asm_rule[QF + p][2];
    const double wp = c_asm_rule[QF + p][3] * cst;
    const double am = asm_sel(mF, ly0, ly1, ly2);
    double au[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) au[u] = asm_sel(inF[u], ly0, ly1, ly2);
    double y0 = 0.0, y1 = 0.0;
    if constexpr (KER != kKerConst) {
      y0 = ly0 * Fx[0] + ly1 * Fx[1] + ly2 * Fx[2];
      y1 = ly0 * Fy[0] + ly1 * Fy[1] + ly2 * Fy[2];
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
      const double lx[3] = {c_asm_rule[QE + q][0], c_asm_rule[QE + q][1], c_asm_rule[QE + q][2]};
      const double dm = am - bm[q];
      const double w = c_asm_rule[QE + q][3] * wp;
      double g = 0.0, s0 = 0.0, s1 = 0.0, b00 = 0.0, b01 = 0.0, b11 = 0.0;
      if constexpr (KER == kKerConst) {
        g = w * dm;
      } else {
        s0 = lx[0] * Ex[0] + lx[1] * Ex[1] + lx[2] * Ex[2] - y0;
        s1 = lx[0] * Ey[0] + lx[1] * Ey[1] + lx[2] * Ey[2] - y1;
        const double r2 = s0 * s0 + s1 * s1;
        // (r2 = 0 only where the points coincide, where d_m = 0 as well)
        if (r2 > 0.0) {
          if constexpr (KER == kKerPD) g = w * dm / (r2 * sqrt(r2));
          else g = w * dm * exp2(-(1.0 + P.s) * log2(r2));   // |x - y|^-(2 + 2s); r2 > 0
        }
        if constexpr (KER == kKerPD) {
          b00 = g * s0 * s0;
          b01 = g * s0 * s1;
          b11 = g * s1 * s1;
        }
      }
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        if (u >= nu) break;
        const double dn = u < 3 ? au[u] - lx[u < 3 ? u : 0] : au[u];
        if constexpr (KER == kKerPD) {     // ([1][0] equals [0][1]: the window copies it)
          acc[4 * u + 0] += dn * b00;
          acc[4 * u + 1] += dn * b01;
          acc[4 * u + 3] += dn * b11;
        } else {
          acc[u] += g * dn;
        }
      }
    }
  }
}

// Window entries per node pair (NC) and distinct values among them (NV: the
// peridynamic 2x2 block is symmetric, [1][0] equals [0][1]); a workgroup
// holds kAsmWaves copies of NV values per reachable node in LDS.
constexpr int kAsmWaves = kAsmBlock / 64;
// Per kernel, measured on the benchmark systems (h = 1/128, 1/96, 1/160):
// kPad lays each element's candidates out in multiples of 64, so that a wave
// step stays in one element and its data is uniform over the wave (fewer
// registers, some idle lanes); kWaves is the occupancy the register
// allocation must allow (three for the fractional and peridynamic kernels,
// at the price of a few spilled registers, beats two).
template <int KER> struct AsmShape {
  static constexpr int NC = KER == kKerPD ? 4 : 1;
  static constexpr int NV = KER == kKerPD ? 3 : 1;
  static constexpr bool kPad = KER != kKerFrac;
  static constexpr int kWaves = KER == kKerConst ? 1 : 3;
};

// One workgroup per free node: its window, accumulated in LDS (dynamic size
// kAsmWaves * NV * WC doubles), then stored (zeros outside the disk).
template <int KER>
__global__ void __launch_bounds__(kAsmBlock, AsmShape<KER>::kWaves) k_assemble_2d(AsmProblem P, double *__restrict__ win) {
  constexpr int NC = AsmShape<KER>::NC, NV = AsmShape<KER>::NV;
  extern __shared__ double sw[];
  __shared__ int se[6][2][3];       // elements holding the node: vertex coordinates
  __shared__ int nE;
  __shared__ int disk[kAsmMaxW];
  const int W2 = P.W * P.W, WV = P.WC * NV;
  const int row = blockIdx.x;
  const int ma = P.c + 1 + row % (P.n - 1), mb = P.c + 1 + row / (P.n - 1);
  for (int i = threadIdx.x; i < kAsmWaves * WV; i += kAsmBlock) sw[i] = 0.0;
  if (threadIdx.x < P.W) disk[threadIdx.x] = P.disk[threadIdx.x];
  if (threadIdx.x == 0) {
    int k = 0;
    for (int ca = ma - 1; ca <= ma; ++ca)
      for (int cb = mb - 1; cb <= mb; ++cb)
        for (int t = 0; t < 2; ++t) {
          if (ca < 0 || cb < 0 || ca >= P.N || cb >= P.N) continue;
          int va[3], vb[3];
          asm_tri(ca, cb, t, va, vb);
          bool holds = false;
          for (int j = 0; j < 3; ++j) holds |= va[j] == ma && vb[j] == mb;
          if (!holds) continue;
          for (int j = 0; j < 3; ++j) {
            se[k][0][j] = va[j];
            se[k][1][j] = vb[j];
          }
          ++k;
        }
    nE = k;
  }
  __syncthreads();
  const int span = 2 * P.R1 + 1;
  const int per_e = span * span * 2;            // partner candidates of one element
  // Candidates per element as laid out over the steps: at least 64, so that
  // one wave step spans at most two elements; padded, a multiple of 64, so
  // that it spans one.
  constexpr bool kPad = AsmShape<KER>::kPad;
  const int per_p = kPad ? (per_e + 63) & ~63 : (per_e >= 64 ? per_e : 64);
  const int items = nE * per_p;
  const double off = P.c * P.h;
  const int lane = threadIdx.x & 63;
  double *mine = sw + (threadIdx.x >> 6) * WV;  // this wave's copy
  constexpr int comp[3] = {0, 1, 3};            // acc's [0][0], [0][1], [1][1] of a 2x2 block
  // shares of the vertices of E, per thread, for the elements of even and odd index
  double es[2][3 * NV];
  for (int k = 0; k < 3 * NV; ++k) es[0][k] = es[1][k] = 0.0;
  // element k's sums: butterfly over the wave, then lane 0 adds to the copy
  auto flush = [&](int k) {
    const int par = kPad ? 0 : k & 1;
#pragma unroll
    for (int q = 0; q < 3 * NV; ++q) {
      double v = par ? es[1][q] : es[0][q];
      for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) {
        const int j = q / NV, c = q - j * NV;
        const int wi = disk[se[k][1][j] - mb + P.R] + (se[k][0][j] - ma);   // (neighbours of m)
        atomicAdd(&mine[wi * NV + c], v);
      }
      if (par) es[1][q] = 0.0;
      else es[0][q] = 0.0;
    }
  };
  int ep = 0;                                   // first element not yet flushed (uniform)
  // the wave's steps: bases are uniform, so every lane runs every step
  int ecur = -1, eac[3] = {0, 0, 0}, ebc[3] = {0, 0, 0};   // padded: the wave's element
  int base0 = (int)threadIdx.x - lane;
  if constexpr (kPad) base0 = __builtin_amdgcn_readfirstlane(base0);
  for (int base = base0; base < items; base += kAsmBlock) {
    const int e0 = base / per_p;                // element of the step's first lane
    while (ep < e0) flush(ep++);                // the wave is past these elements
    const int it = base + lane;
    const int e = kPad ? e0 : it / per_p, f = it - e * per_p;
    const int tf = f & 1, cell = f >> 1;
    const int es_ = e < nE ? e : 0;
    int ea[3], eb[3];
    if constexpr (kPad) {
      if (e0 != ecur && e0 < nE) {
        ecur = e0;
        for (int j = 0; j < 3; ++j) {
          eac[j] = __builtin_amdgcn_readfirstlane(se[e0][0][j]);
          ebc[j] = __builtin_amdgcn_readfirstlane(se[e0][1][j]);
        }
      }
      for (int j = 0; j < 3; ++j) {
        ea[j] = eac[j];
        eb[j] = ebc[j];
      }
    } else {
      for (int j = 0; j < 3; ++j) {
        ea[j] = se[es_][0][j];
        eb[j] = se[es_][1][j];
      }
    }
    // the partner square: cells (x0 .. x0 + span - 1, y0 .. y0 + span - 1)
    // around E's cell (the lower-left vertex of its triangle)
    const int fa0 = ea[0] - P.R1 + cell % span, fb0 = eb[0] - P.R1 + cell / span;
    if (it >= items || f >= per_e || fa0 < 0 || fb0 < 0 || fa0 >= P.N || fb0 >= P.N) continue;
    int fa[3], fb[3];
    asm_tri(fa0, fb0, tf, fa, fb);
    // (|dA|, |dB| <= 3 (2 R1 + 2): 32-bit products suffice)
    const int dA = (ea[0] + ea[1] + ea[2]) - (fa[0] + fa[1] + fa[2]);
    const int dB = (eb[0] + eb[1] + eb[2]) - (fb[0] + fb[1] + fb[2]);
    if ((long long)(dA * dA + dB * dB) > P.thr) continue;
    // union of the vertices of E and F: E's three, then F's not in E
    // (static indices only: the array stays in registers)
    int inF[6] = {-1, -1, -1, -1, -1, -1};
    int nu = 3;
    bool touching = false;
    int mF = -1, mE = 0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (ea[j] == ma && eb[j] == mb) mE = j;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      bool dup = false;
#pragma unroll
      for (int u = 0; u < 3; ++u)
        if (fa[j] == ea[u] && fb[j] == eb[u]) {
          inF[u] = j;
          dup = true;
        }
      if (fa[j] == ma && fb[j] == mb) mF = j;
      touching |= dup;
      if (!dup) {
#pragma unroll
        for (int u = 3; u < 6; ++u)
          if (u == nu) inF[u] = j;
        ++nu;
      }
    }
    double Ex[3], Ey[3], Fx[3], Fy[3];
    for (int j = 0; j < 3; ++j) {
      Ex[j] = ea[j] * P.h - off;
      Ey[j] = eb[j] * P.h - off;
      Fx[j] = fa[j] * P.h - off;
      Fy[j] = fb[j] * P.h - off;
    }
    double acc[6 * NC];
    for (int j = 0; j < 6 * NC; ++j) acc[j] = 0.0;
    if (KER == kKerFrac && touching) {
      asm_pair<KER, 0, 7, 7, 6>(P, Ex, Ey, Fx, Fy, mE, mF, nu, inF, 0.5, acc);
      asm_pair<KER, 7, 6, 0, 7>(P, Ex, Ey, Fx, Fy, mE, mF, nu, inF, 0.5, acc);
    } else {
      asm_pair<KER, 0, 7, 0, 7>(P, Ex, Ey, Fx, Fy, mE, mF, nu, inF, 1.0, acc);
    }
    const double wf = mF >= 0 ? 1.0 : 2.0;
    const bool odd = !kPad && (e & 1);
#pragma unroll
    for (int u = 0; u < 3; ++u)                                     // E's vertices
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        const double v = wf * acc[u * NC + (NC == 1 ? 0 : comp[c])];
        if (odd) es[1][u * NV + c] += v;
        else es[0][u * NV + c] += v;
      }
    // F's other vertices, by vertex index of F: window node (or -1) and share
    int wj[3] = {-1, -1, -1};
    double fv[3 * NV];
#pragma unroll
    for (int k = 0; k < 3 * NV; ++k) fv[k] = 0.0;
#pragma unroll
    for (int u = 3; u < 6; ++u) {
      if (u >= nu) break;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (inF[u] == j) {
          const int da = fa[j] - ma, db = fb[j] - mb;
          if (da >= -P.R && da <= P.R && db >= -P.R && db <= P.R && (long long)(da * da + db * db) <= P.rr)
            wj[j] = disk[db + P.R] + da;
#pragma unroll
          for (int c = 0; c < NV; ++c) fv[j * NV + c] = wf * acc[u * NC + (NC == 1 ? 0 : comp[c])];
        }
    }
    // twelve steps (element of the step, triangle type, vertex index); in
    // each, the lanes that add hold distinct window nodes, and a wave's LDS
    // operations complete in program order (so the adds need not return:
    // nothing waits for them)
    const int de = e - e0;
#pragma unroll
    for (int d = 0; d < (kPad ? 1 : 2); ++d)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (de == d && tf == t && wj[j] >= 0)
#pragma unroll
            for (int c = 0; c < NV; ++c) atomicAdd(&mine[wj[j] * NV + c], fv[j * NV + c]);
  }
  while (ep < nE) flush(ep++);
  __syncthreads();
  // the copies in wave order; the 2x2 blocks as [row comp][window][col comp]
  const int WW = W2 * NC;
  double *out = win + (size_t)row * WW;
  for (int i = threadIdx.x; i < WW; i += kAsmBlock) {
    int wi = i, c = 0;
    if constexpr (KER == kKerPD) {
      const int rc = i / (2 * W2), rest = i - rc * 2 * W2, cc = rest & 1;
      wi = rest >> 1;
      c = rc + cc;                              // (0,0) -> 0, (0,1) and (1,0) -> 1, (1,1) -> 2
    }
    const int db = wi / P.W - P.R, da = wi - (db + P.R) * P.W - P.R;
    double v = 0.0;
    if ((long long)(da * da + db * db) <= P.rr) {
      const int idx = (disk[db + P.R] + da) * NV + c;
      v = sw[idx];
      for (int w = 1; w < kAsmWaves; ++w) v += sw[w * WV + idx];
    }
    out[i] = v;
  }
}

}  // namespace dd
