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
// One workgroup per row: the window accumulates in LDS; the threads take the
// (E, F) candidates of the row in a fixed stride and integrate each pair into
// registers.  The shares of F's vertices go to the window with LDS atomics;
// those of E's three vertices, which every pair of E touches, are summed in
// registers first.  The summation order -- and the last bits -- vary between
// runs.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace dd {

constexpr int kAsmBlock = 256;
constexpr int kKerConst = 0, kKerFrac = 1, kKerPD = 2;

struct AsmProblem {
  int n, c, N;         // cells per side, collar cells, N = n + 2c
  int R, W, R1;        // window half width, 2R + 1, partner search radius in cells
  int kernel;
  double h, phi, s;
  long long thr;       // barycentre test: squared distance in (h/3)^2 units <= thr
};

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
        if constexpr (KER == kKerPD) {     // (the [1][0] entry is copied from [0][1] at the end)
          acc[4 * u + 0] += dn * b00;
          acc[4 * u + 1] += dn * b01;
          acc[4 * u + 3] += dn * b11;
        } else {
          acc[u] += g * dn;
        }
      }
    }
  }
  if constexpr (KER == kKerPD) {
#pragma unroll
    for (int u = 0; u < 6; ++u) acc[4 * u + 2] = acc[4 * u + 1];
  }
}

// One workgroup per free node: its window, accumulated in LDS (dynamic size
// W^2 or 4 W^2 doubles), then stored.
template <int KER>
__global__ void __launch_bounds__(kAsmBlock) k_assemble_2d(AsmProblem P, double *__restrict__ win) {
  extern __shared__ double sw[];
  __shared__ int se[6][2][3];       // elements holding the node: vertex coordinates
  __shared__ int nE;
  constexpr int NC = KER == kKerPD ? 4 : 1;
  const int WW = P.W * P.W * NC;
  const int row = blockIdx.x;
  const int ma = P.c + 1 + row % (P.n - 1), mb = P.c + 1 + row / (P.n - 1);
  for (int i = threadIdx.x; i < WW; i += kAsmBlock) sw[i] = 0.0;
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
  const int items = nE * per_e;
  const double off = P.c * P.h;
  // E's three vertices receive a share of every pair: their sums stay in
  // registers while this thread's items belong to the same E (ecur) and go
  // to the window when it changes (LDS atomics on those few entries would
  // serialise)
  const int W2 = P.W * P.W;
  auto add = [&](int a, int b, const double *v) {
    const int wi = (b - mb + P.R) * P.W + (a - ma + P.R);
    if constexpr (KER == kKerPD) {
      atomicAdd(&sw[(0 * W2 + wi) * 2 + 0], v[0]);
      atomicAdd(&sw[(0 * W2 + wi) * 2 + 1], v[1]);
      atomicAdd(&sw[(1 * W2 + wi) * 2 + 0], v[2]);
      atomicAdd(&sw[(1 * W2 + wi) * 2 + 1], v[3]);
    } else {
      atomicAdd(&sw[wi], v[0]);
    }
  };
  double esum[3 * NC];
  for (int j = 0; j < 3 * NC; ++j) esum[j] = 0.0;
  int ecur = -1;
  auto flush = [&]() {
    if (ecur < 0) return;
    for (int j = 0; j < 3; ++j) add(se[ecur][0][j], se[ecur][1][j], esum + j * NC);
    for (int j = 0; j < 3 * NC; ++j) esum[j] = 0.0;
  };
  for (int it = threadIdx.x; it < items; it += kAsmBlock) {
    const int e = it / per_e, f = it - e * per_e;
    if (e != ecur) {
      flush();
      ecur = e;
    }
    int ea[3], eb[3];
    for (int j = 0; j < 3; ++j) {
      ea[j] = se[e][0][j];
      eb[j] = se[e][1][j];
    }
    // cell of E: the lower-left vertex of its triangle
    const int ca = ea[0], cb = eb[0];
    const int tf = f & 1, cell = f >> 1;
    const int fa0 = ca - P.R1 + cell % span, fb0 = cb - P.R1 + cell / span;
    if (fa0 < 0 || fb0 < 0 || fa0 >= P.N || fb0 >= P.N) continue;
    int fa[3], fb[3];
    asm_tri(fa0, fb0, tf, fa, fb);
    // (|dA|, |dB| <= 3 (2 R1 + 2): 32-bit products suffice)
    const int dA = (ea[0] + ea[1] + ea[2]) - (fa[0] + fa[1] + fa[2]);
    const int dB = (eb[0] + eb[1] + eb[2]) - (fb[0] + fb[1] + fb[2]);
    if ((long long)(dA * dA + dB * dB) > P.thr) continue;
    // union of the vertices of E and F: E's three, then F's not in E
    int inF[6], ua[6], ub[6];
    for (int j = 3; j < 6; ++j) inF[j] = -1;
    int nu = 3;
    for (int j = 0; j < 3; ++j) {
      ua[j] = ea[j];
      ub[j] = eb[j];
      inF[j] = -1;
    }
    bool touching = false;
    int mF = -1, mE = 0;
    for (int j = 0; j < 3; ++j)
      if (ea[j] == ma && eb[j] == mb) mE = j;
    for (int j = 0; j < 3; ++j) {
      int dup = -1;
      for (int u = 0; u < 3; ++u)
        if (fa[j] == ea[u] && fb[j] == eb[u]) dup = u;
      if (fa[j] == ma && fb[j] == mb) mF = j;
      if (dup >= 0) {
        inF[dup] = j;
        touching = true;
      } else {
        ua[nu] = fa[j];
        ub[nu] = fb[j];
        inF[nu] = j;
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
    for (int j = 0; j < 3 * NC; ++j) esum[j] += wf * acc[j];           // E's vertices
#pragma unroll
    for (int u = 3; u < 6; ++u) {                                       // F's other vertices
      if (u >= nu) break;
      const int da = ua[u] - ma, db = ub[u] - mb;
      if (da < -P.R || da > P.R || db < -P.R || db > P.R) continue;
      double v[NC];
      for (int j = 0; j < NC; ++j) v[j] = wf * acc[u * NC + j];
      add(ua[u], ub[u], v);
    }
  }
  flush();
  __syncthreads();
  double *out = win + (size_t)row * WW;
  for (int i = threadIdx.x; i < WW; i += kAsmBlock) out[i] = sw[i];
}

}  // namespace dd
