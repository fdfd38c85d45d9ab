/*
 * Nonlocal P1 stiffness assembly on structured meshes: the seeded problem
 * generator that produces the matrices both the CPU oracle and the GPU solver
 * consume.  It holds none of the solver's arithmetic (no factorisation, no
 * Schur products, no Krylov iteration).
 *
 * Bilinear form (weak form, eq. bil1):
 *     A(u,v) = int int (u(y)-u(x)) (v(y)-v(x)) gamma(x,y) dy dx
 * over (Omega u Gamma^D)^2, with a truncated kernel gamma = phi * 1_{ball}
 * (eqs. scalarkernel / vectorkernel, kernels of eqs. constantkernel,
 * fractionalkernel, peridynamics).  For P1 nodal functions and one ordered
 * element pair (E, F), x in E and y in F, put d_n(x,y) = psi_n(y) - psi_n(x);
 * the pair contributes  int_E int_F d_m d_n gamma  to entry (m, n).  The pair
 * (F, E) contributes the same amount (swap x and y: d -> -d, gamma symmetric),
 * so the row of a node m sums, over the elements E that hold m and every
 * partner F,  (1 + [m not a vertex of F]) * c(E, F)  -- every ordered pair
 * that touches m counted once.  Each row is computed by exactly one thread in
 * a fixed order, so the result does not depend on the thread count.
 *
 * Truncation:
 *   1D  : exact band |x - y| <= delta, integrated exactly (the clipped square
 *         is split into triangles; the edge-midpoint rule is exact for the
 *         degree-2 integrand).
 *   2D  : element pairs whose barycentres are within delta (the barycentre
 *         approximate ball of the section on approximate interaction balls,
 *         taken per element pair so the matrix stays symmetric); 7-point
 *         degree-5 Gauss rule on each triangle.  Pairs that share a vertex
 *         under the fractional kernel use the symmetric mean of the (7-point,
 *         6-point) and (6-point, 7-point) product rules, so no two quadrature
 *         points coincide.
 *
 * Output: a dense window per free row.  Row of free node (a[,b]) stores the
 * entries for nodes (a+da[, b+db]) with |da|,|db| <= R at
 * index (db+R)*(2R+1) + (da+R).  For the vector (peridynamic) kernel each
 * window entry is a 2x2 block, stored [row comp][window][col comp].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { KER_CONST = 0, KER_FRAC = 1, KER_PD = 2 };

/* ------------------------------------------------------------------ 1D -- */

/* Keep the part of a convex polygon with  sx*x + sy*y <= c. */
static int clip_poly(double (*p)[2], int n, double sx, double sy, double c,
                     double (*out)[2]) {
  int m = 0;
  for (int i = 0; i < n; ++i) {
    const double *P = p[i], *Q = p[(i + 1) % n];
    double fp = sx * P[0] + sy * P[1] - c, fq = sx * Q[0] + sy * Q[1] - c;
    if (fp <= 0) { out[m][0] = P[0]; out[m][1] = P[1]; ++m; }
    if ((fp < 0 && fq > 0) || (fp > 0 && fq < 0)) {
      double t = fp / (fp - fq);
      out[m][0] = P[0] + t * (Q[0] - P[0]);
      out[m][1] = P[1] + t * (Q[1] - P[1]);
      ++m;
    }
  }
  return m;
}

/*
 * Row of free node am (extended index) for the 1D constant kernel phi on the
 * band |x-y| <= delta.  Nodes x_a = (a - c) h, a = 0..N.  win has 2R+1 slots.
 */
/* member (optional): per element e of the extended mesh a bit mask of the
 * subdomains k whose hat-Omega_k u Gamma^D_k holds it; then only pairs (e, f)
 * that both lie in subdomain `sub` count, weighted by 1 / zeta(e, f) with zeta
 * the number of subdomains holding both (eqs. zeta, bilinear-multi1). */
static int popcount64(uint64_t v) {
  int n = 0;
  while (v) { v &= v - 1; ++n; }
  return n;
}

static void row_1d(int am, int N, int c, double h, double delta, double phi,
                   int R, double *win, const uint64_t *member, int sub) {
  int R1 = (int)ceil(delta / h) + 1;
  for (int ei = 0; ei < 2; ++ei) {
    int e = am - 1 + ei;                 /* element [e, e+1] holds am */
    if (e < 0 || e >= N) continue;
    double xe = (e - c) * h;
    for (int f = e - R1; f <= e + R1; ++f) {
      if (f < 0 || f >= N) continue;
      double xf = (f - c) * h;
      /* square [xe,xe+h] x [xf,xf+h], clipped to the band */
      double sq[8][2] = {{xe, xf}, {xe + h, xf}, {xe + h, xf + h}, {xe, xf + h}};
      double t1[8][2], t2[8][2];
      int n1 = clip_poly(sq, 4, -1.0, 1.0, delta, t1);   /* y - x <= delta */
      int n2 = clip_poly(t1, n1, 1.0, -1.0, delta, t2);  /* x - y <= delta */
      if (n2 < 3) continue;
      double wf = (am == f || am == f + 1) ? 1.0 : 2.0;
      if (member) {
        const uint64_t both = member[e] & member[f];
        if (!((both >> sub) & 1u)) continue;
        wf /= (double)popcount64(both);
      }
      int verts[4] = {e, e + 1, f, f + 1};
      double acc[4] = {0, 0, 0, 0};
      for (int k = 1; k + 1 < n2; ++k) {
        const double *A = t2[0], *B = t2[k], *C = t2[k + 1];
        double area = 0.5 * fabs((B[0] - A[0]) * (C[1] - A[1]) -
                                 (C[0] - A[0]) * (B[1] - A[1]));
        if (area == 0.0) continue;
        const double *V[3] = {A, B, C};
        for (int q = 0; q < 3; ++q) {
          double x = 0.5 * (V[q][0] + V[(q + 1) % 3][0]);
          double y = 0.5 * (V[q][1] + V[(q + 1) % 3][1]);
          double w = area / 3.0;
          double lx1 = (x - xe) / h, lx0 = 1.0 - lx1;   /* psi_e, psi_{e+1} at x */
          double ly1 = (y - xf) / h, ly0 = 1.0 - ly1;   /* psi_f, psi_{f+1} at y */
          double d[4];
          for (int v = 0; v < 4; ++v) {
            int nd = verts[v];
            double dv = 0.0;
            if (nd == f) dv += ly0;
            if (nd == f + 1) dv += ly1;
            if (nd == e) dv -= lx0;
            if (nd == e + 1) dv -= lx1;
            d[v] = dv;
          }
          double dm = 0.0;
          if (am == f) dm += ly0;
          if (am == f + 1) dm += ly1;
          if (am == e) dm -= lx0;
          if (am == e + 1) dm -= lx1;
          for (int v = 0; v < 4; ++v) acc[v] += w * dm * d[v];
        }
      }
      /* a node listed twice (shared vertex) must receive its d only once */
      for (int v = 0; v < 4; ++v) {
        int dup = 0;
        for (int u = 0; u < v; ++u) dup |= (verts[u] == verts[v]);
        if (dup) continue;
        int off = verts[v] - am;
        if (off < -R || off > R) continue;  /* cannot happen for R >= R1 + 1 */
        win[off + R] += wf * phi * acc[v];
      }
    }
  }
}

/* n cells inside (0,1); collar of c cells; free nodes a = c+1 .. c+n-1. */
int nl_assemble_1d(int n, int c, double delta, double phi, int R, int nthreads,
                   double *win /* (n-1) x (2R+1) */) {
  double h = 1.0 / n;
  int N = n + 2 * c;
  if (R < (int)ceil(delta / h) + 2) return -1;
  memset(win, 0, sizeof(double) * (size_t)(n - 1) * (2 * R + 1));
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
  for (int i = 0; i < n - 1; ++i)
    row_1d(c + 1 + i, N, c, h, delta, phi, R, win + (size_t)i * (2 * R + 1), NULL, 0);
  return 0;
}

/* Rows of the subdomain matrices A^k of eq. subStiffnessMatrix (the form of
 * eq. bilinear-multi1): row p is node row_node[p] (extended index a) of
 * subdomain row_sub[p]; member[e] (e = 0..N-1) as for row_1d. */
int nl_assemble_1d_sub(int n, int c, double delta, double phi, int R, int nthreads,
                       const uint64_t *member, int P, const int *row_node, const int *row_sub,
                       double *win /* P x (2R+1) */) {
  double h = 1.0 / n;
  int N = n + 2 * c;
  if (R < (int)ceil(delta / h) + 2) return -1;
  memset(win, 0, sizeof(double) * (size_t)P * (2 * R + 1));
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
  for (int p = 0; p < P; ++p)
    row_1d(row_node[p], N, c, h, delta, phi, R, win + (size_t)p * (2 * R + 1), member, row_sub[p]);
  return 0;
}

/* ------------------------------------------------------------------ 2D -- */

typedef struct { int np; double l[7][3]; double w[7]; } rule_t;

static rule_t rule7, rule6;
static int rules_ready = 0;

static void init_rules(void) {
  if (rules_ready) return;
  /* 7-point degree-5 rule (Radon; Strang & Fix): centroid plus two orbits */
  double s15 = sqrt(15.0);
  double a1 = (6.0 - s15) / 21.0, b1 = (9.0 + 2.0 * s15) / 21.0;
  double a2 = (6.0 + s15) / 21.0, b2 = (9.0 - 2.0 * s15) / 21.0;
  double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
  rule7.np = 7;
  rule7.l[0][0] = rule7.l[0][1] = rule7.l[0][2] = 1.0 / 3.0; rule7.w[0] = 9.0 / 40.0;
  double orb[2][3] = {{a1, a1, b1}, {a2, a2, b2}};
  double ow[2] = {w1, w2};
  for (int o = 0; o < 2; ++o)
    for (int r = 0; r < 3; ++r) {
      int q = 1 + 3 * o + r;
      rule7.l[q][0] = orb[o][(0 + r) % 3];
      rule7.l[q][1] = orb[o][(1 + r) % 3];
      rule7.l[q][2] = orb[o][(2 + r) % 3];
      rule7.w[q] = ow[o];
    }
  /* 6-point degree-4 rule (Dunavant 1985) */
  double c1 = 0.445948490915965, d1 = 1.0 - 2.0 * c1, v1 = 0.223381589678011;
  double c2 = 0.091576213509771, d2 = 1.0 - 2.0 * c2, v2 = 0.109951743655322;
  double orb6[2][3] = {{c1, c1, d1}, {c2, c2, d2}};
  double ow6[2] = {v1, v2};
  rule6.np = 6;
  for (int o = 0; o < 2; ++o)
    for (int r = 0; r < 3; ++r) {
      int q = 3 * o + r;
      rule6.l[q][0] = orb6[o][(0 + r) % 3];
      rule6.l[q][1] = orb6[o][(1 + r) % 3];
      rule6.l[q][2] = orb6[o][(2 + r) % 3];
      rule6.w[q] = ow6[o];
    }
  rules_ready = 1;
}

/* Triangle t of cell (a,b): vertex grid coordinates (integers). */
static void tri_verts(int a, int b, int t, int va[3], int vb[3]) {
  if (t == 0) { va[0] = a; vb[0] = b; va[1] = a + 1; vb[1] = b; va[2] = a + 1; vb[2] = b + 1; }
  else        { va[0] = a; vb[0] = b; va[1] = a + 1; vb[1] = b + 1; va[2] = a; vb[2] = b + 1; }
}

typedef struct {
  int kernel;          /* KER_* */
  double phi;          /* kernel constant */
  double s;            /* fractional order */
  double h, delta;
  int c, N;            /* collar cells, cells per side incl. collar */
  long thr;            /* barycentre test: D <= thr, D in units (h/3)^2 */
  int R;               /* window half width */
  int W;               /* 2R+1 */
} prob2d_t;

/*
 * Contribution of one ordered pair (E, F) to the row of node (ma, mb), using
 * rule rE on E and rF on F.  out[v] (scalar) or out[v][2][2] (vector) over
 * the union vertex list uva/uvb (nu entries).
 */
static void pair_2d(const prob2d_t *P, const int ea[3], const int eb[3],
                    const int fa[3], const int fb[3], const rule_t *rE,
                    const rule_t *rF, int ma, int mb, int nu, const int *uva,
                    const int *uvb, double *out, double scale) {
  double h = P->h, off = P->c * h;
  double area = 0.5 * h * h;
  /* index of each union vertex in E and F (or -1) */
  int inE[6], inF[6];
  for (int u = 0; u < nu; ++u) {
    inE[u] = inF[u] = -1;
    for (int k = 0; k < 3; ++k) {
      if (ea[k] == uva[u] && eb[k] == uvb[u]) inE[u] = k;
      if (fa[k] == uva[u] && fb[k] == uvb[u]) inF[u] = k;
    }
  }
  int mE = -1, mF = -1;
  for (int k = 0; k < 3; ++k) {
    if (ea[k] == ma && eb[k] == mb) mE = k;
    if (fa[k] == ma && fb[k] == mb) mF = k;
  }
  double Ex[3], Ey[3], Fx[3], Fy[3];
  for (int k = 0; k < 3; ++k) {
    Ex[k] = ea[k] * h - off; Ey[k] = eb[k] * h - off;
    Fx[k] = fa[k] * h - off; Fy[k] = fb[k] * h - off;
  }
  for (int q = 0; q < rE->np; ++q) {
    const double *lx = rE->l[q];
    double x0 = lx[0] * Ex[0] + lx[1] * Ex[1] + lx[2] * Ex[2];
    double x1 = lx[0] * Ey[0] + lx[1] * Ey[1] + lx[2] * Ey[2];
    for (int p = 0; p < rF->np; ++p) {
      const double *ly = rF->l[p];
      double y0 = ly[0] * Fx[0] + ly[1] * Fx[1] + ly[2] * Fx[2];
      double y1 = ly[0] * Fy[0] + ly[1] * Fy[1] + ly[2] * Fy[2];
      double s0 = x0 - y0, s1 = x1 - y1;
      double r2 = s0 * s0 + s1 * s1;
      double w = rE->w[q] * rF->w[p] * area * area * scale;
      double dm = (mF >= 0 ? ly[mF] : 0.0) - (mE >= 0 ? lx[mE] : 0.0);
      if (dm == 0.0) continue;
      if (P->kernel == KER_PD) {
        if (r2 == 0.0) continue;          /* d vanishes there as well */
        double r = sqrt(r2);
        double g = w * P->phi / (r2 * r);
        double B00 = g * s0 * s0, B01 = g * s0 * s1, B11 = g * s1 * s1;
        for (int u = 0; u < nu; ++u) {
          double dn = (inF[u] >= 0 ? ly[inF[u]] : 0.0) - (inE[u] >= 0 ? lx[inE[u]] : 0.0);
          double t = dm * dn;
          double *o = out + 4 * u;
          o[0] += t * B00; o[1] += t * B01; o[2] += t * B01; o[3] += t * B11;
        }
      } else {
        double g;
        if (P->kernel == KER_CONST) {
          g = w * P->phi;
        } else {
          if (r2 == 0.0) continue;        /* never reached: rules differ on touching pairs */
          g = w * P->phi * pow(r2, -(2.0 + 2.0 * P->s) * 0.5);
        }
        for (int u = 0; u < nu; ++u) {
          double dn = (inF[u] >= 0 ? ly[inF[u]] : 0.0) - (inE[u] >= 0 ? lx[inE[u]] : 0.0);
          out[u] += g * dm * dn;
        }
      }
    }
  }
}

/* member (optional): per element of the extended mesh (index 2 (cb N + ca) + t)
 * the bit mask of the subdomains holding it; then only pairs that both lie in
 * subdomain `sub` count, weighted by 1 / zeta(E, F) (eqs. zeta,
 * bilinear-multi1). */
static void row_2d(const prob2d_t *P, int ma, int mb, double *win, const uint64_t *member, int sub) {
  int R1 = (int)ceil(P->delta / P->h) + 1;
  int vec = (P->kernel == KER_PD);
  int W = P->W;
  for (int ca = ma - 1; ca <= ma; ++ca)
    for (int cb = mb - 1; cb <= mb; ++cb)
      for (int t = 0; t < 2; ++t) {
        if (ca < 0 || cb < 0 || ca >= P->N || cb >= P->N) continue;
        int ea[3], eb[3];
        tri_verts(ca, cb, t, ea, eb);
        int holds = 0;
        for (int k = 0; k < 3; ++k) holds |= (ea[k] == ma && eb[k] == mb);
        if (!holds) continue;
        /* barycentre of E in units of h/3 */
        long BEa = ea[0] + ea[1] + ea[2], BEb = eb[0] + eb[1] + eb[2];
        for (int fa0 = ca - R1; fa0 <= ca + R1; ++fa0)
          for (int fb0 = cb - R1; fb0 <= cb + R1; ++fb0)
            for (int tf = 0; tf < 2; ++tf) {
              if (fa0 < 0 || fb0 < 0 || fa0 >= P->N || fb0 >= P->N) continue;
              int fa[3], fb[3];
              tri_verts(fa0, fb0, tf, fa, fb);
              long BFa = fa[0] + fa[1] + fa[2], BFb = fb[0] + fb[1] + fb[2];
              long D = (BEa - BFa) * (BEa - BFa) + (BEb - BFb) * (BEb - BFb);
              if (D > P->thr) continue;
              double zw = 1.0;
              if (member) {
                const uint64_t both = member[2 * (cb * P->N + ca) + t] & member[2 * (fb0 * P->N + fa0) + tf];
                if (!((both >> sub) & 1u)) continue;
                zw = 1.0 / (double)popcount64(both);
              }
              /* union vertex list */
              int uva[6], uvb[6], nu = 0;
              for (int k = 0; k < 3; ++k) { uva[nu] = ea[k]; uvb[nu] = eb[k]; ++nu; }
              int touching = 0, mInF = 0;
              for (int k = 0; k < 3; ++k) {
                int dup = 0;
                for (int u = 0; u < 3; ++u) dup |= (fa[k] == ea[u] && fb[k] == eb[u]);
                touching |= dup;
                if (fa[k] == ma && fb[k] == mb) mInF = 1;
                if (!dup) { uva[nu] = fa[k]; uvb[nu] = fb[k]; ++nu; }
              }
              double wf = (mInF ? 1.0 : 2.0) * zw;
              double acc[24];
              memset(acc, 0, sizeof(acc));
              if (P->kernel == KER_FRAC && touching) {
                pair_2d(P, ea, eb, fa, fb, &rule7, &rule6, ma, mb, nu, uva, uvb, acc, 0.5);
                pair_2d(P, ea, eb, fa, fb, &rule6, &rule7, ma, mb, nu, uva, uvb, acc, 0.5);
              } else {
                pair_2d(P, ea, eb, fa, fb, &rule7, &rule7, ma, mb, nu, uva, uvb, acc, 1.0);
              }
              for (int u = 0; u < nu; ++u) {
                int da = uva[u] - ma, db = uvb[u] - mb;
                if (da < -P->R || da > P->R || db < -P->R || db > P->R) continue;
                int wi = (db + P->R) * W + (da + P->R);
                if (vec) {
                  /* layout [row comp][window][col comp] */
                  win[(0 * W * W + wi) * 2 + 0] += wf * acc[4 * u + 0];
                  win[(0 * W * W + wi) * 2 + 1] += wf * acc[4 * u + 1];
                  win[(1 * W * W + wi) * 2 + 0] += wf * acc[4 * u + 2];
                  win[(1 * W * W + wi) * 2 + 1] += wf * acc[4 * u + 3];
                } else {
                  win[wi] += wf * acc[u];
                }
              }
            }
      }
}

/*
 * 2D assembly on (0,1)^2 with n cells per side and a collar of c cells.
 * Free nodes (a,b) with a,b in c+1 .. c+n-1, row index (b-c-1)(n-1)+(a-c-1).
 * win: (n-1)^2 rows of (2R+1)^2 scalars, or 4 (2R+1)^2 for KER_PD.
 */
int nl_assemble_2d(int n, int c, double delta, int kernel, double phi,
                   double s, int R, int nthreads, double *win) {
  init_rules();
  prob2d_t P;
  P.kernel = kernel; P.phi = phi; P.s = s;
  P.h = 1.0 / n; P.delta = delta; P.c = c; P.N = n + 2 * c;
  double t = 3.0 * delta / P.h;
  P.thr = (long)floor(t * t);
  P.R = R; P.W = 2 * R + 1;
  if (R < (int)ceil(delta / P.h) + 2) return -1;
  size_t rowlen = (size_t)P.W * P.W * (kernel == KER_PD ? 4 : 1);
  size_t nrow = (size_t)(n - 1) * (n - 1);
  memset(win, 0, sizeof(double) * rowlen * nrow);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (long i = 0; i < (long)nrow; ++i) {
    int ia = (int)(i % (n - 1)), ib = (int)(i / (n - 1));
    row_2d(&P, c + 1 + ia, c + 1 + ib, win + (size_t)i * rowlen, NULL, 0);
  }
  return 0;
}

/* Rows of the subdomain matrices A^k (eq. subStiffnessMatrix with the form of
 * eq. bilinear-multi1): row p is extended node row_node[p] = b (N+1) + a of
 * subdomain row_sub[p], in the window layout of nl_assemble_2d. */
int nl_assemble_2d_sub(int n, int c, double delta, int kernel, double phi, double s, int R,
                       int nthreads, const uint64_t *member, int P, const int *row_node,
                       const int *row_sub, double *win) {
  init_rules();
  prob2d_t Q;
  Q.kernel = kernel; Q.phi = phi; Q.s = s;
  Q.h = 1.0 / n; Q.delta = delta; Q.c = c; Q.N = n + 2 * c;
  double t = 3.0 * delta / Q.h;
  Q.thr = (long)floor(t * t);
  Q.R = R; Q.W = 2 * R + 1;
  if (R < (int)ceil(delta / Q.h) + 2) return -1;
  size_t rowlen = (size_t)Q.W * Q.W * (kernel == KER_PD ? 4 : 1);
  memset(win, 0, sizeof(double) * rowlen * (size_t)P);
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
  for (long p = 0; p < (long)P; ++p) {
    int a = row_node[p] % (Q.N + 1), b = row_node[p] / (Q.N + 1);
    row_2d(&Q, a, b, win + (size_t)p * rowlen, member, row_sub[p]);
  }
  return 0;
}
