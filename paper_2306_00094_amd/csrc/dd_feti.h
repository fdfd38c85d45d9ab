// One-level FETI on the device (section "FETI", Algorithm 1): the dual method
// the paper solves the reduced multi-domain problem (eq. discreteSubNonlocal)
// with.  Included at the end of dd_lib.hip; it reuses the substructuring
// context's kernels:
//
//   * a "Dirichlet" context D over the stacked interface copies
//     U = (Gamma_1, ..., Gamma_K): its interiors are the K_II^k, its interface
//     is U with K_UU = blockdiag(A^k_GG) and the couplings A^k_IG into the
//     copy of subdomain k, so its Schur product is S = diag(S_k) (eq.
//     subSchurComplement per subdomain, eq. SchurComplement), its
//     condensation is eq. subForcing and its back substitution eq.
//     backwardSubstitution;
//   * a "Neumann" context N whose blocks are the subdomain matrices A^k with
//     pinned dofs for floating subdomains (section "Pseudoinverse and
//     Cholesky decomposition"), factored and inverted by the batched Cholesky
//     of dd_factor; the interface block W_k of the inverse, its pinned rows
//     and columns set to zero (the Neumann solve with a right-hand side that
//     vanishes at the pins), gives S_k^+ = P_Z W_k P_Z (P_Z the orthogonal
//     projection off ker S_k), kept packed in 16x16 tiles and applied on the
//     matrix cores;
//   * a primal context over the original problem for the FP64 residual check.
//
// The constraint matrices B (one +1 and one -1 per row, consecutive copies of
// a dof), B_D = (B D^-1 B^T)^-1 B D^-1 (eq. preconditioner), G = B Z and the
// coarse matrix (G^T G)^-1 are formed on the host when the context is set up
// (structure and a coarse matrix of at most a few hundred rows); every
// product of the iteration runs in device kernels.  The projected
// preconditioned CG keeps its per-column scalars on the host (one read-back
// of the dot products per step).

namespace dd {

// out[r * ld + c] = scale_r * src[map_r * ldb + c] for c < nrhs (0 for padded
// columns): the stacked right-hand side of the Dirichlet context -- interiors
// b_I, interface copies b_G / zeta (the load of an interface dof split evenly
// over its copies: the constrained problem only sees their sum).
__global__ void k_feti_gather(int nrows, const int *__restrict__ map, const double *__restrict__ scale,
                              const double *__restrict__ b, int ldb, int nrhs, int ld,
                              double *__restrict__ out) {
  const size_t total = (size_t)nrows * ld;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / ld), c = (int)(e % ld);
    out[e] = c < nrhs ? scale[r] * b[(size_t)c * ldb + map[r]] : 0.0;
  }
}

// Global solution: interiors from uI (one row each), every interface dof the
// mean of its copies in uU (copies of dof i: cent[cptr[i] .. cptr[i+1]), in
// increasing order).
__global__ void k_feti_scatter(int NI, const int *__restrict__ imap, const double *__restrict__ uI,
                               int nG, const int *__restrict__ gmap, const int *__restrict__ cptr,
                               const int *__restrict__ cent, const double *__restrict__ uU, int ld,
                               int nrhs, double *__restrict__ u, int ldu) {
  const size_t tot = (size_t)(NI + nG) * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / nrhs), c = (int)(e % nrhs);
    if (r < NI) {
      u[(size_t)c * ldu + imap[r]] = uI[(size_t)r * ld + c];
    } else {
      const int i = r - NI;
      double s = 0.0;
      for (int a = cptr[i]; a < cptr[i + 1]; ++a) s += uU[(size_t)cent[a] * ld + c];
      u[(size_t)c * ldu + gmap[i]] = s / (double)(cptr[i + 1] - cptr[i]);
    }
  }
}

// Column dot products x_c . y_c of n x ld DD-layout vectors, deterministic:
// workgroup b sums rows 64 b .. 64 b + 63 (wave butterfly per column) into
// part[b * ld + c]; k_dot_fin sums the partials in order.
__global__ void __launch_bounds__(kBlock)
k_dot_part(int n, int ld, const double *__restrict__ x, const double *__restrict__ y,
           double *__restrict__ part) {
  __shared__ double lds[kRowsE * kMaxLd];
  const int r0 = blockIdx.x * kRowsE;
  for (int e = threadIdx.x; e < kRowsE * ld; e += kBlock) {
    const int lr = e / ld, c = e - lr * ld, r = r0 + lr;
    lds[e] = r < n ? x[(size_t)r * ld + c] * y[(size_t)r * ld + c] : 0.0;
  }
  __syncthreads();
  for (int c = wave_id(); c < ld; c += kWavesPerBlock) {
    const double s = chunk64_sum(lds, ld, c);
    if (lane_id() == 0) part[(size_t)blockIdx.x * ld + c] = s;
  }
}

__global__ void k_dot_fin(int nparts, int ld, const double *__restrict__ part, double *__restrict__ out) {
  const int c = threadIdx.x;
  if (c >= ld) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(size_t)b * ld + c];
  out[c] = s;
}

// Per-column coefficients, passed by value with the launch (captured when
// the kernel is enqueued: no host buffer that a later step could overwrite
// before the copy runs).
struct ColCoef {
  double a[kMaxLd];
};

// y = y + a_c x (axpy) or y = x + a_c y (xpay) per column c.
__global__ void k_axpy_cols(size_t n, int ld, ColCoef a, const double *__restrict__ x, double *__restrict__ y) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = fma(a.a[e % ld], x[e], y[e]);
}
__global__ void k_xpay_cols(size_t n, int ld, const double *__restrict__ x, ColCoef a, double *__restrict__ y) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * ld;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = fma(a.a[e % ld], y[e], x[e]);
}

// Packs the trailing sub-block [off_k, n_k) x [off_k, n_k) of dense
// column-major blocks (n_k x n_k at koff[k]) into the tile order of
// k_dense_tiles (block of m_k = n_k - off_k rows at toff[k]), with the rows
// and columns of pinned dofs (pinned[uo[k] + i] != 0) set to zero: the
// pinned inverse holds a unit column there, while the Neumann solve takes a
// right-hand side that vanishes at the pins and returns zero at them.
template <typename T>
__global__ void k_pack_sub(int nsub, const T *__restrict__ blocks, const long long *__restrict__ koff,
                           const int *__restrict__ ni, const int *__restrict__ off,
                           const long long *__restrict__ toff, const int *__restrict__ uo,
                           const int *__restrict__ pinned, double *__restrict__ packed) {
  const int k = blockIdx.y;
  if (k >= nsub) return;
  const int n = ni[k], o = off[k], m = n - o, nt = (m + kT - 1) / kT;
  const long long tot = (long long)nt * nt * 256;
  const T *B = blocks + koff[k];
  double *P = packed + toff[k];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(e / 256), pos = (int)(e % 256);
    const int I = t / nt, J = t % nt, l = TileLayout<double>::lane(pos), s = TileLayout<double>::step(pos);
    const int i = I * kT + (l & 15), j = J * kT + 4 * s + (l >> 4);
    const bool keep = i < m && j < m && !pinned[uo[k] + i] && !pinned[uo[k] + j];
    P[e] = keep ? (double)B[(size_t)(o + j) * n + (o + i)] : 0.0;
  }
}

// Seeded test right-hand side of the method autotuner: b[c * ld + i] in
// [-1, 1) from a 64-bit mix of (i, c) (the finaliser of SplitMix64).
__global__ void k_feti_pattern(int n, int nrhs, int ld, double *__restrict__ b) {
  const size_t tot = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / n), i = (int)(e % n);
    unsigned long long z = (unsigned long long)e * 0x9E3779B97F4A7C15ull + 0x1234567ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    b[(size_t)c * ld + i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

}  // namespace dd

namespace {

// CSR on the device (int32 structure, FP64 values).
struct DCsr {
  int nrows = 0;
  int *ptr = nullptr, *col = nullptr;
  double *val = nullptr;
};

struct HCsr {
  int nrows = 0, ncols = 0;
  std::vector<int> ptr{0}, col;
  std::vector<double> val;
  void row_end() { ptr.push_back((int)col.size()); ++nrows; }
  HCsr transpose() const {
    HCsr t;
    t.nrows = ncols;
    t.ncols = nrows;
    t.ptr.assign(ncols + 1, 0);
    for (int c : col) ++t.ptr[c + 1];
    for (int i = 0; i < ncols; ++i) t.ptr[i + 1] += t.ptr[i];
    t.col.resize(col.size());
    t.val.resize(col.size());
    std::vector<int> fill(t.ptr.begin(), t.ptr.end() - 1);
    for (int r = 0; r < nrows; ++r)
      for (int a = ptr[r]; a < ptr[r + 1]; ++a) {
        const int p = fill[col[a]]++;
        t.col[p] = r;
        t.val[p] = val[a];
      }
    return t;
  }
};

}  // namespace

struct dd_feti_ctx {
  dd_ctx *P = nullptr;   // primal context (residual check)
  dd_ctx *D = nullptr;   // Dirichlet context over the stacked interface copies
  hipStream_t stream = nullptr;
  int K = 0, NI = 0, NU = 0, nlam = 0, nc = 0, n_dof = 0, n_gamma = 0, max_nrhs = 0, ldmax = 1;
  std::vector<int> uoff;                    // offset of subdomain k's copy in U
  DCsr B, Bt, BD, BDt, Gm, Gt, GtGi, Q, Qt, Zm, Zt;
  // S^+ blocks W_k (interface block of the pinned inverse), packed tiles
  double *W = nullptr;
  long long *d_wtoff = nullptr;
  int *d_wni = nullptr, *d_wioff = nullptr;
  int2 *d_witems = nullptr;
  int n_wit = 0;
  // map of the stacked right-hand side and the solution scatter
  int *d_bmap = nullptr, *d_cptr = nullptr, *d_cent = nullptr, *d_imap = nullptr, *d_gmap = nullptr;
  double *d_bscale = nullptr;
  // vectors (DD layout, ldmax columns)
  double *lam = nullptr, *r = nullptr, *w = nullptr, *y = nullptr, *p = nullptr, *q = nullptr,
         *d = nullptr, *tU = nullptr, *sU = nullptr, *fU = nullptr, *cz = nullptr, *cz2 = nullptr;
  double *dpart = nullptr, *dout = nullptr;
  double *h_dots = nullptr;                      // pinned
  dd::ColCoef coef{};                            // coefficients of the next axpy / xpay
  bool factored = false;
  // balancing Neumann-Neumann preconditioner of the primal interface problem:
  // scaled restriction R_D (U x Gamma, entries 1 / zeta), its transpose, the
  // coarse space N = R_D^T Z, S N and the inverse of S_0 = N^T S N (formed by
  // the first BDD solve), interface vectors of the primal PCG
  DCsr Rd, Rdt, Nm, Nt, SNm, SNt, S0i;
  std::vector<int> hN_ptr, hN_col;
  std::vector<double> hN_val;
  bool bdd_ready = false;
  double *gx = nullptr, *gr = nullptr, *gz = nullptr, *gp = nullptr, *gq = nullptr, *gt = nullptr,
         *gu = nullptr, *cz3 = nullptr;
  // method chosen by dd_method_autotune (0: not tuned) and its timings
  int method = 0, tuned_nrhs = 0;
  double tune_ms[3] = {0.0, 0.0, 0.0};
  std::string err;
};

namespace {

dd_status ffail(dd_feti_ctx *f, dd_status s, const std::string &m) {
  if (f) f->err = m; else g_setup_error = m;
  return s;
}

#define FTRY(expr)                                            \
  do {                                                        \
    dd_status _s = (expr);                                    \
    if (_s != DD_OK) {                                        \
      if (f->err.empty()) f->err = f->D ? f->D->err : "";     \
      return _s;                                              \
    }                                                         \
  } while (0)

#define FHIP(expr)                                                                         \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) return ffail(f, DD_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

dd_status up_csr(dd_feti_ctx *f, const HCsr &h, DCsr &d) {
  dd_ctx *c = f->D;
  d.nrows = h.nrows;
  std::vector<int> col = h.col;
  std::vector<double> val = h.val;
  if (col.empty()) { col.push_back(0); val.push_back(0.0); }
  TRY(upload(c, &d.ptr, h.ptr.data(), h.ptr.size()));
  TRY(upload(c, &d.col, col.data(), col.size()));
  TRY(upload(c, &d.val, val.data(), val.size()));
  return DD_OK;
}

// out = base + sign * M x (DD layout, ld columns), on the Dirichlet context's stream.
void csr_apply(dd_feti_ctx *f, const DCsr &M, const double *x, int ld, const double *base, double sign,
               double *out) {
  if (M.nrows <= 0) return;
  csr_rows<double>(f->D, M.nrows, M.ptr, M.col, M.val, plain(x), ld, base, sign, out);
}

// Greedy pivoting over the rows of Z (n x nz, column-major): the pinned dofs.
std::vector<int> choose_pins(const double *z, int n, int nz) {
  std::vector<double> Z(z, z + (size_t)n * nz);
  std::vector<int> pins;
  for (int t = 0; t < nz; ++t) {
    int best = 0;
    double bn = -1.0;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int m = 0; m < nz; ++m) s += Z[(size_t)m * n + i] * Z[(size_t)m * n + i];
      if (s > bn) { bn = s; best = i; }
    }
    pins.push_back(best);
    double q[8], nq = std::sqrt(bn);
    for (int m = 0; m < nz; ++m) q[m] = Z[(size_t)m * n + best] / nq;
    for (int i = 0; i < n; ++i) {
      double dot = 0.0;
      for (int m = 0; m < nz; ++m) dot += Z[(size_t)m * n + i] * q[m];
      for (int m = 0; m < nz; ++m) Z[(size_t)m * n + i] -= dot * q[m];
    }
  }
  return pins;
}

// Inverse of a symmetric positive definite n x n matrix (row-major) by
// Cholesky; false if a pivot is not positive.  The result as a dense CSR.
bool spd_inverse_csr(const std::vector<double> &M, int n, HCsr &out) {
  std::vector<double> L((size_t)n * n, 0.0), Li((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = M[(size_t)j * n + j];
    for (int q = 0; q < j; ++q) s -= L[(size_t)j * n + q] * L[(size_t)j * n + q];
    if (!(s > 0.0)) return false;
    L[(size_t)j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = M[(size_t)i * n + j];
      for (int q = 0; q < j; ++q) t -= L[(size_t)i * n + q] * L[(size_t)j * n + q];
      L[(size_t)i * n + j] = t / L[(size_t)j * n + j];
    }
  }
  for (int col = 0; col < n; ++col) {       // (L L^T)^-1 e_col
    std::vector<double> v(n, 0.0);
    v[col] = 1.0;
    for (int i = 0; i < n; ++i) {
      double t = v[i];
      for (int q = 0; q < i; ++q) t -= L[(size_t)i * n + q] * v[q];
      v[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = v[i];
      for (int q = i + 1; q < n; ++q) t -= L[(size_t)q * n + i] * v[q];
      v[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) Li[(size_t)i * n + col] = v[i];
  }
  out = HCsr();
  out.ncols = n;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      out.col.push_back(j);
      out.val.push_back(Li[(size_t)i * n + j]);
    }
    out.row_end();
  }
  return true;
}

// Dot products of the ncols columns of x and y (n rows, ld): into f->h_dots.
dd_status dots(dd_feti_ctx *f, int n, int ld, const double *x, const double *y) {
  if (n <= 0) {
    for (int c = 0; c < ld; ++c) f->h_dots[c] = 0.0;
    return DD_OK;
  }
  const unsigned nb = grid_for(std::max(1, n), kRowsE);
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(kBlock), 0, f->stream, n, ld, x, y, f->dpart);
  hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(kMaxLd), 0, f->stream, (int)nb, ld, f->dpart, f->dout);
  FHIP(hipMemcpyAsync(f->h_dots, f->dout, ld * sizeof(double), hipMemcpyDeviceToHost, f->stream));
  FHIP(hipStreamSynchronize(f->stream));
  return DD_OK;
}

void set_coef(dd_feti_ctx *f, const std::vector<double> &a, int ld) {
  for (int c = 0; c < ld; ++c) f->coef.a[c] = a[c];
}

void axpy(dd_feti_ctx *f, size_t n, int ld, const double *x, double *y) {
  hipLaunchKernelGGL(k_axpy_cols, dim3(std::min(4096u, grid_for(n * ld, 256))), dim3(256), 0, f->stream, n, ld,
                     f->coef, x, y);
}
void xpay(dd_feti_ctx *f, size_t n, int ld, const double *x, double *y) {
  hipLaunchKernelGGL(k_xpay_cols, dim3(std::min(4096u, grid_for(n * ld, 256))), dim3(256), 0, f->stream, n, ld, x,
                     f->coef, y);
}

// S^+ x on U (out may not alias x): project off the kernels, W_k blocks, project.
void spinv(dd_feti_ctx *f, const double *x, double *out, int ld) {
  const double *in = x;
  if (f->nc > 0) {          // t = x - Q Q^T x
    csr_apply(f, f->Qt, x, ld, nullptr, 1.0, f->cz);
    csr_apply(f, f->Q, f->cz, ld, x, -1.0, f->tU);
    in = f->tU;
  }
  const dim3 g(f->n_wit), b(kTW * kWave);
#define DD_WT(NCB)                                                                                  \
  hipLaunchKernelGGL((k_dense_tiles<double, NCB>), g, b, 0, f->stream, f->NU, f->d_witems, f->W,      \
                     f->d_wtoff, f->d_wioff, f->d_wni, in, ld, (const double *)nullptr, 1.0, out, \
                     (const int *)nullptr, (float *)nullptr)
  if (ld <= 16) DD_WT(1);
  else if (ld <= 32) DD_WT(2);
  else DD_WT(4);
#undef DD_WT
  if (f->nc > 0) {
    csr_apply(f, f->Qt, out, ld, nullptr, 1.0, f->cz);
    csr_apply(f, f->Q, f->cz, ld, out, -1.0, out);
  }
}

// S x on U (Dirichlet solves with the K_II^k factors, eq. subSchurComplement).
void sapply(dd_feti_ctx *f, const double *x, double *out, int ld) {
  dd_ctx *c = f->D;
  kig_apply(c, DD_FP64, plain(x), ld, nullptr, 1.0, c->w.yI);
  interior_solve(c, DD_FP64, DD_APPLY_INV, c->w.yI, c->w.wI, ld);
  gamma_apply(c, DD_FP64, plain(x), c->w.wI, ld, nullptr, 1.0, -1.0, out);
}

// F x = B S^+ B^T x on Lambda.
void fapply(dd_feti_ctx *f, const double *x, double *out, int ld) {
  csr_apply(f, f->Bt, x, ld, nullptr, 1.0, f->sU);
  spinv(f, f->sU, f->fU, ld);
  csr_apply(f, f->B, f->fU, ld, nullptr, 1.0, out);
}

// P x = x - G (G^T G)^-1 G^T x (in place allowed).
void project(dd_feti_ctx *f, const double *x, double *out, int ld) {
  if (f->nc == 0) {
    if (out != x)     // (a failure shows at the next checked call on the stream)
      (void)hipMemcpyAsync(out, x, (size_t)f->nlam * ld * sizeof(double), hipMemcpyDeviceToDevice, f->stream);
    return;
  }
  csr_apply(f, f->Gt, x, ld, nullptr, 1.0, f->cz);
  csr_apply(f, f->GtGi, f->cz, ld, nullptr, 1.0, f->cz2);
  csr_apply(f, f->Gm, f->cz2, ld, x, -1.0, out);
}

// M^-1 x = B_D S B_D^T x (scaled Dirichlet preconditioner, eq. preconditioner).
void precond(dd_feti_ctx *f, const double *x, double *out, int ld) {
  csr_apply(f, f->BDt, x, ld, nullptr, 1.0, f->sU);
  sapply(f, f->sU, f->fU, ld);
  csr_apply(f, f->BD, f->fU, ld, nullptr, 1.0, out);
}

// ---------------------------------------------------- balancing Neumann-Neumann --
// q = S x on the interface of the primal context (eq. subSchurComplement summed
// over subdomains): the same three products as one CG iteration of dd_solve.
void primal_schur(dd_feti_ctx *f, const double *x, double *q, int ld) {
  dd_ctx *c = f->P;
  kig_apply(c, DD_FP64, plain(x), ld, nullptr, 1.0, c->w.yI);
  interior_solve(c, DD_FP64, DD_APPLY_INV, c->w.yI, c->w.wI, ld);
  gamma_apply(c, DD_FP64, plain(x), c->w.wI, ld, nullptr, 1.0, -1.0, q);
}

// S N (dense, n_gamma x nc, by columns through the primal Schur product) and
// the inverse of S_0 = N^T S N, once per context.
dd_status bdd_prepare(dd_feti_ctx *f) {
  if (f->bdd_ready) return DD_OK;
  const int nG = f->n_gamma, nc = f->nc, L = f->ldmax;
  if (nc > 0) {
    std::vector<double> Nd((size_t)nG * nc, 0.0), SNd((size_t)nG * nc, 0.0), chunk((size_t)nG * L);
    for (int g = 0; g < nG; ++g)
      for (int a = f->hN_ptr[g]; a < f->hN_ptr[g + 1]; ++a) Nd[(size_t)g * nc + f->hN_col[a]] = f->hN_val[a];
    for (int c0 = 0; c0 < nc; c0 += L) {
      const int m = std::min(L, nc - c0);
      for (int g = 0; g < nG; ++g)
        for (int j = 0; j < L; ++j) chunk[(size_t)g * L + j] = j < m ? Nd[(size_t)g * nc + c0 + j] : 0.0;
      FHIP(hipMemcpyAsync(f->gt, chunk.data(), chunk.size() * sizeof(double), hipMemcpyHostToDevice, f->stream));
      primal_schur(f, f->gt, f->gq, L);
      FHIP(hipMemcpyAsync(chunk.data(), f->gq, chunk.size() * sizeof(double), hipMemcpyDeviceToHost, f->stream));
      FHIP(hipStreamSynchronize(f->stream));
      for (int g = 0; g < nG; ++g)
        for (int j = 0; j < m; ++j) SNd[(size_t)g * nc + c0 + j] = chunk[(size_t)g * L + j];
    }
    std::vector<double> S0((size_t)nc * nc, 0.0);
    for (int g = 0; g < nG; ++g)
      for (int a = f->hN_ptr[g]; a < f->hN_ptr[g + 1]; ++a) {
        const int i = f->hN_col[a];
        const double v = f->hN_val[a];
        for (int j = 0; j < nc; ++j) S0[(size_t)i * nc + j] += v * SNd[(size_t)g * nc + j];
      }
    for (int i = 0; i < nc; ++i)          // symmetric up to rounding: take the mean
      for (int j = 0; j < i; ++j) S0[(size_t)i * nc + j] = S0[(size_t)j * nc + i] =
          0.5 * (S0[(size_t)i * nc + j] + S0[(size_t)j * nc + i]);
    HCsr S0i, SN, SNt;
    if (!spd_inverse_csr(S0, nc, S0i)) return ffail(f, DD_ENOTSPD, "coarse matrix N^T S N not positive definite");
    SN.ncols = nc;
    for (int g = 0; g < nG; ++g) {
      for (int j = 0; j < nc; ++j) {
        SN.col.push_back(j);
        SN.val.push_back(SNd[(size_t)g * nc + j]);
      }
      SN.row_end();
    }
    SNt = SN.transpose();
    dd_status st;
    if ((st = up_csr(f, S0i, f->S0i)) != DD_OK || (st = up_csr(f, SN, f->SNm)) != DD_OK ||
        (st = up_csr(f, SNt, f->SNt)) != DD_OK)
      return ffail(f, st, "uploading the coarse space: " + f->D->err);
  }
  f->bdd_ready = true;
  return DD_OK;
}

// z = M^-1 r = P_0 r + (I - P_0 S) M_NN (I - S P_0) r with P_0 = N S_0^-1 N^T and
// M_NN = R_D^T S^+ R_D (S^+ blockwise over the copies).
void bdd_minv(dd_feti_ctx *f, const double *r, double *z, int ld) {
  const double *t = r;
  if (f->nc > 0) {            // c2 = S_0^-1 N^T r;  t = r - S N c2 (balanced)
    csr_apply(f, f->Nt, r, ld, nullptr, 1.0, f->cz);
    csr_apply(f, f->S0i, f->cz, ld, nullptr, 1.0, f->cz2);
    csr_apply(f, f->SNm, f->cz2, ld, r, -1.0, f->gt);
    t = f->gt;
  }
  csr_apply(f, f->Rd, t, ld, nullptr, 1.0, f->sU);
  spinv(f, f->sU, f->fU, ld);
  if (f->nc > 0) {            // z = u + N (c2 - S_0^-1 (S N)^T u)
    csr_apply(f, f->Rdt, f->fU, ld, nullptr, 1.0, f->gu);
    csr_apply(f, f->SNt, f->gu, ld, nullptr, 1.0, f->cz3);
    csr_apply(f, f->S0i, f->cz3, ld, f->cz2, -1.0, f->cz);
    csr_apply(f, f->Nm, f->cz, ld, f->gu, 1.0, z);
  } else {
    csr_apply(f, f->Rdt, f->fU, ld, nullptr, 1.0, z);
  }
}

}  // namespace

extern "C" {

dd_status dd_feti_setup(const dd_problem *prob, const dd_feti_sub *fs, void *hip_stream, int32_t max_nrhs,
                        dd_feti_ctx **out) {
  if (!out) return ffail(nullptr, DD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!prob || !fs || prob->n_sub < 1) return ffail(nullptr, DD_EINVAL, "problem, subdomains or n_sub < 1");
  if (max_nrhs < 1 || max_nrhs > kMaxLd) return ffail(nullptr, DD_EINVAL, "max_nrhs out of [1, 64]");
  const int K = prob->n_sub, nG = prob->n_gamma;
  // validate the subdomain copies
  for (int k = 0; k < K; ++k) {
    const dd_feti_sub &s = fs[k];
    const std::string tag = "subdomain " + std::to_string(k) + ": ";
    if (s.n_g < 0 || s.n_g > nG || (s.n_g > 0 && (!s.g_map || !s.agg_rowptr || !s.kig_rowptr)))
      return ffail(nullptr, DD_EINVAL, tag + "bad interface copy");
    if (s.n_z < 0 || s.n_z > 8 || (s.n_z > 0 && (!s.z || s.n_z > s.n_g)))
      return ffail(nullptr, DD_EINVAL, tag + "bad kernel basis");
    for (int j = 0; j < s.n_g; ++j)
      if (s.g_map[j] < 0 || s.g_map[j] >= nG || (j > 0 && s.g_map[j] <= s.g_map[j - 1]))
        return ffail(nullptr, DD_EINVAL, tag + "g_map not increasing in [0, n_gamma)");
    if (s.n_g > 0 && s.agg_rowptr[0] != 0) return ffail(nullptr, DD_EINVAL, tag + "agg_rowptr[0] != 0");
    for (int j = 0; j < s.n_g; ++j) {
      if (s.agg_rowptr[j + 1] < s.agg_rowptr[j]) return ffail(nullptr, DD_EINVAL, tag + "agg_rowptr not monotone");
      for (int a = s.agg_rowptr[j]; a < s.agg_rowptr[j + 1]; ++a)
        if (s.agg_col[a] < 0 || s.agg_col[a] >= s.n_g) return ffail(nullptr, DD_EINVAL, tag + "agg_col out of range");
    }
    const int ni = prob->sub[k].n_i;
    if (s.kig_rowptr[0] != 0) return ffail(nullptr, DD_EINVAL, tag + "kig_rowptr[0] != 0");
    for (int i = 0; i < ni; ++i) {
      if (s.kig_rowptr[i + 1] < s.kig_rowptr[i]) return ffail(nullptr, DD_EINVAL, tag + "kig_rowptr not monotone");
      for (int a = s.kig_rowptr[i]; a < s.kig_rowptr[i + 1]; ++a)
        if (s.kig_col[a] < 0 || s.kig_col[a] >= s.n_g) return ffail(nullptr, DD_EINVAL, tag + "kig_col out of range");
    }
  }
  dd_feti_ctx *f = new (std::nothrow) dd_feti_ctx();
  if (!f) return ffail(nullptr, DD_ENOMEM, "host allocation failed");
  auto bail = [&](dd_status s) {
    std::string m = f->err;
    dd_feti_destroy(f);
    g_setup_error = m;
    return s;
  };
  f->stream = (hipStream_t)hip_stream;
  f->K = K;
  f->n_dof = prob->n_dof;
  f->n_gamma = nG;
  f->max_nrhs = max_nrhs;
  f->ldmax = next_pow2(max_nrhs);
  // primal context (validates the problem)
  dd_status st = dd_setup(prob, hip_stream, max_nrhs, &f->P);
  if (st != DD_OK) { f->err = g_setup_error; return bail(st); }
  // --- the Dirichlet context over U -------------------------------------------
  f->uoff.assign(K + 1, 0);
  int NI = 0;
  for (int k = 0; k < K; ++k) {
    f->uoff[k + 1] = f->uoff[k] + fs[k].n_g;
    NI += prob->sub[k].n_i;
  }
  const int NU = f->uoff[K];
  f->NI = NI;
  f->NU = NU;
  if (NU == 0) { f->err = "no interface copies"; return bail(DD_EINVAL); }
  {
    std::vector<dd_subdomain> subs(K);
    std::vector<std::vector<int>> imaps(K), gmaps(K);
    int io = 0;
    for (int k = 0; k < K; ++k) {
      const dd_subdomain &s = prob->sub[k];
      imaps[k].resize(s.n_i);
      for (int i = 0; i < s.n_i; ++i) imaps[k][i] = io + i;
      io += s.n_i;
      gmaps[k].resize(fs[k].n_g);
      for (int j = 0; j < fs[k].n_g; ++j) gmaps[k][j] = f->uoff[k] + j;
      subs[k] = dd_subdomain{s.n_i, s.k_ii, fs[k].n_g, gmaps[k].data(), fs[k].kig_rowptr, fs[k].kig_col,
                             fs[k].kig_val, imaps[k].data()};
    }
    std::vector<int> gam(NU), uptr(NU + 1, 0), ucol;
    std::vector<double> uval;
    for (int u = 0; u < NU; ++u) gam[u] = NI + u;
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < fs[k].n_g; ++j) {
        for (int a = fs[k].agg_rowptr[j]; a < fs[k].agg_rowptr[j + 1]; ++a) {
          ucol.push_back(f->uoff[k] + fs[k].agg_col[a]);
          uval.push_back(fs[k].agg_val[a]);
        }
        uptr[f->uoff[k] + j + 1] = (int)ucol.size();
      }
    if (ucol.empty()) { ucol.push_back(0); uval.push_back(0.0); }
    dd_problem pd{NI + NU, NU, K, subs.data(), gam.data(), uptr.data(), ucol.data(), uval.data()};
    st = dd_setup(&pd, hip_stream, max_nrhs, &f->D);
    if (st != DD_OK) { f->err = "Dirichlet context: " + g_setup_error; return bail(st); }
  }
  dd_ctx *c = f->D;
  // --- constraints B and the multiplicities ----------------------------------------
  std::vector<std::vector<int>> copies(nG);
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < fs[k].n_g; ++j) copies[fs[k].g_map[j]].push_back(f->uoff[k] + j);
  HCsr B, BD;
  B.ncols = BD.ncols = NU;
  for (int i = 0; i < nG; ++i) {
    const auto &cp = copies[i];
    const int z = (int)cp.size();
    if (z == 0) { f->err = "interface dof " + std::to_string(i) + " has no copy"; return bail(DD_EINVAL); }
    for (int a = 0; a + 1 < z; ++a) {
      B.col.push_back(cp[a]); B.val.push_back(1.0);
      B.col.push_back(cp[a + 1]); B.val.push_back(-1.0);
      B.row_end();
    }
    // B_D rows of this dof: (B_i B_i^T)^-1 B_i, with B_i the (z-1) x z chain
    // (D_i = z I cancels); (B_i B_i^T) is tridiagonal [-1 2 -1], solved densely
    if (z >= 2) {
      const int m = z - 1;
      std::vector<double> T((size_t)m * m, 0.0), R((size_t)m * z, 0.0);
      for (int a = 0; a < m; ++a) {
        T[(size_t)a * m + a] = 2.0;
        if (a + 1 < m) T[(size_t)a * m + a + 1] = T[(size_t)(a + 1) * m + a] = -1.0;
        R[(size_t)a * z + a] = 1.0;
        R[(size_t)a * z + a + 1] = -1.0;
      }
      // Gauss-Jordan on [T | R]
      for (int piv = 0; piv < m; ++piv) {
        const double dv = T[(size_t)piv * m + piv];
        for (int j2 = 0; j2 < m; ++j2) T[(size_t)piv * m + j2] /= dv;
        for (int j2 = 0; j2 < z; ++j2) R[(size_t)piv * z + j2] /= dv;
        for (int r2 = 0; r2 < m; ++r2) {
          if (r2 == piv) continue;
          const double fct = T[(size_t)r2 * m + piv];
          if (fct == 0.0) continue;
          for (int j2 = 0; j2 < m; ++j2) T[(size_t)r2 * m + j2] -= fct * T[(size_t)piv * m + j2];
          for (int j2 = 0; j2 < z; ++j2) R[(size_t)r2 * z + j2] -= fct * R[(size_t)piv * z + j2];
        }
      }
      for (int a = 0; a < m; ++a) {
        for (int j2 = 0; j2 < z; ++j2) {
          BD.col.push_back(cp[j2]);
          BD.val.push_back(R[(size_t)a * z + j2]);
        }
        BD.row_end();
      }
    }
  }
  f->nlam = B.nrows;
  if (f->nlam == 0) { f->err = "no constraints (a single subdomain?)"; return bail(DD_EINVAL); }
  // --- kernels: Z (U x nc, block-diagonal), orthonormal Q, G = B Z, (G^T G)^-1 -----
  HCsr Z, Q;
  Z.ncols = Q.ncols = 0;
  std::vector<int> zoff(K + 1, 0);
  for (int k = 0; k < K; ++k) zoff[k + 1] = zoff[k] + fs[k].n_z;
  const int nc = zoff[K];
  f->nc = nc;
  {
    // rows of Z and Q over U
    std::vector<std::vector<std::pair<int, double>>> zr(NU), qr(NU);
    for (int k = 0; k < K; ++k) {
      const int ng = fs[k].n_g, nz = fs[k].n_z;
      if (nz == 0) continue;
      std::vector<double> q(fs[k].z, fs[k].z + (size_t)ng * nz);
      for (int m = 0; m < nz; ++m) {              // modified Gram-Schmidt
        for (int m2 = 0; m2 < m; ++m2) {
          double dt = 0.0;
          for (int j = 0; j < ng; ++j) dt += q[(size_t)m2 * ng + j] * q[(size_t)m * ng + j];
          for (int j = 0; j < ng; ++j) q[(size_t)m * ng + j] -= dt * q[(size_t)m2 * ng + j];
        }
        double nrm = 0.0;
        for (int j = 0; j < ng; ++j) nrm += q[(size_t)m * ng + j] * q[(size_t)m * ng + j];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) { f->err = "subdomain " + std::to_string(k) + ": dependent kernel basis"; return bail(DD_EINVAL); }
        for (int j = 0; j < ng; ++j) q[(size_t)m * ng + j] /= nrm;
      }
      for (int j = 0; j < ng; ++j)
        for (int m = 0; m < nz; ++m) {
          zr[f->uoff[k] + j].push_back({zoff[k] + m, fs[k].z[(size_t)m * ng + j]});
          qr[f->uoff[k] + j].push_back({zoff[k] + m, q[(size_t)m * ng + j]});
        }
    }
    Z.ncols = Q.ncols = nc;
    for (int u = 0; u < NU; ++u) {
      for (auto &e : zr[u]) { Z.col.push_back(e.first); Z.val.push_back(e.second); }
      Z.row_end();
      for (auto &e : qr[u]) { Q.col.push_back(e.first); Q.val.push_back(e.second); }
      Q.row_end();
    }
  }
  HCsr G;
  G.ncols = nc;
  for (int r = 0; r < B.nrows; ++r) {      // G = B Z
    std::vector<double> acc(nc, 0.0);
    std::vector<int> touched;
    for (int a = B.ptr[r]; a < B.ptr[r + 1]; ++a) {
      const int u = B.col[a];
      for (int b2 = Z.ptr[u]; b2 < Z.ptr[u + 1]; ++b2) {
        if (acc[Z.col[b2]] == 0.0) touched.push_back(Z.col[b2]);
        acc[Z.col[b2]] += B.val[a] * Z.val[b2];
      }
    }
    std::sort(touched.begin(), touched.end());
    touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
    for (int cc : touched)
      if (acc[cc] != 0.0) { G.col.push_back(cc); G.val.push_back(acc[cc]); }
    G.row_end();
  }
  HCsr Gt = G.transpose();
  HCsr GtGi;
  GtGi.ncols = nc;
  if (nc > 0) {
    // G^T G (dense, nc x nc) and its inverse by Cholesky (the coarse problem)
    std::vector<double> M((size_t)nc * nc, 0.0);
    for (int r = 0; r < G.nrows; ++r)
      for (int a = G.ptr[r]; a < G.ptr[r + 1]; ++a)
        for (int b2 = G.ptr[r]; b2 < G.ptr[r + 1]; ++b2) M[(size_t)G.col[a] * nc + G.col[b2]] += G.val[a] * G.val[b2];
    if (!spd_inverse_csr(M, nc, GtGi)) { f->err = "G^T G not positive definite"; return bail(DD_ENOTSPD); }
  }
  f->err.clear();
  if ((st = up_csr(f, B, f->B)) != DD_OK) return bail(st);
  if ((st = up_csr(f, B.transpose(), f->Bt)) != DD_OK) return bail(st);
  if ((st = up_csr(f, BD, f->BD)) != DD_OK) return bail(st);
  if ((st = up_csr(f, BD.transpose(), f->BDt)) != DD_OK) return bail(st);
  if ((st = up_csr(f, G, f->Gm)) != DD_OK) return bail(st);
  if ((st = up_csr(f, Gt, f->Gt)) != DD_OK) return bail(st);
  if ((st = up_csr(f, GtGi, f->GtGi)) != DD_OK) return bail(st);
  if ((st = up_csr(f, Q, f->Q)) != DD_OK) return bail(st);
  if ((st = up_csr(f, Q.transpose(), f->Qt)) != DD_OK) return bail(st);
  if ((st = up_csr(f, Z, f->Zm)) != DD_OK) return bail(st);
  if ((st = up_csr(f, Z.transpose(), f->Zt)) != DD_OK) return bail(st);
  {
    // balancing Neumann-Neumann: R_D (row u: the interface dof of copy u,
    // weight 1 / zeta), R_D^T (per dof its copies in subdomain order) and the
    // coarse space N = R_D^T Z (column (k, m): z_k[:, m] / zeta on Gamma_k)
    HCsr Rd;
    Rd.ncols = nG;
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < fs[k].n_g; ++j) {
        const int gi = fs[k].g_map[j];
        Rd.col.push_back(gi);
        Rd.val.push_back(1.0 / (double)copies[gi].size());
        Rd.row_end();
      }
    HCsr Rdt = Rd.transpose(), N;
    N.ncols = nc;
    for (int g = 0; g < nG; ++g) {
      for (int a = Rdt.ptr[g]; a < Rdt.ptr[g + 1]; ++a)
        for (int b2 = Z.ptr[Rdt.col[a]]; b2 < Z.ptr[Rdt.col[a] + 1]; ++b2) {
          N.col.push_back(Z.col[b2]);
          N.val.push_back(Rdt.val[a] * Z.val[b2]);
        }
      N.row_end();
    }
    if ((st = up_csr(f, Rd, f->Rd)) != DD_OK || (st = up_csr(f, Rdt, f->Rdt)) != DD_OK ||
        (st = up_csr(f, N, f->Nm)) != DD_OK || (st = up_csr(f, N.transpose(), f->Nt)) != DD_OK)
      return bail(st);
    f->hN_ptr = N.ptr;
    f->hN_col = N.col;
    f->hN_val = N.val;
  }
  // --- the Neumann context: pinned subdomain matrices, factored and inverted ----------
  {
    std::vector<std::vector<double>> blocks(K);
    std::vector<dd_subdomain> subs(K);
    std::vector<std::vector<int>> imaps(K);
    std::vector<int> pinflag(NU, 0);
    int off = 0;
    for (int k = 0; k < K; ++k) {
      const dd_subdomain &s = prob->sub[k];
      const dd_feti_sub &q = fs[k];
      const int ni = s.n_i, ng = q.n_g, n = ni + ng;
      std::vector<double> &A = blocks[k];
      A.assign((size_t)n * n, 0.0);
      for (int j = 0; j < ni; ++j)
        for (int i = 0; i < ni; ++i) A[(size_t)j * n + i] = s.k_ii[(size_t)j * ni + i];
      for (int i = 0; i < ni; ++i)
        for (int a = q.kig_rowptr[i]; a < q.kig_rowptr[i + 1]; ++a) {
          const int jj = ni + q.kig_col[a];
          A[(size_t)jj * n + i] = q.kig_val[a];
          A[(size_t)i * n + jj] = q.kig_val[a];
        }
      for (int j = 0; j < ng; ++j)
        for (int a = q.agg_rowptr[j]; a < q.agg_rowptr[j + 1]; ++a)
          A[(size_t)(ni + q.agg_col[a]) * n + ni + j] = q.agg_val[a];
      if (q.n_z > 0) {
        for (int pin : choose_pins(q.z, ng, q.n_z)) {
          pinflag[f->uoff[k] + pin] = 1;
          const int pv = ni + pin;
          for (int i = 0; i < n; ++i) A[(size_t)pv * n + i] = A[(size_t)i * n + pv] = 0.0;
          A[(size_t)pv * n + pv] = 1.0;
        }
      }
      imaps[k].resize(n);
      for (int i = 0; i < n; ++i) imaps[k][i] = off + i;
      off += n;
      subs[k] = dd_subdomain{n, A.data(), 0, nullptr, nullptr, nullptr, nullptr, imaps[k].data()};
    }
    std::vector<int> kptr(off + 1, 0);   // every subdomain shares the all-zero K_IG row pointers
    for (int k = 0; k < K; ++k) subs[k].kig_rowptr = kptr.data();
    int dummy = 0;
    double dval = 0.0;
    dd_problem pn{off, 0, K, subs.data(), &dummy, &dummy, &dummy, &dval};
    dd_ctx *N = nullptr;
    st = dd_setup(&pn, hip_stream, 1, &N);
    if (st != DD_OK) { f->err = "Neumann context: " + g_setup_error; return bail(st); }
    blocks.clear();
    st = dd_factor(N, DD_FP64);
    if (st != DD_OK) {
      f->err = "Neumann factor: " + N->err;
      dd_destroy(N);
      return bail(st);
    }
    // W_k = interface block of the inverse, packed into tiles
    std::vector<long long> wtoff(K + 1, 0);
    std::vector<int> wni(K), wioff(K), woff(K);
    for (int k = 0; k < K; ++k) {
      const long long nt = (fs[k].n_g + kT - 1) / kT;
      wtoff[k + 1] = wtoff[k] + nt * nt * 256;
      wni[k] = fs[k].n_g;
      wioff[k] = f->uoff[k];
      woff[k] = prob->sub[k].n_i;
    }
    if ((st = dalloc(c, &f->W, (size_t)std::max<long long>(1, wtoff[K]))) != DD_OK) { dd_destroy(N); return bail(st); }
    int *d_woff = nullptr, *d_nfull = nullptr, *d_pin = nullptr;
    std::vector<int> nfull(K);
    for (int k = 0; k < K; ++k) nfull[k] = prob->sub[k].n_i + fs[k].n_g;
    if ((st = upload(c, &f->d_wtoff, wtoff.data(), wtoff.size())) != DD_OK ||
        (st = upload(c, &f->d_wni, wni.data(), wni.size())) != DD_OK ||
        (st = upload(c, &f->d_wioff, wioff.data(), wioff.size())) != DD_OK ||
        (st = upload(c, &d_woff, woff.data(), woff.size())) != DD_OK ||
        (st = upload(c, &d_nfull, nfull.data(), nfull.size())) != DD_OK ||
        (st = upload(c, &d_pin, pinflag.data(), pinflag.size())) != DD_OK) {
      dd_destroy(N);
      return bail(st);
    }
    hipLaunchKernelGGL((k_pack_sub<double>), dim3(64, K), dim3(256), 0, N->stream, K, (const double *)N->op[0].kinv,
                       N->d_koff, d_nfull, d_woff, f->d_wtoff, f->d_wioff, d_pin, f->W);
    hipError_t he = hipStreamSynchronize(N->stream);
    dd_destroy(N);
    if (he != hipSuccess) { f->err = std::string("packing S^+ blocks: ") + hipGetErrorString(he); return bail(DD_EHIP); }
    // work items of the S^+ blocks: (subdomain, 16-row tile), XCD bins as for K_II^-1
    constexpr int kXcd = 8;
    std::vector<int> order(K);
    for (int k = 0; k < K; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) { return wni[a2] > wni[b2]; });
    std::vector<std::vector<int2>> bins(kXcd);
    long long load[kXcd] = {0};
    for (int k : order) {
      int x = 0;
      for (int y = 1; y < kXcd; ++y)
        if (load[y] < load[x]) x = y;
      const int nt = (wni[k] + kT - 1) / kT;
      load[x] += (long long)nt * nt;
      for (int I = 0; I < nt; ++I) bins[x].push_back(make_int2(k, I));
    }
    size_t blen = 0;
    for (auto &bn : bins) blen = std::max(blen, bn.size());
    std::vector<int2> items;
    for (size_t i = 0; i < blen; ++i)
      for (int x = 0; x < kXcd; ++x) items.push_back(i < bins[x].size() ? bins[x][i] : make_int2(-1, 0));
    f->n_wit = (int)items.size();
    if ((st = upload(c, &f->d_witems, items.data(), items.size())) != DD_OK) return bail(st);
  }
  // --- right-hand side map, solution scatter, vectors ------------------------------------
  {
    std::vector<int> bmap(NI + NU), imap(NI), cptr(nG + 1, 0), cent;
    std::vector<double> bscale(NI + NU, 1.0);
    int r = 0;
    for (int k = 0; k < K; ++k)
      for (int i = 0; i < prob->sub[k].n_i; ++i, ++r) bmap[r] = imap[r] = prob->sub[k].i_map[i];
    for (int k = 0; k < K; ++k)
      for (int j = 0; j < fs[k].n_g; ++j) {
        const int gi = fs[k].g_map[j];
        bmap[NI + f->uoff[k] + j] = prob->gamma_map[gi];
        bscale[NI + f->uoff[k] + j] = 1.0 / (double)copies[gi].size();
      }
    for (int i = 0; i < nG; ++i) {
      for (int u : copies[i]) cent.push_back(u);
      cptr[i + 1] = (int)cent.size();
    }
    if ((st = upload(c, &f->d_bmap, bmap.data(), bmap.size())) != DD_OK ||
        (st = upload(c, &f->d_bscale, bscale.data(), bscale.size())) != DD_OK ||
        (st = upload(c, &f->d_imap, imap.data(), std::max<size_t>(1, imap.size()))) != DD_OK ||
        (st = upload(c, &f->d_gmap, prob->gamma_map, (size_t)std::max(1, nG))) != DD_OK ||
        (st = upload(c, &f->d_cptr, cptr.data(), cptr.size())) != DD_OK ||
        (st = upload(c, &f->d_cent, cent.data(), cent.size())) != DD_OK)
      return bail(st);
  }
  const size_t L = f->ldmax;
  double **lv[] = {&f->lam, &f->r, &f->w, &f->y, &f->p, &f->q, &f->d};
  for (double **v : lv)
    if ((st = dalloc(c, v, (size_t)f->nlam * L)) != DD_OK) return bail(st);
  double **uv[] = {&f->tU, &f->sU, &f->fU};
  for (double **v : uv)
    if ((st = dalloc(c, v, (size_t)NU * L)) != DD_OK) return bail(st);
  double **gv[] = {&f->gx, &f->gr, &f->gz, &f->gp, &f->gq, &f->gt, &f->gu};
  for (double **v : gv)
    if ((st = dalloc(c, v, (size_t)std::max(1, nG) * L)) != DD_OK) return bail(st);
  if ((st = dalloc(c, &f->cz3, (size_t)std::max(1, f->nc) * L)) != DD_OK) return bail(st);
  if ((st = dalloc(c, &f->cz, (size_t)std::max(1, nc) * L)) != DD_OK ||
      (st = dalloc(c, &f->cz2, (size_t)std::max(1, nc) * L)) != DD_OK ||
      (st = dalloc(c, &f->dpart, (size_t)(grid_for(std::max(std::max(f->nlam, NU), NI), kRowsE) + 1) * kMaxLd)) != DD_OK ||
      (st = dalloc(c, &f->dout, kMaxLd)) != DD_OK)
    return bail(st);
  if (hipHostMalloc((void **)&f->h_dots, kMaxLd * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    f->err = "pinned host allocation failed";
    return bail(DD_ENOMEM);
  }
  *out = f;
  return DD_OK;
}

dd_status dd_feti_factor(dd_feti_ctx *f) {
  if (!f) return ffail(nullptr, DD_EINVAL, "ctx is NULL");
  f->err.clear();
  dd_status st = dd_factor(f->D, DD_FP64);
  if (st != DD_OK) return ffail(f, st, "Dirichlet factor: " + f->D->err);
  st = dd_factor(f->P, DD_FP64);
  if (st != DD_OK) return ffail(f, st, "primal factor: " + f->P->err);
  f->factored = true;
  return DD_OK;
}

dd_status dd_feti_solve(dd_feti_ctx *f, const double *b_dev, double *u_dev, int32_t nrhs, int32_t ld,
                        double tol, int32_t max_it, dd_solve_info *info) {
  if (!f) return ffail(nullptr, DD_EINVAL, "ctx is NULL");
  f->err.clear();
  if (!f->factored) return ffail(f, DD_ESTATE, "dd_feti_factor has not run");
  if (nrhs < 1 || nrhs > f->max_nrhs) return ffail(f, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  if (ld < f->n_dof || !b_dev || !u_dev || b_dev == u_dev) return ffail(f, DD_EINVAL, "bad b/u or ld < n_dof");
  if (!(tol > 0.0) || max_it < 1) return ffail(f, DD_EINVAL, "tol <= 0 or max_it < 1");
  dd_ctx *c = f->D;
  const int L = next_pow2(nrhs);
  const size_t nl = (size_t)f->nlam, NU = (size_t)f->NU;
  Work &w = c->w;
  // stacked right-hand side: b_I (interiors), b_G split evenly over the copies
  if (f->NI > 0)
    hipLaunchKernelGGL(k_feti_gather, dim3(std::min(4096u, grid_for((size_t)f->NI * L, 256))), dim3(256), 0,
                       f->stream, f->NI, f->d_bmap, f->d_bscale, b_dev, ld, nrhs, L, w.bI);
  hipLaunchKernelGGL(k_feti_gather, dim3(std::min(4096u, grid_for(NU * L, 256))), dim3(256), 0, f->stream,
                     f->NU, f->d_bmap + f->NI, f->d_bscale + f->NI, b_dev, ld, nrhs, L, w.bG);
  // f = b_U - K_GI K_II^-1 b_I (eq. subForcing per subdomain)
  interior_solve(c, DD_FP64, DD_APPLY_INV, w.bI, w.wI, L);
  gamma_apply(c, DD_FP64, plain(nullptr), w.wI, L, w.bG, 0.0, -1.0, w.rG);    // rG = f
  // d = B S^+ f, e = Z^T f, lambda_0 = G (G^T G)^-1 e
  spinv(f, w.rG, f->fU, L);
  csr_apply(f, f->B, f->fU, L, nullptr, 1.0, f->d);
  if (f->nc > 0) {
    csr_apply(f, f->Zt, w.rG, L, nullptr, 1.0, f->cz);
    csr_apply(f, f->GtGi, f->cz, L, nullptr, 1.0, f->cz2);
    csr_apply(f, f->Gm, f->cz2, L, nullptr, 1.0, f->lam);
  } else {
    FHIP(hipMemsetAsync(f->lam, 0, nl * L * sizeof(double), f->stream));
  }
  // r = d - F lambda_0, w = P r
  fapply(f, f->lam, f->q, L);
  FHIP(hipMemcpyAsync(f->r, f->d, nl * L * sizeof(double), hipMemcpyDeviceToDevice, f->stream));
  std::vector<double> a(L, 0.0), w0(L, 0.0), wy_old(L, 0.0), wyv(L, 0.0);
  for (int col = 0; col < L; ++col) a[col] = -1.0;
  set_coef(f, a, L);
  axpy(f, nl, L, f->q, f->r);
  project(f, f->r, f->w, L);
  FTRY(dots(f, f->nlam, L, f->w, f->w));
  std::vector<int> active(L, 0), its(L, 0);
  for (int col = 0; col < L; ++col) {
    w0[col] = std::sqrt(f->h_dots[col]);
    active[col] = col < nrhs && w0[col] > 0.0;
  }
  bool any = false;
  for (int col = 0; col < L; ++col) any |= active[col] != 0;
  int it = 0;
  while (any && it < max_it) {
    // y = P M^-1 w; beta = (w.y) / (w.y)_old; p = y + beta p
    precond(f, f->w, f->y, L);
    project(f, f->y, f->y, L);
    FTRY(dots(f, f->nlam, L, f->w, f->y));
    for (int col = 0; col < L; ++col) {
      wyv[col] = f->h_dots[col];
      a[col] = (it == 0 || !active[col]) ? 0.0 : wyv[col] / wy_old[col];
    }
    set_coef(f, a, L);
    if (it == 0) FHIP(hipMemsetAsync(f->p, 0, nl * L * sizeof(double), f->stream));
    xpay(f, nl, L, f->y, f->p);
    // q = F p; alpha = (w.y) / (p.q)
    fapply(f, f->p, f->q, L);
    FTRY(dots(f, f->nlam, L, f->p, f->q));
    for (int col = 0; col < L; ++col) {
      const double pq = f->h_dots[col];
      if (active[col] && !(pq > 0.0)) return ffail(f, DD_ENOTSPD, "FETI breakdown: p^T F p <= 0");
      a[col] = active[col] ? wyv[col] / pq : 0.0;
      wy_old[col] = wyv[col];
    }
    set_coef(f, a, L);
    axpy(f, nl, L, f->p, f->lam);
    for (int col = 0; col < L; ++col) a[col] = -a[col];
    set_coef(f, a, L);
    axpy(f, nl, L, f->q, f->r);
    project(f, f->r, f->w, L);
    FTRY(dots(f, f->nlam, L, f->w, f->w));
    ++it;
    any = false;
    for (int col = 0; col < L; ++col)
      if (active[col]) {
        its[col] = it;
        if (std::sqrt(f->h_dots[col]) <= tol * w0[col]) active[col] = 0;
        any |= active[col] != 0;
      }
  }
  // alpha = (G^T G)^-1 G^T (d - F lambda) (eq. forAlpha); u_U = S^+ (f - B^T lambda) - Z alpha (eq. forU)
  fapply(f, f->lam, f->q, L);
  for (int col = 0; col < L; ++col) a[col] = -1.0;
  set_coef(f, a, L);
  FHIP(hipMemcpyAsync(f->r, f->d, nl * L * sizeof(double), hipMemcpyDeviceToDevice, f->stream));
  axpy(f, nl, L, f->q, f->r);
  csr_apply(f, f->Bt, f->lam, L, w.rG, -1.0, f->sU);        // f - B^T lambda
  spinv(f, f->sU, w.uG, L);
  if (f->nc > 0) {
    csr_apply(f, f->Gt, f->r, L, nullptr, 1.0, f->cz);
    csr_apply(f, f->GtGi, f->cz, L, nullptr, 1.0, f->cz2);
    csr_apply(f, f->Zm, f->cz2, L, w.uG, -1.0, w.uG);
  }
  // interiors by eq. backwardSubstitution, then the global solution
  kig_apply(c, DD_FP64, plain(w.uG), L, w.bI, -1.0, w.yI);
  interior_solve(c, DD_FP64, DD_APPLY_INV, w.yI, w.uI, L);
  hipLaunchKernelGGL(k_feti_scatter, dim3(std::min(4096u, grid_for((size_t)(f->NI + f->n_gamma) * nrhs, 256))),
                     dim3(256), 0, f->stream, f->NI, f->d_imap, w.uI, f->n_gamma, f->d_gmap, f->d_cptr, f->d_cent,
                     w.uG, L, nrhs, u_dev, ld);
  FHIP(hipGetLastError());
  FHIP(hipStreamSynchronize(f->stream));
  dd_status result = DD_OK;
  for (int col = 0; col < nrhs; ++col)
    if (active[col]) result = DD_ENOCONV;
  if (info) {
    // FP64 residual of the full system through the primal context
    std::vector<double> rel(nrhs);
    dd_status rs = residual_cols(f->P, b_dev, u_dev, nrhs, ld, rel.data());
    if (rs != DD_OK) return ffail(f, rs, "residual: " + f->P->err);
    for (int col = 0; col < nrhs; ++col) {
      info[col].iters = its[col];
      info[col].refine_steps = 0;
      info[col].used_fallback = 0;
      info[col].converged = !active[col];
      info[col].rel_resid = rel[col];
    }
  }
  if (result == DD_ENOCONV) f->err = "tolerance not reached for at least one column";
  return result;
}

dd_status dd_bdd_solve(dd_feti_ctx *f, const double *b_dev, double *u_dev, int32_t nrhs, int32_t ld, double tol,
                       int32_t max_it, dd_solve_info *info) {
  if (!f) return ffail(nullptr, DD_EINVAL, "ctx is NULL");
  f->err.clear();
  if (!f->factored) return ffail(f, DD_ESTATE, "dd_feti_factor has not run");
  if (nrhs < 1 || nrhs > f->max_nrhs) return ffail(f, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  if (ld < f->n_dof || !b_dev || !u_dev || b_dev == u_dev) return ffail(f, DD_EINVAL, "bad b/u or ld < n_dof");
  if (!(tol > 0.0) || max_it < 1) return ffail(f, DD_EINVAL, "tol <= 0 or max_it < 1");
  FTRY(bdd_prepare(f));
  dd_ctx *c = f->P;
  Work &w = c->w;
  const int L = next_pow2(nrhs), nG = f->n_gamma;
  const size_t ng = (size_t)nG;
  // b in the primal DD layout; reduced forcing g = b_G - K_GI K_II^-1 b_I (eq. subForcing)
  const int n_all = c->NI + nG;
  hipLaunchKernelGGL(k_gather2, dim3(std::min(4096u, grid_for((size_t)n_all * L, 256))), dim3(256), 0, f->stream,
                     c->NI, nG, c->d_imap, c->d_gmap, b_dev, ld, nrhs, L, w.bI, w.bG);
  interior_solve(c, DD_FP64, DD_APPLY_INV, w.bI, w.wI, L);
  gamma_apply(c, DD_FP64, plain(nullptr), w.wI, L, w.bG, 0.0, -1.0, f->gr);      // r = g (x = 0)
  FHIP(hipMemsetAsync(f->gx, 0, ng * L * sizeof(double), f->stream));
  // stop column c when ||r_c|| <= tol ||b_c|| (the stopping rule of dd_solve)
  std::vector<double> stop2(L, 0.0), rz(L, 0.0), a(L, 0.0);
  FTRY(dots(f, c->NI, L, w.bI, w.bI));
  for (int col = 0; col < L; ++col) stop2[col] = f->h_dots[col];
  FTRY(dots(f, nG, L, w.bG, w.bG));
  for (int col = 0; col < L; ++col) stop2[col] = tol * tol * (stop2[col] + f->h_dots[col]);
  FTRY(dots(f, nG, L, f->gr, f->gr));
  std::vector<int> active(L, 0), its(L, 0);
  bool any = false;
  for (int col = 0; col < L; ++col) {
    active[col] = col < nrhs && f->h_dots[col] > stop2[col];
    any |= active[col] != 0;
  }
  if (any) {
    bdd_minv(f, f->gr, f->gz, L);
    FHIP(hipMemcpyAsync(f->gp, f->gz, ng * L * sizeof(double), hipMemcpyDeviceToDevice, f->stream));
    FTRY(dots(f, nG, L, f->gr, f->gz));
    for (int col = 0; col < L; ++col) rz[col] = f->h_dots[col];
  }
  int it = 0;
  while (any && it < max_it) {
    primal_schur(f, f->gp, f->gq, L);                       // q = S p
    FTRY(dots(f, nG, L, f->gp, f->gq));
    for (int col = 0; col < L; ++col) {
      const double pq = f->h_dots[col];
      if (active[col] && !(pq > 0.0)) return ffail(f, DD_ENOTSPD, "BDD breakdown: p^T S p <= 0");
      a[col] = active[col] ? rz[col] / pq : 0.0;
    }
    set_coef(f, a, L);
    axpy(f, ng, L, f->gp, f->gx);                           // x += alpha p
    for (int col = 0; col < L; ++col) a[col] = -a[col];
    set_coef(f, a, L);
    axpy(f, ng, L, f->gq, f->gr);                           // r -= alpha q
    FTRY(dots(f, nG, L, f->gr, f->gr));
    ++it;
    any = false;
    for (int col = 0; col < L; ++col)
      if (active[col]) {
        its[col] = it;
        if (f->h_dots[col] <= stop2[col]) active[col] = 0;
        any |= active[col] != 0;
      }
    if (!any) break;
    bdd_minv(f, f->gr, f->gz, L);                           // z = M^-1 r
    FTRY(dots(f, nG, L, f->gr, f->gz));
    for (int col = 0; col < L; ++col) {
      a[col] = active[col] ? f->h_dots[col] / rz[col] : 0.0;
      if (active[col]) rz[col] = f->h_dots[col];
    }
    set_coef(f, a, L);
    xpay(f, ng, L, f->gz, f->gp);                           // p = z + beta p
  }
  // interiors by eq. backwardSubstitution, then the solution in the caller's layout
  kig_apply(c, DD_FP64, plain(f->gx), L, w.bI, -1.0, w.yI);
  interior_solve(c, DD_FP64, DD_APPLY_INV, w.yI, w.uI, L);
  hipLaunchKernelGGL(k_scatter2, dim3(std::min(4096u, grid_for((size_t)n_all * nrhs, 256))), dim3(256), 0,
                     f->stream, c->NI, nG, c->d_imap, c->d_gmap, w.uI, f->gx, L, nrhs, u_dev, ld);
  FHIP(hipGetLastError());
  FHIP(hipStreamSynchronize(f->stream));
  dd_status result = DD_OK;
  for (int col = 0; col < nrhs; ++col)
    if (active[col]) result = DD_ENOCONV;
  if (info) {
    std::vector<double> rel(nrhs);
    dd_status rs = residual_cols(c, b_dev, u_dev, nrhs, ld, rel.data());
    if (rs != DD_OK) return ffail(f, rs, "residual: " + c->err);
    for (int col = 0; col < nrhs; ++col) {
      info[col].iters = its[col];
      info[col].refine_steps = 0;
      info[col].used_fallback = 0;
      info[col].converged = !active[col];
      info[col].rel_resid = rel[col];
    }
  }
  if (result == DD_ENOCONV) f->err = "tolerance not reached for at least one column";
  return result;
}

dd_status dd_method_solve(dd_feti_ctx *f, int32_t method, const double *b_dev, double *u_dev, int32_t nrhs,
                          int32_t ld, double tol, int32_t max_it, dd_solve_info *info);

dd_status dd_method_autotune(dd_feti_ctx *f, int32_t nrhs, double tol, int32_t max_it, int32_t *method,
                             double *ms) {
  if (!f) return ffail(nullptr, DD_EINVAL, "ctx is NULL");
  f->err.clear();
  if (!f->factored) return ffail(f, DD_ESTATE, "dd_feti_factor has not run");
  if (nrhs < 1 || nrhs > f->max_nrhs) return ffail(f, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  if (!(tol > 0.0) || max_it < 1) return ffail(f, DD_EINVAL, "tol <= 0 or max_it < 1");
  // the primal context's own schedule for the Jacobi-preconditioned method
  {
    dd_solve_opts o;
    dd_default_opts(&o);
    o.tol = tol;
    o.max_it = max_it;
    dd_tune_result tr;
    dd_status st = dd_autotune(f->P, DD_FP64, nrhs, &o, &tr);
    if (st != DD_OK) return ffail(f, st, "primal schedule: " + f->P->err);
  }
  double *b = nullptr, *u = nullptr;
  const size_t n = (size_t)f->n_dof * nrhs;
  if (hipMalloc(&b, n * sizeof(double)) != hipSuccess) return ffail(f, DD_ENOMEM, "autotune right-hand side");
  if (hipMalloc(&u, n * sizeof(double)) != hipSuccess) {
    (void)hipFree(b);
    return ffail(f, DD_ENOMEM, "autotune solution");
  }
  hipLaunchKernelGGL(k_feti_pattern, dim3(std::min(4096u, grid_for(n, 256))), dim3(256), 0, f->stream, f->n_dof,
                     nrhs, f->n_dof, b);
  double best = 1e300;
  int choice = DD_METHOD_FETI;
  double t3[3] = {0.0, 0.0, 0.0};
  dd_status result = DD_OK;
  for (int m = DD_METHOD_FETI; m <= DD_METHOD_JACOBI && result == DD_OK; ++m) {
    double tm = 1e300;
    for (int rep = 0; rep < 3; ++rep) {        // the first run is a warm-up
      if (hipStreamSynchronize(f->stream) != hipSuccess) { result = ffail(f, DD_EHIP, "autotune sync"); break; }
      const auto t0 = std::chrono::steady_clock::now();
      dd_status st = dd_method_solve(f, m, b, u, nrhs, f->n_dof, tol, max_it, nullptr);
      const auto t1 = std::chrono::steady_clock::now();
      if (st == DD_ENOCONV) { tm = 1e300; break; }        // a method that misses the tolerance loses
      if (st != DD_OK) { result = st; break; }
      if (rep > 0) tm = std::min(tm, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    t3[m - 1] = tm;
    if (tm < best) { best = tm; choice = m; }
  }
  (void)hipFree(b);
  (void)hipFree(u);
  if (result != DD_OK) return result;
  f->err.clear();
  f->method = choice;
  f->tuned_nrhs = nrhs;
  for (int i = 0; i < 3; ++i) f->tune_ms[i] = t3[i];
  if (method) *method = choice;
  if (ms)
    for (int i = 0; i < 3; ++i) ms[i] = t3[i];
  return DD_OK;
}

dd_status dd_method_solve(dd_feti_ctx *f, int32_t method, const double *b_dev, double *u_dev, int32_t nrhs,
                          int32_t ld, double tol, int32_t max_it, dd_solve_info *info) {
  if (!f) return ffail(nullptr, DD_EINVAL, "ctx is NULL");
  if (method == DD_METHOD_AUTO) {
    if (!f->method) {
      dd_status st = dd_method_autotune(f, nrhs, tol, max_it, nullptr, nullptr);
      if (st != DD_OK) return st;
    }
    method = f->method;
  }
  switch (method) {
    case DD_METHOD_FETI: return dd_feti_solve(f, b_dev, u_dev, nrhs, ld, tol, max_it, info);
    case DD_METHOD_BDD: return dd_bdd_solve(f, b_dev, u_dev, nrhs, ld, tol, max_it, info);
    case DD_METHOD_JACOBI: {
      f->err.clear();
      if (!f->factored) return ffail(f, DD_ESTATE, "dd_feti_factor has not run");
      dd_solve_opts o;
      dd_default_opts(&o);
      o.tol = tol;
      o.max_it = max_it;
      std::vector<dd_solve_info> tmp(std::max(1, (int)nrhs));
      dd_status st = dd_solve(f->P, DD_FP64, b_dev, u_dev, nrhs, ld, &o, info ? info : tmp.data());
      if (st != DD_OK) f->err = f->P->err;
      return st;
    }
    default: return ffail(f, DD_EINVAL, "unknown method");
  }
}

const char *dd_feti_last_error(const dd_feti_ctx *f) { return f ? f->err.c_str() : g_setup_error.c_str(); }

void dd_feti_destroy(dd_feti_ctx *f) {
  if (!f) return;
  if (f->h_dots) (void)hipHostFree(f->h_dots);
  dd_destroy(f->D);
  dd_destroy(f->P);
  delete f;
}

}  // extern "C"
