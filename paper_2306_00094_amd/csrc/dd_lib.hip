// Host side of the substructuring Schur-complement solver: validation and
// deep copy of the partitioned system, the batched factorisation, and the
// solve pipeline (condensation, preconditioned CG on the interface Schur
// complement, back substitution, mixed-precision refinement), exported
// through the C ABI declared in include/dd.h.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dd.h"
#include "dd_kernels.h"
#include "dd_tiles.h"
#include "dd_assemble.h"
#include "dd_persistent.h"

using namespace dd;

namespace {

thread_local std::string g_setup_error;

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Operators of one precision.
struct Ops {
  void *L = nullptr;       // factor blocks (T)
  void *kinv = nullptr;    // inverse blocks (T), exactly symmetric
  void *ig_val = nullptr;  // K_IG values (T)
  void *g_val = nullptr;   // [K_GG | K_GI] values (T)
  double *diag = nullptr;  // diag(S)
  double *dinv = nullptr;  // 1 / diag(S)
  void *tI_val = nullptr;  // 16x8 units of K_IG (T), wide batches
  void *tG_val = nullptr;  // 16x8 units of [K_GG | K_GI] (T), wide batches
  void *kinv_t = nullptr;  // K_II^{-1} packed into 16x16 tiles (T), wide batches
  bool ready = false;
};

// Per-column solver state in one allocation, so one copy brings it to the host.
struct StateBlock {
  double rz[kMaxLd], alpha[kMaxLd], beta[kMaxLd], stop2[kMaxLd], nrm2[kMaxLd];
  double bnrm2[kMaxLd], rnrm2[kMaxLd];
  double rz2[2 * kMaxLd], rz_prev[kMaxLd];
  int active[kMaxLd], iters[kMaxLd], flag[kMaxLd];
  int act2[2 * kMaxLd], bd[kMaxLd], act_prev[kMaxLd], brk[kMaxLd];
  double ref2[kMaxLd];
};

struct Work {
  // interface (n_gamma x ldmax)
  double *bG, *xG, *rG, *zG, *pG, *qG, *uG, *dG, *tG;
  double *r2G, *z2G;       // second residual / preconditioned residual (three-launch iteration)
  double *qdG;             // D^{-1} q (three-launch iteration)
  // FP32 gather copies of the mixed three-launch iteration: z by parity (like
  // zG / z2G), D^{-1} q and p (n_gamma x ldmax), w (NI x ldmax)
  float *z32A, *z32B, *qd32, *p32, *w32;
  // interior (NI x ldmax)
  double *bI, *yI, *wI, *uI, *dI, *tI;
  double *bnrm2, *rnrm2;   // ldmax
};

}  // namespace

struct dd_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int n_dof = 0, n_gamma = 0, n_sub = 0, NI = 0, max_nrhs = 0, ldmax = 1, max_ni = 0;
  std::vector<int> ni, ioff;
  std::vector<long long> koff;
  long long ktot = 0;
  size_t nnz_ig = 0, nnz_g = 0;
  // structure
  int n_rb = 0, *d_rb_first = nullptr;   // row blocks of kRB rows (never crossing subdomains)
  int n_gram = 0;                         // 16x16 lower output tiles of all K_II^{-1} blocks
  int2 *d_gram_tiles = nullptr;
  // diag(S) on the matrix cores: K_IG^k packed into 16-column strips (positions
  // of every K_IG entry), strip work items, per-subdomain local interface slots
  // and, per interface dof, its slots in subdomain order
  long long vpack = 0;
  int nloc = 0, n_wsq = 0;
  long long *d_vpos = nullptr, *d_voff = nullptr;
  int *d_goff = nullptr, *d_dptr = nullptr, *d_dent = nullptr;
  int4 *d_wsq_items = nullptr;
  double *d_kgg_diag = nullptr;
  int *d_ni = nullptr, *d_ioff = nullptr, *d_rowsub = nullptr, *d_imap = nullptr,
      *d_gmap = nullptr;
  long long *d_koff = nullptr;
  int *d_ig_ptr = nullptr, *d_ig_col = nullptr;
  int *d_g_ptr = nullptr, *d_g_split = nullptr, *d_g_col = nullptr;
  // wide batches on the matrix cores (built when max_nrhs >= 8 and there are
  // interiors): 16x8 units of K_IG over blocks of kTileRbI x 16 interior rows,
  // of [K_GG | K_GI] over blocks of kTileRbG x 16 interface rows (entries
  // [ptr, split) multiply p, [split, ptr+1) multiply w; t_nI, t_nG count 16x8
  // units), and the (subdomain, 16-row tile) work items of the interior solve
  bool tiles = false;
  int t_nrbI = 0, t_nrbG = 0, n_dit = 0;
  size_t t_nI = 0, t_nG = 0;
  int *d_tI_ptr = nullptr, *d_tI_col = nullptr;
  int *d_tG_ptr = nullptr, *d_tG_split = nullptr, *d_tG_col = nullptr;
  double *d_tI_val64 = nullptr, *d_tG_val64 = nullptr;
  int2 *d_dit = nullptr;
  long long t_kpack = 0;              // elements of the packed dense blocks (16x16 tiles)
  long long *d_toff = nullptr;        // per subdomain offset of its packed tiles
  double *d_kii_t = nullptr;          // K_II packed into tiles (FP64 residual of the mixed path)
  double *d_ig_val64 = nullptr, *d_g_val64 = nullptr, *d_kii64 = nullptr;
  Ops op[2];
  Work w{};
  ColState st{};
  StateBlock *d_state = nullptr;
  RedBuf red{};
  int *d_status = nullptr, *d_bad = nullptr;
  size_t max_chunks = 0;
  int *d_solve_mask = nullptr;         // refinement column mask of dd_solve (kMaxLd)
  int gamma_parts = 0;                  // p^T q group sums written by the last interface-row launch
  // host polling
  int *h_nact = nullptr;          // pinned, mapped
  StateBlock *h_state = nullptr;   // pinned copy target of the device state block
  int *h_mask = nullptr;           // pinned staging of per-column masks (kMaxLd)
  double *h_stop2 = nullptr;       // pinned staging of stopping thresholds (kMaxLd)
  int *h_nact_dev = nullptr;
  int nslots = 0;
  std::vector<hipEvent_t> ev;
  std::vector<void *> allocs;
  size_t bytes = 0;
  int use_mfma = 1;
  int direction_kernel = 0;   // 1: keep p in memory, update it with its own kernel
  int classic_cg = 0;         // 1: four launches per CG iteration also where three would do
  int old_trtri = 0;          // 1: L^{-1} by one wave per block column (no LDS panel)
  int panel_potrf = 0;        // 1: Cholesky by two launches per 16-wide panel
  int flow_spin = kFlowSpin;  // bound of each wait in the single-launch Cholesky (sleeps)
  int gather32 = 0;           // 1: untuned mixed three-launch solves gather FP32 vector copies
  int tune_persistent = 0;    // 1: the autotuner also times the cooperative persistent launch
  Gather32 g32{};             // FP32 gather copies of the three-launch iteration being launched
  int *d_flow = nullptr;      // single-launch Cholesky: ticket, timeout, done flags
  double *fac_x = nullptr, *fac_packed = nullptr, *fac_dloc = nullptr;   // factor work space
  bool packed_ready = false;
  int num_cu = 0;
  size_t max_lds = 65536;     // LDS bytes one workgroup may use
  unsigned *d_bar = nullptr;  // persistent-launch barrier: count, generation, abort
  long long spin_limit = 1ll << 20;
  int last_launch = DD_LAUNCH_KERNELS;
  struct GraphEntry {
    int prec, ld, apply, precond, dk, iters, cg3;
    double *x;
    hipGraphExec_t exec;
    double drop;      // residual replacement: the drop factor the direction launches carry
  };
  std::vector<GraphEntry> graphs;
  bool capturing = false;
  // autotuned schedules per precision and batch width (log2)
  struct Tuned {
    bool set = false;
    int apply = 0, launch = 0, dk = 0, check_every = 0, cg3 = 1;
    double ms = 0, inner_tol = 0;
    double drop = 0;            // mixed, replacing schedule: the replacement drop factor
  };
  int force_cg3 = -1;         // autotuner: -1 schedule decides, else the schedule bits (bit 0 three
                              // launches, bit 1 FP32 gathers)
  Tuned tuned[2][7];
  // continuous batching
  struct Batch {
    bool on = false;
    int prec = 0;
    dd_solve_opts o{};
    int ld = 1;
    int state[kMaxLd] = {0}, its[kMaxLd] = {0}, steps[kMaxLd] = {0}, conv[kMaxLd] = {0};
    int stall[kMaxLd] = {0};
    double bn2[kMaxLd] = {0}, rn2[kMaxLd] = {0}, prev[kMaxLd] = {0}, stop2[kMaxLd] = {0};
    // FP32 gathers (mixed): the direction is kept in pG by its own kernel and
    // the FP32-data products gather FP32 copies of it and of w
    bool g32 = false;
    int *d_mask = nullptr, *d_slots = nullptr;
  } batch;
  hipStream_t cap_stream = nullptr;   // capture only (the legacy default stream cannot capture)
  // optional per-phase kernel timing with HIP events (dd_set_timing)
  unsigned timing_mask = 0;
  std::vector<hipEvent_t> tev;          // event pool, pairs (start, stop)
  std::vector<int> tev_phase;           // phase of each recorded pair
  size_t tev_used = 0;
  int tev_cg3_ld = 0;                   // recorded pairs come from a three-launch CG loop of this width
  double t_ms[DD_NPHASES] = {0};
  long long t_count[DD_NPHASES] = {0};
  std::string err;
};

namespace {

dd_status fail(dd_ctx *c, dd_status s, const std::string &m) {
  if (c) c->err = m; else g_setup_error = m;
  return s;
}

#define HIPCHK(ctx, expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail((ctx), DD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_) + \
                                      " (" + std::to_string((int)e_) + ")");       \
  } while (0)

template <typename T>
dd_status dalloc(dd_ctx *c, T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) return fail(c, DD_ENOMEM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  c->allocs.push_back(q);
  c->bytes += n * sizeof(T);
  *p = (T *)q;
  return DD_OK;
}

template <typename T>
dd_status upload(dd_ctx *c, T **p, const T *h, size_t n) {
  dd_status s = dalloc(c, p, n);
  if (s != DD_OK) return s;
  if (n) HIPCHK(c, hipMemcpy(*p, h, n * sizeof(T), hipMemcpyHostToDevice));
  return DD_OK;
}

#define TRY(expr)                  \
  do {                             \
    dd_status s_ = (expr);         \
    if (s_ != DD_OK) return s_;    \
  } while (0)

unsigned grid_for(size_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// --------------------------------------------------------------- validation --
dd_status validate(const dd_problem *p) {
  if (!p) return fail(nullptr, DD_EINVAL, "problem is NULL");
  if (p->n_dof < 1) return fail(nullptr, DD_EINVAL, "n_dof < 1");
  if (p->n_gamma < 0 || p->n_gamma > p->n_dof) return fail(nullptr, DD_EINVAL, "n_gamma out of range");
  if (p->n_sub < 0 || (p->n_sub > 0 && !p->sub)) return fail(nullptr, DD_EINVAL, "n_sub < 0 or sub is NULL");
  if (p->n_gamma > 0 && (!p->gamma_map || !p->kgg_rowptr))
    return fail(nullptr, DD_EINVAL, "gamma_map / kgg_rowptr is NULL");
  std::vector<int> seen(p->n_dof, 0);
  for (int j = 0; j < p->n_gamma; ++j) {
    int g = p->gamma_map[j];
    if (g < 0 || g >= p->n_dof) return fail(nullptr, DD_EINVAL, "gamma_map entry out of range");
    if (seen[g]++) return fail(nullptr, DD_EINVAL, "gamma_map not injective");
  }
  if (p->n_gamma > 0) {
    if (p->kgg_rowptr[0] != 0) return fail(nullptr, DD_EINVAL, "kgg_rowptr[0] != 0");
    for (int j = 0; j < p->n_gamma; ++j) {
      if (p->kgg_rowptr[j + 1] < p->kgg_rowptr[j]) return fail(nullptr, DD_EINVAL, "kgg_rowptr not monotone");
      for (int a = p->kgg_rowptr[j]; a < p->kgg_rowptr[j + 1]; ++a)
        if (p->kgg_col[a] < 0 || p->kgg_col[a] >= p->n_gamma)
          return fail(nullptr, DD_EINVAL, "kgg_col out of range");
    }
  }
  for (int k = 0; k < p->n_sub; ++k) {
    const dd_subdomain &s = p->sub[k];
    std::string tag = "subdomain " + std::to_string(k) + ": ";
    if (s.n_i < 1) return fail(nullptr, DD_EINVAL, tag + "n_i < 1");
    if (s.n_g < 0 || s.n_g > p->n_gamma) return fail(nullptr, DD_EINVAL, tag + "n_g out of range");
    if (!s.k_ii || !s.i_map || !s.kig_rowptr) return fail(nullptr, DD_EINVAL, tag + "NULL array");
    std::vector<char> gs(p->n_gamma, 0);
    for (int g = 0; g < s.n_g; ++g) {
      int v = s.g_map[g];
      if (v < 0 || v >= p->n_gamma) return fail(nullptr, DD_EINVAL, tag + "g_map entry out of range");
      if (gs[v]++) return fail(nullptr, DD_EINVAL, tag + "g_map not injective");
    }
    for (int i = 0; i < s.n_i; ++i) {
      int g = s.i_map[i];
      if (g < 0 || g >= p->n_dof) return fail(nullptr, DD_EINVAL, tag + "i_map entry out of range");
      if (seen[g]++) return fail(nullptr, DD_EINVAL, tag + "dof " + std::to_string(g) + " assigned twice");
    }
    if (s.kig_rowptr[0] != 0) return fail(nullptr, DD_EINVAL, tag + "kig_rowptr[0] != 0");
    for (int i = 0; i < s.n_i; ++i) {
      if (s.kig_rowptr[i + 1] < s.kig_rowptr[i]) return fail(nullptr, DD_EINVAL, tag + "kig_rowptr not monotone");
      for (int a = s.kig_rowptr[i]; a < s.kig_rowptr[i + 1]; ++a)
        if (s.kig_col[a] < 0 || s.kig_col[a] >= s.n_g) return fail(nullptr, DD_EINVAL, tag + "kig_col out of range");
    }
    for (int j = 0; j < s.n_i; ++j)
      for (int i = 0; i < s.n_i; ++i)
        if (!std::isfinite(s.k_ii[(size_t)j * s.n_i + i]))
          return fail(nullptr, DD_EINVAL, tag + "k_ii has a non-finite entry");
  }
  for (int g = 0; g < p->n_dof; ++g)
    if (!seen[g]) return fail(nullptr, DD_EINVAL, "dof " + std::to_string(g) + " is neither interior nor interface");
  return DD_OK;
}

// Block CSR of 16x8 units over row blocks of RB x 16 rows and column blocks of
// kTU = 8 columns.  Row i's entries [ptr[i], mid) (columns in [0, ncol1)) go
// to the first part of its block, entries [mid, ptr[i+1]) (columns in [0,
// ncol2)) to the second, mid = split[i] (or ptr[i+1] when split is null).
// Within a part the column blocks are in increasing order; an entry (row
// block, column block) holds RB units, one per 16-row slice of the block (zero
// where the slice has no entry), so that one slice of the multiplied vector
// serves RB units.  Values are placed in the A-operand order of two steps of
// the 16x16x4 matrix instructions (UnitLayout in dd_tiles.h), zeros elsewhere.
// Returns the number of 16x8 units (entries x RB).
struct TileSet {
  std::vector<int> ptr, split, col;
  std::vector<double> val;
};
constexpr int kTileMinLd = 8;     // narrowest batch served by the tiled products
// 16-row slices per row block: the interface rows (the largest product) share
// each vector slice between two slices of rows; the interior rows K_IG, with
// fewer row blocks, keep one (their launch would otherwise fill the chip
// only half).
constexpr int kTileRbG = 2, kTileRbI = 1;

size_t build_tiles(int nrows, const int *ptr, const int *split, const int *col, const double *val,
                   int ncol1, int ncol2, int RB, TileSet *ts) {
  const int H = RB * kT;
  const int nrb = (nrows + H - 1) / H;
  std::vector<int> slot1((ncol1 + kTU - 1) / kTU + 1, -1), slot2((ncol2 + kTU - 1) / kTU + 1, -1);
  std::vector<int> cb1, cb2;
  size_t nent = 0;
  if (ts) {
    ts->ptr.assign(nrb + 1, 0);
    ts->split.assign(nrb, 0);
    ts->col.clear();
    ts->val.clear();
  }
  for (int rb = 0; rb < nrb; ++rb) {
    const int i0 = rb * H, i1 = std::min(nrows, i0 + H);
    cb1.clear();
    cb2.clear();
    for (int i = i0; i < i1; ++i) {
      const int mid = split ? split[i] : ptr[i + 1];
      for (int a = ptr[i]; a < mid; ++a) {
        const int cb = col[a] / kTU;
        if (slot1[cb] < 0) { slot1[cb] = 0; cb1.push_back(cb); }
      }
      for (int a = mid; a < ptr[i + 1]; ++a) {
        const int cb = col[a] / kTU;
        if (slot2[cb] < 0) { slot2[cb] = 0; cb2.push_back(cb); }
      }
    }
    std::sort(cb1.begin(), cb1.end());
    std::sort(cb2.begin(), cb2.end());
    const size_t base = nent;
    for (size_t t = 0; t < cb1.size(); ++t) slot1[cb1[t]] = (int)(base + t);
    for (size_t t = 0; t < cb2.size(); ++t) slot2[cb2[t]] = (int)(base + cb1.size() + t);
    nent += cb1.size() + cb2.size();
    if (ts) {
      for (int cb : cb1) ts->col.push_back(cb);
      ts->split[rb] = (int)ts->col.size();
      for (int cb : cb2) ts->col.push_back(cb);
      ts->ptr[rb + 1] = (int)ts->col.size();
      ts->val.resize(nent * RB * kUV, 0.0);
      for (int i = i0; i < i1; ++i) {
        const int mid = split ? split[i] : ptr[i + 1];
        const int h = (i - i0) / kT, ii = (i - i0) % kT;
        for (int a = ptr[i]; a < ptr[i + 1]; ++a) {
          const int t = a < mid ? slot1[col[a] / kTU] : slot2[col[a] / kTU];
          const int kk = col[a] % kTU;
          // U[ii][kk] of slice h is held by lane (kk % 4) * 16 + ii at step kk / 4
          ts->val[((size_t)t * RB + h) * kUV + UnitLayout::pos((kk % 4) * kT + ii, kk / 4)] += val[a];
        }
      }
    }
    for (int cb : cb1) slot1[cb] = -1;
    for (int cb : cb2) slot2[cb] = -1;
  }
  return nent * RB;
}

// Tiles of a problem (interior rows x interface columns, interface rows x
// [interface | interior] columns) counted from its CSR input.
void count_problem_tiles(const dd_problem *p, size_t *nI, size_t *nG) {
  std::vector<int> iptr(1, 0), icol;
  int NI = 0;
  for (int k = 0; k < p->n_sub; ++k) NI += p->sub[k].n_i;
  iptr.reserve(NI + 1);
  std::vector<std::vector<int>> gi(p->n_gamma);
  int r = 0;
  for (int k = 0; k < p->n_sub; ++k) {
    const dd_subdomain &s = p->sub[k];
    for (int i = 0; i < s.n_i; ++i, ++r) {
      for (int a = s.kig_rowptr[i]; a < s.kig_rowptr[i + 1]; ++a) {
        const int g = s.g_map[s.kig_col[a]];
        icol.push_back(g);
        gi[g].push_back(r);
      }
      iptr.push_back((int)icol.size());
    }
  }
  *nI = build_tiles(NI, iptr.data(), nullptr, icol.data(), nullptr, p->n_gamma, 1, kTileRbI, nullptr);
  std::vector<int> gptr(1, 0), gsplit, gcol;
  for (int j = 0; j < p->n_gamma; ++j) {
    for (int a = p->kgg_rowptr[j]; a < p->kgg_rowptr[j + 1]; ++a) gcol.push_back(p->kgg_col[a]);
    gsplit.push_back((int)gcol.size());
    for (int v : gi[j]) gcol.push_back(v);
    gptr.push_back((int)gcol.size());
  }
  *nG = build_tiles(p->n_gamma, gptr.data(), gsplit.data(), gcol.data(), nullptr, p->n_gamma,
                    std::max(1, NI), kTileRbG, nullptr);
}

size_t footprint_bytes(const dd_problem *p, dd_precision prec, int max_nrhs) {
  size_t NI = 0, kt = 0, nig = 0;
  for (int k = 0; k < p->n_sub; ++k) {
    NI += p->sub[k].n_i;
    kt += (size_t)p->sub[k].n_i * p->sub[k].n_i;
    nig += p->sub[k].kig_rowptr[p->sub[k].n_i];
  }
  size_t ngg = p->n_gamma ? (size_t)p->kgg_rowptr[p->n_gamma] : 0;
  size_t ld = next_pow2(std::max(1, max_nrhs));
  size_t b = 0;
  b += NI * 4 * 3 + p->n_gamma * 4 + p->n_sub * 16;                 // maps
  b += (NI + 1) * 4 + nig * 12 + (p->n_gamma + 1) * 8 + (ngg + nig) * 12;  // CSR (FP64)
  b += kt * 8;                                                        // K_II
  size_t s = prec == DD_MIXED ? 4 : 8;
  b += 2 * kt * s + p->n_gamma * 16;                                  // L, K^-1, diag
  if (prec == DD_MIXED) {
    b += (nig + ngg + nig) * 4;                                       // FP32 values
    b += 2 * kt * 8 + p->n_gamma * 16;    // FP64 factors of the fallback (formed on first use)
  }
  if (max_nrhs >= kTileMinLd && p->n_sub > 0 && p->n_gamma > 0) {    // tiles of the wide batches
    size_t tI = 0, tG = 0;
    count_problem_tiles(p, &tI, &tG);
    const size_t nrbI = (NI + kT * kTileRbI - 1) / (kT * kTileRbI),
                 nrbG = (p->n_gamma + kT * kTileRbG - 1) / (kT * kTileRbG);
    b += (tI + tG) * (4 + kUV * 8) + (nrbI + 1) * 4 + (2 * nrbG + 1) * 4 + NI * 8 / kT + 64;
    if (prec == DD_MIXED) b += (tI + tG) * kUV * 4;
    size_t kp = 0;                       // packed K_II (FP64) and K_II^{-1} (T)
    for (int k = 0; k < p->n_sub; ++k) {
      const size_t nt = (p->sub[k].n_i + kT - 1) / kT;
      kp += nt * nt * 256;
    }
    b += kp * 8 + kp * s + (p->n_sub + 1) * 8;
    if (prec == DD_MIXED) b += kp * 8;  // the FP64 fallback's packed inverse
  }
  b += (12 * (size_t)p->n_gamma + 6 * NI) * ld * 8;                   // work vectors
  b += (4 * (size_t)p->n_gamma + NI) * ld * 4;                        // FP32 gather copies
  size_t chunks = std::max<size_t>((p->n_gamma + kGChunk - 1) / kGChunk,
                                   (std::max<size_t>(p->n_gamma, NI) + kRowsE - 1) / kRowsE) + 1;
  b += 3 * chunks * kMaxLd * 8;
  b += (chunks / kPGroup + 1) * (kMaxLd * 8 + kCounterStride * 4);
  if (p->n_sub > 0) {                     // factor work space: X, packed K_IG strips, diag(S) parts
    b += kt * 8;
    for (int k = 0; k < p->n_sub; ++k)
      b += ((size_t)(p->sub[k].n_i + 15) / 16) * ((p->sub[k].n_g + 15) / 16) * 256 * 8 + p->sub[k].n_g * 8;
  }
  return b;
}

// ------------------------------------------------------------ launchers --
template <int C, typename VT>
void launch_csr(dd_ctx *c, int nrows, const int *ptr, const int *col, const VT *val,
                Src x, int ld, const double *base, double sign, double *out, double *dir) {
  if (nrows <= 0) return;
  if (x.z)
    hipLaunchKernelGGL((k_csr_rows<C, VT, true>), dim3(grid_for(nrows, kWavesPerBlock)), dim3(kBlock), 0,
                       c->stream, nrows, ptr, col, val, x, ld, base, sign, out,
                       dir ? c->n_gamma : 0, dir);
  else
    hipLaunchKernelGGL((k_csr_rows<C, VT, false>), dim3(grid_for(nrows, kWavesPerBlock)), dim3(kBlock), 0,
                       c->stream, nrows, ptr, col, val, x, ld, base, sign, out, 0, (double *)nullptr);
}

template <typename VT>
void csr_rows(dd_ctx *c, int nrows, const int *ptr, const int *col, const VT *val,
              Src x, int ld, const double *base, double sign, double *out, double *dir = nullptr) {
  switch (std::min(ld, 16)) {
    case 1: launch_csr<1, VT>(c, nrows, ptr, col, val, x, ld, base, sign, out, dir); break;
    case 2: launch_csr<2, VT>(c, nrows, ptr, col, val, x, ld, base, sign, out, dir); break;
    case 4: launch_csr<4, VT>(c, nrows, ptr, col, val, x, ld, base, sign, out, dir); break;
    case 8: launch_csr<8, VT>(c, nrows, ptr, col, val, x, ld, base, sign, out, dir); break;
    default: launch_csr<16, VT>(c, nrows, ptr, col, val, x, ld, base, sign, out, dir); break;
  }
}

template <int C, typename MT, typename AT>
void launch_dense(dd_ctx *c, const MT *blocks, const double *y, int ld, const double *base,
                  double sign, double *out, const int *sptr, const int *scol, const double *sval,
                  const double *sx, float *out32) {
  if (c->NI <= 0) return;
  hipLaunchKernelGGL((k_dense_rows<C, MT, AT>), dim3(grid_for(c->NI, kWavesPerBlock)),
                     dim3(kBlock), 0, c->stream, c->NI, blocks, c->d_koff, c->d_ioff, c->d_ni,
                     c->d_rowsub, y, ld, base, sign, out, sptr, scol, sval, sx, out32);
}

template <typename MT, typename AT>
void dense_rows(dd_ctx *c, const MT *blocks, const double *y, int ld, const double *base,
                double sign, double *out, const int *sptr = nullptr, const int *scol = nullptr,
                const double *sval = nullptr, const double *sx = nullptr, float *out32 = nullptr) {
  switch (std::min(ld, 16)) {
    case 1: launch_dense<1, MT, AT>(c, blocks, y, ld, base, sign, out, sptr, scol, sval, sx, out32); break;
    case 2: launch_dense<2, MT, AT>(c, blocks, y, ld, base, sign, out, sptr, scol, sval, sx, out32); break;
    case 4: launch_dense<4, MT, AT>(c, blocks, y, ld, base, sign, out, sptr, scol, sval, sx, out32); break;
    case 8: launch_dense<8, MT, AT>(c, blocks, y, ld, base, sign, out, sptr, scol, sval, sx, out32); break;
    default: launch_dense<16, MT, AT>(c, blocks, y, ld, base, sign, out, sptr, scol, sval, sx, out32); break;
  }
}

// Event pair recorded by the launch itself at the start and the end of one
// kernel of a timed phase (hipExtLaunchKernelGGL): the kernel's own duration,
// without the gap that events recorded between launches add.
bool kernel_events(dd_ctx *c, int phase, hipEvent_t *e0, hipEvent_t *e1) {
  if (!((c->timing_mask >> phase) & 1u) || c->capturing) return false;
  if (c->tev_used + 2 > c->tev.size()) {
    for (int i = 0; i < 256; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      c->tev.push_back(e);
    }
    c->tev_phase.resize(c->tev.size() / 2, 0);
  }
  *e0 = c->tev[c->tev_used];
  *e1 = c->tev[c->tev_used + 1];
  c->tev_phase[c->tev_used / 2] = phase;
  c->tev_used += 2;
  return true;
}

template <int C, typename VT>
void launch_gamma(dd_ctx *c, const VT *val, Src p, const double *z, int ld,
                  const double *base, double c1, double c2, double *out, int dot, double *pout,
                  const double *dinv, double *qd) {
  if (c->n_gamma <= 0) return;
  dim3 g(grid_for(c->n_gamma, kGChunk)), b(kGRows * kWave);
  if (dot) c->gamma_parts = (int)((g.x + kPGroup - 1) / kPGroup);   // group sums
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = dot && kernel_events(c, DD_PHASE_GAMMA, &e0, &e1);   // CG iterations only
  if (p.z) {
    if (timed)
      hipExtLaunchKernelGGL((k_gamma_rows<C, VT, true>), g, b, 0, c->stream, e0, e1, 0, c->n_gamma, c->d_g_ptr,
                            c->d_g_split, c->d_g_col, val, p, z, ld, base, c1, c2, out, dot, pout, c->red, c->st, dinv, qd, c->g32);
    else
      hipLaunchKernelGGL((k_gamma_rows<C, VT, true>), g, b, 0, c->stream, c->n_gamma, c->d_g_ptr,
                         c->d_g_split, c->d_g_col, val, p, z, ld, base, c1, c2, out, dot, pout, c->red, c->st, dinv, qd, c->g32);
  } else if (c->g32.p) {       // FP32 gathers of p and w (FP32-data products of the mixed path)
    constexpr auto kern = k_gamma_rows<C, VT, false, kGLanes, GUnroll<C>::U, false, kGRows, true>;
    if (timed)
      hipExtLaunchKernelGGL(kern, g, b, 0, c->stream, e0, e1, 0, c->n_gamma, c->d_g_ptr,
                            c->d_g_split, c->d_g_col, val, p, z, ld, base, c1, c2, out, dot, pout, c->red, c->st, dinv, qd, c->g32);
    else
      hipLaunchKernelGGL(kern, g, b, 0, c->stream, c->n_gamma, c->d_g_ptr,
                         c->d_g_split, c->d_g_col, val, p, z, ld, base, c1, c2, out, dot, pout, c->red, c->st, dinv, qd, c->g32);
  } else {
    if (timed)
      hipExtLaunchKernelGGL((k_gamma_rows<C, VT, false>), g, b, 0, c->stream, e0, e1, 0, c->n_gamma, c->d_g_ptr,
                            c->d_g_split, c->d_g_col, val, p, z, ld, base, c1, c2, out, dot, pout, c->red, c->st, dinv, qd, c->g32);
    else
      hipLaunchKernelGGL((k_gamma_rows<C, VT, false>), g, b, 0, c->stream, c->n_gamma, c->d_g_ptr,
                         c->d_g_split, c->d_g_col, val, p, z, ld, base, c1, c2, out, dot, pout, c->red, c->st, dinv, qd, c->g32);
  }
}

// Update-kernel launch shape: cpw chunks of kRowsE rows per workgroup (more
// chunks per workgroup for narrow batches; the chunk partials do not change).
inline int upd_cpw(int ld) { return ld >= 4 ? 1 : 4 / ld; }
inline unsigned upd_grid(int n_gamma, int ld) {
  unsigned ch = grid_for(n_gamma, kRowsE);
  unsigned w = (unsigned)upd_cpw(ld);
  return (ch + w - 1) / w;
}

// Workgroups of the direction launch that ends a split update: each reduces
// the chunk partials of its column block (redundantly), so more of them cost
// L2 reads and fewer of them leave CUs idle for the direction update.  (Its
// 512-thread workgroups run one per CU.)
constexpr unsigned kDirStateGrid = 256;
inline unsigned direction_state_grid(int ld) {
  const unsigned ncb = (unsigned)(ld / std::min(ld, kDirCols));
  // workgroup 0 (the column state) and the row workgroups together fill at
  // most one workgroup per CU: one more would wait for a second round
  return 1 + ncb * std::max(1u, (kDirStateGrid - 1) / ncb);
}

// CG update launch; the elements per thread follow from the batch width.
// red: 0 single-level reduction, 1 grouped, 2 split (mode 1, one chunk per
// workgroup; the direction launch k_cg_direction_state reduces the chunk
// partials and finishes the step).
void launch_update(dd_ctx *c, int mode, int ld, int nrhs, const double *dinv, double *x, double *r,
                   double *z, double *p, const double *q, int precond, int *host_nact,
                   int init_p_is_z, const int *mask, int npq, int red = 0, const int *run = nullptr) {
  if (c->n_gamma <= 0) return;
  const int cpw = upd_cpw(ld);
  const dim3 g(upd_grid(c->n_gamma, ld)), b(kBlock);
  const int E = std::max(1, cpw * kRowsE * ld / kBlock);
  if (cpw != 1) red = 0;
#define DD_UPD(EE)                                                                                        \
  if (red == 2)                                                                                           \
    hipLaunchKernelGGL((k_cg_update<EE, 2>), g, b, 0, c->stream, mode, c->n_gamma, ld, nrhs, dinv, x,      \
                       r, z, p, q, c->red, c->st, precond, host_nact, init_p_is_z, mask, npq, cpw, c->g32.p, run); \
  else if (red == 1)                                                                                      \
    hipLaunchKernelGGL((k_cg_update<EE, 1>), g, b, 0, c->stream, mode, c->n_gamma, ld, nrhs, dinv, x,      \
                       r, z, p, q, c->red, c->st, precond, host_nact, init_p_is_z, mask, npq, cpw, c->g32.p, run); \
  else                                                                                                    \
    hipLaunchKernelGGL((k_cg_update<EE>), g, b, 0, c->stream, mode, c->n_gamma, ld, nrhs, dinv, x,         \
                       r, z, p, q, c->red, c->st, precond, host_nact, init_p_is_z, mask, npq, cpw, c->g32.p, run)
  switch (E) {
    case 1: DD_UPD(1); break;
    case 2: DD_UPD(2); break;
    case 4: DD_UPD(4); break;
    case 8: DD_UPD(8); break;
    default: DD_UPD(16); break;
  }
#undef DD_UPD
}

// (qd != nullptr: also qd = D^{-1} out, with D^{-1} = dinv or the identity)
template <typename VT>
void gamma_rows(dd_ctx *c, const VT *val, Src p, const double *z, int ld,
                const double *base, double c1, double c2, double *out, int dot, double *pout,
                const double *dinv = nullptr, double *qd = nullptr) {
  switch (std::min(ld, 8)) {
    case 1: launch_gamma<1, VT>(c, val, p, z, ld, base, c1, c2, out, dot, pout, dinv, qd); break;
    case 2: launch_gamma<2, VT>(c, val, p, z, ld, base, c1, c2, out, dot, pout, dinv, qd); break;
    case 4: launch_gamma<4, VT>(c, val, p, z, ld, base, c1, c2, out, dot, pout, dinv, qd); break;
    default: launch_gamma<8, VT>(c, val, p, z, ld, base, c1, c2, out, dot, pout, dinv, qd); break;
  }
}

Src plain(const double *x) { return Src{x, nullptr, nullptr, nullptr}; }

void colnorm2(dd_ctx *c, int nrows, int ld, const double *v, double *acc) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_colnorm2, dim3(grid_for(nrows, kRowsE)), dim3(kBlock), 0, c->stream,
                     nrows, ld, v, c->red, acc);
}

// squared column norms of a DD-layout vector pair (interior, interface)
dd_status dd_norm2(dd_ctx *c, int ld, const double *vI, const double *vG, double *acc) {
  HIPCHK(c, hipMemsetAsync(acc, 0, kMaxLd * sizeof(double), c->stream));
  colnorm2(c, c->NI, ld, vI, acc);
  colnorm2(c, c->n_gamma, ld, vG, acc);
  return DD_OK;
}

// z_I = (K_II)^{-1} y_I with the operators of precision `prec`.
void interior_solve(dd_ctx *c, int prec, int apply, const double *y, double *z, int ld) {
  if (c->NI <= 0) return;
  if (apply == DD_APPLY_TRSM) {
    int ncolw = std::min(ld, 16);
    dim3 grid(c->n_sub, ld / ncolw);
    if (prec == DD_FP64)
      hipLaunchKernelGGL((k_trsm_apply<double, double>), grid, dim3(kBlock), 0, c->stream,
                         (const double *)c->op[0].L, c->d_koff, c->d_ioff, c->d_ni, y, z, ld, ncolw);
    else
      hipLaunchKernelGGL((k_trsm_apply<float, float>), grid, dim3(kBlock), 0, c->stream,
                         (const float *)c->op[1].L, c->d_koff, c->d_ioff, c->d_ni, y, z, ld, ncolw);
    return;
  }
  if (ld >= 8 && c->n_rb > 0) {      // wide batches: kRB rows per wave share the y loads
    const dim3 g(grid_for(c->n_rb, kWavesPerBlock)), b(kBlock);
    if (prec == DD_FP64)
      hipLaunchKernelGGL((k_dense_rows_rb<8, double, double>), g, b, 0, c->stream, c->n_rb, c->d_rb_first,
                         (const double *)c->op[0].kinv, c->d_koff, c->d_ioff, c->d_ni, c->d_rowsub, y, ld, z,
                         c->g32.w);
    else
      hipLaunchKernelGGL((k_dense_rows_rb<8, float, float>), g, b, 0, c->stream, c->n_rb, c->d_rb_first,
                         (const float *)c->op[1].kinv, c->d_koff, c->d_ioff, c->d_ni, c->d_rowsub, y, ld, z,
                         c->g32.w);
    return;
  }
  // (c->g32.w: FP32 copy of w for the FP32-data gathers of the interface rows)
  if (prec == DD_FP64)
    dense_rows<double, double>(c, (const double *)c->op[0].kinv, y, ld, nullptr, 1.0, z, nullptr, nullptr,
                               nullptr, nullptr, c->g32.w);
  else
    dense_rows<float, float>(c, (const float *)c->op[1].kinv, y, ld, nullptr, 1.0, z, nullptr, nullptr,
                             nullptr, nullptr, c->g32.w);
}

// y = K_IG x (+ base, sign) with the coupling values of `prec`.
// y = base + sign * K_IG x; with an on-the-fly direction x and dir != nullptr
// the launch also stores that direction (all interface rows) into dir.
void kig_apply(dd_ctx *c, int prec, Src x, int ld, const double *base, double sign,
               double *out, double *dir = nullptr) {
  if (prec == DD_FP64)
    csr_rows<double>(c, c->NI, c->d_ig_ptr, c->d_ig_col, (const double *)c->op[0].ig_val, x, ld,
                     base, sign, out, dir);
  else
    csr_rows<float>(c, c->NI, c->d_ig_ptr, c->d_ig_col, (const float *)c->op[1].ig_val, x, ld,
                    base, sign, out, dir);
}

void gamma_apply(dd_ctx *c, int prec, Src p, const double *z, int ld, const double *base,
                 double c1, double c2, double *out, int dot = 0, double *pout = nullptr,
                 const double *dinv = nullptr, double *qd = nullptr) {
  if (prec == DD_FP64)
    gamma_rows<double>(c, (const double *)c->op[0].g_val, p, z, ld, base, c1, c2, out, dot, pout, dinv, qd);
  else
    gamma_rows<float>(c, (const float *)c->op[1].g_val, p, z, ld, base, c1, c2, out, dot, pout, dinv, qd);
}

// ------------------------------------------------- tiled wide batches --
// (batches of kTileMinLd or more columns; dd_tiles.h)
template <typename VT, int NCB, bool DOT>
void launch_tile_rows_t(dd_ctx *c, bool interface_rows, const VT *val, const double *x1,
                        const double *x2, int ld, const double *base, double c1, double c2,
                        double *out, const int *run, const float *x1f, const float *x2f) {
  const int nrb = interface_rows ? c->t_nrbG : c->t_nrbI;
  const int nrows = interface_rows ? c->n_gamma : c->NI;
  if (nrb <= 0) return;
  const dim3 g(nrb), b(kTW * kWave);
  const int *ptr = interface_rows ? c->d_tG_ptr : c->d_tI_ptr;
  const int *split = interface_rows ? c->d_tG_split : nullptr;
  const int *col = interface_rows ? c->d_tG_col : c->d_tI_col;
  const int n2 = interface_rows ? c->NI : 0;
  if (DOT) c->gamma_parts = (int)((g.x + kPGroup - 1) / kPGroup);   // group sums of p^T q
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto launch = [&](auto kern) {
    if (DOT && kernel_events(c, DD_PHASE_GAMMA, &e0, &e1))
      hipExtLaunchKernelGGL(kern, g, b, 0, c->stream, e0, e1, 0, nrb, nrows, ptr, split, col, val, x1,
                            c->n_gamma, x2, n2, ld, base, c1, c2, out, c->red, run, x1f, x2f);
    else
      hipLaunchKernelGGL(kern, g, b, 0, c->stream, nrb, nrows, ptr, split, col, val, x1, c->n_gamma, x2, n2,
                         ld, base, c1, c2, out, c->red, run, x1f, x2f);
  };
  // two entries' operands in flight per wave: three or four measured slower on
  // the peridynamic 32-column batch (FP64 interface launch 78 -> 81 us with
  // three; FP32 57 us with two or three, 59 with four)
  constexpr int kDepth = 2;
  if (interface_rows) launch(k_tile_rows<VT, NCB, DOT, kDepth, kTileRbG>);
  else launch(k_tile_rows<VT, NCB, DOT, kDepth, kTileRbI>);
}

// out = base + c1 * (tiled K_IG or K_GG) x1 + c2 * (tiled K_GI) x2 with the
// coupling values of `prec` (interface_rows: [K_GG | K_GI], else K_IG).  With
// both parts c2 must be c1 or -c1 (the kernel sums both parts in one
// accumulator).
// (x1f, x2f: FP32 copies of x1, x2 for the FP32 units; nullptr: none)
template <bool DOT>
void tile_rows(dd_ctx *c, int prec, bool interface_rows, const double *x1, const double *x2, int ld,
               const double *base, double c1, double c2, double *out, const int *run = nullptr,
               const float *x1f = nullptr, const float *x2f = nullptr) {
  // FP64 values straight from the setup copies: the FP64 residual of the mixed
  // path runs on contexts whose FP64 operators were never formed
  const void *v = prec == DD_FP64 ? (interface_rows ? (const void *)c->d_tG_val64 : (const void *)c->d_tI_val64)
                                  : (interface_rows ? c->op[prec].tG_val : c->op[prec].tI_val);
#define DD_TR(NCB)                                                                                     \
  if (prec == DD_FP64)                                                                                 \
    launch_tile_rows_t<double, NCB, DOT>(c, interface_rows, (const double *)v, x1, x2, ld, base, c1, c2, out, run, \
                                         nullptr, nullptr);                                            \
  else                                                                                                 \
    launch_tile_rows_t<float, NCB, DOT>(c, interface_rows, (const float *)v, x1, x2, ld, base, c1, c2, out, run, \
                                        x1f, x2f)
  if (ld <= 16) { DD_TR(1); }
  else if (ld <= 32) { DD_TR(2); }
  else { DD_TR(4); }
#undef DD_TR
}

// w = base + sign * B y for the dense interior blocks B (kinv of `prec`, or the
// FP64 blocks K_II themselves when kii is set).
// (w32: also an FP32 copy of w when not nullptr)
void dense_tiles(dd_ctx *c, int prec, bool kii, const double *y, int ld, const double *base, double sign,
                 double *w, const int *run = nullptr, float *w32 = nullptr) {
  if (c->n_dit <= 0) return;
  const dim3 g(c->n_dit), b(kTW * kWave);
#define DD_DT(MT, NCB, BLK)                                                                                \
  hipLaunchKernelGGL((k_dense_tiles<MT, NCB>), g, b, 0, c->stream, c->NI, c->d_dit, (const MT *)(BLK),   \
                     c->d_toff, c->d_ioff, c->d_ni, y, ld, base, sign, w, run, w32)
  if (kii || prec == DD_FP64) {
    const void *blk = kii ? (const void *)c->d_kii_t : c->op[DD_FP64].kinv_t;
    if (ld <= 16) DD_DT(double, 1, blk);
    else if (ld <= 32) DD_DT(double, 2, blk);
    else DD_DT(double, 4, blk);
  } else {
    const void *blk = c->op[DD_MIXED].kinv_t;
    if (ld <= 16) DD_DT(float, 1, blk);
    else if (ld <= 32) DD_DT(float, 2, blk);
    else DD_DT(float, 4, blk);
  }
#undef DD_DT
}

// ------------------------------------------------ three-launch iteration --
// Launches K1 and K2 of CG iteration k (see k_cg_kig): K2's state
// workgroup, one workgroup per 64-row interface slice, then the row
// workgroups.
template <int C, int E, typename VT>
void launch_cg_kig_t(dd_ctx *c, const VT *val, int mode, int par, int ld, const CgVec &v,
                     const int *mask) {
  const unsigned nsl = grid_for(c->n_gamma, kRowsE);
  const unsigned g = nsl + grid_for(c->NI, kWavesPerBlock);
  if (c->g32.z_old)
    hipLaunchKernelGGL((k_cg_kig<C, E, VT, true>), dim3(g), dim3(kBlock), 0, c->stream, mode, par, c->NI,
                       (int)nsl, c->d_ig_ptr, c->d_ig_col, val, c->n_gamma, ld, v, c->w.yI, c->red, c->st,
                       mask, c->gamma_parts, c->g32);
  else
    hipLaunchKernelGGL((k_cg_kig<C, E, VT>), dim3(g), dim3(kBlock), 0, c->stream, mode, par, c->NI,
                       (int)nsl, c->d_ig_ptr, c->d_ig_col, val, c->n_gamma, ld, v, c->w.yI, c->red, c->st,
                       mask, c->gamma_parts, c->g32);
}

template <typename VT>
void launch_cg_kig(dd_ctx *c, const VT *val, int mode, int par, int ld, const CgVec &v,
                   const int *mask) {
  switch (ld) {
    case 1: launch_cg_kig_t<1, 1, VT>(c, val, mode, par, ld, v, mask); break;
    case 2: launch_cg_kig_t<2, 1, VT>(c, val, mode, par, ld, v, mask); break;
    case 4: launch_cg_kig_t<4, 1, VT>(c, val, mode, par, ld, v, mask); break;
    case 8: launch_cg_kig_t<8, 2, VT>(c, val, mode, par, ld, v, mask); break;
    case 16: launch_cg_kig_t<16, 4, VT>(c, val, mode, par, ld, v, mask); break;
    case 32: launch_cg_kig_t<16, 8, VT>(c, val, mode, par, ld, v, mask); break;
    default: launch_cg_kig_t<16, 16, VT>(c, val, mode, par, ld, v, mask); break;
  }
}

template <int C, typename MT, typename AT>
void launch_cg_dense_t(dd_ctx *c, const MT *kinv, int mode, int par, int ld, int nrhs, const CgVec &v,
                       const int *mask, int *host_nact) {
  const unsigned nsl = grid_for(c->n_gamma, kRowsE) + 1;     // slices and the state workgroup
  if (ld >= 8 && c->n_rb > 0) {
    const unsigned nrb = grid_for(c->n_rb, kWavesPerBlock);
#define DD_K2RB(G)                                                                                     \
  hipLaunchKernelGGL((k_cg_dense_rb<8, MT, AT, G>), dim3(nsl + nrb), dim3(kBlock), 0, c->stream, mode,     \
                     par, c->n_rb, (int)nsl, c->d_rb_first, kinv, c->d_koff, c->d_ioff, c->d_ni,           \
                     c->d_rowsub, c->w.yI, ld, c->w.wI, c->n_gamma, nrhs, v.z, v.p, c->red, c->st, mask, \
                     host_nact, c->g32)
    if (c->g32.w) DD_K2RB(true);
    else DD_K2RB(false);
#undef DD_K2RB
  } else {
    const unsigned nrb = grid_for(c->NI, kWavesPerBlock);
#define DD_K2(G)                                                                                        \
  hipLaunchKernelGGL((k_cg_dense<C, MT, AT, G>), dim3(nsl + nrb), dim3(kBlock), 0, c->stream, mode, par,    \
                     c->NI, (int)nsl, kinv, c->d_koff, c->d_ioff, c->d_ni, c->d_rowsub, c->w.yI, ld,        \
                     c->w.wI, c->n_gamma, nrhs, v.z, v.p, c->red, c->st, mask, host_nact, c->g32)
    if (c->g32.w) DD_K2(true);
    else DD_K2(false);
#undef DD_K2
  }
}

template <typename MT, typename AT>
void launch_cg_dense(dd_ctx *c, const MT *kinv, int mode, int par, int ld, int nrhs, const CgVec &v,
                     const int *mask, int *host_nact) {
  switch (std::min(ld, 8)) {
    case 1: launch_cg_dense_t<1, MT, AT>(c, kinv, mode, par, ld, nrhs, v, mask, host_nact); break;
    case 2: launch_cg_dense_t<2, MT, AT>(c, kinv, mode, par, ld, nrhs, v, mask, host_nact); break;
    case 4: launch_cg_dense_t<4, MT, AT>(c, kinv, mode, par, ld, nrhs, v, mask, host_nact); break;
    default: launch_cg_dense_t<8, MT, AT>(c, kinv, mode, par, ld, nrhs, v, mask, host_nact); break;
  }
}

// ---------------------------------------------------------------- factor --
// Single-launch left-looking Cholesky for blocks of up to 16 * 4 * 16 rows
// (row tiles per wave held in registers: the smallest OWN >= ceil(tiles / 4)).
// Returns false (nothing launched) when the blocks are larger.
template <typename T>
bool launch_potrf_flow(dd_ctx *c, T *L, T *Xd) {
  const int ntmax = (c->max_ni + 15) / 16, need = (ntmax + 3) / 4;
  const dim3 grid((unsigned)(c->n_sub * ntmax)), blk(kBlock);
  unsigned *ticket = (unsigned *)c->d_flow;
  int *timeout = c->d_flow + 1, *done = c->d_flow + 2;
#define DD_FLOW(OWN)                                                                                  \
  hipLaunchKernelGGL((k_potrf_flow<T, OWN>), grid, blk, 0, c->stream, L, c->d_koff, c->d_ni, c->n_sub, \
                     ntmax, c->d_status, ticket, done, timeout, Xd, c->flow_spin)
  if (need <= 2) DD_FLOW(2);
  else if (need <= 4) DD_FLOW(4);
  else if (need <= 6) DD_FLOW(6);
  else if (need <= 8) DD_FLOW(8);
  else if (need <= 10) DD_FLOW(10);
  else if (need <= 12) DD_FLOW(12);
  else if (need <= 16) DD_FLOW(16);
  else return false;
#undef DD_FLOW
  return true;
}

template <typename T>
dd_status factor_impl(dd_ctx *c, int pi) {
  Ops &o = c->op[pi];
  T *L = (T *)o.L, *Kinv = (T *)o.kinv;
  // copy (and convert) K_II into the factor buffer
  size_t n = (size_t)c->ktot;
  if (pi == DD_FP64)
    hipLaunchKernelGGL((k_copy<double>), dim3(1024), dim3(256), 0, c->stream, n, c->d_kii64, (double *)L);
  else
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, c->stream, n, c->d_kii64, (float *)L);
  HIPCHK(c, hipGetLastError());
  // work space of the MFMA inverse path, kept for later factorisations: X = L^{-1}
  // (FP64-sized, serves both precisions), K_IG packed into strips (packed once:
  // the values do not change after setup), per-subdomain diag(S) parts
  const bool mfma_inv = c->n_sub > 0 && c->use_mfma;
  const int ntmax = (c->max_ni + 15) / 16;
  const size_t trtri_lds = ((size_t)ntmax * 256 + 2 * kWavesPerBlock * 256) * sizeof(T);
  const bool panel_trtri = trtri_lds <= c->max_lds && !c->old_trtri;
  if (mfma_inv && !c->fac_x) {
    dd_status st;
    if ((st = dalloc(c, &c->fac_x, n)) != DD_OK) return st;
    if (c->n_gamma > 0) {
      if ((st = dalloc(c, &c->fac_packed, (size_t)c->vpack)) != DD_OK) return st;
      if ((st = dalloc(c, &c->fac_dloc, (size_t)c->nloc)) != DD_OK) return st;
    }
  }
  T *X = mfma_inv ? (T *)c->fac_x : nullptr;
  if (c->n_sub > 0) HIPCHK(c, hipMemsetAsync(c->d_status, 0, c->n_sub * sizeof(int), c->stream));
  bool flow = false;
  if (c->use_mfma && c->n_sub > 0 && !c->panel_potrf) {
    // one launch; it also writes the diagonal blocks of X
    HIPCHK(c, hipMemsetAsync(c->d_flow, 0, (2 + 2 * (size_t)c->n_sub * ntmax) * sizeof(int), c->stream));
    flow = launch_potrf_flow<T>(c, L, panel_trtri ? X : nullptr);
    HIPCHK(c, hipGetLastError());
  }
  if (!flow) {
    // panel by panel: the diagonal block and the rows below it (one workgroup per
    // subdomain), then the trailing update of all subdomains' tiles
    for (int J = 0; J < ntmax; ++J) {
      hipLaunchKernelGGL((k_potrf_panel<T>), dim3(c->n_sub), dim3(kBlock), 0, c->stream, L, c->d_koff,
                         c->d_ni, c->d_status, J);
      const int m = c->max_ni - kNB * (J + 1);
      if (m > 0) {
        const int t16 = (m + 15) / 16;
        const int nt = t16 * (t16 + 1) / 2;
        hipLaunchKernelGGL((k_potrf_update<T>), dim3(grid_for(nt, kWavesPerBlock), c->n_sub), dim3(kBlock), 0,
                           c->stream, L, c->d_koff, c->d_ni, J, c->use_mfma);
      }
    }
  }
  HIPCHK(c, hipGetLastError());
  // the pivots are checked once at the end (a failed pivot is replaced by 1, so
  // the rest of the factorisation stays finite)
  HIPCHK(c, hipMemsetAsync(c->d_bad, 0, sizeof(int), c->stream));
  if (c->n_sub == 0) {
    // no interiors: nothing to invert (S = K_GG)
  } else if (c->use_mfma) {
    // K_II^{-1} = X^T X with X = L^{-1}, both steps on MFMA (X in a temporary block set);
    // diag(S) from the column sums of squares of X K_IG, also on MFMA
    double *packed = c->fac_packed, *dloc = c->fac_dloc;
    if (c->n_gamma > 0 && !c->packed_ready) {
      // strips without nonzeros keep zero parts (never written by k_schur_wsq)
      HIPCHK(c, hipMemsetAsync(packed, 0, (size_t)c->vpack * sizeof(double), c->stream));
      HIPCHK(c, hipMemsetAsync(dloc, 0, (size_t)c->nloc * sizeof(double), c->stream));
      if (c->nnz_ig > 0)
        hipLaunchKernelGGL(k_pack_strips, dim3(std::min<unsigned>(grid_for(c->nnz_ig, 256), 4096)), dim3(256), 0,
                           c->stream, (long long)c->nnz_ig, c->d_ig_val64, c->d_vpos, packed);
      HIPCHK(c, hipGetLastError());
      c->packed_ready = true;
    }
    dim3 gt(c->n_sub, ntmax);
    if (panel_trtri) {
      if (!flow)      // the flow factorisation wrote the diagonal blocks already
        hipLaunchKernelGGL((k_trtri_diag<T>), gt, dim3(kWave), 0, c->stream, (const T *)L, X, c->d_koff, c->d_ni);
      HIPCHK(c, hipGetLastError());
      if (ntmax > 1) {
        HIPCHK(c, hipFuncSetAttribute((const void *)k_trtri_panel<T>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)trtri_lds));
        hipLaunchKernelGGL((k_trtri_panel<T>), dim3(c->n_sub, ntmax - 1), dim3(kBlock), trtri_lds, c->stream,
                           (const T *)L, X, c->d_koff, c->d_ni);
      }
    } else {
      hipLaunchKernelGGL((k_trtri<T>), gt, dim3(kWave), 0, c->stream, (const T *)L, X, c->d_koff, c->d_ni);
    }
    HIPCHK(c, hipGetLastError());
    if (c->n_gram > 0)
      hipLaunchKernelGGL((k_gram<T>), dim3(grid_for(c->n_gram, kWavesPerBlock)), dim3(kBlock), 0, c->stream,
                         (const T *)X, Kinv, c->d_koff, c->d_ni, c->d_gram_tiles, c->n_gram);
    HIPCHK(c, hipGetLastError());
    if (c->n_gamma > 0) {
      if (c->n_wsq > 0)
        hipLaunchKernelGGL((k_schur_wsq<T>), dim3(c->n_wsq), dim3(kBlock), 0, c->stream, (const T *)X, packed,
                           c->d_koff, c->d_voff, c->d_ni, c->d_goff, c->d_wsq_items, dloc);
      hipLaunchKernelGGL(k_schur_diag_sum, dim3(grid_for(c->n_gamma, 256)), dim3(256), 0, c->stream,
                         c->n_gamma, c->d_kgg_diag, c->d_dptr, c->d_dent, dloc, o.diag, o.dinv, c->d_bad);
      HIPCHK(c, hipGetLastError());
    }
  } else {
    dim3 ginv(c->n_sub, (c->max_ni + kInvCols - 1) / kInvCols);
    hipLaunchKernelGGL((k_inverse<T>), ginv, dim3(kBlock), 0, c->stream, (const T *)L, Kinv,
                       c->d_koff, c->d_ni);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL((k_symmetrize<T>), dim3(c->n_sub, 64), dim3(256), 0, c->stream, Kinv,
                       c->d_koff, c->d_ni);
    HIPCHK(c, hipGetLastError());
  }
  if (c->tiles && c->n_sub > 0) {   // K_II^{-1} in the tile order of the wide-batch interior solves
    hipLaunchKernelGGL((k_pack_tiles<T>), dim3(64, c->n_sub), dim3(256), 0, c->stream, c->n_sub,
                       (const T *)Kinv, c->d_koff, c->d_toff, c->d_ni, (T *)o.kinv_t);
    HIPCHK(c, hipGetLastError());
  }
  if (pi == DD_MIXED) {
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, c->stream, c->nnz_ig, c->d_ig_val64,
                       (float *)o.ig_val);
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, c->stream, c->nnz_g, c->d_g_val64,
                       (float *)o.g_val);
    if (c->tiles) {
      hipLaunchKernelGGL(k_units_to_f32, dim3(1024), dim3(256), 0, c->stream, c->t_nI / kTileRbI, kTileRbI,
                         c->d_tI_val64, (float *)o.tI_val);
      hipLaunchKernelGGL(k_units_to_f32, dim3(1024), dim3(256), 0, c->stream, c->t_nG / kTileRbG, kTileRbG,
                         c->d_tG_val64, (float *)o.tG_val);
    }
    HIPCHK(c, hipGetLastError());
  }
  if (c->n_gamma > 0 && !(c->n_sub > 0 && c->use_mfma))
    hipLaunchKernelGGL((k_schur_diag<T>), dim3(grid_for(c->n_gamma, kWavesPerBlock)), dim3(kBlock),
                       0, c->stream, c->n_gamma, c->d_g_ptr, c->d_g_split, c->d_g_col,
                       c->d_g_val64, (const T *)Kinv, c->d_koff, c->d_ioff, c->d_ni, c->d_rowsub,
                       o.diag, o.dinv, c->d_bad);
  HIPCHK(c, hipGetLastError());
  int bad = 0, flow_timeout = 0;
  std::vector<int> status(c->n_sub);
  if (c->n_sub > 0)
    HIPCHK(c, hipMemcpyAsync(status.data(), c->d_status, c->n_sub * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if (flow) HIPCHK(c, hipMemcpyAsync(&flow_timeout, c->d_flow + 1, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (flow_timeout) return fail(c, DD_EHIP, "factorisation: a block column waited too long for its predecessors");
  for (int k = 0; k < c->n_sub; ++k)
    if (status[k])
      return fail(c, DD_ENOTSPD, "subdomain " + std::to_string(k) + " not SPD at column " +
                                     std::to_string(status[k] - 1));
  if (bad)
    return fail(c, DD_ENOTSPD, "diag(S) not positive at interface row " + std::to_string(bad - 1));
  o.ready = true;
  return DD_OK;
}

dd_status ensure_ops(dd_ctx *c, int pi) {
  Ops &o = c->op[pi];
  if (o.L) return DD_OK;
  size_t s = pi == DD_FP64 ? 8 : 4;
  void *p;
  auto al = [&](void **dst, size_t bytes) -> dd_status {
    hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 1));
    if (e != hipSuccess) return fail(c, DD_ENOMEM, "hipMalloc of factor storage failed");
    c->allocs.push_back(p);
    c->bytes += bytes;
    *dst = p;
    return DD_OK;
  };
  TRY(al(&o.L, c->ktot * s));
  TRY(al(&o.kinv, c->ktot * s));
  TRY(al((void **)&o.diag, c->n_gamma * 8));
  TRY(al((void **)&o.dinv, c->n_gamma * 8));
  if (c->tiles) TRY(al(&o.kinv_t, (size_t)c->t_kpack * s));
  if (pi == DD_FP64) {
    o.ig_val = c->d_ig_val64;
    o.g_val = c->d_g_val64;
    o.tI_val = c->d_tI_val64;
    o.tG_val = c->d_tG_val64;
  } else {
    TRY(al(&o.ig_val, c->nnz_ig * 4));
    TRY(al(&o.g_val, c->nnz_g * 4));
    if (c->tiles) {
      TRY(al(&o.tI_val, c->t_nI * kUV * 4));
      TRY(al(&o.tG_val, c->t_nG * kUV * 4));
    }
  }
  return DD_OK;
}

// ----------------------------------------------------------- phase timing --
struct PhaseTimer {
  dd_ctx *c;
  int phase;
  bool on;
  PhaseTimer(dd_ctx *c_, int ph)
      : c(c_), phase(ph), on(((c_->timing_mask >> ph) & 1u) && !c_->capturing) {
    if (!on) return;
    if (c->tev_used + 2 > c->tev.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
        c->tev.push_back(e);
      }
      c->tev_phase.resize(c->tev.size() / 2, 0);
    }
    (void)hipEventRecord(c->tev[c->tev_used], c->stream);
  }
  ~PhaseTimer() {
    if (!on) return;
    (void)hipEventRecord(c->tev[c->tev_used + 1], c->stream);
    c->tev_phase[c->tev_used / 2] = phase;
    c->tev_used += 2;
  }
};

// Accumulate the recorded pairs (the stream must be idle).  When the pairs
// come from a three-launch CG loop (tev_cg3_ld > 0; h holds its final column
// state), its interface-row launches that swept the matrix are those of
// iterations 0 .. K-1, K the largest iteration count of its columns: the launch
// of iteration K and those enqueued after it return at once (every column had
// stopped) and are left out.
void collect_timing(dd_ctx *c, const StateBlock *h) {
  long keep_gamma = -1;                  // < 0: every interface-row pair counts
  if (c->tev_cg3_ld > 0 && h) {
    keep_gamma = 0;
    for (int j = 0; j < c->tev_cg3_ld; ++j) keep_gamma = std::max<long>(keep_gamma, h->iters[j]);
  }
  c->tev_cg3_ld = 0;
  for (size_t i = 0; i + 1 < c->tev_used; i += 2) {
    const int ph = c->tev_phase[i / 2];
    if (ph == DD_PHASE_GAMMA && keep_gamma >= 0) {
      if (keep_gamma == 0) continue;
      --keep_gamma;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->tev[i], c->tev[i + 1]) == hipSuccess) {
      c->t_ms[ph] += ms;
      c->t_count[ph] += 1;
    }
  }
  c->tev_used = 0;
}

// K1, K2 and K3 of iteration k (modes 0 and 1); r_{k-1} and z_{k-1} are in
// rG / zG for even k and in r2G / z2G for odd k.
void cg3_iteration(dd_ctx *c, int prec, int k, int mode, int ld, int nrhs, int precond, double *x,
                   const int *mask, int *host_nact, bool gather32) {
  Work &w = c->w;
  const Ops &op = c->op[prec];
  const int par = k & 1;
  const double *dinv = precond ? op.dinv : nullptr;
  CgVec v{dinv, x, par ? w.r2G : w.rG, par ? w.rG : w.r2G, par ? w.z2G : w.zG, par ? w.zG : w.z2G,
          w.pG, w.qG, w.qdG};
  // the FP32-data products of the mixed path gather FP32 copies of z, D^{-1} q, p and w
  if (prec == DD_MIXED && gather32)
    c->g32 = Gather32{par ? w.z32B : w.z32A, par ? w.z32A : w.z32B, w.qd32, w.p32, w.w32, w.qd32};
  struct ResetG32 { dd_ctx *c; ~ResetG32() { c->g32 = Gather32{}; } } reset_g32{c};
  {
    PhaseTimer t(c, DD_PHASE_KIG);
    if (prec == DD_FP64) launch_cg_kig<double>(c, (const double *)op.ig_val, mode, par, ld, v, mask);
    else launch_cg_kig<float>(c, (const float *)op.ig_val, mode, par, ld, v, mask);
  }
  {
    PhaseTimer t(c, DD_PHASE_INTERIOR);
    if (prec == DD_FP64)
      launch_cg_dense<double, double>(c, (const double *)op.kinv, mode, par, ld, nrhs, v, mask, host_nact);
    else
      launch_cg_dense<float, float>(c, (const float *)op.kinv, mode, par, ld, nrhs, v, mask, host_nact);
  }
  gamma_apply(c, prec, plain(w.pG), w.wI, ld, nullptr, 1.0, -1.0, w.qG, 1, nullptr, dinv, w.qdG);
}

// ------------------------------------------------------------------ solve --
struct CoreOpts {
  int max_it;
  int precond;
  int apply;
  int check_every;
  int launch;
  int cg3;        // bit 0: three launches per CG iteration where possible; bit 1: FP32 gathers (mixed)
  int reliable = 0;   // DD_MIXED, tiled: iterations between FP64 residual replacements (0: none)
  double replace_drop = 0.0;   // residual reduction after which a column is due for one
};

// Untuned solves run three launches per iteration (k_cg_kig) at every batch
// width, so a column's arithmetic never depends on the batch.  The autotuner
// may choose four per width (wide batches run them faster: the three-launch
// K_IG kernel holds more registers there).

// ------------------------------------------------------ persistent launch --
template <int C, typename VT, typename MT, typename AT>
dd_status launch_persistent_t(dd_ctx *c, PArgs<VT, MT> &a) {
  auto kern = k_pcg_persistent<C, VT, MT, AT>;
  int nb = 0;
  HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kPBlock, 0));
  if (nb < 1) return fail(c, DD_EHIP, "persistent kernel does not fit on a compute unit");
  int grid = nb * c->num_cu;
  HIPCHK(c, hipMemsetAsync(c->d_bar, 0, 4 * sizeof(unsigned), c->stream));
  void *args[] = {(void *)&a};
  {
    PhaseTimer t(c, DD_PHASE_LOOP);
    HIPCHK(c, hipLaunchCooperativeKernel((const void *)kern, dim3(grid), dim3(kPBlock), args, 0,
                                         c->stream));
  }
  return DD_OK;
}

template <typename VT, typename MT, typename AT>
dd_status launch_persistent(dd_ctx *c, int prec, int ld, int nrhs, int max_it, int precond,
                            double *x, double *pA, double *pB) {
  const Ops &op = c->op[prec];
  Work &w = c->w;
  PArgs<VT, MT> a;
  a.NI = c->NI; a.nG = c->n_gamma; a.ld = ld; a.nrhs = nrhs; a.max_it = max_it;
  a.use_precond = precond;
  a.ig_ptr = c->d_ig_ptr; a.ig_col = c->d_ig_col; a.ig_val = (const VT *)op.ig_val;
  a.kinv = (const MT *)op.kinv; a.koff = c->d_koff; a.ioff = c->d_ioff; a.ni = c->d_ni;
  a.rowsub = c->d_rowsub;
  a.g_ptr = c->d_g_ptr; a.g_split = c->d_g_split; a.g_col = c->d_g_col; a.g_val = (const VT *)op.g_val;
  a.dinv = op.dinv;
  a.x = x; a.r = w.rG; a.z = w.zG; a.pA = pA; a.pB = pB; a.q = w.qG; a.y = w.yI; a.w = w.wI;
  a.red = c->red; a.st = c->st; a.go = c->st.flag + 1;
  a.bar = GridBar{c->d_bar, c->d_bar + 1, c->d_bar + 2, c->spin_limit};
  switch (std::min(ld, 8)) {
    case 1: return launch_persistent_t<1, VT, MT, AT>(c, a);
    case 2: return launch_persistent_t<2, VT, MT, AT>(c, a);
    case 4: return launch_persistent_t<4, VT, MT, AT>(c, a);
    default: return launch_persistent_t<8, VT, MT, AT>(c, a);
  }
}

// The tiled wide-batch products serve this solve: schedule bit 2, tiles built,
// a batch of kTileMinLd or more columns, explicit inverses, no persistent launch.
bool use_tiles(const dd_ctx *c, int sched, int ld, int apply, int launch) {
  return (sched & 4) && c->tiles && ld >= kTileMinLd && apply != DD_APPLY_TRSM &&
         launch != DD_LAUNCH_PERSISTENT && c->NI > 0 && c->n_gamma > 0;
}

// One substructuring solve on DD-layout data:
//   g = bG - K_GI K_II^{-1} bI;  CG on S x = g until ||r_c||^2 <= stop2[c];
//   uI = K_II^{-1} (bI - K_IG x);  uG = x.
// stop2 must be set on the device before the call.  iters[c] and active[c]
// are left in the column state.
dd_status core_solve(dd_ctx *c, int prec, const double *bI, const double *bG, double *uI,
                     double *uG, int ld, int nrhs, const CoreOpts &o) {
  Work &w = c->w;
  const Ops &op = c->op[prec];
  // Wide batches on the matrix cores (schedule bit 2): tiled coupling products
  // and interior solves, the direction kept in memory by its own kernel.
  const bool tl = use_tiles(c, o.cg3, ld, o.apply, o.launch);
  // Residual replacement (mixed precision on the tiled path, FP64 operators
  // formed): the directions take S p with the FP32 operators, while the
  // condensation, the back substitution and, every `rel` iterations, the
  // residual r = g - S x come from the FP64 ones.  One Krylov space then
  // reaches the FP64 accuracy, where refinement restarts it per step.
  const int rel = (tl && prec == DD_MIXED && o.reliable > 0 && c->op[DD_FP64].ready &&
                   c->op[DD_FP64].kinv_t && c->n_gamma > 0) ? o.reliable : 0;
  const int cprec = rel ? DD_FP64 : prec;    // operators of condensation and back substitution
  double *gG = w.r2G;                        // condensed right-hand side g (unused by the tiled loop)
  // condensation (eq. subForcing summed over subdomains): r = bG - K_GI K_II^{-1} bI
  if (tl) {
    dense_tiles(c, cprec, false, bI, ld, nullptr, 1.0, w.wI);
    tile_rows<false>(c, cprec, true, nullptr, w.wI, ld, bG, 0.0, -1.0, w.rG);
    if (rel)
      HIPCHK(c, hipMemcpyAsync(gG, w.rG, (size_t)c->n_gamma * ld * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
  } else {
    interior_solve(c, prec, o.apply, bI, w.wI, ld);
    gamma_apply(c, prec, plain(nullptr), w.wI, ld, bG, 0.0, -1.0, w.rG);
  }
  // Three launches per iteration where the interiors exist and their inverse
  // is applied (k_cg_kig); otherwise four (K_IG, interior solve, interface
  // rows, update), which the persistent kernel also runs.
  const bool cg3 = !tl && (o.cg3 & 1) && c->NI > 0 && c->n_gamma > 0 && o.apply != DD_APPLY_TRSM &&
                   o.launch != DD_LAUNCH_PERSISTENT && !c->classic_cg;
  const int dkv = (c->direction_kernel || tl) ? 1 : 0;
  // FP32 gather copies for the FP32-data products (mixed): in the three-launch
  // iteration, or in the four-launch one with the direction kept by its kernel
  const bool g32 = !tl && (o.cg3 & 2) && prec == DD_MIXED && c->NI > 0 && c->n_gamma > 0 &&
                   o.apply != DD_APPLY_TRSM && o.launch != DD_LAUNCH_PERSISTENT &&
                   (cg3 || c->direction_kernel);
  const int sched = (cg3 ? 1 : 0) | (g32 ? 2 : 0) | (tl ? 4 : 0);
  // tiled mixed path: FP32 copies of p and w for the FP32 unit products
  // (which round their slices to FP32 anyway: the same sums from half the
  // slice bytes)
  const bool s32 = tl && prec == DD_MIXED;
  float *p32 = s32 ? w.p32 : nullptr, *w32 = s32 ? w.w32 : nullptr;
  struct ResetG32 { dd_ctx *c; ~ResetG32() { c->g32 = Gather32{}; } } reset_g32{c};
  c->tev_cg3_ld = cg3 ? ld : 0;
  // CG init: x = 0, z = D^-1 r, previous direction 0 (beta = 0)
  double *pA = w.pG, *pB = w.xG;
  if (c->n_gamma == 0)            // no init kernel to clear the breakdown flag
    HIPCHK(c, hipMemsetAsync(c->st.flag, 0, sizeof(int), c->stream));
  if (cg3)                        // iteration 0: start every column (p_0 = z_0, q_0 = S p_0)
    cg3_iteration(c, prec, 0, 0, ld, nrhs, o.precond, uG, nullptr, nullptr, g32);
  else if (c->n_gamma > 0) {
    // four launches: p (from the init and the direction kernel) and w (from the
    // interior solve) also written in FP32 for the gathers of the loop below
    if (g32) c->g32 = Gather32{nullptr, nullptr, nullptr, w.p32, w.w32, nullptr};
    // tiled mixed path: p also in FP32 (from the init and the direction
    // launch), the slices the FP32 unit products load
    if (s32) c->g32 = Gather32{nullptr, nullptr, nullptr, w.p32, nullptr, nullptr};
    launch_update(c, 0, ld, nrhs, op.dinv, uG, w.rG, w.zG, pA, w.qG, o.precond, nullptr,
                  dkv, nullptr, 0, tl ? 1 : 0);
  }
  HIPCHK(c, hipGetLastError());
  if (o.launch == DD_LAUNCH_PERSISTENT && o.apply != DD_APPLY_TRSM && c->n_gamma > 0) {
    dd_status ps = prec == DD_FP64
                       ? launch_persistent<double, double, double>(c, prec, ld, nrhs, o.max_it, o.precond, uG, pA, pB)
                       : launch_persistent<float, float, float>(c, prec, ld, nrhs, o.max_it, o.precond, uG, pA, pB);
    if (ps != DD_OK) return ps;
    unsigned abort_flag = 0;
    HIPCHK(c, hipMemcpyAsync(&abort_flag, c->d_bar + 2, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (abort_flag) return fail(c, DD_EHIP, "persistent CG kernel aborted: a grid barrier wait exceeded its limit");
    c->last_launch = DD_LAUNCH_PERSISTENT;
    kig_apply(c, prec, plain(uG), ld, bI, -1.0, w.yI);
    interior_solve(c, prec, o.apply, w.yI, uI, ld);
    HIPCHK(c, hipGetLastError());
    return DD_OK;
  }
  c->last_launch = DD_LAUNCH_KERNELS;
  // host polling with a lag: iteration `it` writes h_nact[it % nslots] = active + 1
  const int lag = std::min(8, std::max(1, o.check_every > 0 ? o.check_every : 2));
  std::vector<int> ring_it(c->nslots, -1);
  int it = 0;
  int observed = 0;       // last iteration whose result the host has seen
  bool stop = c->n_gamma == 0;
  // one CG iteration (S p, alpha, updates, beta); nact_dst receives
  // (active columns + 1) from the update kernel when non-null.  The tiled
  // iteration's launches do nothing once no column iterates (the flag the
  // last direction launch, or the initialisation, left in st.flag[1]): the
  // host enqueues up to check_every iterations past the last one needed.
  const int *run = tl ? c->st.flag + 1 : nullptr;
  auto iteration = [&](double *&pA_, double *&pB_, int *nact_dst, bool replace) -> dd_status {
    // direction p = z + beta p_prev, formed where it is gathered (or kept in pA)
    const bool dk = dkv != 0;
    Src P = dk ? plain(pA_) : Src{nullptr, w.zG, pA_, c->st.beta};
    if (dk && g32) P.x32 = w.p32;
    // S p (eq. subSchurComplement, summed): y = K_IG p, w = K_II^{-1} y, q = K_GG p - K_GI w
    // (formed at the K_IG gathers, which also store it into pB for the rest of
    // the iteration; without interiors the interface rows form and store it)
    const bool p_at_gamma = !dk && c->NI == 0;
    if (tl) {
      {
        PhaseTimer t(c, DD_PHASE_KIG);
        tile_rows<false>(c, prec, false, pA_, nullptr, ld, nullptr, 1.0, 0.0, w.yI, run, p32);
      }
      {
        PhaseTimer t(c, DD_PHASE_INTERIOR);
        dense_tiles(c, prec, false, w.yI, ld, nullptr, 1.0, w.wI, run, w32);
      }
      tile_rows<true>(c, prec, true, pA_, w.wI, ld, nullptr, 1.0, -1.0, w.qG, run, p32, w32);
    } else {
      {
        PhaseTimer t(c, DD_PHASE_KIG);
        kig_apply(c, prec, P, ld, nullptr, 1.0, w.yI, dk ? nullptr : pB_);
      }
      {
        PhaseTimer t(c, DD_PHASE_INTERIOR);
        interior_solve(c, prec, o.apply, w.yI, w.wI, ld);
      }
      // (timed, when asked, by events the launch itself records: kernel_events)
      gamma_apply(c, prec, (dk || p_at_gamma) ? P : plain(pB_), w.wI, ld, nullptr, 1.0, -1.0, w.qG, 1,
                  p_at_gamma ? pB_ : nullptr);
    }
    {
      PhaseTimer t(c, DD_PHASE_UPDATE);
      launch_update(c, 1, ld, nrhs, op.dinv, uG, w.rG, w.zG, dk ? pA_ : pB_, w.qG, o.precond,
                    tl ? nullptr : nact_dst, 0, nullptr, c->gamma_parts, tl ? 2 : 0, run);
    }
    if (tl && replace) {
      // the FP64 residual of the new x, q = g - K_GG x + K_GI K_II^{-1} K_IG x
      // (q, y and w are free until the next step), takes the place of r in
      // every iterating column.  The launches do nothing unless the last
      // direction launch found a column whose residual fell by the drop
      // factor since the last replacement (st.flag[2]).
      const int *due = c->st.flag + 2;
      tile_rows<false>(c, DD_FP64, false, uG, nullptr, ld, nullptr, 1.0, 0.0, w.yI, due);
      dense_tiles(c, DD_FP64, false, w.yI, ld, nullptr, 1.0, w.wI, due);
      tile_rows<false>(c, DD_FP64, true, uG, w.wI, ld, gG, -1.0, 1.0, w.qG, due);
      launch_update(c, 3, ld, nrhs, op.dinv, uG, w.rG, w.zG, pA_, w.qG, o.precond, nullptr, 0, nullptr, 0,
                    2, due);
    }
    if (tl) {        // the split update's state and the direction in one launch
      hipLaunchKernelGGL(k_cg_direction_state, dim3(direction_state_grid(ld)), dim3(kDirBlock), 0, c->stream,
                         c->n_gamma, ld, w.zG,
                         pA_, c->red, c->st, (int)upd_grid(c->n_gamma, ld), nact_dst, c->g32.p, run,
                         o.replace_drop * o.replace_drop);
    } else if (dk) {
      unsigned gd = std::min(4096u, grid_for((size_t)c->n_gamma * ld, kBlock));
      hipLaunchKernelGGL(k_cg_direction, dim3(gd), dim3(kBlock), 0, c->stream, c->n_gamma, ld,
                         w.zG, pA_, c->st, c->g32.p);
    } else {
      std::swap(pA_, pB_);
    }
    HIPCHK(c, hipGetLastError());
    return DD_OK;
  };
  // CG iteration k >= 1 in either scheme
  // (replace: this iteration ends with the residual replacement)
  auto step = [&](int k, double *&pA_, double *&pB_, int *nact_dst, bool replace) -> dd_status {
    if (!cg3) return iteration(pA_, pB_, nact_dst, replace);
    cg3_iteration(c, prec, k, 1, ld, nrhs, o.precond, uG, nullptr, nact_dst, g32);
    HIPCHK(c, hipGetLastError());
    return DD_OK;
  };
  if (o.launch == DD_LAUNCH_GRAPH && !stop) {
    // G iterations per graph (even, so the direction buffers return to place)
    int G = std::max(2, std::min(32, o.check_every > 0 ? o.check_every : 4));
    G += G & 1;
    // with residual replacement, a second graph of G iterations whose last
    // one replaces the residual, replayed every relG / G launches (relG: the
    // period rounded up to a multiple of G)
    const int relG = rel ? (rel + G - 1) / G * G : 0;
    auto graph_exec = [&](bool rb, hipGraphExec_t &exec) -> dd_status {
      const int key = sched | (rb ? 8 : 0);
      exec = nullptr;
      for (auto &g : c->graphs)
        if (g.prec == prec && g.ld == ld && g.apply == o.apply && g.precond == o.precond &&
            g.dk == dkv && g.iters == G && g.x == uG && g.cg3 == key && g.drop == o.replace_drop)
          exec = g.exec;
      if (!exec) {
        if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;     // kernels are recorded, not run
        hipError_t eb = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (eb != hipSuccess) {
          c->stream = user;
          return fail(c, DD_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(eb));
        }
        c->capturing = true;
        dd_status cs = DD_OK;
        double *qa = pA, *qb = pB;
        for (int i = 0; i < G && cs == DD_OK; ++i)     // iterations 1..G (odd k first)
          cs = step(1 + i, qa, qb, i == G - 1 ? c->h_nact_dev : nullptr, rb && i == G - 1);
        c->capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(c->cap_stream, &graph);
        c->stream = user;
        if (cs != DD_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return cs;
        }
        if (ee != hipSuccess)
          return fail(c, DD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
        ee = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ee != hipSuccess)
          return fail(c, DD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ee));
        c->graphs.push_back({prec, ld, o.apply, o.precond, dkv, G, key, uG, exec, o.replace_drop});
      }
      return DD_OK;
    };
    hipGraphExec_t exec = nullptr, exec_rel = nullptr;
    TRY(graph_exec(false, exec));
    if (rel) TRY(graph_exec(true, exec_rel));
    // replay; look at the result of launch n - 1 while launch n runs.  The
    // number of active columns only decreases, so a later value is as good.
    ((volatile int *)c->h_nact)[0] = 0;
    int launches = 0;
    const int max_launch = (o.max_it + G - 1) / G;
    while (launches < max_launch) {
      {
        PhaseTimer t(c, DD_PHASE_LOOP);
        const bool rb = rel && ((launches + 1) * G) % relG == 0;
        HIPCHK(c, hipGraphLaunch(rb ? exec_rel : exec, c->stream));
      }
      HIPCHK(c, hipEventRecord(c->ev[launches % c->nslots], c->stream));
      ++launches;
      if (launches >= 2) {
        HIPCHK(c, hipEventSynchronize(c->ev[(launches - 2) % c->nslots]));
        if (((volatile int *)c->h_nact)[0] == 1) break;
      }
    }
    c->last_launch = DD_LAUNCH_GRAPH;
  } else {
    // The update kernel of iteration `it` stores (active columns + 1) into
    // host memory h_nact[it % nslots]; the host waits for that value of
    // iteration it - lag by reading it (no event per iteration: an event
    // record adds a release of the caches and a gap between kernels).
    volatile int *hn = (volatile int *)c->h_nact;
    auto wait_slot = [&](int s2) -> dd_status {
      for (long spins = 1; hn[s2] == 0; ++spins) {
        if ((spins & 255) == 0) {
          hipError_t q = hipStreamQuery(c->stream);
          if (q == hipSuccess) {               // stream drained: the value must be there
            if (hn[s2] == 0) return fail(c, DD_EHIP, "CG state not published by the update kernel");
            break;
          }
          if (q != hipErrorNotReady)
            return fail(c, DD_EHIP, std::string("hipStreamQuery: ") + hipGetErrorString(q));
        }
      }
      return DD_OK;
    };
    while (!stop && it < o.max_it) {
      ++it;
      int slot = it % c->nslots;
      hn[slot] = 0;
      TRY(step(it, pA, pB, c->h_nact_dev + slot, rel > 0 && it % rel == 0));
      ring_it[slot] = it;
      // look at iteration it - lag, never more than nslots in flight
      int target = it - lag;
      while (observed < target) {
        int s2 = (observed + 1) % c->nslots;
        TRY(wait_slot(s2));
        ++observed;
        if (hn[s2] == 1) {
          stop = true;
          break;
        }
      }
    }
  }
  c->g32 = Gather32{};
  // back substitution (eq. backwardSubstitution): uI = K_II^{-1} (bI - K_IG uG)
  if (tl) {
    tile_rows<false>(c, cprec, false, uG, nullptr, ld, bI, -1.0, 0.0, w.yI);
    dense_tiles(c, cprec, false, w.yI, ld, nullptr, 1.0, uI);
  } else {
    kig_apply(c, prec, plain(uG), ld, bI, -1.0, w.yI);
    interior_solve(c, prec, o.apply, w.yI, uI, ld);
  }
  HIPCHK(c, hipGetLastError());
  return DD_OK;
}

// Squared stopping threshold of the inner (FP32-operator) CG of one
// refinement step: the relative reduction inner_tol of the current FP64
// residual, but never tighter than half the outer target tol * ||b||, so the
// last step stops as soon as the outer tolerance can be met instead of
// reducing the residual by inner_tol once more.
// Inner tolerance when neither the caller nor the autotuner chose one: the
// FP32 operators limit what one step can gain to about 1e-5..1e-6, and a
// step that stops there needs two steps for a 1e-9 target instead of three.
constexpr double kInnerTol = 1e-5;
// Residual replacement of the mixed tiled solve: every kReplacePeriod
// iterations the FP64 residual may take the place of the recurrence one; it
// does when some column's residual has fallen by the factor kReplaceDrop (in
// the direction launch) since the last replacement.  The recurrence, on FP32
// operators, drifts from the true residual by about 1e-5 of the residual at
// the last replacement, so the drift stays a small fraction of the current
// residual, and the solve stops at kReplaceStop times the target so that the
// drift since the last replacement stays inside it.
constexpr int kReplacePeriod = 8;
constexpr double kReplaceDrop = 1e-2;
constexpr double kReplaceStop = 0.7;
inline double resolve_inner_tol(const dd_ctx *c, int prec, int ld, double requested) {
  if (requested > 0.0) return requested;
  int lg = 0;
  while ((1 << lg) < ld) ++lg;
  const auto &t = c->tuned[prec][lg];
  return (t.set && t.inner_tol > 0.0) ? t.inner_tol : kInnerTol;
}
inline double inner_stop2(double inner_tol, double tol, double rn2, double bn2) {
  return std::max(inner_tol * inner_tol * rn2, 0.25 * tol * tol * bn2);
}

// breakdown_fails = false (inner solves of the mixed refinement): a breakdown
// of the FP32-operator CG (p^T S p <= 0 for an S that is positive definite
// but ill-conditioned beyond FP32) is not an error; the refinement step then
// fails to reduce the FP64 residual, and the column stalls and falls back to
// the FP64 path.
dd_status fetch_state(dd_ctx *c, StateBlock *h, bool breakdown_fails = true) {
  HIPCHK(c, hipMemcpyAsync(h, c->d_state, sizeof(StateBlock), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->tev_used) collect_timing(c, h);
  if (h->flag[0] && breakdown_fails) return fail(c, DD_ENOTSPD, "CG breakdown: p^T S p <= 0");
  return DD_OK;
}

// FP64 full-system residual in DD layout: rI = bI - K_II uI - K_IG uG,
// rG = bG - K_GI uI - K_GG uG.
void full_residual(dd_ctx *c, const double *bI, const double *bG, const double *uI,
                   const double *uG, double *rI, double *rG, int ld, bool tiles = false) {
  if (tiles) {      // the tiled products (FP64 values); rI passes through y
    tile_rows<false>(c, DD_FP64, false, uG, nullptr, ld, bI, -1.0, 0.0, c->w.yI);
    dense_tiles(c, DD_FP64, true, uI, ld, c->w.yI, -1.0, rI);
    tile_rows<false>(c, DD_FP64, true, uG, uI, ld, bG, -1.0, -1.0, rG);
    return;
  }
  dense_rows<double, double>(c, c->d_kii64, uI, ld, bI, -1.0, rI, c->d_ig_ptr, c->d_ig_col,
                             c->d_ig_val64, uG);
  gamma_rows<double>(c, c->d_g_val64, plain(uG), uI, ld, bG, -1.0, -1.0, rG, 0, nullptr);
}

// ||b_c - A u_c||_2 / ||b_c||_2 of caller-layout columns (column-major n_dof x
// nrhs, leading dimension ld) with the FP64 blocks of the context.
dd_status residual_cols(dd_ctx *c, const double *b, const double *u, int nrhs, int ld, double *rel) {
  const int L = next_pow2(nrhs);
  Work &w = c->w;
  const int n_all = c->NI + c->n_gamma;
  const unsigned g = std::min(4096u, grid_for((size_t)n_all * L, 256));
  hipLaunchKernelGGL(k_gather2, dim3(g), dim3(256), 0, c->stream, c->NI, c->n_gamma, c->d_imap, c->d_gmap, b,
                     ld, nrhs, L, w.bI, w.bG);
  hipLaunchKernelGGL(k_gather2, dim3(g), dim3(256), 0, c->stream, c->NI, c->n_gamma, c->d_imap, c->d_gmap, u,
                     ld, nrhs, L, w.uI, w.uG);
  full_residual(c, w.bI, w.bG, w.uI, w.uG, w.tI, w.tG, L);
  hipLaunchKernelGGL(k_norm2, dim3(grid_for((size_t)n_all, kRowsE)), dim3(kBlock), 0, c->stream, c->NI,
                     c->n_gamma, L, w.bI, w.bG, c->red, w.bnrm2, 0.0, (double *)nullptr);
  hipLaunchKernelGGL(k_norm2, dim3(grid_for((size_t)n_all, kRowsE)), dim3(kBlock), 0, c->stream, c->NI,
                     c->n_gamma, L, w.tI, w.tG, c->red, w.rnrm2, 0.0, (double *)nullptr);
  HIPCHK(c, hipGetLastError());
  StateBlock &h = *c->h_state;
  TRY(fetch_state(c, &h, false));
  for (int j = 0; j < nrhs; ++j)
    rel[j] = h.bnrm2[j] > 0.0 ? std::sqrt(h.rnrm2[j] / h.bnrm2[j]) : std::sqrt(h.rnrm2[j]);
  return DD_OK;
}

}  // namespace

// =================================================================== C ABI ==
extern "C" {

void dd_default_opts(dd_solve_opts *o) {
  if (!o) return;
  o->tol = 1e-10;
  o->max_it = 1000;
  o->precond = 1;
  o->max_refine = 8;
  o->inner_tol = 0.0;             // automatic: the tuned value, else kInnerTol
  o->fp64_fallback = 1;
  o->apply = DD_APPLY_AUTO;
  o->launch = DD_LAUNCH_AUTO;
  o->check_every = 0;
  o->verify = 1;
  o->gather32 = -1;
  o->tiles = -1;
  o->reliable = -1;
}

const char *dd_last_error(const dd_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_setup_error.c_str();
}

dd_status dd_footprint(const dd_problem *prob, dd_precision prec, int32_t max_nrhs, size_t *bytes) {
  if (!prob || !bytes || prob->n_sub < 0 || (prob->n_sub > 0 && !prob->sub))
    return fail(nullptr, DD_EINVAL, "bad arguments");
  if (max_nrhs < 1 || max_nrhs > kMaxLd) return fail(nullptr, DD_EINVAL, "max_nrhs out of [1, 64]");
  *bytes = footprint_bytes(prob, prec, max_nrhs);
  return DD_OK;
}

void dd_destroy(dd_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  for (void *p : c->allocs) (void)hipFree(p);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->h_nact) (void)hipHostFree(c->h_nact);
  if (c->h_state) (void)hipHostFree(c->h_state);
  if (c->h_mask) (void)hipHostFree(c->h_mask);
  if (c->h_stop2) (void)hipHostFree(c->h_stop2);
  delete c;
}

dd_status dd_setup(const dd_problem *p, void *hip_stream, int32_t max_nrhs, dd_ctx **out) {
  if (!out) return fail(nullptr, DD_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_nrhs < 1 || max_nrhs > kMaxLd) return fail(nullptr, DD_EINVAL, "max_nrhs out of [1, 64]");
  dd_status vs = validate(p);
  if (vs != DD_OK) return vs;
  dd_ctx *c = new (std::nothrow) dd_ctx();
  if (!c) return fail(nullptr, DD_ENOMEM, "host allocation failed");
  auto bail = [&](dd_status s) {
    g_setup_error = c->err;
    dd_destroy(c);
    return s;
  };
  c->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&c->device);
  c->n_dof = p->n_dof;
  c->n_gamma = p->n_gamma;
  c->n_sub = p->n_sub;
  c->max_nrhs = max_nrhs;
  c->ldmax = next_pow2(max_nrhs);
  if (const char *e = getenv("DD_NO_MFMA")) c->use_mfma = atoi(e) ? 0 : 1;
  if (const char *e = getenv("DD_DIRECTION_KERNEL")) c->direction_kernel = atoi(e) ? 1 : 0;
  if (const char *e = getenv("DD_CLASSIC_CG")) c->classic_cg = atoi(e) ? 1 : 0;
  if (const char *e = getenv("DD_BLOCKWAVE_TRTRI")) c->old_trtri = atoi(e) ? 1 : 0;
  if (const char *e = getenv("DD_PANEL_POTRF")) c->panel_potrf = atoi(e) ? 1 : 0;
  if (const char *e = getenv("DD_FLOW_SPIN")) c->flow_spin = std::max(0, std::min(atoi(e), kFlowSpin));
  if (const char *e = getenv("DD_GATHER32")) c->gather32 = atoi(e) ? 1 : 0;
  if (const char *e = getenv("DD_TUNE_PERSISTENT")) c->tune_persistent = atoi(e) ? 1 : 0;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
      c->num_cu = prop.multiProcessorCount;
      c->max_lds = prop.sharedMemPerBlock;
    }
    if (c->num_cu <= 0) c->num_cu = 1;
  }
  // host-side structure
  c->ni.resize(c->n_sub);
  c->ioff.resize(c->n_sub);
  c->koff.resize(c->n_sub);
  long long kt = 0;
  int NI = 0;
  for (int k = 0; k < c->n_sub; ++k) {
    c->ni[k] = p->sub[k].n_i;
    c->ioff[k] = NI;
    c->koff[k] = kt;
    NI += p->sub[k].n_i;
    kt += (long long)p->sub[k].n_i * p->sub[k].n_i;
    c->max_ni = std::max(c->max_ni, p->sub[k].n_i);
  }
  c->NI = NI;
  c->ktot = kt;
  std::vector<int> rowsub(NI), imap(NI);
  size_t nig = 0;
  for (int k = 0; k < c->n_sub; ++k) nig += (size_t)p->sub[k].kig_rowptr[p->sub[k].n_i];
  std::vector<int> igptr(NI + 1, 0), igcol(nig);
  std::vector<double> igval(nig);
  {
    size_t at = 0;
    for (int k = 0; k < c->n_sub; ++k) {
      const dd_subdomain &s = p->sub[k];
      for (int i = 0; i < s.n_i; ++i) {
        const int r = c->ioff[k] + i;
        rowsub[r] = k;
        imap[r] = s.i_map[i];
        for (int a = s.kig_rowptr[i]; a < s.kig_rowptr[i + 1]; ++a, ++at) {
          igcol[at] = s.g_map[s.kig_col[a]];
          igval[at] = s.kig_val[a];
        }
        igptr[r + 1] = (int)at;
      }
    }
  }
  // interface rows: [K_GG entries | K_GI entries (transposes of K_IG^k), by
  // increasing interior row], filled by counting
  std::vector<int> gptr(c->n_gamma + 1, 0), gsplit(c->n_gamma, 0);
  for (int j = 0; j < c->n_gamma; ++j) gptr[j + 1] = p->kgg_rowptr[j + 1] - p->kgg_rowptr[j];
  for (size_t a = 0; a < nig; ++a) ++gptr[igcol[a] + 1];
  for (int j = 0; j < c->n_gamma; ++j) gptr[j + 1] += gptr[j];
  std::vector<int> gcol(gptr[c->n_gamma]);
  std::vector<double> gval(gptr[c->n_gamma]);
  {
    std::vector<int> fill(c->n_gamma);
    for (int j = 0; j < c->n_gamma; ++j) {
      const int b = p->kgg_rowptr[j], len = p->kgg_rowptr[j + 1] - b;
      if (len) {
        memcpy(&gcol[gptr[j]], p->kgg_col + b, sizeof(int) * len);
        memcpy(&gval[gptr[j]], p->kgg_val + b, sizeof(double) * len);
      }
      gsplit[j] = fill[j] = gptr[j] + len;
    }
    for (int r = 0; r < NI; ++r)
      for (int a = igptr[r]; a < igptr[r + 1]; ++a) {
        const int j = igcol[a];
        gcol[fill[j]] = r;
        gval[fill[j]++] = igval[a];
      }
  }
  c->nnz_ig = igcol.size();
  c->nnz_g = gcol.size();
  std::vector<int> ni32(c->ni.begin(), c->ni.end());
  dd_status s;
  if ((s = upload(c, &c->d_ni, ni32.data(), c->n_sub)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_ioff, c->ioff.data(), c->n_sub)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_koff, c->koff.data(), c->n_sub)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_rowsub, rowsub.data(), NI)) != DD_OK) return bail(s);
  {
    std::vector<int> rbf;
    for (int k = 0; k < c->n_sub; ++k)
      for (int t = 0; t < p->sub[k].n_i; t += kRB) rbf.push_back(c->ioff[k] + t);
    c->n_rb = (int)rbf.size();
    if ((s = upload(c, &c->d_rb_first, rbf.data(), rbf.size())) != DD_OK) return bail(s);
    std::vector<int2> gt;
    for (int k = 0; k < c->n_sub; ++k) {
      const int nt = (p->sub[k].n_i + 15) / 16;
      for (int I = 0; I < nt; ++I)
        for (int J = 0; J <= I; ++J) gt.push_back(make_int2(k, (I << 16) | J));
    }
    c->n_gram = (int)gt.size();
    if ((s = upload(c, &c->d_gram_tiles, gt.data(), gt.size())) != DD_OK) return bail(s);
  }
  {
    std::vector<long long> voff(c->n_sub + 1, 0), vpos;
    std::vector<int> goff(c->n_sub + 1, 0);
    std::vector<int4> items;
    vpos.reserve(igval.size());
    for (int k = 0; k < c->n_sub; ++k) {
      const dd_subdomain &sd = p->sub[k];
      const int nt = (sd.n_i + 15) / 16, ns = (sd.n_g + 15) / 16;
      voff[k + 1] = voff[k] + (long long)nt * ns * 256;
      goff[k + 1] = goff[k] + sd.n_g;
      std::vector<int> kf(ns, INT_MAX), kl(ns, -1);
      for (int i = 0; i < sd.n_i; ++i)
        for (int a = sd.kig_rowptr[i]; a < sd.kig_rowptr[i + 1]; ++a) {
          const int jl = sd.kig_col[a], J = jl / 16, K = i / 16;
          kf[J] = std::min(kf[J], K);
          kl[J] = std::max(kl[J], K);
          vpos.push_back(voff[k] + ((long long)J * nt + K) * 256 + ((i % 16) / 4 * 16 + jl % 16) * 4 + i % 4);
        }
      for (int J = 0; J < ns; ++J)
        if (kl[J] >= 0) items.push_back(make_int4(k, J, kf[J], kl[J]));
    }
    {
      // Workgroup b runs on XCD b % 8 (round-robin dispatch), and each XCD has
      // its own L2: give every subdomain's strips one XCD, so its X_k is cached
      // once.  Subdomains go to XCDs by decreasing work (tile products), each to
      // the least loaded; within an XCD the longest strips come first, and the
      // XCD lists are interleaved (k = -1 pads a short list).
      constexpr int kXcd = 8;
      auto work = [&](const int4 &it) {
        const int nt = (p->sub[it.x].n_i + 15) / 16;
        long long w = 0;
        for (int I = it.z; I < nt; ++I) w += std::min(I, it.w) - it.z + 1;
        return w;
      };
      std::vector<long long> wk(c->n_sub, 0);
      for (const int4 &it : items) wk[it.x] += work(it);
      std::vector<int> order(c->n_sub);
      for (int k = 0; k < c->n_sub; ++k) order[k] = k;
      std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) { return wk[a2] > wk[b2]; });
      std::vector<int> xcd_of(c->n_sub, 0);
      long long load[kXcd] = {0};
      for (int k : order) {
        int x = 0;
        for (int y = 1; y < kXcd; ++y)
          if (load[y] < load[x]) x = y;
        xcd_of[k] = x;
        load[x] += wk[k];
      }
      std::vector<std::vector<int4>> bins(kXcd);
      for (const int4 &it : items) bins[xcd_of[it.x]].push_back(it);
      size_t len = 0;
      for (auto &b : bins) {
        std::stable_sort(b.begin(), b.end(), [&](const int4 &u, const int4 &v) { return work(u) > work(v); });
        len = std::max(len, b.size());
      }
      items.clear();
      for (size_t i = 0; i < len; ++i)
        for (int x = 0; x < kXcd; ++x) items.push_back(i < bins[x].size() ? bins[x][i] : make_int4(-1, 0, 0, 0));
    }
    std::vector<int> dptr(c->n_gamma + 1, 0), dent(goff[c->n_sub]);
    for (int k = 0; k < c->n_sub; ++k)
      for (int jl = 0; jl < p->sub[k].n_g; ++jl) ++dptr[p->sub[k].g_map[jl] + 1];
    for (int j = 0; j < c->n_gamma; ++j) dptr[j + 1] += dptr[j];
    {
      std::vector<int> fill(dptr.begin(), dptr.end() - 1);
      for (int k = 0; k < c->n_sub; ++k)
        for (int jl = 0; jl < p->sub[k].n_g; ++jl) dent[fill[p->sub[k].g_map[jl]]++] = goff[k] + jl;
    }
    std::vector<double> kd(c->n_gamma, 0.0);
    for (int j = 0; j < c->n_gamma; ++j)
      for (int a = p->kgg_rowptr[j]; a < p->kgg_rowptr[j + 1]; ++a)
        if (p->kgg_col[a] == j) kd[j] += p->kgg_val[a];
    c->vpack = voff[c->n_sub];
    c->nloc = goff[c->n_sub];
    c->n_wsq = (int)items.size();
    if ((s = upload(c, &c->d_vpos, vpos.data(), vpos.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_voff, voff.data(), voff.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_goff, goff.data(), goff.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_wsq_items, items.data(), items.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_dptr, dptr.data(), dptr.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_dent, dent.data(), dent.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_kgg_diag, kd.data(), kd.size())) != DD_OK) return bail(s);
  }
  if ((s = upload(c, &c->d_imap, imap.data(), NI)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_gmap, p->gamma_map, c->n_gamma)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_kii64, (size_t)kt)) != DD_OK) return bail(s);
  for (int k = 0; k < c->n_sub; ++k)          // straight from the caller's blocks
    if (c->ni[k] > 0 &&
        hipMemcpy(c->d_kii64 + c->koff[k], p->sub[k].k_ii, sizeof(double) * (size_t)c->ni[k] * c->ni[k],
                  hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "hipMemcpy of K_II failed";
      return bail(DD_EHIP);
    }
  if ((s = upload(c, &c->d_ig_ptr, igptr.data(), NI + 1)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_ig_col, igcol.data(), igcol.size())) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_ig_val64, igval.data(), igval.size())) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_g_ptr, gptr.data(), c->n_gamma + 1)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_g_split, gsplit.data(), c->n_gamma)) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_g_col, gcol.data(), gcol.size())) != DD_OK) return bail(s);
  if ((s = upload(c, &c->d_g_val64, gval.data(), gval.size())) != DD_OK) return bail(s);
  // tiles of the wide-batch products (matrix cores)
  if (c->ldmax >= kTileMinLd && c->n_sub > 0 && c->n_gamma > 0 && !getenv("DD_NO_TILES")) {
    TileSet ti, tg;
    c->t_nI = build_tiles(NI, igptr.data(), nullptr, igcol.data(), igval.data(), c->n_gamma, 1, kTileRbI, &ti);
    c->t_nG = build_tiles(c->n_gamma, gptr.data(), gsplit.data(), gcol.data(), gval.data(), c->n_gamma,
                          std::max(1, NI), kTileRbG, &tg);
    c->t_nrbI = (NI + kT * kTileRbI - 1) / (kT * kTileRbI);
    c->t_nrbG = (c->n_gamma + kT * kTileRbG - 1) / (kT * kTileRbG);
    // Interior-solve work items (subdomain, 16-row tile).  Workgroup b runs on
    // XCD b % 8: every subdomain's items go to one XCD (its slices of y are then
    // cached in one L2), subdomains by decreasing work to the least loaded XCD,
    // and the eight lists are interleaved (k = -1 pads a short list).
    constexpr int kXcd = 8;
    std::vector<int> order(c->n_sub);
    for (int k = 0; k < c->n_sub; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) { return c->ni[a2] > c->ni[b2]; });
    std::vector<std::vector<int2>> bins(kXcd);
    long long load[kXcd] = {0};
    for (int k : order) {
      int x = 0;
      for (int y = 1; y < kXcd; ++y)
        if (load[y] < load[x]) x = y;
      const int nt = (c->ni[k] + kT - 1) / kT;
      load[x] += (long long)nt * nt;
      for (int I = 0; I < nt; ++I) bins[x].push_back(make_int2(k, I));
    }
    size_t blen = 0;
    for (auto &bn : bins) blen = std::max(blen, bn.size());
    std::vector<int2> items;
    for (size_t i = 0; i < blen; ++i)
      for (int x = 0; x < kXcd; ++x) items.push_back(i < bins[x].size() ? bins[x][i] : make_int2(-1, 0));
    c->n_dit = (int)items.size();
    for (TileSet *t : {&ti, &tg})          // uploads need at least one element
      if (t->col.empty()) {
        t->col.push_back(0);
        t->val.assign((size_t)kTileRbG * kUV, 0.0);
      }
    if ((s = upload(c, &c->d_tI_ptr, ti.ptr.data(), ti.ptr.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_tI_col, ti.col.data(), ti.col.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_tI_val64, ti.val.data(), ti.val.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_tG_ptr, tg.ptr.data(), tg.ptr.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_tG_split, tg.split.data(), tg.split.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_tG_col, tg.col.data(), tg.col.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_tG_val64, tg.val.data(), tg.val.size())) != DD_OK) return bail(s);
    if ((s = upload(c, &c->d_dit, items.data(), items.size())) != DD_OK) return bail(s);
    std::vector<long long> toff(c->n_sub + 1, 0);
    for (int k = 0; k < c->n_sub; ++k) {
      const long long nt = (c->ni[k] + kT - 1) / kT;
      toff[k + 1] = toff[k] + nt * nt * 256;
    }
    c->t_kpack = toff[c->n_sub];
    if ((s = upload(c, &c->d_toff, toff.data(), toff.size())) != DD_OK) return bail(s);
    if ((s = dalloc(c, &c->d_kii_t, (size_t)c->t_kpack)) != DD_OK) return bail(s);
    hipLaunchKernelGGL((k_pack_tiles<double>), dim3(64, c->n_sub), dim3(256), 0, c->stream, c->n_sub,
                       c->d_kii64, c->d_koff, c->d_toff, c->d_ni, c->d_kii_t);
    if (hipGetLastError() != hipSuccess) {
      c->err = "packing of K_II failed";
      return bail(DD_EHIP);
    }
    c->tiles = true;
  }
  // work vectors
  size_t nG = (size_t)std::max(1, c->n_gamma) * c->ldmax, nI = (size_t)std::max(1, NI) * c->ldmax;
  Work &w = c->w;
  double **gv[] = {&w.bG, &w.xG, &w.rG, &w.zG, &w.pG, &w.qG, &w.uG, &w.dG, &w.tG, &w.r2G, &w.z2G, &w.qdG};
  for (double **q : gv)
    if ((s = dalloc(c, q, nG)) != DD_OK) return bail(s);
  double **iv[] = {&w.bI, &w.yI, &w.wI, &w.uI, &w.dI, &w.tI};
  for (double **q : iv)
    if ((s = dalloc(c, q, nI)) != DD_OK) return bail(s);
  float **gf[] = {&w.z32A, &w.z32B, &w.qd32, &w.p32};
  for (float **q : gf)
    if ((s = dalloc(c, q, nG)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &w.w32, nI)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_state, 1)) != DD_OK) return bail(s);
  {
    StateBlock *sb = c->d_state;
    w.bnrm2 = sb->bnrm2;
    w.rnrm2 = sb->rnrm2;
    c->st.rz = sb->rz;
    c->st.alpha = sb->alpha;
    c->st.beta = sb->beta;
    c->st.stop2 = sb->stop2;
    c->st.nrm2 = sb->nrm2;
    c->st.active = sb->active;
    c->st.iters = sb->iters;
    c->st.flag = sb->flag;
    c->st.rz2 = sb->rz2;
    c->st.act2 = sb->act2;
    c->st.bd = sb->bd;
    c->st.rz_prev = sb->rz_prev;
    c->st.act_prev = sb->act_prev;
    c->st.brk = sb->brk;
    c->st.ref2 = sb->ref2;
    if (hipMemset(sb, 0, sizeof(StateBlock)) != hipSuccess) {
      c->err = "hipMemset failed";
      return bail(DD_EHIP);
    }
  }
  c->max_chunks = std::max((size_t)(c->n_gamma + kGChunk - 1) / kGChunk,
                           (size_t)(std::max(c->n_gamma, NI) + kRowsE - 1) / kRowsE) + 1;
  if ((s = dalloc(c, &c->red.part0, c->max_chunks * kMaxLd)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->red.part1, c->max_chunks * kMaxLd)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->red.part2, c->max_chunks * kMaxLd)) != DD_OK) return bail(s);
  const size_t ngroups = c->max_chunks / kPGroup + 1;
  if ((s = dalloc(c, &c->red.part3, ngroups * kMaxLd)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->red.gcount, ngroups * kCounterStride)) != DD_OK) return bail(s);
  if (hipMemset(c->red.gcount, 0, ngroups * kCounterStride * sizeof(unsigned)) != hipSuccess) {
    c->err = "hipMemset failed";
    return bail(DD_EHIP);
  }
  if ((s = dalloc(c, &c->red.counter, 8)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_status, c->n_sub)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_flow, 2 + 2 * (size_t)c->n_sub * ((c->max_ni + 15) / 16))) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_bar, 4)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->batch.d_mask, kMaxLd)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_solve_mask, kMaxLd)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->batch.d_slots, kMaxLd)) != DD_OK) return bail(s);
  if ((s = dalloc(c, &c->d_bad, 1)) != DD_OK) return bail(s);
  if (hipMemset(c->red.counter, 0, 8 * sizeof(unsigned)) != hipSuccess) {
    c->err = "hipMemset failed";
    return bail(DD_EHIP);
  }
  c->nslots = 16;
  if (hipHostMalloc((void **)&c->h_nact, c->nslots * sizeof(int), hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer((void **)&c->h_nact_dev, c->h_nact, 0) != hipSuccess ||
      hipHostMalloc((void **)&c->h_state, sizeof(StateBlock), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->h_mask, kMaxLd * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&c->h_stop2, kMaxLd * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    c->err = "pinned host allocation failed";
    return bail(DD_ENOMEM);
  }
  c->ev.resize(c->nslots);
  for (auto &e : c->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      c->err = "hipEventCreate failed";
      return bail(DD_EHIP);
    }
  *out = c;
  return DD_OK;
}

dd_status dd_factor(dd_ctx *c, dd_precision prec) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  c->err.clear();
  TRY(ensure_ops(c, prec));
  c->op[prec].ready = false;
  return prec == DD_FP64 ? factor_impl<double>(c, DD_FP64) : factor_impl<float>(c, DD_MIXED);
}

dd_status dd_schur_apply(dd_ctx *c, dd_precision prec, const double *p_dev, double *q_dev,
                         int32_t nrhs, int32_t ld) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(c, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  if (ld < c->n_gamma || !p_dev || !q_dev) return fail(c, DD_EINVAL, "bad p/q or ld");
  int L = next_pow2(nrhs);
  Work &w = c->w;
  std::vector<int> id(c->n_gamma);
  for (int j = 0; j < c->n_gamma; ++j) id[j] = j;
  int *d_id = nullptr;
  HIPCHK(c, hipMalloc(&d_id, std::max<size_t>(1, id.size()) * sizeof(int)));
  HIPCHK(c, hipMemcpy(d_id, id.data(), id.size() * sizeof(int), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_gather, dim3(256), dim3(256), 0, c->stream, c->n_gamma, d_id, p_dev, ld, nrhs, L, w.tG);
  kig_apply(c, prec, plain(w.tG), L, nullptr, 1.0, w.yI);
  interior_solve(c, prec, DD_APPLY_INV, w.yI, w.wI, L);
  gamma_apply(c, prec, plain(w.tG), w.wI, L, nullptr, 1.0, -1.0, w.qG);
  hipLaunchKernelGGL(k_scatter, dim3(256), dim3(256), 0, c->stream, c->n_gamma, d_id, w.qG, L, nrhs, q_dev, ld);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  (void)hipFree(d_id);
  return DD_OK;
}

dd_status dd_get_factor(dd_ctx *c, dd_precision prec, int32_t k, double *out) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  if (k < 0 || k >= c->n_sub || !out) return fail(c, DD_EINVAL, "bad subdomain index or out");
  size_t n = c->ni[k], nn = n * n;
  if (prec == DD_FP64) {
    HIPCHK(c, hipMemcpy(out, (double *)c->op[0].L + c->koff[k], nn * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(nn);
    HIPCHK(c, hipMemcpy(f.data(), (float *)c->op[1].L + c->koff[k], nn * 4, hipMemcpyDeviceToHost));
    for (size_t e = 0; e < nn; ++e) out[e] = f[e];
  }
  for (size_t j = 0; j < n; ++j)
    for (size_t i = 0; i < j; ++i) out[j * n + i] = 0.0;
  return DD_OK;
}

dd_status dd_autotune(dd_ctx *c, dd_precision prec, int32_t nrhs, const dd_solve_opts *base,
                      dd_tune_result *out) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (c->batch.on) return fail(c, DD_ESTATE, "a batch is open on this context");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(c, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  dd_solve_opts o;
  if (base) o = *base; else dd_default_opts(&o);
  double *b = nullptr, *u = nullptr;
  size_t n = (size_t)c->n_dof * nrhs;
  HIPCHK(c, hipMalloc(&b, n * sizeof(double)));
  if (hipMalloc(&u, n * sizeof(double)) != hipSuccess) {
    (void)hipFree(b);
    return fail(c, DD_ENOMEM, "autotune buffers");
  }
  struct Free2 { double *a, *b; ~Free2() { (void)hipFree(a); (void)hipFree(b); } } fr{b, u};
  hipLaunchKernelGGL(k_fill_rhs, dim3(256), dim3(256), 0, c->stream, c->n_dof, nrhs, c->n_dof,
                     0x5eedull, b);
  HIPCHK(c, hipGetLastError());
  struct Cand { int apply, launch, dk, ce, cg3; double drop = 0.0; };
  std::vector<Cand> cands;
  // three-launch iteration (when there are interiors), then the four-launch
  // one with the direction formed at the gathers or kept by its own kernel
  if (c->NI > 0 && !c->classic_cg) {
    for (int lag : {1, 2, 4}) cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 0, lag, 1});
    for (int g : {2, 4}) cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 0, g, 1});
    if (prec == DD_MIXED) {      // the FP32-data products gathering FP32 vector copies
      for (int lag : {1, 2}) cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 0, lag, 3});
      cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 0, 4, 3});
    }
  }
  for (int lag : {1, 2, 4}) cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 0, lag, 0});
  for (int g : {2, 4}) cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 0, g, 0});
  cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 1, 2, 0});
  cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 1, 4, 0});
  if (prec == DD_MIXED && c->NI > 0) {   // the same with FP32 gathers
    cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 1, 2, 2});
    cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 1, 4, 2});
  }
  // batches of kTileMinLd or more columns: the tiled matrix-core products
  // (mixed precision with the FP64 factor formed: they replace residuals,
  // and each launch mode is timed at four drop factors)
  const bool can_replace = prec == DD_MIXED && o.reliable != 0 && !(o.inner_tol > 0.0) &&
                           c->op[DD_FP64].ready && c->op[DD_FP64].kinv_t;
  if (c->tiles && next_pow2(nrhs) >= kTileMinLd) {
    if (can_replace) {
      for (double drop : {1e-2, 3e-3, 1e-3, 1e-4}) {
        cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 1, 2, 4, drop});
        cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 1, 4, 4, drop});
      }
    } else {
      cands.push_back({DD_APPLY_INV, DD_LAUNCH_KERNELS, 1, 2, 4});
      cands.push_back({DD_APPLY_INV, DD_LAUNCH_GRAPH, 1, 4, 4});
    }
  }
  cands.push_back({DD_APPLY_TRSM, DD_LAUNCH_KERNELS, 0, 2, 0});
  // The cooperative persistent launch is timed only on request
  // (DD_TUNE_PERSISTENT=1): it has never won, and its first launch creates the
  // runtime's cooperative-dispatch state, which then lives until the process
  // exits.
  if (c->tune_persistent) cands.push_back({DD_APPLY_INV, DD_LAUNCH_PERSISTENT, 0, 0, 0});
  const int saved_dk = c->direction_kernel;
  int lg = 0;
  while ((1 << lg) < next_pow2(nrhs)) ++lg;
  c->tuned[prec][lg].set = false;
  double best = 1e30;
  Cand bc = cands[0];
  for (const Cand &cd : cands) {
    dd_solve_opts oc = o;
    oc.apply = cd.apply;
    oc.launch = cd.launch;
    oc.check_every = cd.ce;
    if (cd.drop > 0.0) oc.inner_tol = cd.drop;
    c->direction_kernel = cd.dk;
    c->force_cg3 = cd.cg3;
    dd_status s = dd_solve(c, prec, b, u, nrhs, c->n_dof, &oc, nullptr);   // warm-up (captures graphs)
    if (s != DD_OK && s != DD_ENOCONV) continue;
    const int reps = 3;
    auto t0 = std::chrono::steady_clock::now();
    for (int r = 0; r < reps && s == DD_OK; ++r) s = dd_solve(c, prec, b, u, nrhs, c->n_dof, &oc, nullptr);
    auto t1 = std::chrono::steady_clock::now();
    if (s != DD_OK && s != DD_ENOCONV) continue;
    double ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / reps;
    if (ms < best) {
      best = ms;
      bc = cd;
    }
  }
  // mixed precision: the inner tolerance, with the schedule just chosen
  double best_itol = o.inner_tol > 0.0 ? o.inner_tol : kInnerTol;
  int ncand = (int)cands.size();
  // (not for a tiled schedule that replaces residuals: that solve never
  // refines, and inner_tol set its replacement points instead)
  const bool replaces = can_replace && (bc.cg3 & 4);
  if (prec == DD_MIXED && !(o.inner_tol > 0.0) && !replaces) {
    for (double itol : {1e-4, 1e-5, 1e-6}) {
      dd_solve_opts oc = o;
      oc.apply = bc.apply;
      oc.launch = bc.launch;
      oc.check_every = bc.ce;
      oc.inner_tol = itol;
      c->direction_kernel = bc.dk;
      c->force_cg3 = bc.cg3;
      dd_status s = dd_solve(c, prec, b, u, nrhs, c->n_dof, &oc, nullptr);
      if (s != DD_OK) continue;
      const int reps = 3;
      auto t0 = std::chrono::steady_clock::now();
      for (int r = 0; r < reps && s == DD_OK; ++r) s = dd_solve(c, prec, b, u, nrhs, c->n_dof, &oc, nullptr);
      auto t1 = std::chrono::steady_clock::now();
      if (s != DD_OK) continue;
      ++ncand;
      double ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / reps;
      if (ms < best) {
        best = ms;
        best_itol = itol;
      }
    }
  }
  c->direction_kernel = saved_dk;
  c->force_cg3 = -1;
  c->err.clear();
  const double best_drop = replaces ? bc.drop : 0.0;
  auto &t = c->tuned[prec][lg];
  t.drop = best_drop;
  t.set = true;
  t.apply = bc.apply;
  t.launch = bc.launch;
  t.dk = bc.dk;
  t.cg3 = bc.cg3;
  t.check_every = bc.ce;
  t.ms = best;
  t.inner_tol = prec == DD_MIXED ? best_itol : 0.0;
  if (out) {
    out->apply = bc.apply;
    out->launch = bc.launch;
    out->direction_kernel = bc.dk;
    out->check_every = bc.ce;
    out->ms_per_solve = best;
    out->candidates = ncand;
    out->inner_tol = best_drop > 0.0 ? best_drop : t.inner_tol;
    out->three_launch = bc.cg3;
  }
  return DD_OK;
}

// ------------------------------------------------------------ batching --
namespace {

unsigned grid1d(size_t n) { return std::max(1u, std::min(4096u, grid_for(n, 256))); }

dd_status batch_mask(dd_ctx *c, const int *m) {
  HIPCHK(c, hipMemcpyAsync(c->batch.d_mask, m, kMaxLd * sizeof(int), hipMemcpyHostToDevice, c->stream));
  return DD_OK;
}

// Change the column stride of the resident vectors (results per column are
// unaffected: the arithmetic of a column does not depend on the stride).
dd_status batch_relayout(dd_ctx *c, int ln) {
  auto &B = c->batch;
  if (ln == B.ld) return DD_OK;
  Work &w = c->w;
  double **gv[] = {&w.bG, &w.uG, &w.tG, &w.rG, &w.zG, &w.pG, &w.dG};
  double **iv[] = {&w.bI, &w.uI, &w.tI};
  for (double **v : gv) {
    hipLaunchKernelGGL(k_relayout, dim3(grid1d((size_t)c->n_gamma * ln)), dim3(256), 0, c->stream,
                       c->n_gamma, B.ld, ln, *v, w.qG);
    std::swap(*v, w.qG);
  }
  for (double **v : iv) {
    hipLaunchKernelGGL(k_relayout, dim3(grid1d((size_t)c->NI * ln)), dim3(256), 0, c->stream, c->NI,
                       B.ld, ln, *v, w.yI);
    std::swap(*v, w.yI);
  }
  HIPCHK(c, hipGetLastError());
  B.ld = ln;
  return DD_OK;
}

int batch_need_ld(const dd_ctx *c) {
  int hi = 0;
  for (int j = 0; j < kMaxLd; ++j)
    if (c->batch.state[j] != DD_SLOT_FREE) hi = j + 1;
  return next_pow2(std::max(1, hi));
}

// Start the CG of the masked columns on the right-hand side (rI, rG):
// condensation, then the masked CG initialisation; the CG right-hand side's
// interior part is kept in tI for the back substitution.
dd_status batch_start_cg(dd_ctx *c, const int *mask, const double *rI, const double *rG) {
  auto &B = c->batch;
  Work &w = c->w;
  const Ops &op = c->op[B.prec];
  const int ld = B.ld;
  TRY(batch_mask(c, mask));
  if (rI != w.tI)
    hipLaunchKernelGGL(k_cols_update, dim3(grid1d((size_t)c->NI * ld)), dim3(256), 0, c->stream,
                       (size_t)c->NI * ld, ld, 0.0, rI, w.tI, B.d_mask);
  interior_solve(c, B.prec, DD_APPLY_INV, w.tI, w.wI, ld);
  gamma_apply(c, B.prec, plain(nullptr), w.wI, ld, rG, 0.0, -1.0, w.qG);
  std::vector<double> st2(B.stop2, B.stop2 + kMaxLd);
  HIPCHK(c, hipMemcpyAsync(c->st.stop2, st2.data(), kMaxLd * 8, hipMemcpyHostToDevice, c->stream));
  // first direction: z itself when the direction kernel keeps it (FP32
  // gathers), else none (formed as z + 0 p where it is gathered)
  if (c->n_gamma > 0)
    launch_update(c, 2, ld, kMaxLd, op.dinv, w.dG, w.rG, w.zG, w.pG, w.qG, B.o.precond, nullptr,
                  B.g32 ? 1 : 0, (const int *)B.d_mask, 0);
  HIPCHK(c, hipGetLastError());
  return DD_OK;
}

}  // namespace

dd_status dd_batch_begin(dd_ctx *c, dd_precision prec, const dd_solve_opts *opts) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (c->batch.on) return fail(c, DD_ESTATE, "a batch is already open");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  auto &B = c->batch;
  int *dm = B.d_mask, *ds = B.d_slots;
  B = dd_ctx::Batch();
  B.d_mask = dm;
  B.d_slots = ds;
  if (opts) B.o = *opts; else dd_default_opts(&B.o);
  if (!(B.o.tol > 0.0) || B.o.max_it < 1) return fail(c, DD_EINVAL, "tol <= 0 or max_it < 1");
  if (B.o.inner_tol < 0.0 || B.o.inner_tol >= 1.0) return fail(c, DD_EINVAL, "inner_tol not in [0,1)");
  if (B.o.inner_tol == 0.0) B.o.inner_tol = kInnerTol;
  B.prec = prec;
  B.g32 = prec == DD_MIXED && B.o.gather32 == 1 && c->NI > 0 && c->n_gamma > 0;
  B.ld = 1;
  B.on = true;
  HIPCHK(c, hipMemsetAsync(c->st.active, 0, kMaxLd * sizeof(int), c->stream));
  HIPCHK(c, hipMemsetAsync(c->st.flag, 0, 2 * sizeof(int), c->stream));
  return DD_OK;
}

dd_status dd_batch_end(dd_ctx *c) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->batch.on = false;
  HIPCHK(c, hipMemsetAsync(c->st.active, 0, kMaxLd * sizeof(int), c->stream));
  return DD_OK;
}

dd_status dd_batch_admit(dd_ctx *c, const int32_t *slots, int32_t ncol, const double *b_dev, int32_t ld) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  auto &B = c->batch;
  if (!B.on) return fail(c, DD_ESTATE, "no batch is open");
  if (ncol < 1 || !slots || !b_dev || ld < c->n_dof) return fail(c, DD_EINVAL, "bad admit arguments");
  std::vector<int> mask(kMaxLd, 0);
  for (int j = 0; j < ncol; ++j) {
    int sl = slots[j];
    if (sl < 0 || sl >= c->max_nrhs) return fail(c, DD_EINVAL, "slot out of [0, max_nrhs)");
    if (B.state[sl] != DD_SLOT_FREE || mask[sl]) return fail(c, DD_EINVAL, "slot not free");
    mask[sl] = 1;
  }
  for (int j = 0; j < ncol; ++j) B.state[slots[j]] = DD_SLOT_RUNNING;
  TRY(batch_relayout(c, batch_need_ld(c)));
  const int L = B.ld;
  Work &w = c->w;
  HIPCHK(c, hipMemcpyAsync(B.d_slots, slots, ncol * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_gather_cols, dim3(grid1d((size_t)c->NI * ncol)), dim3(256), 0, c->stream, c->NI,
                     c->d_imap, b_dev, ld, ncol, B.d_slots, L, w.bI);
  if (c->n_gamma)
    hipLaunchKernelGGL(k_gather_cols, dim3(grid1d((size_t)c->n_gamma * ncol)), dim3(256), 0, c->stream,
                       c->n_gamma, c->d_gmap, b_dev, ld, ncol, B.d_slots, L, w.bG);
  TRY(batch_mask(c, mask.data()));
  hipLaunchKernelGGL(k_cols_update, dim3(grid1d((size_t)c->NI * L)), dim3(256), 0, c->stream,
                     (size_t)c->NI * L, L, 0.0, (const double *)nullptr, w.uI, B.d_mask);
  hipLaunchKernelGGL(k_cols_update, dim3(grid1d((size_t)c->n_gamma * L)), dim3(256), 0, c->stream,
                     (size_t)c->n_gamma * L, L, 0.0, (const double *)nullptr, w.uG, B.d_mask);
  TRY(dd_norm2(c, L, w.bI, w.bG, w.bnrm2));
  std::vector<double> bn(kMaxLd);
  HIPCHK(c, hipMemcpyAsync(bn.data(), w.bnrm2, kMaxLd * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int j = 0; j < kMaxLd; ++j)
    if (mask[j]) {
      B.bn2[j] = bn[j];
      B.rn2[j] = bn[j];
      B.its[j] = B.steps[j] = B.conv[j] = B.stall[j] = 0;
      B.prev[j] = -1.0;
      B.stop2[j] = B.prec == DD_FP64 ? B.o.tol * B.o.tol * bn[j]
                                     : inner_stop2(B.o.inner_tol, B.o.tol, bn[j], bn[j]);
    }
  return batch_start_cg(c, mask.data(), w.bI, w.bG);
}

dd_status dd_batch_step(dd_ctx *c, int32_t iters, int32_t *state_host) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  auto &B = c->batch;
  if (!B.on) return fail(c, DD_ESTATE, "no batch is open");
  Work &w = c->w;
  const Ops &op = c->op[B.prec];
  const int L = B.ld;
  const int prec = B.prec;
  bool any = false;
  for (int j = 0; j < kMaxLd; ++j) any |= B.state[j] == DD_SLOT_RUNNING;
  if (any && iters > 0 && c->n_gamma > 0 && B.g32) {
    // direction kept in pG; its FP32 copy is refreshed here because the
    // admissions and retirements in between change the column stride
    hipLaunchKernelGGL(k_to_f32, dim3(grid1d((size_t)c->n_gamma * L)), dim3(256), 0, c->stream,
                       (size_t)c->n_gamma * L, (const double *)w.pG, w.p32);
    c->g32 = Gather32{nullptr, nullptr, nullptr, w.p32, w.w32, nullptr};
    struct ResetG32 { dd_ctx *c; ~ResetG32() { c->g32 = Gather32{}; } } reset_g32{c};
    Src P = plain(w.pG);
    P.x32 = w.p32;
    const unsigned gd = std::min(4096u, grid_for((size_t)c->n_gamma * L, kBlock));
    for (int it = 0; it < iters; ++it) {
      kig_apply(c, prec, P, L, nullptr, 1.0, w.yI);
      interior_solve(c, prec, DD_APPLY_INV, w.yI, w.wI, L);          // also w in FP32
      gamma_apply(c, prec, P, w.wI, L, nullptr, 1.0, -1.0, w.qG, 1, nullptr);
      launch_update(c, 1, L, kMaxLd, op.dinv, w.dG, w.rG, w.zG, w.pG, w.qG, B.o.precond, nullptr, 0,
                    nullptr, c->gamma_parts);
      hipLaunchKernelGGL(k_cg_direction, dim3(gd), dim3(kBlock), 0, c->stream, c->n_gamma, L, w.zG,
                         w.pG, c->st, w.p32);
    }
    HIPCHK(c, hipGetLastError());
  } else if (any && iters > 0 && c->n_gamma > 0) {
    double *pA = w.pG, *pB = w.xG;
    for (int it = 0; it < iters; ++it) {
      Src P{nullptr, w.zG, pA, c->st.beta};
      const bool p_at_gamma = c->NI == 0;     // no K_IG rows to store the direction
      kig_apply(c, prec, P, L, nullptr, 1.0, w.yI, pB);
      interior_solve(c, prec, DD_APPLY_INV, w.yI, w.wI, L);
      gamma_apply(c, prec, p_at_gamma ? P : plain(pB), w.wI, L, nullptr, 1.0, -1.0, w.qG, 1,
                  p_at_gamma ? pB : nullptr);
      launch_update(c, 1, L, kMaxLd, op.dinv, w.dG, w.rG, w.zG, pB, w.qG, B.o.precond, nullptr, 0,
                    nullptr, c->gamma_parts);
      std::swap(pA, pB);
    }
    // keep the current direction in pG (the buffer the next step reads)
    if (pA != w.pG) std::swap(w.pG, w.xG);
    HIPCHK(c, hipGetLastError());
  }
  StateBlock &h = *c->h_state;
  TRY(fetch_state(c, &h, prec == DD_FP64));   // mixed: an inner breakdown stalls the slot
  // slots whose CG finished: back substitution of the correction and update of u
  std::vector<int> fin(kMaxLd, 0);
  bool anyfin = false;
  for (int j = 0; j < kMaxLd; ++j) {
    if (B.state[j] != DD_SLOT_RUNNING) continue;
    bool stopped = !h.active[j];
    if (stopped || h.iters[j] >= B.o.max_it) {
      fin[j] = 1;
      anyfin = true;
    }
  }
  if (anyfin) {
    TRY(batch_mask(c, fin.data()));
    kig_apply(c, prec, plain(w.dG), L, w.tI, -1.0, w.yI);
    interior_solve(c, prec, DD_APPLY_INV, w.yI, w.dI, L);
    hipLaunchKernelGGL(k_axpy_masked, dim3(grid1d((size_t)c->NI * L)), dim3(256), 0, c->stream,
                       (size_t)c->NI * L, L, w.dI, w.uI, B.d_mask);
    hipLaunchKernelGGL(k_axpy_masked, dim3(grid1d((size_t)c->n_gamma * L)), dim3(256), 0, c->stream,
                       (size_t)c->n_gamma * L, L, w.dG, w.uG, B.d_mask);
    HIPCHK(c, hipGetLastError());
    for (int j = 0; j < kMaxLd; ++j)
      if (fin[j]) {
        B.its[j] += h.iters[j];
        B.steps[j] += 1;
      }
    if (prec == DD_FP64) {
      for (int j = 0; j < kMaxLd; ++j)
        if (fin[j]) {
          B.state[j] = DD_SLOT_DONE;
          B.conv[j] = h.nrm2[j] <= B.stop2[j];
          B.rn2[j] = h.nrm2[j];
        }
    } else {
      // FP64 residual of the finished columns; refine, finish or fall back
      full_residual(c, w.bI, w.bG, w.uI, w.uG, w.yI, w.qG, L);
      TRY(dd_norm2(c, L, w.yI, w.qG, w.rnrm2));
      std::vector<double> rn(kMaxLd);
      HIPCHK(c, hipMemcpyAsync(rn.data(), w.rnrm2, kMaxLd * 8, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      std::vector<int> again(kMaxLd, 0);
      bool anyagain = false;
      for (int j = 0; j < kMaxLd; ++j) {
        if (!fin[j]) continue;
        B.rn2[j] = rn[j];
        if (rn[j] <= B.o.tol * B.o.tol * B.bn2[j]) {
          B.state[j] = DD_SLOT_DONE;
          B.conv[j] = 1;
          continue;
        }
        if (B.prev[j] >= 0.0 && rn[j] > 0.25 * B.prev[j]) ++B.stall[j];
        if (B.stall[j] >= 2 || B.steps[j] >= B.o.max_refine) {
          B.state[j] = B.o.fp64_fallback ? DD_SLOT_FALLBACK : DD_SLOT_DONE;
          B.conv[j] = 0;
          continue;
        }
        B.prev[j] = rn[j];
        B.stop2[j] = inner_stop2(B.o.inner_tol, B.o.tol, rn[j], B.bn2[j]);
        again[j] = 1;
        anyagain = true;
      }
      if (anyagain) TRY(batch_start_cg(c, again.data(), w.yI, w.qG));
    }
  }
  if (state_host)
    for (int j = 0; j < c->max_nrhs; ++j) state_host[j] = B.state[j];
  return DD_OK;
}

dd_status dd_batch_retire(dd_ctx *c, const int32_t *slots, int32_t ncol, double *u_dev, int32_t ld,
                          dd_solve_info *info) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  auto &B = c->batch;
  if (!B.on) return fail(c, DD_ESTATE, "no batch is open");
  if (ncol < 1 || !slots || (!u_dev && ncol) || ld < c->n_dof) return fail(c, DD_EINVAL, "bad retire arguments");
  for (int j = 0; j < ncol; ++j) {
    int sl = slots[j];
    if (sl < 0 || sl >= kMaxLd || B.state[sl] == DD_SLOT_FREE || B.state[sl] == DD_SLOT_RUNNING)
      return fail(c, DD_EINVAL, "slot is not finished");
  }
  Work &w = c->w;
  HIPCHK(c, hipMemcpyAsync(B.d_slots, slots, ncol * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_scatter_cols, dim3(grid1d((size_t)c->NI * ncol)), dim3(256), 0, c->stream, c->NI,
                     c->d_imap, w.uI, B.ld, ncol, B.d_slots, u_dev, ld);
  if (c->n_gamma)
    hipLaunchKernelGGL(k_scatter_cols, dim3(grid1d((size_t)c->n_gamma * ncol)), dim3(256), 0, c->stream,
                       c->n_gamma, c->d_gmap, w.uG, B.ld, ncol, B.d_slots, u_dev, ld);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int j = 0; j < ncol; ++j) {
    int sl = slots[j];
    if (info) {
      info[j].iters = B.its[sl];
      info[j].refine_steps = B.prec == DD_MIXED ? B.steps[sl] : 0;
      info[j].used_fallback = 0;
      info[j].converged = B.conv[sl];
      info[j].rel_resid = B.bn2[sl] > 0 ? std::sqrt(B.rn2[sl] / B.bn2[sl]) : std::sqrt(B.rn2[sl]);
    }
    B.state[sl] = DD_SLOT_FREE;
  }
  return batch_relayout(c, batch_need_ld(c));
}

dd_status dd_set_timing(dd_ctx *c, uint32_t phase_mask, int32_t reset) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (reset) {
    c->tev_used = 0;
    for (int i = 0; i < DD_NPHASES; ++i) {
      c->t_ms[i] = 0.0;
      c->t_count[i] = 0;
    }
  } else if (c->tev_used > 0) {       // keep what was recorded so far
    HIPCHK(c, hipMemcpyAsync(c->h_state, c->d_state, sizeof(StateBlock), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    collect_timing(c, c->h_state);
  }
  c->timing_mask = phase_mask & ((1u << DD_NPHASES) - 1u);
  return DD_OK;
}

dd_status dd_get_timing(dd_ctx *c, double *ms, int64_t *launches) {
  if (!c || !ms || !launches) return fail(c, DD_EINVAL, "NULL argument");
  HIPCHK(c, hipMemcpyAsync(c->h_state, c->d_state, sizeof(StateBlock), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->tev_used) collect_timing(c, c->h_state);
  for (int i = 0; i < DD_NPHASES; ++i) {
    ms[i] = c->t_ms[i];
    launches[i] = c->t_count[i];
  }
  return DD_OK;
}

dd_status dd_get_schur_diag(dd_ctx *c, dd_precision prec, double *out) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  if (!out) return fail(c, DD_EINVAL, "out is NULL");
  HIPCHK(c, hipMemcpy(out, c->op[prec].diag, c->n_gamma * 8, hipMemcpyDeviceToHost));
  return DD_OK;
}

dd_status dd_solve(dd_ctx *c, dd_precision prec, const double *b_dev, double *u_dev, int32_t nrhs,
                   int32_t ld, const dd_solve_opts *opts, dd_solve_info *info) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (c->batch.on) return fail(c, DD_ESTATE, "a batch is open on this context");
  c->err.clear();
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(c, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  if (ld < c->n_dof || !b_dev || !u_dev) return fail(c, DD_EINVAL, "bad b/u or ld < n_dof");
  if (b_dev == u_dev) return fail(c, DD_EINVAL, "b and u alias");
  dd_solve_opts o;
  if (opts) o = *opts; else dd_default_opts(&o);
  if (!(o.tol > 0.0) || o.max_it < 1) return fail(c, DD_EINVAL, "tol <= 0 or max_it < 1");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  if (prec == DD_MIXED && (o.max_refine < 1 || o.inner_tol < 0.0 || o.inner_tol >= 1.0))
    return fail(c, DD_EINVAL, "max_refine < 1 or inner_tol not in [0,1)");
  if (o.reliable < -1) return fail(c, DD_EINVAL, "reliable < -1");
  const int L = next_pow2(nrhs);
  const double itol_requested = o.inner_tol;
  if (prec == DD_MIXED) o.inner_tol = resolve_inner_tol(c, prec, L, o.inner_tol);
  int use_cg3 = 1;
  double tuned_drop = 0.0;
  struct RestoreDk {
    dd_ctx *c;
    int v;
    ~RestoreDk() { c->direction_kernel = v; }
  } restore_dk{c, c->direction_kernel};
  {
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    const auto &t = c->tuned[prec][lg];
    if (t.set && (o.apply == DD_APPLY_AUTO || o.launch == DD_LAUNCH_AUTO)) {
      if (o.apply == DD_APPLY_AUTO) o.apply = t.apply;
      if (o.launch == DD_LAUNCH_AUTO) {
        o.launch = t.launch;
        c->direction_kernel = t.dk;
        use_cg3 = t.cg3;
        if (o.check_every == 0) o.check_every = t.check_every;
      }
    }
    if (t.set) tuned_drop = t.drop;
  }
  if (c->force_cg3 >= 0) use_cg3 = c->force_cg3;
  if (c->gather32 || o.gather32 == 1) use_cg3 |= 2;
  if (o.gather32 == 0) use_cg3 &= ~2;
  if (prec != DD_MIXED) use_cg3 &= ~2;    // FP32 gathers serve FP32 data only
  if (o.tiles == 1) use_cg3 |= 4;
  if (o.tiles == 0) use_cg3 &= ~4;
  CoreOpts co{o.max_it, o.precond, o.apply == DD_APPLY_TRSM ? DD_APPLY_TRSM : DD_APPLY_INV,
              o.check_every,
              (o.launch == DD_LAUNCH_PERSISTENT || o.launch == DD_LAUNCH_GRAPH) ? o.launch : DD_LAUNCH_KERNELS,
              use_cg3};
  const bool tl = use_tiles(c, co.cg3, L, co.apply, co.launch);
  // residual replacement in the mixed solve (tiled path, FP64 operators formed)
  if (prec == DD_MIXED && o.reliable != 0) co.reliable = o.reliable < 0 ? kReplacePeriod : o.reliable;
  co.replace_drop = itol_requested > 0.0 ? itol_requested : (tuned_drop > 0.0 ? tuned_drop : kReplaceDrop);
  const bool replacing = tl && co.reliable > 0 && c->op[DD_FP64].ready && c->op[DD_FP64].kinv_t &&
                         c->n_gamma > 0;
  Work &w = c->w;
  // gather b into the DD layout (both parts in one launch)
  const int n_all = c->NI + c->n_gamma;
  hipLaunchKernelGGL(k_gather2, dim3(std::min(4096u, grid_for((size_t)n_all * L, 256))), dim3(256), 0,
                     c->stream, c->NI, c->n_gamma, c->d_imap, c->d_gmap, b_dev, ld, nrhs, L, w.bI, w.bG);
  HIPCHK(c, hipGetLastError());
  // squared column norms of a stacked [vI; vG] (optionally stop2 = f2 * norm)
  auto norm2 = [&](const double *vI, const double *vG, double *out, double f2, double *stop2) {
    hipLaunchKernelGGL(k_norm2, dim3(grid_for((size_t)n_all, kRowsE)), dim3(kBlock), 0, c->stream,
                       c->NI, c->n_gamma, L, vI, vG, c->red, out, f2, stop2);
  };
  auto scatter = [&]() {
    hipLaunchKernelGGL(k_scatter2, dim3(std::min(4096u, grid_for((size_t)n_all * nrhs, 256))), dim3(256),
                       0, c->stream, c->NI, c->n_gamma, c->d_imap, c->d_gmap, w.uI, w.uG, L, nrhs,
                       u_dev, ld);
  };
  auto axpy = [&](const int *dmask) {
    size_t nIe = (size_t)c->NI * L, nGe = (size_t)c->n_gamma * L;
    hipLaunchKernelGGL(k_axpy2_masked, dim3(std::min(4096u, grid_for(nIe + nGe, 256))), dim3(256), 0,
                       c->stream, nIe, nGe, L, w.dI, w.dG, w.uI, w.uG, dmask);
  };
  // zero the right-hand side columns of t that take no part in an inner solve
  auto zero_unmasked = [&](const int *mask) -> dd_status {
    for (int j = 0; j < nrhs; ++j)
      if (!mask[j]) {
        if (c->NI) HIPCHK(c, hipMemset2DAsync(w.tI + j, L * 8, 0, 8, c->NI, c->stream));
        if (c->n_gamma) HIPCHK(c, hipMemset2DAsync(w.tG + j, L * 8, 0, 8, c->n_gamma, c->stream));
      }
    return DD_OK;
  };
  std::vector<double> bn2(kMaxLd, 0.0), rn2(kMaxLd, 0.0);
  std::vector<int> its(kMaxLd, 0), conv(kMaxLd, 0), steps(kMaxLd, 0), fb(kMaxLd, 0);
  StateBlock &h = *c->h_state;
  dd_status result = DD_OK;

  if (prec == DD_FP64) {
    norm2(w.bI, w.bG, w.bnrm2, o.tol * o.tol, c->st.stop2);
    dd_status s = core_solve(c, DD_FP64, w.bI, w.bG, w.uI, w.uG, L, nrhs, co);
    if (s != DD_OK) return s;
    if (o.verify) {
      full_residual(c, w.bI, w.bG, w.uI, w.uG, w.tI, w.tG, L, tl);
      norm2(w.tI, w.tG, w.rnrm2, 0.0, nullptr);
    }
    scatter();
    HIPCHK(c, hipGetLastError());
    TRY(fetch_state(c, &h));              // one wait for the whole solve
    for (int j = 0; j < nrhs; ++j) {
      its[j] = h.iters[j];
      conv[j] = !h.active[j];
      bn2[j] = h.bnrm2[j];
      rn2[j] = o.verify ? h.rnrm2[j] : h.nrm2[j];
    }
  } else {
    // Mixed precision iterative refinement on the full system (FP64 residual):
    //   r = b - A u;  inner DD solve with FP32 operators;  u += d.
    // Step 0 solves with r = b straight into u; its stopping thresholds come
    // from ||b|| on the device, so no host round trip precedes it.
    int *mask = c->h_mask;
    double *st2 = c->h_stop2;
    {
      // with residual replacement step 0 aims at the outer tolerance itself
      // (with a margin for the residual's drift since the last replacement)
      const double f20 = replacing ? kReplaceStop * kReplaceStop * o.tol * o.tol
                                   : std::max(o.inner_tol * o.inner_tol, 0.25 * o.tol * o.tol);
      norm2(w.bI, w.bG, w.bnrm2, f20, c->st.stop2);
      dd_status s = core_solve(c, DD_MIXED, w.bI, w.bG, w.uI, w.uG, L, nrhs, co);
      if (s != DD_OK) return s;
    }
    for (int j = 0; j < kMaxLd; ++j) mask[j] = j < nrhs ? 1 : 0;     // columns of the last inner solve
    std::vector<double> prev(kMaxLd, -1.0);
    std::vector<int> stall(kMaxLd, 0), done(kMaxLd, 0), need_fb(kMaxLd, 0), undo(kMaxLd, 0);
    for (int j = nrhs; j < kMaxLd; ++j) done[j] = 1;
    for (int step = 1;; ++step) {
      full_residual(c, w.bI, w.bG, w.uI, w.uG, w.tI, w.tG, L, tl);
      norm2(w.tI, w.tG, w.rnrm2, 0.0, nullptr);
      TRY(fetch_state(c, &h, false));     // inner iterations, ||b||, ||r||: one wait per step
      bool any = false, undo_any = false;
      for (int j = 0; j < kMaxLd; ++j) undo[j] = 0;
      for (int j = 0; j < nrhs; ++j) {
        if (mask[j]) {
          its[j] += h.iters[j];
          steps[j] += 1;
        }
        bn2[j] = h.bnrm2[j];
        rn2[j] = h.rnrm2[j];
        if (step == 1) prev[j] = bn2[j];  // the residual before the first step is b
        const int stepped = mask[j];
        mask[j] = 0;
        if (done[j]) continue;
        if (rn2[j] <= o.tol * o.tol * bn2[j]) { done[j] = 1; conv[j] = 1; continue; }
        // a step that made the residual larger (operators too inaccurate in
        // FP32 for this system) is undone, and the column goes to the FP64 path
        if (stepped && rn2[j] > prev[j]) {
          undo[j] = 1;
          undo_any = true;
          rn2[j] = prev[j];
          done[j] = 1;
          need_fb[j] = 1;
          continue;
        }
        if (rn2[j] > 0.25 * prev[j]) {    // reduction worse than 0.5 in norm
          if (++stall[j] >= 2) { done[j] = 1; need_fb[j] = 1; continue; }
        }
        if (step >= o.max_refine) { done[j] = 1; need_fb[j] = 1; continue; }
        prev[j] = rn2[j];
        mask[j] = 1;
        st2[j] = inner_stop2(o.inner_tol, o.tol, rn2[j], bn2[j]);
        any = true;
      }
      if (undo_any) {
        // u -= d (step 0 solved into u itself: u = 0), and t = b - A u again
        // for the columns the FP64 path finishes
        int *dm = c->d_solve_mask;
        HIPCHK(c, hipMemcpyAsync(dm, undo.data(), kMaxLd * sizeof(int), hipMemcpyHostToDevice, c->stream));
        size_t nIe = (size_t)c->NI * L, nGe = (size_t)c->n_gamma * L;
        hipLaunchKernelGGL(k_undo2_masked, dim3(std::min(4096u, grid_for(nIe + nGe, 256))), dim3(256), 0,
                           c->stream, nIe, nGe, L, w.dI, w.dG, w.uI, w.uG, dm, step == 1 ? 1 : 0);
        HIPCHK(c, hipGetLastError());
        full_residual(c, w.bI, w.bG, w.uI, w.uG, w.tI, w.tG, L, tl);
      }
      if (!any) break;
      for (int j = nrhs; j < kMaxLd; ++j) { mask[j] = 0; st2[j] = 0.0; }
      for (int j = 0; j < nrhs; ++j) if (!mask[j]) st2[j] = 0.0;
      HIPCHK(c, hipMemcpyAsync(c->d_solve_mask, mask, kMaxLd * sizeof(int), hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(c->st.stop2, st2, kMaxLd * 8, hipMemcpyHostToDevice, c->stream));
      TRY(zero_unmasked(mask));
      dd_status s = core_solve(c, DD_MIXED, w.tI, w.tG, w.dI, w.dG, L, nrhs, co);
      if (s != DD_OK) return s;
      axpy(c->d_solve_mask);
      HIPCHK(c, hipGetLastError());
    }
    // FP64 fallback for columns whose refinement stalled
    bool anyfb = false;
    for (int j = 0; j < nrhs; ++j) anyfb |= (need_fb[j] != 0);
    if (anyfb && o.fp64_fallback) {
      if (!c->op[DD_FP64].ready) {
        dd_status s = dd_factor(c, DD_FP64);
        if (s != DD_OK) return s;
      }
      for (int j = 0; j < kMaxLd; ++j) {
        mask[j] = (j < nrhs && need_fb[j]) ? 1 : 0;
        st2[j] = mask[j] ? o.tol * o.tol * bn2[j] : 0.0;
      }
      HIPCHK(c, hipMemcpyAsync(c->d_solve_mask, mask, kMaxLd * sizeof(int), hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(c->st.stop2, st2, kMaxLd * 8, hipMemcpyHostToDevice, c->stream));
      TRY(zero_unmasked(mask));           // t still holds the last residual
      dd_status s = core_solve(c, DD_FP64, w.tI, w.tG, w.dI, w.dG, L, nrhs, co);
      if (s != DD_OK) return s;
      axpy(c->d_solve_mask);
      full_residual(c, w.bI, w.bG, w.uI, w.uG, w.tI, w.tG, L, tl);
      norm2(w.tI, w.tG, w.rnrm2, 0.0, nullptr);
      TRY(fetch_state(c, &h));
      for (int j = 0; j < nrhs; ++j) {
        if (mask[j]) {
          its[j] += h.iters[j];
          fb[j] = 1;
        }
        rn2[j] = h.rnrm2[j];
      }
    }
    for (int j = 0; j < nrhs; ++j) conv[j] = rn2[j] <= o.tol * o.tol * bn2[j] * (1.0 + 1e-12);
    scatter();
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  for (int j = 0; j < nrhs; ++j) {
    if (!conv[j]) result = DD_ENOCONV;
    if (info) {
      info[j].iters = its[j];
      info[j].refine_steps = steps[j];
      info[j].used_fallback = fb[j];
      info[j].converged = conv[j];
      info[j].rel_resid = bn2[j] > 0.0 ? std::sqrt(rn2[j] / bn2[j]) : std::sqrt(rn2[j]);
    }
  }
  if (result == DD_ENOCONV) c->err = "tolerance not reached for at least one column";
  return result;
}

dd_status dd_assemble_2d(int32_t n, int32_t collar, double delta, int32_t kernel, double phi, double s,
                         int32_t R, double *win_dev, void *hip_stream) {
  if (n < 2 || collar < 0 || !(delta > 0.0) || !win_dev)
    return fail(nullptr, DD_EINVAL, "n < 2, collar < 0, delta <= 0 or win_dev NULL");
  if (kernel != kKerConst && kernel != kKerFrac && kernel != kKerPD)
    return fail(nullptr, DD_EINVAL, "unknown kernel");
  AsmProblem P;
  P.n = n;
  P.c = collar;
  P.N = n + 2 * collar;
  P.kernel = kernel;
  P.h = 1.0 / n;
  P.phi = phi;
  P.s = s;
  P.R1 = (int)std::ceil(delta / P.h) + 1;
  if (R < P.R1 + 1) return fail(nullptr, DD_EINVAL, "R < ceil(delta / h) + 2: the window misses partners");
  P.R = R;
  P.W = 2 * R + 1;
  const double t = 3.0 * delta / P.h;
  P.thr = (long long)std::floor(t * t);
  if (P.W > kAsmMaxW) return fail(nullptr, DD_EINVAL, "window wider than 128 nodes");
  asm_disk(P, delta);
  const size_t lds = (size_t)kAsmWaves * P.WC * (kernel == kKerPD ? AsmShape<kKerPD>::NV : 1) * sizeof(double);
  if (lds > 65536) return fail(nullptr, DD_EINVAL, "window copies of more than 64 KiB per row");
  hipStream_t st = (hipStream_t)hip_stream;
  static double rules[13][4];             // static: the copy below may run after the return
  static bool rules_set = false;
  if (!rules_set) {
    asm_rule_table(rules);
    rules_set = true;
  }
  hipError_t ec = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_asm_rule), rules, sizeof(rules), 0,
                                         hipMemcpyHostToDevice, st);
  if (ec != hipSuccess) return fail(nullptr, DD_EHIP, std::string("quadrature rules: ") + hipGetErrorString(ec));
  const dim3 grid((unsigned)((n - 1) * (n - 1))), block(kAsmBlock);
  if (kernel == kKerConst)
    hipLaunchKernelGGL(k_assemble_2d<kKerConst>, grid, block, lds, st, P, win_dev);
  else if (kernel == kKerFrac)
    hipLaunchKernelGGL(k_assemble_2d<kKerFrac>, grid, block, lds, st, P, win_dev);
  else
    hipLaunchKernelGGL(k_assemble_2d<kKerPD>, grid, block, lds, st, P, win_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, DD_EHIP, std::string("k_assemble_2d: ") + hipGetErrorString(e));
  return DD_OK;
}

}  // extern "C"

#include "dd_feti.h"
#include "dd_noalloc.h"

