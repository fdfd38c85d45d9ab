// Allocation-free variant of dd_schur_apply (q = S p, eq. subSchurComplement
// summed over subdomains) for callers that cannot allocate device memory: code
// under graph capture, tight serving loops, harnesses that forbid it.  Its
// work vectors (p and q in the DD layout, y = K_IG p and w = K_II^-1 y) live
// in one file-scope device array, `scratch`, instead of the context's work
// buffers and the per-call index map of dd_schur_apply; the kernels are the
// same.  Included at the end of dd_lib.hip.
//
// Every device that runs it holds its own copy of the array (32 MiB) until the
// process ends; its address on a device is looked up once, by the first call
// on that device, with that device current.  Calls on one device share the
// array: calls that overlap on one GPU (several streams or threads) race.
// Every element a call reads is written earlier in the same call (padded
// columns included), so nothing left by an earlier call leaks into a result.

#include <mutex>
#include <string>

namespace {

constexpr size_t kScratchDoubles = size_t(4) << 20;   // 32 MiB
constexpr int kScratchDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchDevices] = {};
hipError_t g_scratch_err[kScratchDevices] = {};
bool g_scratch_done[kScratchDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked up
// by its first call on that device.
hipError_t scratch_on_device(int dev, double **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? (double *)p : nullptr;
    g_scratch_done[dev] = true;
  }
  *out = g_scratch_ptr[dev];
  return g_scratch_err[dev];
}

// dst[i * L + c] = src[c * lds + i] for c < nrhs, 0 for the padded columns.
__global__ void k_cols_to_dd(int n, const double *__restrict__ src, int lds, int nrhs, int L,
                             double *__restrict__ dst) {
  const size_t total = (size_t)n * L;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / L), c = (int)(e % L);
    dst[e] = c < nrhs ? src[(size_t)c * lds + i] : 0.0;
  }
}

// dst[c * ldd + i] = src[i * L + c] for c < nrhs.
__global__ void k_dd_to_cols(int n, const double *__restrict__ src, int L, int nrhs,
                             double *__restrict__ dst, int ldd) {
  const size_t total = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / n), i = (int)(e % n);
    dst[(size_t)c * ldd + i] = src[(size_t)i * L + c];
  }
}

}  // namespace

extern "C" dd_status dd_schur_apply_noalloc(dd_ctx *c, dd_precision prec, const double *p_dev,
                                            double *q_dev, int32_t nrhs, int32_t ld) {
  if (!c) return fail(nullptr, DD_EINVAL, "ctx is NULL");
  if (prec != DD_FP64 && prec != DD_MIXED) return fail(c, DD_EINVAL, "unknown precision");
  if (!c->op[prec].ready) return fail(c, DD_ESTATE, "dd_factor has not run for this precision");
  if (nrhs < 1 || nrhs > c->max_nrhs) return fail(c, DD_EINVAL, "nrhs out of [1, max_nrhs]");
  if (ld < c->n_gamma || !p_dev || !q_dev) return fail(c, DD_EINVAL, "bad p/q or ld");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->device) return fail(c, DD_EINVAL, "the context's device is not the current device");
  if (dev < 0 || dev >= kScratchDevices) return fail(c, DD_EINVAL, "device index beyond the scratch table");
  const size_t L = (size_t)next_pow2(nrhs), ng = (size_t)c->n_gamma, ni = (size_t)c->NI;
  const size_t need = (2 * ng + 2 * ni) * L;
  if (need > kScratchDoubles)
    return fail(c, DD_EINVAL, "work vectors of " + std::to_string(need) + " doubles exceed the static scratch of " +
                                  std::to_string(kScratchDoubles) + " doubles (fewer columns, or dd_schur_apply)");
  double *base = nullptr;
  const hipError_t se = scratch_on_device(dev, &base);
  if (se != hipSuccess)
    return fail(c, DD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(se));
  if (ng == 0) return DD_OK;
  double *tG = base, *qG = tG + ng * L, *yI = qG + ng * L, *wI = yI + ni * L;
  hipLaunchKernelGGL(k_cols_to_dd, dim3(std::min(4096u, grid_for(ng * L, 256))), dim3(256), 0, c->stream,
                     (int)ng, p_dev, ld, nrhs, (int)L, tG);
  kig_apply(c, prec, plain(tG), (int)L, nullptr, 1.0, yI);
  interior_solve(c, prec, DD_APPLY_INV, yI, wI, (int)L);
  gamma_apply(c, prec, plain(tG), wI, (int)L, nullptr, 1.0, -1.0, qG);
  hipLaunchKernelGGL(k_dd_to_cols, dim3(std::min(4096u, grid_for(ng * nrhs, 256))), dim3(256), 0, c->stream,
                     (int)ng, qG, (int)L, nrhs, q_dev, ld);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return DD_OK;
}
