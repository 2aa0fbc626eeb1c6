// Dense log-likelihood of one small field with no allocation at call time
// (the DENSE-mode tlr_generate + tlr_potrf + tlr_loglik sequence as one call,
// for callers that cannot allocate device memory: code under HIP graph
// capture, tight serving loops).  Every intermediate lives in the file-scope
// device array `scratch`, which each GPU holds from the library's first use
// on it until the process ends; host code addresses it only through the
// per-device pointer hipGetSymbolAddress returns.
//
// Eq. (1): l = -n/2 log(2 pi) - 1/2 log|Sigma| - 1/2 z^T Sigma^{-1} z, with
// Sigma (Eq. (MaternCov)) generated whole, factored as one tile (blocked
// POTRF plus the inverse factor), log|Sigma| = 2 sum log L_ii and
// z^T Sigma^{-1} z = ||L^{-1} z||^2.
#include "tlr.h"
#include "common.h"
#include "kernels.h"
#include "chol.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

namespace tlri {
extern thread_local char g_last_error[256];   // tlr_last_error's text (runtime.hip)
}

using namespace tlrk;

namespace {
constexpr int64_t kNoAllocMaxN = 2048;
// layout (doubles): Sigma / L (n x n, ld n) | L^{-1} (n x n) | POTRF work (64 n) |
// y (n) | Matérn table | scalars (log-diagonal, quad, info)
constexpr int64_t kOffInv = kNoAllocMaxN * kNoAllocMaxN;
constexpr int64_t kOffWork = 2 * kOffInv;
constexpr int64_t kOffY = kOffWork + 64 * kNoAllocMaxN;
constexpr int64_t kOffTab = kOffY + kNoAllocMaxN;
constexpr int64_t kOffScal = kOffTab + kTabSize;
constexpr int64_t kScratchDoubles = kOffScal + 16;
}  // namespace

// 8.5 Mi doubles (68 MB) per GPU
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// the device's address of `scratch` (looked up once per device, with that device current)
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

__global__ void set_u64_kernel(unsigned long long* p, unsigned long long v) { *p = v; }

}  // namespace

extern "C" tlr_status tlr_dense_loglik_noalloc(int64_t n, const double* d_x, const double* d_y, const double* d_z,
                                               const double theta[3], double* ll, double* logdet, double* quad,
                                               int64_t* info, void* stream) {
  if (info) *info = 0;
  if (!d_x || !d_y || !d_z || !theta || n < 1) return TLR_EINVAL;
  if (n > kNoAllocMaxN) {
    snprintf(tlri::g_last_error, sizeof(tlri::g_last_error), "tlr_dense_loglik_noalloc: n = %lld exceeds the maximum %lld", (long long)n,
             (long long)kNoAllocMaxN);
    return TLR_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  MaternParams p{};
  double tab[kTabSize];
  if (!matern_setup(theta[0], theta[1], theta[2], &p, tab)) return TLR_EINVAL;
  p.metric = kMetricEuclid;
  p.radius = 0.0;
  double* S = nullptr;
#define NA_CHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) {                                                               \
      snprintf(tlri::g_last_error, sizeof(tlri::g_last_error), "%s in %s (noalloc.hip)", hipGetErrorName(e_), #x); \
      (void)hipGetLastError();                                                            \
      return TLR_EHIP;                                                                    \
    }                                                                                     \
  } while (0)
  NA_CHK(scratch_ptr(&S));
  double* T = S;
  double* Inv = S + kOffInv;
  double* work = S + kOffWork;
  double* yv = S + kOffY;
  double* dtab = S + kOffTab;
  double* scal = S + kOffScal;   // [0] sum log L_ii, [1] quad, [2] info (as 64 bits)
  unsigned long long* dinfo = reinterpret_cast<unsigned long long*>(scal + 2);
  NA_CHK(hipMemcpyAsync(dtab, tab, kTabSize * sizeof(double), hipMemcpyHostToDevice, s));
  p.tab = dtab;
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(1), 0, s, dinfo, ~0ull);
  NA_CHK(hipGetLastError());
  NA_CHK(launch_matern_block(p, d_x, d_y, 0, n, 0, n, T, n, false, s));
  NA_CHK(tile_potrf_inv(T, n, n, Inv, n, dinfo, 0, work, s));
  NA_CHK(launch_logdiag(T, n, n, scal, s));
  NA_CHK(launch_gemv_n(Inv, n, n, n, d_z, 1.0, 0.0, yv, s));
  NA_CHK(launch_dot(yv, yv, n, scal + 1, s));
  double hs[3] = {0, 0, 0};
  NA_CHK(hipMemcpyAsync(hs, scal, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  NA_CHK(hipStreamSynchronize(s));
#undef NA_CHK
  unsigned long long iv;
  static_assert(sizeof(iv) == sizeof(double), "64-bit info");
  std::memcpy(&iv, &hs[2], sizeof(iv));
  if (iv != ~0ull) {
    if (info) *info = (int64_t)iv;
    return TLR_ENOTSPD;
  }
  const double ld = 2.0 * hs[0], q = hs[1];
  if (ll) *ll = -0.5 * (double)n * std::log(2.0 * M_PI) - 0.5 * ld - 0.5 * q;
  if (logdet) *logdet = ld;
  if (quad) *quad = q;
  return TLR_OK;
}
