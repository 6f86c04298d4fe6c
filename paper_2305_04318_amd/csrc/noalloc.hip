// pl_profile_loglik_noalloc: pl_profile_loglik with its workspace taken from
// a fixed device array of this library instead of the caller, for callers
// that cannot allocate device memory.
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy, at its own address, from the first use on that device
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host that name is only a stand-in for the symbol); it uses
// the device address obtained once per device with hipGetSymbolAddress.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace {

__device__ __align__(256) char scratch[PL_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device, looked up on the
// first call with that device current.
int scratch_on_current_device(void** ptr) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return PL_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PL_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return PL_OK;
}

}  // namespace

extern "C" int pl_profile_loglik_noalloc(const double* locs, const double* y, const double* X,
                                         int64_t n, int64_t p, const double* omega, int64_t K,
                                         const double* lambda, int64_t M, pl_result* out,
                                         double* beta_hat, double* xvx_inv, const pl_opts* opts,
                                         void* stream) {
  if (n < 2 || n > (1 << 30)) return -4;
  if (p < 1 || p >= n || p > PL_MAX_P) return -5;
  if (K < 1 || K > (1 << 24)) return -7;
  if (M < 1 || M > PL_MAX_M) return -9;
  if (opts && opts->precision != PL_FP64 && opts->precision != PL_MIXED) return -13;
  if (opts && opts->chunk < 0) return -13;
  const size_t cap = PL_NOALLOC_SCRATCH_BYTES;

  // the largest omega count per call whose workspace fits the array
  size_t need = 0;
  int rc = pl_workspace_size(n, p, 1, M, opts, &need);
  if (rc > 0) return rc;      // PL_E_UNSUPPORTED: PL_MIXED with M + p > PL_MAX_Q_MIXED
  if (rc < 0) return -13;     // the sizes were checked above: a bad option
  if (need > cap) return PL_E_SCRATCH;
  int64_t lo = 1, hi = K;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (pl_workspace_size(n, p, mid, M, opts, &need) == PL_OK && need <= cap)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t kc = lo;

  void* work = nullptr;
  rc = scratch_on_current_device(&work);
  if (rc != PL_OK) return rc;
  // Successive chunks reuse the array in stream order; every buffer the
  // call needs cleared is cleared by its own kernels.
  for (int64_t c0 = 0; c0 < K; c0 += kc) {
    const int64_t kk = std::min<int64_t>(kc, K - c0);
    rc = pl_profile_loglik(locs, y, X, n, p, omega ? omega + 5 * c0 : nullptr, kk, lambda, M,
                           out ? out + c0 * M : nullptr,
                           beta_hat ? beta_hat + c0 * M * p : nullptr,
                           xvx_inv ? xvx_inv + c0 * p * p : nullptr, opts, work, cap, stream);
    if (rc != PL_OK) return rc;
  }
  return PL_OK;
}
