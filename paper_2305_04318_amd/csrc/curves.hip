// Profile curves of sigma and of single regression coefficients from the
// records of the path (Sections 3.4 and 3.5: the profile likelihood
// for beta_p and for sigma, and Step 6's maximisation over the evaluated
// (omega, lambda) points).
#include <math.h>

#include <vector>

#include "common.h"

namespace plk {
namespace {

constexpr int CURVE_THREADS = 256;

__device__ __forceinline__ bool usable(int32_t info) {
  return info == 0 || info == PL_INFO_FALLBACK;
}

// Value of one (omega, lambda) record at one grid point.  which < 0: sigma
// curve at value g; which = j >= 0: coefficient j fixed at g.
__device__ __forceinline__ double curve_value(const pl_result& r, const double* __restrict__ beta_hat,
                                              const double* __restrict__ xvx_inv, int64_t rec,
                                              int k, double lam, int n, int p, int which,
                                              double g) {
  const double LOG2PI = 1.8378770664093454836;
  const double jterm = (lam - 1.0) * r.jacobian;
  if (which < 0) {
    // equation "profileSigma": beta at its MLE, sigma fixed
    const double s2 = g * g;
    return -0.5 * (r.ssq_resid / s2 + n * log(s2) + r.logdet_v + n * LOG2PI) + jterm;
  }
  // beta_j fixed at g: the other coefficients and sigma at their constrained
  // MLEs; the minimal SSR grows by (g - betahat_j)^2 / [(X^T V^-1 X)^-1]_jj
  const double d = g - beta_hat[rec * p + which];
  const double vjj = xvx_inv[(int64_t)k * p * p + which * p + which];
  const double ssr = r.ssq_resid + d * d / vjj;
  return -0.5 * (n * log(ssr / n) + r.logdet_v + n * LOG2PI + n) + jterm;
}

// One workgroup per grid point: the maximum over every usable record and the
// index of the (first) record attaining it.
__global__ __launch_bounds__(CURVE_THREADS) void k_curves(
    const pl_result* __restrict__ rec, const double* __restrict__ beta_hat,
    const double* __restrict__ xvx_inv, int n, int p, int K, int M,
    const double* __restrict__ lam, const double* __restrict__ sgrid, int Gs,
    const double* __restrict__ bgrid, int Gb, double* __restrict__ prof_sigma,
    int64_t* __restrict__ arg_sigma, double* __restrict__ prof_beta,
    int64_t* __restrict__ arg_beta) {
  __shared__ double bv[CURVE_THREADS];
  __shared__ int64_t bi[CURVE_THREADS];
  const int gp = blockIdx.x;
  int which;
  double g;
  if (gp < Gs) {
    which = -1;
    g = sgrid[gp];
  } else {
    which = (gp - Gs) / Gb;
    g = bgrid[gp - Gs];
  }
  double best = -INFINITY;
  int64_t arg = -1;
  const int64_t R = (int64_t)K * M;
  for (int64_t r = threadIdx.x; r < R; r += CURVE_THREADS) {
    const pl_result x = rec[r];
    if (!usable(x.info)) continue;
    const int k = (int)(r / M), m = (int)(r % M);
    const double v = curve_value(x, beta_hat, xvx_inv, r, k, lam[m], n, p, which, g);
    if (v > best) {  // strictly greater: the first index wins within a thread
      best = v;
      arg = r;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int w = CURVE_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double ov = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      const double cv = bv[threadIdx.x];
      const int64_t ci = bi[threadIdx.x];
      // larger value wins; equal values keep the smaller record index
      if (ov > cv || (ov == cv && oi >= 0 && (ci < 0 || oi < ci))) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (which < 0) {
      prof_sigma[gp] = bv[0];
      if (arg_sigma) arg_sigma[gp] = bi[0];
    } else {
      prof_beta[gp - Gs] = bv[0];
      if (arg_beta) arg_beta[gp - Gs] = bi[0];
    }
  }
}

size_t al(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace
}  // namespace plk

using namespace plk;

extern "C" int pl_curves_workspace_size(int64_t p, int64_t M, int64_t Gs, int64_t Gb,
                                        size_t* bytes) {
  if (p < 1 || p > PL_MAX_P) return -1;
  if (M < 1 || M > PL_MAX_M) return -2;
  if (Gs < 0 || Gs > (1 << 20)) return -3;
  if (Gb < 0 || Gb > (1 << 20)) return -4;
  if (!bytes) return -5;
  *bytes = al(M * sizeof(double)) + al(Gs * sizeof(double)) + al(p * Gb * sizeof(double));
  return PL_OK;
}

extern "C" int pl_profile_curves(const pl_result* rec, const double* beta_hat,
                                 const double* xvx_inv, int64_t n, int64_t p, int64_t K,
                                 const double* lambda, int64_t M, const double* sigma_grid,
                                 int64_t Gs, const double* beta_grid, int64_t Gb,
                                 double* prof_sigma, int64_t* arg_sigma, double* prof_beta,
                                 int64_t* arg_beta, void* work, size_t work_bytes,
                                 void* stream) {
  if (!rec) return -1;
  if (Gb > 0 && !beta_hat) return -2;
  if (Gb > 0 && !xvx_inv) return -3;
  if (n < 2 || n > (1 << 30)) return -4;
  if (p < 1 || p >= n || p > PL_MAX_P) return -5;
  if (K < 1 || K > (1 << 24)) return -6;
  if (!lambda) return -7;
  if (M < 1 || M > PL_MAX_M) return -8;
  for (int64_t m = 0; m < M; ++m)
    if (!isfinite(lambda[m])) return -7;
  if (Gs < 0 || Gs > (1 << 20) || (Gs > 0 && !sigma_grid)) return -10;
  for (int64_t g = 0; g < Gs; ++g)
    if (!(sigma_grid[g] > 0.0) || !isfinite(sigma_grid[g])) return -9;
  if (Gb < 0 || Gb > (1 << 20) || (Gb > 0 && !beta_grid)) return -12;
  for (int64_t g = 0; g < p * Gb; ++g)
    if (!isfinite(beta_grid[g])) return -11;
  if (Gs > 0 && !prof_sigma) return -13;
  if (Gb > 0 && !prof_beta) return -15;
  size_t need = 0;
  pl_curves_workspace_size(p, M, Gs, Gb, &need);
  if (!work) return -17;
  if (work_bytes < need) return -18;
  if (Gs + p * Gb == 0) return PL_OK;
  if (Gs + p * Gb > (1 << 30)) return -10;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)work;
  double* lam_d = (double*)w;
  double* sg_d = (double*)(w + al(M * sizeof(double)));
  double* bg_d = (double*)(w + al(M * sizeof(double)) + al(Gs * sizeof(double)));
  if (stage_h2d(lam_d, lambda, M * sizeof(double), s) != hipSuccess ||
      stage_h2d(sg_d, sigma_grid, Gs * sizeof(double), s) != hipSuccess ||
      stage_h2d(bg_d, beta_grid, p * Gb * sizeof(double), s) != hipSuccess)
    return PL_E_HIP;
  hipLaunchKernelGGL(k_curves, dim3((unsigned)(Gs + p * Gb)), dim3(CURVE_THREADS), 0, s, rec,
                     beta_hat, xvx_inv, (int)n, (int)p, (int)K, (int)M, lam_d, sg_d, (int)Gs, bg_d,
                     (int)Gb, prof_sigma, arg_sigma, prof_beta, arg_beta);
  return hipGetLastError() == hipSuccess ? PL_OK : PL_E_HIP;
}
