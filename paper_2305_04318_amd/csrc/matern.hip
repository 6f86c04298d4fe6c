// Matern correlation with geometric anisotropy (Section 2.1) and the
// covariance build V = R + nu^2 I (equation (1); Step 1 of Section 3.3).
//
// rho depends on a pair of locations only through the scaled distance
// x = sqrt(8 kappa) d, so per omega the library tabulates the smooth function
// h(u) = log rho(e^u) + e^u, u = log x, as NP Chebyshev pieces of NC terms on
// [log X_LO, log x_hi].  h is analytic in the strip |Im u| < pi/2 (K_kappa has
// no zeros with |arg z| <= pi/2), so pieces of width ~0.29 in u converge far
// below double precision at 16 terms.  The nodes come from a trapezoid-rule
// evaluation of K_kappa(x) = int_0^inf exp(-x cosh t) cosh(kappa t) dt
// (DLMF 10.32.9), which converges geometrically for this analytic, doubly
// exponentially decaying integrand.  Each matrix element then costs one
// sqrt, one log, one exp and a 16-term Clenshaw sum; x < X_LO (points far
// closer than the range) falls back to the quadrature itself.
#include <math.h>

#include "common.h"

namespace plk {

// log(e^x K_nu(x)), x > 0, by the trapezoid rule on the even integrand of
// DLMF 10.32.9 with a running log-sum-exp.  The step is a quarter of the
// peak width ~ 1/sqrt(max(nu, x, 1)); the sum stops once the (unimodal)
// log-integrand has dropped 60 below its maximum.
__device__ double log_scaled_kv_quad(double nu, double x) {
  const double h = 0.25 / sqrt(fmax(fmax(nu, x), 1.0));
  double m = -INFINITY, s = 0.0, prev = -INFINITY;
  for (int k = 0; k < 400000; ++k) {
    const double u = k * h;
    const double sh = sinh(0.5 * u);
    const double a = nu * u;
    // -x (cosh u - 1) + log cosh(nu u)
    const double f = -2.0 * x * sh * sh + a + log1p(exp(-2.0 * a)) - M_LN2;
    const double w = (k == 0) ? 0.5 : 1.0;
    if (f > m) {
      s = s * exp(m - f) + w;
      m = f;
    } else {
      s += w * exp(f - m);
    }
    if (f < m - 60.0 && f < prev) break;
    prev = f;
  }
  return m + log(s * h);
}

// h(u) = log rho(x) + x at x = e^u, from the quadrature.
__device__ double h_direct(const MaternParams& P, double u) {
  const double x = exp(u);
  return P.log_norm + P.kappa * u + log_scaled_kv_quad(P.kappa, x);
}

// rho(x) for one element given the omega's table (NP*NC doubles).
__device__ __forceinline__ double rho_eval(const MaternParams& P, const double* tab, double d2) {
  const double x = P.sqrt8k * sqrt(d2);
  if (x <= X_ZERO) return 1.0;
  if (x >= P.x_hi) return 0.0;
  if (x < X_LO) {
    const double lr = P.log_norm + P.kappa * log(x) + log_scaled_kv_quad(P.kappa, x) - x;
    return fmin(exp(lr), 1.0);
  }
  const double t = (log(x) - P.u_a) * P.inv_w;
  // t lies in [0, NP) for finite x in [X_LO, x_hi); the clamp keeps the
  // table read in bounds for any input (a NaN coordinate included)
  int piece = (t >= 0.0 && t < (double)NP) ? (int)t : (t >= (double)NP ? NP - 1 : 0);
  const double s = 2.0 * (t - (double)piece) - 1.0;
  const double s2 = s + s;
  const double* c = tab + piece * NC;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int mm = NC - 1; mm >= 1; --mm) {
    const double tmp = fma(s2, b1, c[mm] - b2);
    b2 = b1;
    b1 = tmp;
  }
  const double hv = fma(s, b1, c[0] - b2);
  return fmin(exp(hv - x), 1.0);
}

// ---- table construction ---------------------------------------------------

__global__ void k_cheb_nodes(const MaternParams* __restrict__ mp, double* __restrict__ nodes, int K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * NP * NC) return;
  const int j = (int)(idx % NC);
  const int piece = (int)((idx / NC) % NP);
  const int k = (int)(idx / (NP * NC));
  const MaternParams P = mp[k];
  const double w = 1.0 / P.inv_w;
  const double sj = cos(M_PI * (j + 0.5) / NC);
  const double u = P.u_a + (piece + 0.5 + 0.5 * sj) * w;
  nodes[idx] = h_direct(P, u);
}

__global__ void k_cheb_coeffs(const double* __restrict__ nodes, double* __restrict__ tables, int K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * NP * NC) return;
  const int mm = (int)(idx % NC);
  const int64_t base = idx - mm;
  double acc = 0.0;
  for (int j = 0; j < NC; ++j) acc += nodes[base + j] * cos(M_PI * mm * (j + 0.5) / NC);
  acc *= 2.0 / NC;
  if (mm == 0) acc *= 0.5;
  tables[idx] = acc;
}

hipError_t launch_cheb_tables(const MaternParams* mp, double* nodes, double* tables, int K,
                              hipStream_t s) {
  const int64_t total = (int64_t)K * NP * NC;
  const int blocks = (int)((total + 255) / 256);
  hipLaunchKernelGGL(k_cheb_nodes, dim3(blocks), dim3(256), 0, s, mp, nodes, K);
  hipLaunchKernelGGL(k_cheb_coeffs, dim3(blocks), dim3(256), 0, s, nodes, tables, K);
  return hipGetLastError();
}

// ---- covariance tiles -----------------------------------------------------
// One workgroup per (omega, lower tile (I,J)).  Column coordinates and the
// omega's table are staged in LDS; thread (r, h) owns row r of the tile and
// every other column, so each column store is one contiguous 1 KB run.

// MODE 0: packed FP64 tiles (full diagonal tiles); MODE 1: column-major,
// lower triangle only; MODE 2: packed FP64 tiles plus an FP32 copy.
template <int MODE>
__device__ __forceinline__ void matern_tile(const MaternParams& P, const double* tab,
                                            const double* __restrict__ locs, int n, int I, int J,
                                            double* C, int64_t ldc, float* C32, const double* cx,
                                            const double* cy) {
  const int r = threadIdx.x & (T - 1);
  const int hh = threadIdx.x >> 7;
  const int gi = I * T + r;
  if (gi >= n) return;
  const double xi = locs[2 * gi], yi = locs[2 * gi + 1];
  const int cmax = min(T, n - J * T);
  for (int c = hh; c < cmax; c += 2) {
    const int gj = J * T + c;
    if (MODE == 1 && gj > gi) continue;
    double v;
    if (gi == gj) {
      v = 1.0 + P.nugget;
    } else {
      const double dx = xi - cx[c], dy = yi - cy[c];
      const double u1 = P.cosA * dx - P.sinA * dy;
      const double u2 = P.sinA * dx + P.cosA * dy;
      const double a = u1 * P.inv_phix, b = u2 * P.inv_phiy;
      v = rho_eval(P, tab, a * a + b * b);
    }
    C[(int64_t)c * ldc + r] = v;
    if (MODE == 2) C32[(int64_t)c * ldc + r] = (float)v;
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_matern(Lay lay, double* __restrict__ mats,
                                                int64_t stride64, float* __restrict__ m32,
                                                int64_t stride32,
                                                const double* __restrict__ locs,
                                                const MaternParams* __restrict__ mp,
                                                const double* __restrict__ tables, int ntiles,
                                                int G) {
  __shared__ double tab[NP * NC];
  __shared__ double cx[T], cy[T];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / ntiles;
  const int t = wg % ntiles;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int J = t - I * (I + 1) / 2;
  const double* tk = tables + (int64_t)k * NP * NC;
  for (int i = threadIdx.x; i < NP * NC; i += blockDim.x) tab[i] = tk[i];
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    const int gj = J * T + i;
    cx[i] = gj < lay.n ? locs[2 * gj] : 0.0;
    cy[i] = gj < lay.n ? locs[2 * gj + 1] : 0.0;
  }
  __syncthreads();
  const MaternParams P = mp[k];
  const int64_t off = lay.tile_off(I, J);
  double* C = mats + (int64_t)k * stride64 + off;
  float* C32 = (MODE == 2) ? m32 + (int64_t)k * stride32 + off : nullptr;
  matern_tile<MODE>(P, tab, locs, lay.n, I, J, C, lay.tile_ld(I), C32, cx, cy);
}

hipError_t launch_matern_packed(const Lay& lay, double* mats, const double* locs,
                                const MaternParams* mp, const double* tables, int K,
                                hipStream_t s) {
  const int ntiles = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntiles;
  hipLaunchKernelGGL(k_matern<0>, dim3(G), dim3(256), 0, s, lay, mats, lay.mstride, (float*)nullptr,
                     (int64_t)0, locs, mp, tables, ntiles, G);
  return hipGetLastError();
}

hipError_t launch_matern_mixed(const Lay& lay, double* m64, int64_t stride64, float* m32,
                               const double* locs, const MaternParams* mp, const double* tables,
                               int K, hipStream_t s) {
  const int ntiles = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntiles;
  hipLaunchKernelGGL(k_matern<2>, dim3(G), dim3(256), 0, s, lay, m64, stride64, m32, lay.mstride,
                     locs, mp, tables, ntiles, G);
  return hipGetLastError();
}

hipError_t launch_matern_colmajor(double* V, int64_t ld, int n, const double* locs,
                                  const MaternParams* mp, const double* tables, int K,
                                  hipStream_t s) {
  Lay lay{};
  lay.kind = 1;
  lay.n = n;
  lay.Nv = (n + T - 1) / T;
  lay.ld = ld;
  lay.mstride = ld * (int64_t)n;
  const int ntiles = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntiles;
  hipLaunchKernelGGL(k_matern<1>, dim3(G), dim3(256), 0, s, lay, V, lay.mstride, (float*)nullptr,
                     (int64_t)0, locs, mp, tables, ntiles, G);
  return hipGetLastError();
}

}  // namespace plk
