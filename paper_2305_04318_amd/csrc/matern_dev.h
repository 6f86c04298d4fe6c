// Device side of the Matern correlation (Section 2.1): the quadrature
// evaluation of K_kappa, the per-element table evaluation and the tile task.
#pragma once

#include <math.h>

#include "common.h"

namespace plk {

// log(e^x K_nu(x)), x > 0, by the trapezoid rule on the even integrand of
// DLMF 10.32.9 with a running log-sum-exp.  The step is a quarter of the
// peak width ~ 1/sqrt(max(nu, x, 1)); the sum stops once the (unimodal)
// log-integrand has dropped 60 below its maximum.
static __device__ double log_scaled_kv_quad(double nu, double x) {
  const double h = 0.25 / sqrt(fmax(fmax(nu, x), 1.0));
  // exp(-2 nu u) on the grid u = k h as a running product (relative error at
  // most ~k eps, far below the tables' accuracy): one exponential per term
  // fewer
  const double ratio = exp(-2.0 * nu * h);
  double e2a = 1.0;
  double m = -INFINITY, s = 0.0, prev = -INFINITY;
  for (int k = 0; k < 400000; ++k, e2a *= ratio) {
    const double u = k * h;
    const double sh = sinh(0.5 * u);
    const double a = nu * u;
    // -x (cosh u - 1) + log cosh(nu u)
    const double f = -2.0 * x * sh * sh + a + log1p(e2a) - M_LN2;
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

// g(w) = log rho(x) at x = sqrt(w) > 0, from the quadrature:
// log rho = log_norm + kappa log x + log K_kappa(x), K from e^x K by - x.
static __device__ double g_direct(const MaternParams& P, double w) {
  const double x = sqrt(w);
  return P.log_norm + P.kappa * log(x) + (log_scaled_kv_quad(P.kappa, x) - x);
}

// rho for one element given d^2 (the squared anisotropic distance) and the
// omega's table (TABLE doubles: per piece, the power-basis coefficients of the
// Chebyshev interpolant of rho itself in the local variable s).  The piece
// comes from the binary exponent and mantissa of w = 8 kappa d^2 (no
// logarithm), the value from a Horner sum clamped to [0, 1] (no exp).
__device__ __forceinline__ double rho_eval(const MaternParams& P, const double* tab, double d2) {
  const double w = P.k8 * d2;
  if (w == 0.0) return 1.0;
  if (w >= P.w_hi) return 0.0;
  if (w < 0x1p-20) return fmin(exp(g_direct(P, w)), 1.0);  // 2^W_E_LO
  int e;
  const double m = frexp(w, &e);            // w = m 2^e, m in [0.5, 1)
  const double t = (2.0 * m - 1.0) * PB;    // position in the binade, [0, PB)
  int j = (int)t;
  j = j < 0 ? 0 : (j >= PB ? PB - 1 : j);
  int piece = (e - 1 - W_E_LO) * PB + j;
  // in range for every finite w in [2^W_E_LO, w_hi); the clamp keeps the
  // table read in bounds for any input (a NaN coordinate included)
  piece = piece < 0 ? 0 : (piece >= NPIECE ? NPIECE - 1 : piece);
  const double s = 2.0 * (t - (double)j) - 1.0;
  const double* a = tab + piece * NC;  // power-basis coefficients in s
  double r = a[NC - 1];
#pragma unroll
  for (int mm = NC - 2; mm >= 0; --mm) r = fma(r, s, a[mm]);
  return fmin(fmax(r, 0.0), 1.0);
}

// ---- covariance tiles -----------------------------------------------------
// One workgroup per (omega, lower tile (I,J)).  Column coordinates and the
// omega's table are staged in LDS; thread (r, h) owns row r of the tile and
// every other column, so each column store is one contiguous 1 KB run.

// MODE 0: packed FP64 tiles (full diagonal tiles); MODE 1: column-major,
// lower triangle only; MODE 2: packed FP64 tiles plus an FP32 copy; MODE 3:
// column-major, lower triangle only, FP32 only (C32; C is not written).
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
    if ((MODE == 1 || MODE == 3) && gj > gi) continue;
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
    if (MODE != 3) C[(int64_t)c * ldc + r] = v;
    if (MODE == 2 || MODE == 3) C32[(int64_t)c * ldc + r] = (float)v;
  }
}

// One T x T tile (I, J) of V for one omega: the omega's table and the tile's
// column coordinates are staged in smem (TABLE + 2T doubles).  C points at the
// tile (leading dimension ldc); MODE 2 also writes C32, MODE 3 only C32.
template <int MODE>
__device__ __forceinline__ void dev_matern_tile(const Lay& lay, const MaternParams& P,
                                                const double* __restrict__ tab_g,
                                                const double* __restrict__ locs, int I, int J,
                                                double* C, int64_t ldc, float* C32, double* smem) {
  double* tab = smem;
  double* cx = smem + TABLE;
  double* cy = cx + T;
  for (int i = threadIdx.x; i < TABLE; i += blockDim.x) tab[i] = tab_g[i];
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    const int gj = J * T + i;
    cx[i] = gj < lay.n ? locs[2 * gj] : 0.0;
    cy[i] = gj < lay.n ? locs[2 * gj + 1] : 0.0;
  }
  __syncthreads();
  matern_tile<MODE>(P, tab, locs, lay.n, I, J, C, ldc, C32, cx, cy);
}

}  // namespace plk
