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

// rho for one element given w = 8 kappa d^2 (d the anisotropic distance) and
// the omega's table (TABLE doubles, 16-byte aligned: per piece, the
// power-basis coefficients of the Chebyshev interpolant of rho itself in the
// local variable s, the coefficient of s^m scaled by 8^-m).  For w >= 2^W_E_LO,
// a normal double, the piece is the binary exponent and the top two mantissa
// bits of w (PB = 4 pieces per binade) and s the remaining mantissa bits,
// read off its bit pattern (no logarithm); the value is a Horner sum in s / 8
// clamped to [0, 1] (no exp).  w_hi: the omega's underflow point (P.w_hi).
// rho_table covers w >= 2^W_E_LO (RHO_W_LO), rho_small the rest.
constexpr double RHO_W_LO = 0x1p-20;

// rho for 0 <= w < 2^W_E_LO: 1 at w = 0 (coincident locations), else the
// quadrature directly.
__device__ __forceinline__ double rho_small(const MaternParams& P, double w) {
  return w == 0.0 ? 1.0 : fmin(exp(g_direct(P, w)), 1.0);
}

__device__ __forceinline__ double rho_table(const double* tab, double w, double w_hi) {
  static_assert(PB == 4 && NC % 2 == 0, "two mantissa bits per piece; coefficient pairs");
  const long long u = __double_as_longlong(w);
  const int hi = (int)(u >> 32);
  // exponent and top two mantissa bits, relative to 2^W_E_LO; the clamp
  // keeps the table read in bounds for any input (a NaN or infinite w
  // included, which the final test maps to 0)
  int piece = (hi >> 18) - ((1023 + W_E_LO) << 2);
  piece = max(0, min(piece, NPIECE - 1));
  // the piece's byte offset, opaque to the compiler: otherwise it folds the
  // bias above into five separate address constants instead of one base
  // address with the five reads' immediate offsets
  int off = piece * (NC * 8);
  asm volatile("" : "+v"(off));
  // the other 50 mantissa bits under exponent 0: v = 1 + f / 4 with f the
  // position in the piece, in [0, 1); s / 8 = v - 9 / 8 in [-1/8, 1/8), exact
  const double v = __longlong_as_double((long long)(((unsigned long long)((hi & 0x3FFFF) | 0x3FF00000) << 32) |
                                                    (unsigned long long)(u & 0xffffffffLL)));
  const double s8 = v - 1.125;
  typedef double pair __attribute__((ext_vector_type(2)));
  const pair* a2 = reinterpret_cast<const pair*>(reinterpret_cast<const char*>(tab) + off);
  double a[NC];
#pragma unroll
  for (int q = 0; q < NC / 2; ++q) {
    const pair t = a2[q];
    a[2 * q] = t.x;
    a[2 * q + 1] = t.y;
  }
  double r = a[NC - 1];
#pragma unroll
  for (int mm = NC - 2; mm >= 0; --mm) r = fma(r, s8, a[mm]);
  r = fmin(fmax(r, 0.0), 1.0);
  return w < w_hi ? r : 0.0;
}

// Whether w takes the quadrature (NaN does not: the table path maps it to 0).
__device__ __forceinline__ bool rho_needs_quad(double w) { return w < RHO_W_LO && w != 0.0; }

__device__ __forceinline__ double rho_eval(const MaternParams& P, const double* tab, double w,
                                           double w_hi) {
  return w < RHO_W_LO ? rho_small(P, w) : rho_table(tab, w, w_hi);
}

// ---- covariance tiles -----------------------------------------------------
// One workgroup per (omega, lower tile (I,J)).  Column coordinates and the
// omega's table are staged in LDS; thread (r, h) owns row r of the tile and
// every other column, so each column store is one contiguous 1 KB run.

// MODE 0: packed FP64 tiles (full diagonal tiles); MODE 1: column-major,
// lower triangle only; MODE 2: packed FP64 tiles plus an FP32 copy; MODE 3:
// column-major, lower triangle only, FP32 only (C32; C is not written).
// SPLIT: the elements that need the quadrature (rho_needs_quad) are stored as
// 0 and left to matern_tile_quad; each wave writes flags[wave] = whether it
// left any.  The quadrature's call holds more than twice the registers of
// the table path, so keeping it out of this loop doubles the resident waves.

// w = 8 kappa d^2 = |M (dx, dy)|^2: rotation by phi_A, the two range scales
// and sqrt(8 kappa) in one 2 x 2 map (m11, m12, m21, m22)
struct WMap {
  double m11, m12, m21, m22;
  __device__ __forceinline__ explicit WMap(const MaternParams& P) {
    const double sk = sqrt(P.k8);
    m11 = sk * P.inv_phix * P.cosA;
    m12 = -sk * P.inv_phix * P.sinA;
    m21 = sk * P.inv_phiy * P.sinA;
    m22 = sk * P.inv_phiy * P.cosA;
  }
  __device__ __forceinline__ double w(double xi, double yi, double xj, double yj) const {
    const double dx = xi - xj, dy = yi - yj;
    const double u1 = fma(m12, dy, m11 * dx);
    const double u2 = fma(m22, dy, m21 * dx);
    return fma(u1, u1, u2 * u2);
  }
};

template <int MODE, bool SPLIT = false>
__device__ __forceinline__ void matern_tile(const MaternParams& P, const double* tab,
                                            const double* __restrict__ locs, int n, int I, int J,
                                            double* C, int64_t ldc, float* C32, const double* cx,
                                            const double* cy, uint8_t* flags = nullptr) {
  const int r = threadIdx.x & (T - 1);
  const int hh = threadIdx.x >> 7;
  const int gi = I * T + r;
  bool quad = false;  // SPLIT: an element of this lane left to the quadrature launch
  if (gi < n) {
    const double xi = locs[2 * gi], yi = locs[2 * gi + 1];
    const int cmax = min(T, n - J * T);
    const WMap M(P);
    // read once: the stores below may alias P as far as the compiler knows
    const double w_hi = P.w_hi, vdiag = 1.0 + P.nugget;
    for (int c = hh; c < cmax; c += 2) {
      const int gj = J * T + c;
      if ((MODE == 1 || MODE == 3) && gj > gi) continue;
      double v;
      if (gi == gj) {
        v = vdiag;
      } else {
        const double w = M.w(xi, yi, cx[c], cy[c]);
        if constexpr (SPLIT) {
          const bool q = rho_needs_quad(w);
          quad |= q;
          v = q ? 0.0 : (w == 0.0 ? 1.0 : rho_table(tab, w, w_hi));
        } else {
          v = rho_eval(P, tab, w, w_hi);
        }
      }
      if (MODE != 3) C[(int64_t)c * ldc + r] = v;
      if (MODE == 2 || MODE == 3) C32[(int64_t)c * ldc + r] = (float)v;
    }
  }
  if constexpr (SPLIT) {
    const bool any = __any(quad);
    if ((threadIdx.x & 63) == 0) flags[threadIdx.x >> 6] = any ? 1 : 0;
  }
}

// The elements of tile (I, J) that matern_tile<MODE, true> left to the
// quadrature: the same w, bit for bit (same map, same coordinates), then
// rho_small.  Coordinates straight from global memory (few tiles get here).
template <int MODE>
__device__ __forceinline__ void matern_tile_quad(const MaternParams& P,
                                                 const double* __restrict__ locs, int n, int I,
                                                 int J, double* C, int64_t ldc, float* C32) {
  const int r = threadIdx.x & (T - 1);
  const int hh = threadIdx.x >> 7;
  const int gi = I * T + r;
  if (gi >= n) return;
  const double xi = locs[2 * gi], yi = locs[2 * gi + 1];
  const int cmax = min(T, n - J * T);
  const WMap M(P);
  for (int c = hh; c < cmax; c += 2) {
    const int gj = J * T + c;
    if (gj == gi || ((MODE == 1 || MODE == 3) && gj > gi)) continue;
    const double w = M.w(xi, yi, locs[2 * gj], locs[2 * gj + 1]);
    if (!rho_needs_quad(w)) continue;
    const double v = rho_small(P, w);
    if (MODE != 3) C[(int64_t)c * ldc + r] = v;
    if (MODE == 2 || MODE == 3) C32[(int64_t)c * ldc + r] = (float)v;
  }
}

// One T x T tile (I, J) of V for one omega: the omega's table and the tile's
// column coordinates are staged in smem (TABLE + 2T doubles).  C points at the
// tile (leading dimension ldc); MODE 2 also writes C32, MODE 3 only C32.
template <int MODE, bool SPLIT = false>
__device__ __forceinline__ void dev_matern_tile(const Lay& lay, const MaternParams& P,
                                                const double* __restrict__ tab_g,
                                                const double* __restrict__ locs, int I, int J,
                                                double* C, int64_t ldc, float* C32, double* smem,
                                                uint8_t* flags = nullptr) {
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
  matern_tile<MODE, SPLIT>(P, tab, locs, lay.n, I, J, C, ldc, C32, cx, cy, flags);
}

}  // namespace plk
