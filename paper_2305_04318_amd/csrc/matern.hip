// Matern correlation with geometric anisotropy (Section 2.1) and the
// covariance build V = R + nu^2 I (equation (1); Step 1 of Section 3.3).
//
// rho depends on a pair of locations only through the scaled distance
// x = sqrt(8 kappa) d, so per omega the library tabulates rho(sqrt w) in
// w = x^2 = 8 kappa d^2: Chebyshev pieces of NC terms, PB pieces uniform in
// the mantissa of each binade [2^e, 2^(e+1)) of w.  The only singularity on
// or near the positive axis is at w = 0 (K_kappa has no zeros with
// |arg z| <= pi/2), which lies at least 2 PB + 1 half-widths from every
// piece, so the pieces converge geometrically (NC = 10 terms on PB = 4
// pieces match the quadrature to its own accuracy, ~2.6e-13 absolute in rho).
// V needs absolute accuracy, so rho itself is tabulated rather than log rho
// (which would cost an exp per element).  Each piece's Chebyshev interpolant
// is stored as power-basis coefficients in the piece's local variable
// s in [-1, 1] (its coefficients decay geometrically, so the conversion adds
// only rounding of the order of the leading terms): a matrix element costs
// its binary exponent and mantissa and a 10-term Horner sum (9 FMAs, against
// 18 operations for a Clenshaw sum) -- no square root, logarithm or
// exponential.  The node values come from a trapezoid-rule evaluation of
// K_kappa(x) = int_0^inf exp(-x cosh t) cosh(kappa t) dt (DLMF 10.32.9),
// which converges geometrically for this analytic, doubly exponentially
// decaying integrand; w < 2^W_E_LO (points far closer than the range) uses
// the quadrature itself.
#include <math.h>

#include "matern_dev.h"

namespace plk {

// ---- table construction ---------------------------------------------------

__global__ void k_cheb_nodes(const MaternParams* __restrict__ mp, double* __restrict__ nodes, int K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * TABLE) return;
  const int j = (int)(idx % NC);
  const int piece = (int)((idx / NC) % NPIECE);
  const int k = (int)(idx / TABLE);
  const MaternParams P = mp[k];
  const int bin = piece / PB, sub = piece % PB;
  const double sj = cos(M_PI * (j + 0.5) / NC);
  // node j of piece `sub` of binade W_E_LO + bin, in the mantissa of w
  const double w = ldexp(1.0 + (sub + 0.5 + 0.5 * sj) / PB, W_E_LO + bin);
  // rho underflows beyond w_hi (rho_eval returns 0 there)
  nodes[idx] = w < P.w_hi ? exp(g_direct(P, w)) : 0.0;
}

__global__ void k_cheb_coeffs(const double* __restrict__ nodes, double* __restrict__ tables, int K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * TABLE) return;
  const int mm = (int)(idx % NC);
  const int64_t base = idx - mm;
  double acc = 0.0;
  for (int j = 0; j < NC; ++j) acc += nodes[base + j] * cos(M_PI * mm * (j + 0.5) / NC);
  acc *= 2.0 / NC;
  if (mm == 0) acc *= 0.5;
  tables[idx] = acc;
}

// Chebyshev coefficients c_0 .. c_{NC-1} of one piece (c_0 already halved)
// -> power-basis coefficients a_j of sum_m c_m T_m(s), in place, through the
// integer coefficients of T_m (T_{m+1} = 2 s T_m - T_{m-1}); stored as
// a_j 8^j, the coefficients in s / 8 (exact: a power of two).
__global__ void k_cheb_mono(double* __restrict__ tables, int K) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * NPIECE) return;
  double* c = tables + idx * NC;
  double cm[NC], a[NC], t0[NC], t1[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    cm[j] = c[j];
    t0[j] = t1[j] = 0.0;
  }
  t0[0] = 1.0;  // T_0
  t1[1] = 1.0;  // T_1
#pragma unroll
  for (int j = 0; j < NC; ++j) a[j] = cm[0] * t0[j] + cm[1] * t1[j];
#pragma unroll
  for (int m = 2; m < NC; ++m) {
    double t2[NC];
    t2[0] = -t0[0];
#pragma unroll
    for (int j = 1; j < NC; ++j) t2[j] = 2.0 * t1[j - 1] - t0[j];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      a[j] = fma(cm[m], t2[j], a[j]);
      t0[j] = t1[j];
      t1[j] = t2[j];
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) c[j] = ldexp(a[j], 3 * j);
}

hipError_t launch_cheb_tables(const MaternParams* mp, double* nodes, double* tables, int K,
                              hipStream_t s) {
  const int64_t total = (int64_t)K * TABLE;
  const int blocks = (int)((total + 255) / 256);
  hipLaunchKernelGGL(k_cheb_nodes, dim3(blocks), dim3(256), 0, s, mp, nodes, K);
  hipLaunchKernelGGL(k_cheb_coeffs, dim3(blocks), dim3(256), 0, s, nodes, tables, K);
  const int64_t pieces = (int64_t)K * NPIECE;
  hipLaunchKernelGGL(k_cheb_mono, dim3((unsigned)((pieces + 255) / 256)), dim3(256), 0, s, tables,
                     K);
  return hipGetLastError();
}

// Lower tile t of the packed order (row-major over I, then J <= I).
__device__ __forceinline__ void tile_of(int t, int& I, int& J) {
  I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  J = t - I * (I + 1) / 2;
}

// SPLIT: flags holds 4 bytes per tile (one per wave; see matern_tile).
template <int MODE, bool SPLIT = false>
__global__ __launch_bounds__(256) void k_matern(Lay lay, double* __restrict__ mats,
                                                int64_t stride64, float* __restrict__ m32,
                                                int64_t stride32,
                                                const double* __restrict__ locs,
                                                const MaternParams* __restrict__ mp,
                                                const double* __restrict__ tables, int ntiles,
                                                int G, uint8_t* __restrict__ flags) {
  __shared__ __attribute__((aligned(16))) double smem[TABLE + 2 * T];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / ntiles;
  const int t = wg % ntiles;
  int I, J;
  tile_of(t, I, J);
  const int64_t off = lay.tile_off(I, J);
  double* C = (MODE != 3) ? mats + (int64_t)k * stride64 + off : nullptr;
  float* C32 = (MODE == 2 || MODE == 3) ? m32 + (int64_t)k * stride32 + off : nullptr;
  // an uneven batch: the unit's own order and locations
  const double* lk = lay.units ? lay.units[k].locs : locs;
  dev_matern_tile<MODE, SPLIT>(lay_of(lay, k), mp[k], tables + (int64_t)k * TABLE, lk, I, J, C,
                               lay.tile_ld(I), C32, smem,
                               SPLIT ? flags + ((int64_t)k * ntiles + t) * 4 : nullptr);
}

// After k_matern<MODE, true>: one workgroup per omega walks its tiles' flags
// (staged through LDS 256 at a time) and computes, in the flagged tiles, the
// elements left to the quadrature (pairs within about 1e-3 of the range:
// a few tiles per omega at most in practice).
template <int MODE>
__global__ __launch_bounds__(256) void k_matern_quad(Lay lay, double* __restrict__ mats,
                                                     int64_t stride64, float* __restrict__ m32,
                                                     int64_t stride32,
                                                     const double* __restrict__ locs,
                                                     const MaternParams* __restrict__ mp,
                                                     const uint8_t* __restrict__ flags,
                                                     int ntiles) {
  __shared__ uint32_t fl[256];
  const int k = blockIdx.x;
  const Lay L = lay_of(lay, k);
  const double* lk = lay.units ? lay.units[k].locs : locs;
  const uint32_t* f = reinterpret_cast<const uint32_t*>(flags) + (int64_t)k * ntiles;
  for (int t0 = 0; t0 < ntiles; t0 += 256) {
    __syncthreads();  // the previous block of flags is read
    fl[threadIdx.x] = t0 + (int)threadIdx.x < ntiles ? f[t0 + threadIdx.x] : 0u;
    __syncthreads();
    const int nb = min(256, ntiles - t0);
    for (int i = 0; i < nb; ++i) {
      if (fl[i] == 0u) continue;  // uniform: every lane reads the same word
      int I, J;
      tile_of(t0 + i, I, J);
      const int64_t off = lay.tile_off(I, J);
      double* C = mats + (int64_t)k * stride64 + off;
      float* C32 = MODE == 2 ? m32 + (int64_t)k * stride32 + off : nullptr;
      matern_tile_quad<MODE>(mp[k], lk, L.n, I, J, C, lay.tile_ld(I), C32);
    }
  }
}

// The split build needs 4 bytes per tile per omega of flag_ws (the table
// nodes' TABLE doubles per omega); without it, or past that, the one-launch
// form with the quadrature inline.
static bool split_ok(int ntiles, const uint8_t* flag_ws) {
  return flag_ws != nullptr && (reinterpret_cast<uintptr_t>(flag_ws) & 3) == 0 &&
         (int64_t)ntiles * 4 <= (int64_t)TABLE * (int64_t)sizeof(double);
}

hipError_t launch_matern_packed(const Lay& lay, double* mats, const double* locs,
                                const MaternParams* mp, const double* tables, int K,
                                hipStream_t s, uint8_t* flag_ws) {
  const int ntiles = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntiles;
  if (split_ok(ntiles, flag_ws)) {
    hipLaunchKernelGGL((k_matern<0, true>), dim3(G), dim3(256), 0, s, lay, mats, lay.mstride,
                       (float*)nullptr, (int64_t)0, locs, mp, tables, ntiles, G, flag_ws);
    hipLaunchKernelGGL(k_matern_quad<0>, dim3(K), dim3(256), 0, s, lay, mats, lay.mstride,
                       (float*)nullptr, (int64_t)0, locs, mp, flag_ws, ntiles);
  } else {
    hipLaunchKernelGGL((k_matern<0, false>), dim3(G), dim3(256), 0, s, lay, mats, lay.mstride,
                       (float*)nullptr, (int64_t)0, locs, mp, tables, ntiles, G, (uint8_t*)nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_matern_mixed(const Lay& lay, double* m64, int64_t stride64, float* m32,
                               const double* locs, const MaternParams* mp, const double* tables,
                               int K, hipStream_t s, uint8_t* flag_ws) {
  const int ntiles = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntiles;
  if (split_ok(ntiles, flag_ws)) {
    hipLaunchKernelGGL((k_matern<2, true>), dim3(G), dim3(256), 0, s, lay, m64, stride64, m32,
                       lay.mstride, locs, mp, tables, ntiles, G, flag_ws);
    hipLaunchKernelGGL(k_matern_quad<2>, dim3(K), dim3(256), 0, s, lay, m64, stride64, m32,
                       lay.mstride, locs, mp, flag_ws, ntiles);
  } else {
    hipLaunchKernelGGL((k_matern<2, false>), dim3(G), dim3(256), 0, s, lay, m64, stride64, m32,
                       lay.mstride, locs, mp, tables, ntiles, G, (uint8_t*)nullptr);
  }
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
  hipLaunchKernelGGL((k_matern<1, false>), dim3(G), dim3(256), 0, s, lay, V, lay.mstride,
                     (float*)nullptr, (int64_t)0, locs, mp, tables, ntiles, G, (uint8_t*)nullptr);
  return hipGetLastError();
}

// FP32 column-major V: every element computed in FP64 as above, rounded once.
hipError_t launch_matern_colmajor_f32(float* V, int64_t ld, int n, const double* locs,
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
  hipLaunchKernelGGL((k_matern<3, false>), dim3(G), dim3(256), 0, s, lay, (double*)nullptr,
                     (int64_t)0, V, lay.mstride, locs, mp, tables, ntiles, G, (uint8_t*)nullptr);
  return hipGetLastError();
}

}  // namespace plk
