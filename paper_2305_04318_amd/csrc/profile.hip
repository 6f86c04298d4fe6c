// Box-Cox right-hand sides and Jacobian (Section 2; equation (2)'s third
// term), and the p x p stage of Step 3 (Steps 5-8 of Section 3.3) that turns
// the cross products into beta-hat, sigma-hat^2 and the profile
// log-likelihood (equations "betahat", (4), "profile", Appendix "remlpro").
#include <math.h>

#include "finalize_dev.h"

namespace plk {

__global__ void k_fill(double* p, double v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
hipError_t launch_fill(double* p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

// rhs is n rows of TB values: [y'(lambda_1) .. y'(lambda_M) | X_1 .. X_p | 0 ..]
// (y' = expm1(lambda log y)/lambda, log y at lambda = 0).
__global__ void k_boxcox_rhs(const double* __restrict__ y, const double* __restrict__ X,
                             const double* __restrict__ lam, int n, int p, int M, int TB,
                             double* __restrict__ rhs) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * TB) return;
  const int i = (int)(idx / TB), a = (int)(idx % TB);
  double v = 0.0;
  if (a < M) {
    const double ly = log(y[i]);
    const double l = lam[a];
    v = (l == 0.0) ? ly : expm1(l * ly) / l;
  } else if (a < M + p) {
    v = X[(int64_t)(a - M) * n + i];
  }
  rhs[idx] = v;
}

// J = sum log y_i in one workgroup (fixed summation order) and the y > 0 flag.
__global__ __launch_bounds__(1024) void k_jacobian(const double* __restrict__ y, int n,
                                                   double* __restrict__ jac,
                                                   int32_t* __restrict__ flags) {
  __shared__ double red[1024];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double s = 0.0;
  int lbad = 0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double v = y[i];
    if (!(v > 0.0) || !isfinite(v)) lbad = 1;
    else s += log(v);
  }
  red[threadIdx.x] = s;
  if (lbad) atomicOr(&bad, 1);
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    jac[0] = red[0];
    flags[0] = bad;
  }
}

hipError_t launch_boxcox_rhs(const double* y, const double* X, const double* lam, int n, int p,
                             int M, double* rhs, double* jac, int32_t* flags, hipStream_t s) {
  const int TB = ((M + p) + 15) / 16 * 16;
  const int64_t total = (int64_t)n * TB;
  hipLaunchKernelGGL(k_boxcox_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, y, X,
                     lam, n, p, M, TB, rhs);
  hipLaunchKernelGGL(k_jacobian, dim3(1), dim3(1024), 0, s, y, n, jac, flags);
  return hipGetLastError();
}

// Copy the right-hand sides into each omega's bordered tile row (column i of
// the bordered panel is rhs row i) and clear the final TB x TB tile.  In an
// uneven batch each omega takes its dataset's right-hand sides and order;
// columns at or beyond n are not written (never read as data).
__host__ __device__ inline int64_t border_span(const Lay& lay) {
  return (int64_t)lay.Nv * T * lay.TB + (int64_t)lay.TB * lay.TB;
}

template <typename TS>
__global__ void k_border_init(Lay lay, TS* __restrict__ mats, const double* __restrict__ rhs,
                              int K) {
  const int64_t per = border_span(lay);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= per * K) return;
  const int k = (int)(idx / per);
  const int64_t e = idx % per;
  TS* base = mats + (int64_t)k * lay.mstride;
  const int64_t panel = (int64_t)lay.Nv * T * lay.TB;
  if (e < panel) {
    const int n = lay.units ? lay.units[k].n : lay.n;
    if (e < (int64_t)n * lay.TB)
      base[lay.tile_off(lay.Nv, 0) + e] = (TS)rhs[(lay.units ? lay.units[k].rhs : 0) + e];
  } else {
    base[lay.tile_off(lay.Nv, lay.Nv) + (e - panel)] = (TS)0;
  }
}

hipError_t launch_border_init(const Lay& lay, double* mats, const double* rhs, int K,
                              hipStream_t s) {
  const int64_t total = border_span(lay) * K;
  hipLaunchKernelGGL(k_border_init<double>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     lay, mats, rhs, K);
  return hipGetLastError();
}

hipError_t launch_border_init_f32(const Lay& lay, float* mats, const double* rhs, int K,
                                  hipStream_t s) {
  const int64_t total = border_span(lay) * K;
  hipLaunchKernelGGL(k_border_init<float>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     lay, mats, rhs, K);
  return hipGetLastError();
}

static_assert(T * (T + 1) % 4 == 0, "right-hand sides follow the tile in LDS, 16-byte aligned");

// ---- mixed form: back substitution x0 = L^-T Z -----------------------------------
// The FP32 factorisation leaves Z^T = (L^-1 B)^T in the bordered tile row.  x0
// (n rows of TB values, FP64) starts as Z and is swept from the bottom tile row:
//   k_bs_diag(I)   : X_I <- W_I^T X_I           (W_I = L_II^-1, one workgroup per omega)
//   k_bs_update(I) : X_J <- X_J - L_IJ^T X_I   (J < I, one workgroup per (omega, J))
// TB (16, 32, 48 or 64: the mixed form takes M + p <= 64) is a template
// parameter so that the per-thread column loop is straight-line code.  Thread (r, h) owns
// row r of the output tile and the contiguous columns h*TB/2 .. h*TB/2+TB/2-1;
// a wave has one h, so its reads of the right-hand sides are LDS broadcasts.

__global__ void k_bs_init(Lay lay, const float* __restrict__ m32, const int32_t* __restrict__ info,
                          double* __restrict__ X, int K) {
  const int64_t per = x0_stride(lay);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= per * K) return;
  const int k = (int)(idx / per);
  const int64_t e = idx % per;
  const int n = lay.units ? lay.units[k].n : lay.n;
  // bordered panel: element (a, i) at i*TB + a, the same index as x0 row i,
  // column a; rows at or beyond n are never read
  if (e < (int64_t)n * lay.TB)
    X[idx] = (double)m32[(int64_t)k * lay.mstride + lay.tile_off(lay.Nv, 0) + e];
}

// Ls[c][r] (stride T + 1) = G[c][r] for the T x T column-major tile G, rows
// r >= valid_rows as zero.  Every thread (blockDim.x == 256) issues all 16 of
// its 16-byte loads before its first LDS store.
constexpr int STAGE_PER = T * T / 4 / 256;
__device__ __forceinline__ void stage_tile_t(float* Ls, const float* __restrict__ G, int valid_rows) {
  float4 v[STAGE_PER];
#pragma unroll
  for (int u = 0; u < STAGE_PER; ++u)
    v[u] = *reinterpret_cast<const float4*>(G + 4 * (threadIdx.x + 256 * u));
#pragma unroll
  for (int u = 0; u < STAGE_PER; ++u) {
    const int idx = 4 * (threadIdx.x + 256 * u), col = idx / T, row = idx % T;
    float* dst = Ls + col * (T + 1) + row;
    dst[0] = (row + 0 < valid_rows) ? v[u].x : 0.0f;
    dst[1] = (row + 1 < valid_rows) ? v[u].y : 0.0f;
    dst[2] = (row + 2 < valid_rows) ? v[u].z : 0.0f;
    dst[3] = (row + 3 < valid_rows) ? v[u].w : 0.0f;
  }
}

// Xs[c][a] = (float) Xg[c][a] for the T x TB block of right-hand sides; rows
// c >= valid_rows read as zero.  Loads go to a clamped (always valid) address
// and are selected afterwards, so all of a thread's loads are in flight at once.
template <int TB>
__device__ __forceinline__ void stage_rhs(float* Xs, const double* __restrict__ Xg, int valid_rows) {
  constexpr int PER = T * TB / 256;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int idx = 256 * u + threadIdx.x;
    const bool ok = idx / TB < valid_rows;
    v[u] = Xg[ok ? idx : 0];
    v[u] = ok ? v[u] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) Xs[256 * u + threadIdx.x] = (float)v[u];
}

// out[m] = sum_c Ls[r][c]-row . Xs[c][h*NC + m] over c < rows (NC = TB / 2)
template <int TB>
__device__ __forceinline__ void bs_rowdot(const float* Ls, const float* Xs, int r, int h, int rows,
                                          float (&out)[TB / 2]) {
  constexpr int NC = TB / 2;
  const float* lrow = Ls + r * (T + 1);
  const float* xcol = Xs + h * NC;
#pragma unroll
  for (int m = 0; m < NC; ++m) out[m] = 0.0f;
#pragma unroll 4
  for (int c = 0; c < rows; ++c) {
    const float l = lrow[c];
    const float4* xv = reinterpret_cast<const float4*>(xcol + c * TB);
#pragma unroll
    for (int m4 = 0; m4 < NC / 4; ++m4) {
      const float4 x = xv[m4];
      out[4 * m4 + 0] += l * x.x;
      out[4 * m4 + 1] += l * x.y;
      out[4 * m4 + 2] += l * x.z;
      out[4 * m4 + 3] += l * x.w;
    }
  }
}

// Half of a tile (its 64 columns from col0) transposed into Ls (64 x (T+1));
// rows c >= valid_rows read as zero.  G points at the tile.
constexpr int HALF_PER = 64 * T / 4 / 256;
__device__ __forceinline__ void stage_half_t(float* Ls, const float* __restrict__ G, int col0,
                                             int valid_rows) {
  float4 v[HALF_PER];
#pragma unroll
  for (int u = 0; u < HALF_PER; ++u)
    v[u] = *reinterpret_cast<const float4*>(G + (int64_t)col0 * T + 4 * (threadIdx.x + 256 * u));
#pragma unroll
  for (int u = 0; u < HALF_PER; ++u) {
    const int idx = 4 * (threadIdx.x + 256 * u), col = idx / T, row = idx % T;
    float* dst = Ls + col * (T + 1) + row;
    dst[0] = (row + 0 < valid_rows) ? v[u].x : 0.0f;
    dst[1] = (row + 1 < valid_rows) ? v[u].y : 0.0f;
    dst[2] = (row + 2 < valid_rows) ? v[u].z : 0.0f;
    dst[3] = (row + 3 < valid_rows) ? v[u].w : 0.0f;
  }
}

// out[m] = sum_c Ls[r][c] Xs[c][q NC + m] over c < rows (NC = TB / 4): the
// quarter-width form of bs_rowdot for a half-tile stage, same order of sums
template <int TB>
__device__ __forceinline__ void bs_rowdot4(const float* Ls, const float* Xs, int r, int q,
                                           int rows, float (&out)[TB / 4]) {
  constexpr int NC = TB / 4;
  const float* lrow = Ls + r * (T + 1);
  const float* xcol = Xs + q * NC;
#pragma unroll
  for (int m = 0; m < NC; ++m) out[m] = 0.0f;
#pragma unroll 4
  for (int c = 0; c < rows; ++c) {
    const float l = lrow[c];
    const float4* xv = reinterpret_cast<const float4*>(xcol + c * TB);
#pragma unroll
    for (int m4 = 0; m4 < NC / 4; ++m4) {
      const float4 x = xv[m4];
      out[4 * m4 + 0] += l * x.x;
      out[4 * m4 + 1] += l * x.y;
      out[4 * m4 + 2] += l * x.z;
      out[4 * m4 + 3] += l * x.w;
    }
  }
}

template <int TB>
__global__ __launch_bounds__(256) void k_bs_diag(Lay lay, const float* __restrict__ W32,
                                                 const int32_t* __restrict__ info,
                                                 double* __restrict__ X, int I) {
  extern __shared__ __attribute__((aligned(16))) float bsm[];  // T x (T+1) tile, T x TB rhs
  float* Ls = bsm;
  float* Xs = bsm + T * (T + 1);  // T (T + 1) = 16512 floats: 16-byte aligned
  constexpr int NC = TB / 2;
  const int k = blockIdx.x;
  if (info[k] != 0) return;
  const int tid = threadIdx.x, r = tid & (T - 1), h = tid >> 7;
  const int ri = lay_of(lay, k).rows(I);
  double* Xi = X + (int64_t)k * x0_stride(lay) + (int64_t)I * T * TB;
  stage_tile_t(Ls, W32 + ((int64_t)k * lay.Nv + I) * T * T, T);
  stage_rhs<TB>(Xs, Xi, ri);
  __syncthreads();
  float out[NC];
  bs_rowdot<TB>(Ls, Xs, r, h, ri, out);
  if (r < ri) {
    double* dst = Xi + r * TB + h * NC;
#pragma unroll
    for (int m = 0; m < NC; ++m) dst[m] = (double)out[m];
  }
}

// x_J -= L_IJ^T x_I for one (omega, J < I).  The tile is staged one half
// (64 of its columns) at a time, so that the LDS block (64 (T+1) + T TB floats)
// lets three workgroups share a compute unit; thread (r, q) produces row
// 64 half + r of x_J for a quarter of the right-hand sides.
template <int TB>
__global__ __launch_bounds__(256) void k_bs_update(Lay lay, const float* __restrict__ m32,
                                                   const int32_t* __restrict__ info,
                                                   double* __restrict__ X, int I) {
  extern __shared__ __attribute__((aligned(16))) float bsm[];
  float* Ls = bsm;
  float* Xs = bsm + 64 * (T + 1);  // 64 (T + 1) = 8256 floats: 16-byte aligned
  constexpr int NC = TB / 4;
  const int k = blockIdx.x / I;
  const int J = blockIdx.x % I;
  if (info[k] != 0) return;
  const int tid = threadIdx.x, r = tid & 63, q = tid >> 6;
  const int ri = lay_of(lay, k).rows(I);
  const double* Xi = X + (int64_t)k * x0_stride(lay) + (int64_t)I * T * TB;
  double* Xj = X + (int64_t)k * x0_stride(lay) + (int64_t)J * T * TB;
  // tile (I, J): rows in block I (the contraction index), columns in block J
  const float* G = m32 + (int64_t)k * lay.mstride + lay.tile_off(I, J);
  stage_rhs<TB>(Xs, Xi, ri);
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    stage_half_t(Ls, G, 64 * half, ri);
    __syncthreads();
    float out[NC];
    bs_rowdot4<TB>(Ls, Xs, r, q, ri, out);
    // tile row J < I is complete (T rows)
    double* dst = Xj + (64 * half + r) * TB + q * NC;
    double cur[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) cur[m] = dst[m];
#pragma unroll
    for (int m = 0; m < NC; ++m) dst[m] = cur[m] - (double)out[m];
    __syncthreads();  // Ls is restaged for the second half
  }
}

template <int TB>
static void backsolve_sweep(const Lay& lay, const float* m32, const float* W32, const int32_t* info,
                            double* X, int K, hipStream_t s) {
  const size_t lds = (size_t)(T * (T + 1) + T * TB) * sizeof(float);
  const size_t lds_half = (size_t)(64 * (T + 1) + T * TB) * sizeof(float);
  for (int I = lay.Nv - 1; I >= 0; --I) {
    hipLaunchKernelGGL(k_bs_diag<TB>, dim3(K), dim3(256), lds, s, lay, W32, info, X, I);
    if (I > 0)
      hipLaunchKernelGGL(k_bs_update<TB>, dim3(K * I), dim3(256), lds_half, s, lay, m32, info, X,
                         I);
  }
}

hipError_t launch_backsolve(const Lay& lay, const float* m32, const float* W32,
                            const int32_t* info, double* X, int K, hipStream_t s) {
  if (lay.TB != 16 && lay.TB != 32 && lay.TB != 48 && lay.TB != 64) return hipErrorInvalidValue;
  const int64_t total = x0_stride(lay) * K;
  hipLaunchKernelGGL(k_bs_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, lay, m32,
                     info, X, K);
  switch (lay.TB) {
    case 16: backsolve_sweep<16>(lay, m32, W32, info, X, K, s); break;
    case 32: backsolve_sweep<32>(lay, m32, W32, info, X, K, s); break;
    case 48: backsolve_sweep<48>(lay, m32, W32, info, X, K, s); break;
    default: backsolve_sweep<64>(lay, m32, W32, info, X, K, s); break;
  }
  return hipGetLastError();
}

// OR the fallback flag into every record of omega k (after an FP64 redo).
__global__ void k_mark_fallback(pl_result* out, int M) {
  for (int m = threadIdx.x; m < M; m += blockDim.x) out[m].info |= PL_INFO_FALLBACK;
}
hipError_t launch_mark_fallback(pl_result* out, int M, hipStream_t s) {
  hipLaunchKernelGGL(k_mark_fallback, dim3(1), dim3(64), 0, s, out, M);
  return hipGetLastError();
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i32, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// ---- mixed form: the cross products from the refined slots ----------------------
// red[b TB + a] = -(1/2) sum_t (slot_t[a][b] + slot_t[b][a]) over the omega's
// lower tiles t, in tile order.  One workgroup per omega, one thread per
// (a, b) pair: the tile loop is unrolled so that many loads are in flight
// (one wave summing every pair in turn was bound by load latency).
__global__ __launch_bounds__(256) void k_slot_reduce(const double* __restrict__ slots, int ntile,
                                                     int TB, double* __restrict__ red,
                                                     int64_t red_stride) {
  const int k = blockIdx.x;
  const int64_t tile = (int64_t)TB * TB;
  const double* sk = slots + (int64_t)k * ntile * tile;
  for (int pr = threadIdx.x; pr < TB * TB; pr += 256) {
    const int a = pr / TB, b = pr % TB;
    double v = 0.0;
#pragma unroll 8
    for (int t = 0; t < ntile; ++t) v += sk[t * tile + a * TB + b] + sk[t * tile + b * TB + a];
    red[(int64_t)k * red_stride + b * TB + a] = -0.5 * v;
  }
}

hipError_t launch_slot_reduce(const Lay& lay, const double* slots, double* red,
                              int64_t red_stride, int K, hipStream_t s) {
  const int ntile = lay.Nv * (lay.Nv + 1) / 2;
  hipLaunchKernelGGL(k_slot_reduce, dim3(K), dim3(256), 0, s, slots, ntile, lay.TB, red,
                     red_stride);
  return hipGetLastError();
}

// ---- p x p stage (dev_finalize) -----------------------------------------------------
// One wave per omega.  S: the Schur tile of the bordered FP64 factorisation, or
// (mixed form, sred non-null) the reduced cross products of k_slot_reduce.
// An uneven batch takes each omega's order, Jacobian, y check and record
// index from its UnitInfo (out, beta and xvi are then the batch's arrays).
__global__ __launch_bounds__(64) void k_finalize(Lay lay, const double* __restrict__ mats,
                                                 const double* __restrict__ sred,
                                                 int64_t sred_stride,
                                                 const double* __restrict__ logdet,
                                                 const int32_t* __restrict__ info,
                                                 const double* __restrict__ jac,
                                                 const int32_t* __restrict__ flags,
                                                 const double* __restrict__ lam, int n, int p,
                                                 int M, pl_result* __restrict__ out,
                                                 double* __restrict__ beta,
                                                 double* __restrict__ xvi) {
  __shared__ double smem[FIN_SMEM_DOUBLES];
  const int k = blockIdx.x;
  const int TB = lay.TB;
  const double* S = sred ? sred + (int64_t)k * sred_stride
                         : mats + (int64_t)k * lay.mstride + lay.tile_off(lay.Nv, lay.Nv);
  const int ds = lay.units ? lay.units[k].ds : 0;
  const int64_t om = lay.units ? lay.units[k].om : k;
  dev_finalize(S, TB, logdet[k], info[k], jac[ds], flags[ds] != 0, lam,
               lay.units ? lay.units[k].n : n, p, M, out + om * M,
               beta ? beta + om * M * p : nullptr, xvi ? xvi + om * p * p : nullptr, smem);
}

hipError_t launch_finalize(const Lay& lay, const double* mats, const double* sred,
                           int64_t sred_stride,
                           const double* logdet, const int32_t* info, const double* jac,
                           const int32_t* flags, const double* lam, int n, int p, int M, int K,
                           pl_result* out, double* beta, double* xvi, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(K), dim3(64), 0, s, lay, mats, sred, sred_stride, logdet,
                     info, jac,
                     flags, lam, n, p, M, out, beta, xvi);
  return hipGetLastError();
}

}  // namespace plk
