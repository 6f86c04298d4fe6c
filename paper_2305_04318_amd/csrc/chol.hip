// Blocked Cholesky V = L L^T and its log-determinant (Step 2 of Section 3.3),
// left-looking over block columns of width T, batched over omega.
//
// Step J of the factorisation:
//   k_gemm_col : C_IJ -= L_I,0:J L_J,0:J^T for every tile row I >= J (MFMA f64)
//   k_potrf    : C_JJ = L_JJ L_JJ^T in LDS, log|V| += 2 sum log L_jj,
//                W_J = L_JJ^{-1} (triangular inverse, also in LDS)
//   k_trsm     : L_IJ = C_IJ W_J^T for I > J (MFMA f64)
// With the packed bordered layout the right-hand sides are extra tile rows
// under V, so the same steps produce Z = L^{-1}[Y'|X] (Step 3) and, in the
// final tile, minus the cross products (y,X)^T V^{-1} (y,X) (Step 4).
//
// MFMA v_mfma_f64_16x16x4f64 operand layout (64 lanes, checked on gfx950):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane
// j + 16 (i % 4), item i / 4.  The kernels pass the B-panel fragment as the
// first operand, so a lane's accumulator item e holds C[16i + (lane & 15)]
// [16j + (lane >> 4) + 4e] of C = A B^T: sixteen lanes cover 16 consecutive
// rows of one column, a contiguous 128-byte run in column-major storage.
#include <math.h>

#include "common.h"

namespace plk {

typedef double d4 __attribute__((ext_vector_type(4)));

// acc[i][j] += A[16i + ., 0:kmax] * B[16j + ., 0:kmax]^T for a 64x64 wave
// tile.  A, B are column-major panels (column k at +k*ld); rows at or beyond
// arows / brows and columns at or beyond kmax read as zero.
__device__ __forceinline__ void mfma_nt64(d4 (&acc)[4][4], const double* __restrict__ A,
                                          int64_t lda, int arows, const double* __restrict__ B,
                                          int64_t ldb, int brows, int kmax, int lane) {
  const int lr = lane & 15, lk = lane >> 4;
  const int ni = min(4, (arows + 15) >> 4);
  const int nj = min(4, (brows + 15) >> 4);
  bool av[4], bv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    av[i] = (16 * i + lr) < arows;
    bv[i] = (16 * i + lr) < brows;
  }
  const double* pa = A + lr;
  const double* pb = B + lr;
#pragma unroll 2
  for (int k0 = 0; k0 < kmax; k0 += 4) {
    const int kk = k0 + lk;
    const bool kv = kk < kmax;
    const double* ca = pa + (int64_t)kk * lda;
    const double* cb = pb + (int64_t)kk * ldb;
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = (kv && av[i]) ? ca[16 * i] : 0.0;
      b[i] = (kv && bv[i]) ? cb[16 * i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i < ni) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j < nj) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
        }
      }
    }
  }
}

// C[r][c] (op)= acc for the valid part of a 64x64 wave tile.
template <bool SUB>
__device__ __forceinline__ void store64(double* C, int64_t ldc, const d4 (&acc)[4][4], int arows,
                                        int brows, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * i + lr;
    if (r >= arows) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * j + lg + 4 * e;
        if (c < brows) {
          double* p = C + (int64_t)c * ldc + r;
          if (SUB) *p -= acc[i][j][e];
          else *p = acc[i][j][e];
        }
      }
    }
  }
}

// ---- left-looking update of block column J -----------------------------------
__global__ __launch_bounds__(256) void k_gemm_col(Lay lay, double* __restrict__ mats,
                                                  const int32_t* __restrict__ info, int J, int nI,
                                                  int G) {
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + wg % nI;
  if (info[k] != 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  if (I == J && wc > wr) return;  // strictly upper part of a diagonal tile
  const int arows = lay.rows(I) - 64 * wr;
  const int brows = lay.rows(J) - 64 * wc;
  if (arows <= 0 || brows <= 0) return;
  double* base = mats + (int64_t)k * lay.mstride;
  const double* A = base + lay.tile_off(I, 0) + 64 * wr;
  const double* B = base + lay.tile_off(J, 0) + 64 * wc;
  const int kmax = min(J * T, lay.n);
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  mfma_nt64(acc, A, lay.tile_ld(I), arows, B, lay.tile_ld(J), brows, kmax, lane);
  const int64_t ldc = lay.tile_ld(I);
  double* C = base + lay.tile_off(I, J) + 64 * wr + 64 * wc * ldc;
  store64<true>(C, ldc, acc, arows, brows, lane);
}

hipError_t launch_gemm_col(const Lay& lay, double* mats, const int32_t* info, int J, int nI,
                           int K, hipStream_t s) {
  const int G = K * nI;
  hipLaunchKernelGGL(k_gemm_col, dim3(G), dim3(256), 0, s, lay, mats, info, J, nI, G);
  return hipGetLastError();
}

// ---- diagonal tile: factor and invert in LDS ------------------------------
constexpr int LDA = T + 1;  // LDS column stride

__global__ __launch_bounds__(256) void k_potrf(Lay lay, double* __restrict__ mats,
                                               double* __restrict__ Wbuf,
                                               double* __restrict__ logdet,
                                               int32_t* __restrict__ info, int J) {
  __shared__ double a[T * LDA];
  __shared__ double red[256];
  const int k = blockIdx.x;
  if (info[k] != 0) return;
  const int tid = threadIdx.x;
  const int nv = lay.rows(J);
  double* C = mats + (int64_t)k * lay.mstride + lay.tile_off(J, J);
  const int64_t ld = lay.tile_ld(J);
  for (int idx = tid; idx < T * T; idx += 256) {
    const int c = idx / T, r = idx % T;
    double v;
    if (r < nv && c < nv) v = (r >= c) ? C[(int64_t)c * ld + r] : 0.0;
    else v = (r == c) ? 1.0 : 0.0;
    a[c * LDA + r] = v;
  }
  __syncthreads();

  // Right-looking column sweep; column j is scaled by 1/sqrt(d_j) during step
  // j+1, which touches disjoint columns, so one barrier per column suffices.
  const int r = tid & (T - 1);
  const int half = tid >> 7;
  double rs_prev = 1.0;
  for (int j = 0; j < nv; ++j) {
    const double d = a[j * LDA + j];
    if (!(d > 0.0)) {  // same value in every thread: uniform exit
      if (tid == 0) info[k] = J * T + j + 1;
      return;
    }
    const double invd = 1.0 / d;
    if (r > j) {
      const double arj = a[j * LDA + r] * invd;
      for (int c = j + 1 + half; c <= r; c += 2) a[c * LDA + r] -= arj * a[j * LDA + c];
    }
    if (j > 0 && half == 0 && r >= j - 1) a[(j - 1) * LDA + r] *= rs_prev;
    rs_prev = 1.0 / sqrt(d);
    __syncthreads();
  }
  if (nv > 0 && half == 0 && r >= nv - 1) a[(nv - 1) * LDA + r] *= rs_prev;
  __syncthreads();

  // log-determinant contribution and the factor itself
  red[tid] = (tid < nv) ? log(a[tid * LDA + tid]) : 0.0;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) logdet[k] += 2.0 * red[0];
  for (int idx = tid; idx < T * T; idx += 256) {
    const int c = idx / T, rr = idx % T;
    if (rr < nv && c < nv && rr >= c) C[(int64_t)c * ld + rr] = a[c * LDA + rr];
  }

  // In-place inverse of the unit-padded lower factor, last column first:
  // W_jj = 1/L_jj, W_rj = -W_jj sum_{m=j+1..r} W_rm L_mj.
  for (int j = T - 1; j >= 0; --j) {
    double t = 0.0;
    if (tid > j && tid < T) {
      for (int m = j + 1; m <= tid; ++m) t += a[m * LDA + tid] * a[j * LDA + m];
    }
    __syncthreads();
    const double wjj = 1.0 / a[j * LDA + j];
    if (tid > j && tid < T) a[j * LDA + tid] = -wjj * t;
    __syncthreads();
    if (tid == 0) a[j * LDA + j] = wjj;
    __syncthreads();
  }
  double* W = Wbuf + (int64_t)k * T * T;
  for (int idx = tid; idx < T * T; idx += 256) {
    const int c = idx / T, rr = idx % T;
    W[idx] = a[c * LDA + rr];
  }
}

hipError_t launch_potrf(const Lay& lay, double* mats, double* W, double* logdet, int32_t* info,
                        int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf, dim3(K), dim3(256), 0, s, lay, mats, W, logdet, info, J);
  return hipGetLastError();
}

// ---- panel solve L_IJ = C_IJ W_J^T for the nI tile rows below J -----------
__global__ __launch_bounds__(256) void k_trsm(Lay lay, double* __restrict__ mats,
                                              const double* __restrict__ Wbuf,
                                              const int32_t* __restrict__ info, int J, int nI,
                                              int G) {
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + 1 + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I) - 64 * wr;
  const int brows = lay.rows(J) - 64 * wc;
  const bool active = arows > 0 && brows > 0;
  double* base = mats + (int64_t)k * lay.mstride;
  const int64_t ldc = lay.tile_ld(I);
  double* Ct = base + lay.tile_off(I, J);
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (active) {
    const double* W = Wbuf + (int64_t)k * T * T + 64 * wc;
    mfma_nt64(acc, Ct + 64 * wr, ldc, arows, W, T, brows, lay.rows(J), lane);
  }
  __syncthreads();  // every wave has read C_IJ before any overwrites it
  if (active) store64<false>(Ct + 64 * wr + 64 * wc * ldc, ldc, acc, arows, brows, lane);
}

hipError_t launch_trsm(const Lay& lay, double* mats, const double* W, const int32_t* info, int J,
                       int nI, int K, hipStream_t s) {
  const int G = K * nI;
  hipLaunchKernelGGL(k_trsm, dim3(G), dim3(256), 0, s, lay, mats, W, info, J, nI, G);
  return hipGetLastError();
}

}  // namespace plk
