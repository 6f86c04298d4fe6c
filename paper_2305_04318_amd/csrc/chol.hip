// Blocked Cholesky V = L L^T and its log-determinant (Step 2 of Section 3.3),
// left-looking over block columns of width T, batched over omega.
//
// Step J of the factorisation:
//   k_col_update : C_IJ -= L_I,0:J L_J,0:J^T for every tile row I >= J (MFMA);
//                  the diagonal tile's workgroup also updates the bordered
//                  row's tile (k_col_update_mx in the mixed form; k_gemm_col
//                  for the plain layout and bordered heights above 32)
//   k_potrf      : C_JJ = L_JJ L_JJ^T, log|V| += 2 sum log L_jj,
//                  W_J = L_JJ^{-1} (triangular inverse), register-blocked, FP64
//   k_trsm       : L_IJ = C_IJ W_J^T for I > J (MFMA)
// and after the last block column k_border_block updates the bordered row's
// own block.
// With the packed bordered layout the right-hand sides are extra tile rows
// under V, so the same steps produce Z = L^{-1}[Y'|X] (Step 3) and, in the
// final tile, minus the cross products (y,X)^T V^{-1} (y,X) (Step 4).
//
// Two forms share these kernels:
//   FP64  : every tile in FP64, FP64 MFMA.
//   mixed : the factor is stored in FP32 and off-diagonal updates use FP32
//           MFMA; panel solves (k_trsm_mx_dma) widen the FP32 tiles to FP64
//           MFMA and round L once; each diagonal tile is updated with FP64
//           accumulation from the original FP64 V and factored in FP64, and
//           the log-determinant is accumulated in FP64.
//
// MFMA operand layouts (64 lanes, checked on gfx950): A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k.  Results: v_mfma_f64_16x16x4f64 puts D[i][j] in lane
// j + 16 (i % 4), item i / 4; v_mfma_f32_16x16x4f32 in lane j + 16 (i / 4),
// item i % 4.  The kernels pass the B-panel fragment as the first operand, so
// sixteen consecutive lanes hold 16 consecutive rows of one result column.
#include <math.h>
#include <stdlib.h>

#include <algorithm>

#include "tiles.h"

namespace plk {

// ---- left-looking update of block column J ---------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_col(Lay lay, double* __restrict__ mats,
                                                     const int32_t* __restrict__ info, int J, int nI,
                                                     int G) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  dev_gemm_col<VEC>(lay_of(lay, k), mats + (int64_t)k * lay.mstride, J, I,
                    reinterpret_cast<double*>(lds_raw));
}

// Mixed form.  Off-diagonal tiles: FP32 storage, FP32 MFMA whose partial
// sums are accumulated in FP64, subtracted from V's FP64 tile and rounded to
// FP32 once.  The diagonal tile: FP64 MFMA on the FP32 panels, subtracted from
// the FP64 tile of V, written to an FP64 scratch tile for k_potrf.
// The FP32 partial sums span 4 * flush products (flush = FP32 MFMA k-steps per
// FP64 fold): 1, 2 or 4, chosen by the caller (default MX_FLUSH; pl_autotune
// measures the speed/accuracy trade-off per workload).
// DMA: whole packed tiles (I < Nv) take the direct-to-LDS core (lds of at
// least F32_DMA_LDS_BYTES).
template <bool VEC, int FLUSH, bool DMA = false>
__device__ __forceinline__ void dev_col_mx(const Lay& lay, float* __restrict__ m32,
                                           const double* __restrict__ m64, int64_t m64stride,
                                           int k, int I, int J, float* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  const int war = arows - 64 * wr, wbr = brows - 64 * wc;
  const int ni = nblk(war), nj = nblk(wbr);
  float* base = m32 + (int64_t)k * lay.mstride;
  const int kmax = min(J * T, lay.n);
  const bool act = ni > 0 && nj > 0;
  d4 acc[4][4];
  zero_acc<double>(acc);
  if (DMA && lay.kind == 0 && I < lay.Nv) {
    if (arows <= 0 || brows <= 0) return;  // a tile past an uneven unit's order (uniform)
    if (arows < T) {
      // the last tile row: column-split plan
      wg_gemm_nt_f32x64_dma<FLUSH, true>(acc, lds, base + lay.tile_off(I, 0),
                                                base + lay.tile_off(J, 0), kmax, true,
                                                (arows + 15) >> 4);
      const double* Cin = m64 ? m64 + (int64_t)k * m64stride + lay.tile_off(I, J) : nullptr;
      float* C = base + lay.tile_off(I, J);
      if (Cin) sub_store_split<float>(Cin, T, C, T, acc, wave, arows, brows, lane);
      else sub_store_split<float>(C, T, C, T, acc, wave, arows, brows, lane);
      return;
    }
    wg_gemm_nt_f32x64_dma<FLUSH>(acc, lds, base + lay.tile_off(I, 0), base + lay.tile_off(J, 0),
                                 kmax, act, ni);
  } else {
    wg_gemm_nt_f32x64<FLUSH>(acc, lds, base + lay.tile_off(I, 0), lay.tile_ld(I), arows,
                             base + lay.tile_off(J, 0), lay.tile_ld(J), brows, kmax, act, ni);
  }
  if (act) {
    const int64_t ldc = lay.tile_ld(I);
    float* C = base + lay.tile_off(I, J) + 64 * wr + 64 * wc * ldc;
    if (I < lay.Nv && m64) {
      // V's own tile from the FP64 copy: the update is subtracted in FP64
      const double* Cin = m64 + (int64_t)k * m64stride + lay.tile_off(I, J) + 64 * wr + 64 * wc * T;
      store64_l<float, true>(Cin, T, C, ldc, acc, war, wbr, lane);
    } else {
      store64_l<float, true>(C, ldc, C, ldc, acc, war, wbr, lane);
    }
  }
}

// Mixed form, diagonal tile J: FP64 MFMA on the FP32 panel, subtracted from V's
// FP64 tile, written to the FP64 scratch tile that k_potrf reads (the blocks
// on and below the diagonal; k_potrf reads no other).  BORDER: the bordered
// row's FP32 tile is updated in the same workgroup (FP64 MFMA on the FP32
// panels, one rounding to FP32), so the off-diagonal work does not give that
// 16- or 32-row tile a workgroup of its own.  Balanced plan of
// wg_gemm_diag_border.
template <bool VEC, bool BORDER>
__device__ __forceinline__ void dev_diag_mx(const Lay& lay, float* __restrict__ m32,
                                            const double* __restrict__ m64, int64_t m64stride,
                                            double* __restrict__ dscratch, int k, int J,
                                            float* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rows = lay.rows(J);
  if (rows <= 0) return;  // a tile past an uneven unit's order (uniform)
  float* base = m32 + (int64_t)k * lay.mstride;
  const float* P = base + lay.tile_off(J, 0);
  const int kmax = min(J * T, lay.n);
  // J = 0: no update; V's lower blocks are copied to the scratch tile
  const int nbr = (BORDER && kmax > 0) ? lay.TB / 16 : 0;
  const int qrows = nbr > 0 ? lay.q : 0;
  d4 acc[4][4];
  zero_acc<double>(acc);
  wg_gemm_diag_border<VEC, float, true>(acc, lds, P, rows, base + lay.tile_off(lay.Nv, 0),
                                        lay.TB, qrows, nbr, kmax, lay.tile_ld(J));
  double* Cout = dscratch + (int64_t)k * T * T;
  float* Cb = base + lay.tile_off(lay.Nv, J);
  if (m64) {
    const double* Cin = m64 + (int64_t)k * m64stride + lay.tile_off(J, J);
    sub_store_diag_bal(Cin, T, Cout, T, Cb, lay.TB, acc, wave, rows, qrows, nbr, lane);
  } else {
    // no FP64 copy (the plain FP32 matrix of pl_chol_batched): V's tile as stored
    sub_store_diag_bal(base + lay.tile_off(J, J), lay.tile_ld(J), Cout, T, Cb, lay.TB, acc, wave,
                       rows, qrows, nbr, lane);
  }
}

// Mixed-form block-column update in one launch: the K diagonal tiles (FP64
// MFMA, with the bordered row's tile on the idle wave; about twice as long
// as an FP32 tile) are dispatched first, the off-diagonal tiles (FP32 MFMA
// with FP64 folds) after them, so the diagonal work overlaps the bulk of the
// update instead of running as a launch of K workgroups of its own.
template <int FLUSH, bool BORDER>
__global__ __launch_bounds__(256, 2) void k_col_update_mx(Lay lay, float* __restrict__ m32,
                                                          const double* __restrict__ m64,
                                                          int64_t m64stride,
                                                          double* __restrict__ dscratch,
                                                          const int32_t* __restrict__ info, int J,
                                                          int nOff, int K) {
  __shared__ __attribute__((aligned(16)))
  char lds_raw[F32_DMA_LDS_BYTES > GEMM_LDS_BYTES ? F32_DMA_LDS_BYTES : GEMM_LDS_BYTES];
  float* lds = reinterpret_cast<float*>(lds_raw);
  const int b = blockIdx.x;
  if (b < K) {
    if (info[b] != 0) return;  // uniform for the workgroup
    dev_diag_mx<true, BORDER>(lay_of(lay, b), m32, m64, m64stride, dscratch, b, J, lds);
    return;
  }
  const int G = K * nOff;
  const int wg = xcd_remap(b - K, G);
  const int k = wg / nOff, r = wg % nOff;
  if (info[k] != 0) return;
  dev_col_mx<true, FLUSH, true>(lay_of(lay, k), m32, m64, m64stride, k, J + 1 + r, J, lds);
}

// Mixed form on a plain column-major FP32 matrix (pl_chol_batched with
// PL_MIXED): no bordered row and no FP64 copy of V, so each tile's update is
// subtracted from the FP32 tile itself (promoted to FP64).  The K diagonal
// tiles come first, then the nOff tiles below each.
template <int FLUSH>
__global__ __launch_bounds__(256, 2) void k_col_update_mx_plain(Lay lay, float* __restrict__ m32,
                                                                double* __restrict__ dscratch,
                                                                const int32_t* __restrict__ info,
                                                                int J, int nOff, int K) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  float* lds = reinterpret_cast<float*>(lds_raw);
  const int b = blockIdx.x;
  if (b < K) {
    if (info[b] != 0) return;  // uniform for the workgroup
    dev_diag_mx<true, false>(lay, m32, nullptr, 0, dscratch, b, J, lds);
    return;
  }
  const int G = K * nOff;
  const int wg = xcd_remap(b - K, G);
  const int k = wg / nOff, r = wg % nOff;
  if (info[k] != 0) return;
  dev_col_mx<true, FLUSH>(lay, m32, nullptr, 0, k, J + 1 + r, J, lds);
}

static bool vec_ok(const Lay& lay, const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0 && (lay.kind == 0 || (lay.ld % 2) == 0);
}

hipError_t launch_gemm_col(const Lay& lay, double* mats, const int32_t* info, int J, int nI,
                           int K, hipStream_t s) {
  const int G = K * nI;
  if (vec_ok(lay, mats))
    hipLaunchKernelGGL(k_gemm_col<true>, dim3(G), dim3(256), 0, s, lay, mats, info, J, nI, G);
  else
    hipLaunchKernelGGL(k_gemm_col<false>, dim3(G), dim3(256), 0, s, lay, mats, info, J, nI, G);
  return hipGetLastError();
}

hipError_t launch_gemm_col_mx(const Lay& lay, float* m32, const double* m64, int64_t m64stride,
                              double* dscratch, const int32_t* info, int J, int nI, int K,
                              int flush, hipStream_t s) {
  // nI counts the tile rows from J down (the diagonal tile included).  A
  // bordered row of at most 32 rows (the last of the nI rows when J > 0) is
  // folded into the diagonal tile's workgroup; a taller one (M + p up to 64)
  // is updated as one more off-diagonal tile row.
  if (!(lay.kind == 0 && lay.q > 0 && lay.TB <= 64)) return hipErrorInvalidValue;
  const bool border = lay.TB <= 32;
  const int nOff = (J > 0) ? nI - (border ? 2 : 1) : 0;  // tiles strictly below the diagonal
  const int G = K * (nOff + 1);
#define PL_MX_LAUNCH(F, B)                                                                     \
  hipLaunchKernelGGL((k_col_update_mx<F, B>), dim3(G), dim3(256), 0, s, lay, m32, m64, m64stride, \
                     dscratch, info, J, nOff, K)
  switch (flush * 2 + (border ? 1 : 0)) {
    case 3: PL_MX_LAUNCH(1, true); break;
    case 2: PL_MX_LAUNCH(1, false); break;
    case 5: PL_MX_LAUNCH(2, true); break;
    case 4: PL_MX_LAUNCH(2, false); break;
    case 9: PL_MX_LAUNCH(4, true); break;
    case 8: PL_MX_LAUNCH(4, false); break;
    default:
      return hipErrorInvalidValue;
  }
#undef PL_MX_LAUNCH
  return hipGetLastError();
}

hipError_t launch_col_update_mx_plain(const Lay& lay, float* m32, double* dscratch,
                                      const int32_t* info, int J, int K, int flush,
                                      hipStream_t s) {
  // 16-byte loads of every column: the matrix and ld must keep 4-float alignment
  if (!(lay.kind == 1 && lay.ld % 4 == 0 && (reinterpret_cast<uintptr_t>(m32) & 15) == 0))
    return hipErrorInvalidValue;
  if (J < 0 || J >= lay.Nv) return hipErrorInvalidValue;
  const int nOff = (J > 0) ? lay.Nv - 1 - J : 0;  // J = 0: no update below the diagonal
  const int G = K * (nOff + 1);
  switch (flush) {
    case 1:
      hipLaunchKernelGGL(k_col_update_mx_plain<1>, dim3(G), dim3(256), 0, s, lay, m32, dscratch,
                         info, J, nOff, K);
      break;
    case 2:
      hipLaunchKernelGGL(k_col_update_mx_plain<2>, dim3(G), dim3(256), 0, s, lay, m32, dscratch,
                         info, J, nOff, K);
      break;
    case 4:
      hipLaunchKernelGGL(k_col_update_mx_plain<4>, dim3(G), dim3(256), 0, s, lay, m32, dscratch,
                         info, J, nOff, K);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- diagonal tile: factor and invert (dev_potrf) ---------------------------------
// MODE 0 (FP64 form): the tile is read from and L written back to the packed
//   matrix, W (FP64) to Wbuf[k].  MODE 1 (mixed form): the tile is read from
//   the FP64 scratch tile, L is not kept, W is written in FP32 to slot J of
//   the omega's inverse table (the back substitution needs every W_J).
template <int MODE>
__global__ __launch_bounds__(256, 2) void k_potrf(Lay lay, double* __restrict__ mats,
                                               double* __restrict__ Wbuf, float* __restrict__ W32,
                                               double* __restrict__ logdet,
                                               int32_t* __restrict__ info, int J) {
  __shared__ double smem[POTRF_BLK_SMEM_DOUBLES];
  const int k = blockIdx.x;
  if (info[k] != 0) return;
  const Lay L = lay_of(lay, k);
  if (MODE == 0)
    dev_potrf_blk<0>(L, mats + (int64_t)k * lay.mstride + lay.tile_off(J, J), lay.tile_ld(J),
                     Wbuf + (int64_t)k * T * T, nullptr, logdet + k, info + k, J, smem);
  else
    dev_potrf_blk<1>(L, Wbuf + (int64_t)k * T * T, T, nullptr,
                     W32 + ((int64_t)k * lay.Nv + J) * T * T, logdet + k, info + k, J, smem);
}

hipError_t launch_potrf(const Lay& lay, double* mats, double* W, double* logdet, int32_t* info,
                        int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf<0>, dim3(K), dim3(256), 0, s, lay, mats, W, (float*)nullptr, logdet,
                     info, J);
  return hipGetLastError();
}

// Plain FP32 matrix: the FP64 tile from dscratch[k], L_JJ rounded into the
// matrix, W_J to the omega's single FP32 slot W32[k].
__global__ __launch_bounds__(256, 2) void k_potrf_mx_plain(Lay lay, float* __restrict__ m32,
                                                        double* __restrict__ dscratch,
                                                        float* __restrict__ W32,
                                                        double* __restrict__ logdet,
                                                        int32_t* __restrict__ info, int J) {
  __shared__ double smem[POTRF_BLK_SMEM_DOUBLES];
  const int k = blockIdx.x;
  if (info[k] != 0) return;
  dev_potrf_blk<2>(lay, dscratch + (int64_t)k * T * T, T, nullptr, W32 + (int64_t)k * T * T,
               logdet + k, info + k, J, smem, m32 + (int64_t)k * lay.mstride + lay.tile_off(J, J),
               lay.tile_ld(J));
}

hipError_t launch_potrf_mx_plain(const Lay& lay, float* m32, double* dscratch, float* W32,
                                 double* logdet, int32_t* info, int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf_mx_plain, dim3(K), dim3(256), 0, s, lay, m32, dscratch, W32, logdet,
                     info, J);
  return hipGetLastError();
}

hipError_t launch_potrf_mx(const Lay& lay, double* dscratch, float* W32, double* logdet,
                           int32_t* info, int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf<1>, dim3(K), dim3(256), 0, s, lay, (double*)nullptr, dscratch, W32,
                     logdet, info, J);
  return hipGetLastError();
}
// ---- FP64 block-column update with the bordered row folded in -------------------
// Each omega has 1 + nOff workgroups, dispatched omega after omega: first the
// diagonal tile J, whose update runs on the three waves of its lower
// quadrants while the fourth (its quadrant lies above the diagonal) updates
// the bordered row's tile when that is at most 32 rows high, then the
// off-diagonal tiles of column J.  The 16-row bordered tiles, which would
// take a whole workgroup for one block row of MFMA work, no longer occupy
// workgroups of their own.  Consecutive logical workgroups share an XCD
// (xcd_remap), so an omega's panels are read through one L2.
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_col_update(Lay lay, double* __restrict__ mats,
                                                       const int32_t* __restrict__ info, int J,
                                                       int border, int nOff, int G) {
  __shared__ __attribute__((aligned(16)))
  char lds_raw[UPD_DMA_LDS_BYTES > GEMM_LDS_BYTES ? UPD_DMA_LDS_BYTES : GEMM_LDS_BYTES];
  double* lds = reinterpret_cast<double*>(lds_raw);
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / (nOff + 1), r = wg % (nOff + 1);
  if (info[k] != 0) return;  // uniform for the workgroup
  double* base = mats + (int64_t)k * lay.mstride;
  const Lay L = lay_of(lay, k);
  if (r == 0) dev_gemm_diag_border<VEC>(L, base, J, border != 0, lds);
  else if (VEC && lay.kind == 0 && J + r < lay.Nv) dev_gemm_col_dma(L, base, J, J + r, lds);
  else dev_gemm_col<VEC>(L, base, J, J + r, lds);  // the bordered row taller than 32
}

hipError_t launch_col_update(const Lay& lay, double* mats, const int32_t* info, int J, int K,
                             hipStream_t s) {
  if (lay.kind != 0 || J <= 0 || J >= lay.Nv) return hipErrorInvalidValue;
  const bool has_border = lay.kind == 0 && lay.q > 0;
  const bool border = has_border && lay.TB <= 32;
  // off-diagonal tile rows J+1 .. Nv-1, and the bordered row unless the
  // diagonal workgroup takes it
  const int nOff = (lay.Nv - 1 - J) + ((has_border && !border) ? 1 : 0);
  const int G = K * (nOff + 1);
  if (vec_ok(lay, mats))
    hipLaunchKernelGGL(k_col_update<true>, dim3(G), dim3(256), 0, s, lay, mats, info, J,
                       border ? 1 : 0, nOff, G);
  else
    hipLaunchKernelGGL(k_col_update<false>, dim3(G), dim3(256), 0, s, lay, mats, info, J,
                       border ? 1 : 0, nOff, G);
  return hipGetLastError();
}

// ---- the bordered row's own block after the last block column ------------------
// C_B -= Q Q^T: Q is the bordered rows' panel (q rows; the packed tiles
// (Nv, 0..Nv-1) form one TB x Nv T column-major block, leading dimension TB)
// over its n valid columns, C_B the final TB x TB tile (Step 4's cross
// products).  A 16- or 32-row product with k = n gives one wave of a GEMM
// workgroup almost all the MFMA work and a long, latency-bound chunk loop.
// Here the four waves of a workgroup take interleaved groups of 4 U columns,
// load their fragments straight from global memory (16 lanes read 16
// consecutive rows of one column), use each fragment as both MFMA operands,
// and sum their partial blocks through LDS in wave order.
template <int NB>
__global__ __launch_bounds__(256) void k_border_block(Lay lay, double* __restrict__ mats,
                                                      const int32_t* __restrict__ info) {
  constexpr int TBC = 16 * NB, U = NB == 1 ? 8 : 4;
  __shared__ double part[4][TBC * TBC];
  const int k = blockIdx.x;
  if (info[k] != 0) return;  // uniform for the workgroup
  double* base = mats + (int64_t)k * lay.mstride;
  const double* Q = base + lay.tile_off(lay.Nv, 0);
  double* C = base + lay.tile_off(lay.Nv, lay.Nv);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int n = lay.units ? lay.units[k].n : lay.n, q = lay.q;
  const int64_t ld = lay.TB;
  d4 acc[NB][NB];
#pragma unroll
  for (int ib = 0; ib < NB; ++ib)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
  const int ngroups = (n + 4 * U - 1) / (4 * U);
  for (int g = wave; g < ngroups; g += 4) {
    double v[U][NB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = g * 4 * U + 4 * u + lk;
      const int cc = col < n ? col : n - 1;
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        const int row = 16 * ib + lr;
        const int rc = row < q ? row : q - 1;  // clamped: always a valid element
        v[u][ib] = Q[(int64_t)cc * ld + rc];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = g * 4 * U + 4 * u + lk;
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
        if (col >= n || 16 * ib + lr >= q) v[u][ib] = 0.0;
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) acc[ib][jb] = MF<double>::op(v[u][jb], v[u][ib], acc[ib][jb]);
    }
  }
#pragma unroll
  for (int ib = 0; ib < NB; ++ib)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        part[wave][(16 * jb + MF<double>::col(lk, e)) * TBC + 16 * ib + lr] = acc[ib][jb][e];
  __syncthreads();
  for (int idx = tid; idx < TBC * TBC; idx += 256) {
    const int r = idx % TBC, c = idx / TBC;
    if (r < q && c < q)
      C[(int64_t)c * ld + r] -= ((part[0][idx] + part[1][idx]) + part[2][idx]) + part[3][idx];
  }
}

hipError_t launch_border_block(const Lay& lay, double* mats, const int32_t* info, int K,
                               hipStream_t s) {
  if (lay.kind != 0 || lay.q <= 0 || lay.q > 32 || lay.n <= 0) return hipErrorInvalidValue;
  if (lay.TB == 16)
    hipLaunchKernelGGL(k_border_block<1>, dim3(K), dim3(256), 0, s, lay, mats, info);
  else
    hipLaunchKernelGGL(k_border_block<2>, dim3(K), dim3(256), 0, s, lay, mats, info);
  return hipGetLastError();
}

// ---- panel solve L_IJ = C_IJ W_J^T for nI tile rows from I0 down -----------
// TS double: W from Wbuf[k]; TS float: W from slot J of the omega's table.
template <typename TS, bool VEC>
__global__ __launch_bounds__(256, 2) void k_trsm(Lay lay, TS* __restrict__ mats,
                                                 const TS* __restrict__ Wbuf,
                                                 const int32_t* __restrict__ info, int J, int I0,
                                                 int nI, int G, int64_t wstride) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = I0 + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  dev_trsm<TS, VEC, MX_FLUSH, 2>(lay_of(lay, k), mats + (int64_t)k * lay.mstride,
                                 Wbuf + (int64_t)k * wstride, J, I, reinterpret_cast<TS*>(lds_raw));
}

// FP64 panel solve of the packed layout (tile rows J + 1 .. J + nI): whole
// tiles on the direct-to-LDS core, chunks of 8 columns in three stages
// (49.5 KB of LDS) and no staging registers, so three workgroups share a CU
// (each tile is only 128 columns deep; the extra workgroups hide the load
// latency); the bordered row's tile (tile row Nv) on dev_trsm_border.
__global__ __launch_bounds__(256, 3) void k_trsm_dma(Lay lay, double* __restrict__ mats,
                                                     const double* __restrict__ Wbuf,
                                                     const int32_t* __restrict__ info, int J,
                                                     int nI, int G) {
  __shared__ __attribute__((aligned(16))) char lds_raw[dma_lds_bytes<TRSM_KC, TRSM_NST>()];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + 1 + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  const Lay L = lay_of(lay, k);
  double* base = mats + (int64_t)k * lay.mstride;
  const double* W = Wbuf + (int64_t)k * T * T;
  if (I < lay.Nv) {
    dev_trsm_dma<TRSM_KC, TRSM_NST>(L, base, W, J, I, reinterpret_cast<double*>(lds_raw));
    return;
  }
  if (lay.q <= 0) return;  // no bordered row: nothing below the last tile row
  switch (lay.TB) {
    case 16: dev_trsm_border<1>(L, base, W, J); break;
    case 32: dev_trsm_border<2>(L, base, W, J); break;
    case 48: dev_trsm_border<3>(L, base, W, J); break;
    default: dev_trsm_border<4>(L, base, W, J); break;
  }
}

// Mixed-form panel solve of the packed layout (tile rows J + 1 .. J + nI):
// whole tiles in FP64 MFMA on FP32 panels loaded straight into LDS (chunks of
// 16 columns in three stages, 51 KB, three workgroups per CU), the bordered
// row's tile on dev_trsm_border<., float>.  W from slot J of the omega's
// table (wstride floats per omega).
__global__ __launch_bounds__(256, 3) void k_trsm_mx_dma(Lay lay, float* __restrict__ m32,
                                                        const float* __restrict__ Wbuf,
                                                        const int32_t* __restrict__ info, int J,
                                                        int nI, int G, int64_t wstride) {
  __shared__ __attribute__((aligned(16))) char lds_raw[f32dma_lds_bytes<TRSM_MX_KC, TRSM_MX_NST>()];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + 1 + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  const Lay L = lay_of(lay, k);
  float* base = m32 + (int64_t)k * lay.mstride;
  const float* W = Wbuf + (int64_t)k * wstride;
  if (I < lay.Nv) {
    dev_trsm_mx_dma(L, base, W, J, I, reinterpret_cast<float*>(lds_raw));
    return;
  }
  if (lay.q <= 0) return;  // no bordered row: nothing below the last tile row
  switch (lay.TB) {
    case 16: dev_trsm_border<1, float>(L, base, W, J); break;
    case 32: dev_trsm_border<2, float>(L, base, W, J); break;
    case 48: dev_trsm_border<3, float>(L, base, W, J); break;
    default: dev_trsm_border<4, float>(L, base, W, J); break;
  }
}

hipError_t launch_trsm(const Lay& lay, double* mats, const double* W, const int32_t* info, int J,
                       int nI, int K, hipStream_t s) {
  const int64_t ws = (int64_t)T * T;
  const bool vec = vec_ok(lay, mats) && (reinterpret_cast<uintptr_t>(W) & 15) == 0;
  const int I0 = J + 1;
  if (vec && lay.kind == 0 && (lay.q == 0 || lay.TB <= 64)) {
    if (nI > 0) {
      const int G = K * nI;
      hipLaunchKernelGGL(k_trsm_dma, dim3(G), dim3(256), 0, s, lay, mats, W, info, J, nI, G);
    }
  } else if (nI > 0) {
    const int G = K * nI;
    if (vec)
      hipLaunchKernelGGL((k_trsm<double, true>), dim3(G), dim3(256), 0, s, lay, mats, W, info, J,
                         I0, nI, G, ws);
    else
      hipLaunchKernelGGL((k_trsm<double, false>), dim3(G), dim3(256), 0, s, lay, mats, W, info, J,
                         I0, nI, G, ws);
  }
  return hipGetLastError();
}

hipError_t launch_trsm_mx(const Lay& lay, float* m32, const float* W32, const int32_t* info, int J,
                          int nI, int K, hipStream_t s) {
  if (nI <= 0) return hipSuccess;
  const int G = K * nI;
  const int64_t ws = (int64_t)lay.Nv * T * T;
  if (lay.kind == 0 && (lay.q == 0 || lay.TB <= 64))
    hipLaunchKernelGGL(k_trsm_mx_dma, dim3(G), dim3(256), 0, s, lay, m32,
                       W32 + (int64_t)J * T * T, info, J, nI, G, ws);
  else
    hipLaunchKernelGGL((k_trsm<float, true>), dim3(G), dim3(256), 0, s, lay, m32,
                       W32 + (int64_t)J * T * T, info, J, J + 1, nI, G, ws);
  return hipGetLastError();
}

hipError_t launch_trsm_mx_plain(const Lay& lay, float* m32, const float* W32,
                                const int32_t* info, int J, int K, hipStream_t s) {
  if (!(lay.kind == 1 && lay.ld % 4 == 0 && (reinterpret_cast<uintptr_t>(m32) & 15) == 0))
    return hipErrorInvalidValue;
  const int nI = lay.Nv - J - 1;
  if (nI <= 0) return hipSuccess;
  const int G = K * nI;
  hipLaunchKernelGGL((k_trsm<float, true>), dim3(G), dim3(256), 0, s, lay, m32, W32, info, J,
                     J + 1, nI, G, (int64_t)T * T);
  return hipGetLastError();
}

// ---- mixed form: FP64 cross products from x0 -------------------------------------
// For SPD V the functional f(x) = 2 B^T x - x^T V x is maximised at x = V^-1 B
// with value B^T V^-1 B, and f(x*) - f(x0) = (x*-x0)^T V (x*-x0): evaluating f
// at the FP32-solve x0 in FP64 against the FP64 V gives the cross products with
// an error second order in the solve error -- one FP64 refinement step applied
// to the quadratic forms.  With refine = 0 the first-order B^T x0 is used.
// Workgroup (omega, lower tile (I,J)) writes its q x q share to its own slot:
//   Y = V_IJ x0_J on MFMA f64 (the GEMM core, x0 as a TB x T column-major panel),
//   M = x0_I^T Y;  slot = -(M + M^T) for I > J,  2 B_I^T x0_I - M for I = J.
// The slots are summed in a fixed order by k_finalize (deterministic).
// acc[i][0:NB] += A[0:128, 0:kmax] B[0:16 NB, 0:kmax]^T: the GEMM core for a
// B of at most 16 NB rows (x0_J), with an LDS stage sized for those rows
// instead of 128, so that more workgroups fit a compute unit.  The quadratic
// forms stream V once with little arithmetic per byte, so resident
// workgroups (loads in flight) bound them, not the MFMAs.  Same two-set
// register pipeline and guarded loads as wg_gemm_nt; only the waves of the
// first wave column (B rows 0 .. 16 NB - 1) multiply.
template <int NB>
__device__ __forceinline__ void wg_gemm_rhs(d4 (&acc)[4][4], double* lds,
                                            const double* __restrict__ A, int64_t lda, int arows,
                                            const double* __restrict__ B, int64_t ldb, int brows,
                                            int kmax, bool do_mfma, int ni) {
  constexpr int N = 2, KC = 16, PPC = T / N;
  constexpr int BR = 16 * NB, LB = BR + 4, BPPC = BR / N, BPIECES = KC * BPPC;
  constexpr int BQ = (BPIECES + 255) / 256;  // B pieces per thread
  constexpr int STAGE = KC * (LROW + LB);
  typedef dbl2 V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  ni = __builtin_amdgcn_readfirstlane(ni);
  do_mfma = __builtin_amdgcn_readfirstlane((int)do_mfma) != 0;
  V ra[2][4], rb[2][BQ];
  auto fetch = [&](int k0, auto setc) {
    constexpr int S = decltype(setc)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      ra[S][q] = fetch_piece<double, true>(A, lda, arows, k0 + col, kmax, row);
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int idx = tid + 256 * q;
      if (idx < BPIECES) {
        const int col = idx / BPPC, row = (idx % BPPC) * N;
        rb[S][q] = fetch_piece<double, true>(B, ldb, brows, k0 + col, kmax, row);
      }
    }
  };
  auto stash = [&](auto setc) {
    constexpr int S = decltype(setc)::value;
    double* sa = lds + S * STAGE;
    double* sb = sa + KC * LROW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      *reinterpret_cast<V*>(sa + col * LROW + row) = ra[S][q];
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int idx = tid + 256 * q;
      if (idx < BPIECES) {
        const int col = idx / BPPC, row = (idx % BPPC) * N;
        *reinterpret_cast<V*>(sb + col * LB + row) = rb[S][q];
      }
    }
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  fetch(0, S0{});
  if (nchunks > 1) fetch(KC, S1{});
  stash(S0{});
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  auto step = [&](int c, auto setc, auto other) {
    constexpr int S = decltype(setc)::value;
    if (c + 2 < nchunks) fetch((c + 2) * KC, setc);
    if (do_mfma) {
      const double* sa = lds + S * STAGE + 64 * wr + lr;
      const double* sb = lds + S * STAGE + KC * LROW + lr;
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        double a[4], b[NB];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = sa[kk * LROW + 16 * i];
#pragma unroll
        for (int j = 0; j < NB; ++j) b[j] = sb[kk * LB + 16 * j];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i < ni) {
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[i][j] = MF<double>::op(b[j], a[i], acc[i][j]);
          }
        }
      }
    }
    if (c + 1 < nchunks) stash(other);
    __syncthreads();
  };
  for (int c = 0; c < nchunks; c += 2) {
    step(c, S0{}, S1{});
    if (c + 1 < nchunks) step(c + 1, S1{}, S0{});
  }
}

// LDS of k_qform: the core's two stages, then Y ((T + 1) TB) and x0_I (T TB)
template <int TB>
constexpr int qform_lds_doubles() {
  return std::max(2 * 16 * (LROW + TB + 4), (2 * T + 1) * TB);
}

template <int TB>
__global__ __launch_bounds__(256, TB == 16 ? 3 : (TB == 32 ? 2 : 1)) void k_qform(Lay lay, const double* __restrict__ m64,
                                                  int64_t stride64, const double* __restrict__ X,
                                                  const double* __restrict__ rhs,
                                                  const int32_t* __restrict__ info,
                                                  double* __restrict__ slots, int refine,
                                                  int ntile, int G) {
  __shared__ __attribute__((aligned(16))) double lds[qform_lds_doubles<TB>()];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / ntile;
  const int t = wg % ntile;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int J = t - I * (I + 1) / 2;
  if (info[k] != 0) return;  // uniform for the workgroup
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int q = lay.q;
  const Lay L = lay_of(lay, k);
  const int ri = L.rows(I), rj = L.rows(J);
  const double* Xk = X + (int64_t)k * x0_stride(lay);
  double* slot = slots + ((int64_t)k * ntile + t) * TB * TB;
  const double* Xi = Xk + (int64_t)I * T * TB;   // x0_I: element (r, a) at r*TB + a
  // B_I, same layout (an uneven batch: the unit's dataset's right-hand sides)
  const double* Bi = rhs + (lay.units ? lay.units[k].rhs : 0) + (int64_t)I * T * TB;
  // LDS after the core: Y = V_IJ x0_J column-major with the odd stride T + 1
  // (the pair loop below reads 16 columns of Y at once), then x0_I (the
  // block is sized for whichever of the two uses is larger).
  constexpr int LY = T + 1;
  double* Ys = lds;
  double* Xs = lds + LY * TB;
  if (refine) {
    const int war = ri - 64 * wr, wbr = q - 64 * wc;
    const int ni = nblk(war), nj = nblk(wbr);
    const bool act = ni > 0 && nj > 0;
    d4 acc[4][4];
    zero_acc<double>(acc);
    // B = x0_J has q <= TB rows: TB / 16 block columns
    wg_gemm_rhs<TB / 16>(acc, lds, m64 + (int64_t)k * stride64 + lay.tile_off(I, J), T, ri,
                         Xk + (int64_t)J * T * TB, TB, q, rj, act, ni);
    // the core ends with a barrier: the LDS stages are free for Y
    if (act) store64<double, false>(Ys + 64 * wr + 64 * wc * LY, LY, Ys + 64 * wr + 64 * wc * LY, LY,
                                    acc, war, wbr, lane);
  }
  // stage x0_I, and on a diagonal tile fold B_I into Y: since V_II is
  // symmetric, 2 B_I^T x0_I - x0_I^T V_II x0_I = (2 B_I - V_II x0_I)^T x0_I
  // (without refinement the slot is B_I^T x0_I, so Y is replaced by B_I).
  // Loads use a clamped address and a select, so they are all in flight at once.
  constexpr int PER = T * TB / 256;
  double xv[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int idx = 256 * u + tid;
    const bool ok = idx / TB < ri;
    xv[u] = Xi[ok ? idx : 0];
    xv[u] = ok ? xv[u] : 0.0;
  }
  if (refine) __syncthreads();  // Y is complete
#pragma unroll
  for (int u = 0; u < PER; ++u) Xs[256 * u + tid] = xv[u];
  if (I == J) {
    double bv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = 256 * u + tid;
      const bool ok = idx / TB < ri;
      bv[u] = Bi[ok ? idx : 0];
      bv[u] = ok ? bv[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = 256 * u + tid, r = idx / TB, a = idx % TB;
      Ys[a * LY + r] = refine ? 2.0 * bv[u] - Ys[a * LY + r] : bv[u];
    }
  }
  __syncthreads();
  for (int pr = tid; pr < TB * TB; pr += 256) {
    const int a = pr / TB, b = pr % TB;
    double v = 0.0;
    if (I == J) {
#pragma unroll 8
      for (int r = 0; r < ri; ++r) v += Ys[a * LY + r] * Xs[r * TB + b];
    } else if (refine) {
      double mab = 0.0, mba = 0.0;
#pragma unroll 8
      for (int r = 0; r < ri; ++r) {
        mab += Xs[r * TB + a] * Ys[b * LY + r];
        mba += Xs[r * TB + b] * Ys[a * LY + r];
      }
      v = -(mab + mba);
    }
    slot[pr] = v;
  }
}

hipError_t launch_qform(const Lay& lay, const double* m64, int64_t stride64, const double* X,
                        const double* rhs, const int32_t* info, double* slots, int refine, int K,
                        hipStream_t s) {
  const int ntile = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntile;
  if (lay.TB == 16)
    hipLaunchKernelGGL(k_qform<16>, dim3(G), dim3(256), 0, s, lay, m64, stride64, X, rhs, info,
                       slots, refine, ntile, G);
  else if (lay.TB == 32)
    hipLaunchKernelGGL(k_qform<32>, dim3(G), dim3(256), 0, s, lay, m64, stride64, X, rhs, info,
                       slots, refine, ntile, G);
  else if (lay.TB == 48)
    hipLaunchKernelGGL(k_qform<48>, dim3(G), dim3(256), 0, s, lay, m64, stride64, X, rhs, info,
                       slots, refine, ntile, G);
  else if (lay.TB == 64)
    hipLaunchKernelGGL(k_qform<64>, dim3(G), dim3(256), 0, s, lay, m64, stride64, X, rhs, info,
                       slots, refine, ntile, G);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace plk
