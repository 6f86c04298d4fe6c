// Blocked Cholesky V = L L^T and its log-determinant (Step 2 of Section 3.3),
// left-looking over block columns of width T, batched over omega.
//
// Step J of the factorisation:
//   k_gemm_col : C_IJ -= L_I,0:J L_J,0:J^T for every tile row I >= J (MFMA f64)
//   k_potrf    : C_JJ = L_JJ L_JJ^T, log|V| += 2 sum log L_jj,
//                W_J = L_JJ^{-1} (triangular inverse), register-blocked
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
typedef double dbl2 __attribute__((ext_vector_type(2)));

// ---- workgroup GEMM core: acc += A[0:128, 0:kmax] B[0:128, 0:kmax]^T ----------
// 256 threads = 4 waves in a 2x2 grid, each owning a 64x64 quarter of the
// 128x128 result as 4x4 MFMA blocks.  The k range is consumed in chunks of
// KC columns, double-buffered through LDS: every thread fetches 4 + 4
// 16-byte pieces of the next chunk from global memory while the waves run
// the current chunk's 4 x 16 MFMAs, then writes them to the other LDS stage;
// one barrier per chunk.  Rows at or beyond arows / brows and columns at or
// beyond kmax are fetched as zero.
constexpr int KC = 16;
constexpr int LROW = T + 4;                        // LDS stride per k column
constexpr int GEMM_LDS = 2 * 2 * KC * LROW;        // doubles: 2 stages x {A, B}

template <bool VEC>
__device__ __forceinline__ dbl2 fetch2(const double* __restrict__ P, int64_t ld, int rows, int k,
                                       int kmax, int row) {
  dbl2 v = {0.0, 0.0};
  if (k < kmax) {
    const double* p = P + (int64_t)k * ld + row;
    if (VEC && row + 1 < rows) {
      v = *reinterpret_cast<const dbl2*>(p);
    } else {
      if (row < rows) v.x = p[0];
      if (row + 1 < rows) v.y = p[1];
    }
  }
  return v;
}

template <bool VEC>
__device__ __forceinline__ void wg_gemm_nt(d4 (&acc)[4][4], double* lds, const double* __restrict__ A,
                                           int64_t lda, int arows, const double* __restrict__ B,
                                           int64_t ldb, int brows, int kmax, bool do_mfma, int ni,
                                           int nj) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  dbl2 ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx >> 6, row = (idx & 63) * 2;
      ra[q] = fetch2<VEC>(A, lda, arows, k0 + col, kmax, row);
      rb[q] = fetch2<VEC>(B, ldb, brows, k0 + col, kmax, row);
    }
  };
  auto stash = [&](int stage) {
    double* sa = lds + (stage * 2 + 0) * KC * LROW;
    double* sb = lds + (stage * 2 + 1) * KC * LROW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx >> 6, row = (idx & 63) * 2;
      *reinterpret_cast<dbl2*>(sa + col * LROW + row) = ra[q];
      *reinterpret_cast<dbl2*>(sb + col * LROW + row) = rb[q];
    }
  };
  fetch(0);
  stash(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) fetch((c + 1) * KC);
    if (do_mfma) {
      const double* sa = lds + ((c & 1) * 2 + 0) * KC * LROW + 64 * wr + lr;
      const double* sb = lds + ((c & 1) * 2 + 1) * KC * LROW + 64 * wc + lr;
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = sa[kk * LROW + 16 * i];
          b[i] = sb[kk * LROW + 16 * i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i < ni) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (j < nj) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (more) stash((c + 1) & 1);
    __syncthreads();
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

__device__ __forceinline__ int nblk(int rows) { return rows <= 0 ? 0 : min(4, (rows + 15) >> 4); }

// ---- left-looking update of block column J -----------------------------------
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_col(Lay lay, double* __restrict__ mats,
                                                  const int32_t* __restrict__ info, int J, int nI,
                                                  int G) {
  __shared__ double lds[GEMM_LDS];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  const int war = arows - 64 * wr, wbr = brows - 64 * wc;
  const int ni = nblk(war), nj = nblk(wbr);
  const bool act = ni > 0 && nj > 0 && !(I == J && wc > wr);
  double* base = mats + (int64_t)k * lay.mstride;
  const int kmax = min(J * T, lay.n);
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  wg_gemm_nt<VEC>(acc, lds, base + lay.tile_off(I, 0), lay.tile_ld(I), arows,
                  base + lay.tile_off(J, 0), lay.tile_ld(J), brows, kmax, act, ni, nj);
  if (act) {
    const int64_t ldc = lay.tile_ld(I);
    store64<true>(base + lay.tile_off(I, J) + 64 * wr + 64 * wc * ldc, ldc, acc, war, wbr, lane);
  }
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

// ---- diagonal tile: factor and invert, register-blocked -----------------------
// Thread t owns the 8x8 block (rows 8*(t/16).., columns 8*(t%16)..) of the
// unit-padded tile; LDS only broadcasts one column (and one row) per step, with
// two alternating buffers so that a single barrier separates the steps.
//  factor (right-looking): publish column j unscaled; every owner of a lower
//    block updates a_rc -= a_rj a_cj / a_jj for c > j; owners of column j
//    scale it by 1/sqrt(a_jj).
//  inverse (in place, W = L^-1 row by row): at step m scale W's row m by
//    1/L_mm (it then holds its final values), publish it and L's column m;
//    W_rc -= L_rm W_mc for r > m, c < m; W_rm = -L_rm / L_mm; W_mm = 1/L_mm.
__global__ __launch_bounds__(256) void k_potrf(Lay lay, double* __restrict__ mats,
                                               double* __restrict__ Wbuf,
                                               double* __restrict__ logdet,
                                               int32_t* __restrict__ info, int J) {
  __shared__ double bc0[2][T];
  __shared__ double bc1[2][T];
  __shared__ double dinv[T];
  __shared__ double red[256];
  const int k = blockIdx.x;
  if (info[k] != 0) return;
  const int tid = threadIdx.x, bi = tid >> 4, bj = tid & 15;
  const bool low = bi >= bj;
  const int nv = lay.rows(J);
  double* C = mats + (int64_t)k * lay.mstride + lay.tile_off(J, J);
  const int64_t ld = lay.tile_ld(J);
  double a[8][8];
#pragma unroll
  for (int rr = 0; rr < 8; ++rr)
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int r = 8 * bi + rr, c = 8 * bj + cc;
      double v;
      if (r < nv && c < nv) v = (r >= c) ? C[(int64_t)c * ld + r] : 0.0;
      else v = (r == c) ? 1.0 : 0.0;
      a[rr][cc] = v;
    }

  for (int jb = 0; jb < T / 8; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int j = 8 * jb + jj;
      const int buf = jj & 1;
      if (bj == jb) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) bc0[buf][8 * bi + rr] = a[rr][jj];
      }
      __syncthreads();
      const double d = bc0[buf][j];
      if (!(d > 0.0)) {  // the same value in every thread: uniform exit
        if (tid == 0) info[k] = J * T + j + 1;
        return;
      }
      if (low && bj >= jb) {
        const double invd = 1.0 / d;
        double cr[8], cc8[8];
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) cr[rr] = bc0[buf][8 * bi + rr] * invd;
        // columns c <= j of the owner block get a zero multiplier instead of a
        // per-element branch, so the 64 FMAs run unconditionally
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8)
          cc8[c8] = (bj > jb || c8 > jj) ? bc0[buf][8 * bj + c8] : 0.0;
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
#pragma unroll
          for (int c8 = 0; c8 < 8; ++c8) a[rr][c8] = fma(-cr[rr], cc8[c8], a[rr][c8]);
        if (bj == jb) {
          const double sc = 1.0 / sqrt(d);
#pragma unroll
          for (int rr = 0; rr < 8; ++rr)
            if (bi > jb || rr >= jj) a[rr][jj] *= sc;
        }
      }
    }
  }

  // log|V| contribution, 1/L_jj, and the factor itself
  double sl = 0.0;
  if (bi == bj) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      const int r = 8 * bi + rr;
      if (r < nv) sl += log(a[rr][rr]);
      dinv[r] = 1.0 / a[rr][rr];
    }
  }
  red[tid] = sl;
  if (low) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        if (r < nv && c < nv && r >= c) C[(int64_t)c * ld + r] = a[rr][cc];
      }
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) logdet[k] += 2.0 * red[0];

  for (int mb = 0; mb < T / 8; ++mb) {
#pragma unroll
    for (int mm = 0; mm < 8; ++mm) {
      const int m = 8 * mb + mm;
      const int buf = mm & 1;
      if (low && bj == mb) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) bc0[buf][8 * bi + rr] = a[rr][mm];
      }
      if (low && bi == mb) {
        // row m of W is complete up to the factor 1/L_mm
        const double dm = dinv[m];
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) {
          if (bj < mb || c8 < mm) a[mm][c8] *= dm;
          bc1[buf][8 * bj + c8] = a[mm][c8];
        }
      }
      __syncthreads();
      const double wmm = dinv[m];
      if (low && bi >= mb && bj <= mb) {
        double lr[8], wv[8];
        // rows r <= m and columns c >= m get zero multipliers (no branches)
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) lr[rr] = (bi > mb || rr > mm) ? bc0[buf][8 * bi + rr] : 0.0;
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) wv[c8] = (bj < mb || c8 < mm) ? bc1[buf][8 * bj + c8] : 0.0;
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
#pragma unroll
          for (int c8 = 0; c8 < 8; ++c8) a[rr][c8] = fma(-lr[rr], wv[c8], a[rr][c8]);
        if (bj == mb) {
          // column m becomes W_rm = -L_rm / L_mm (r > m), W_mm = 1 / L_mm
#pragma unroll
          for (int rr = 0; rr < 8; ++rr) {
            if (bi > mb || rr > mm) a[rr][mm] = -lr[rr] * wmm;
          }
          if (bi == mb) a[mm][mm] = wmm;
        }
      }
    }
  }
  double* W = Wbuf + (int64_t)k * T * T;
#pragma unroll
  for (int rr = 0; rr < 8; ++rr)
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int r = 8 * bi + rr, c = 8 * bj + cc;
      W[c * T + r] = (low && r >= c) ? a[rr][cc] : 0.0;
    }
}

hipError_t launch_potrf(const Lay& lay, double* mats, double* W, double* logdet, int32_t* info,
                        int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf, dim3(K), dim3(256), 0, s, lay, mats, W, logdet, info, J);
  return hipGetLastError();
}

// ---- panel solve L_IJ = C_IJ W_J^T for the nI tile rows below J -----------
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_trsm(Lay lay, double* __restrict__ mats,
                                              const double* __restrict__ Wbuf,
                                              const int32_t* __restrict__ info, int J, int nI,
                                              int G) {
  __shared__ double lds[GEMM_LDS];
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + 1 + wg % nI;
  if (info[k] != 0) return;  // uniform for the workgroup
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  const int war = arows - 64 * wr, wbr = brows - 64 * wc;
  const int ni = nblk(war), nj = nblk(wbr);
  const bool act = ni > 0 && nj > 0;
  double* Ct = mats + (int64_t)k * lay.mstride + lay.tile_off(I, J);
  const int64_t ldc = lay.tile_ld(I);
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // the core's final barrier orders every read of C_IJ before the overwrite
  wg_gemm_nt<VEC>(acc, lds, Ct, ldc, arows, Wbuf + (int64_t)k * T * T, T, brows, brows, act, ni, nj);
  if (act) store64<false>(Ct + 64 * wr + 64 * wc * ldc, ldc, acc, war, wbr, lane);
}

hipError_t launch_trsm(const Lay& lay, double* mats, const double* W, const int32_t* info, int J,
                       int nI, int K, hipStream_t s) {
  const int G = K * nI;
  if (vec_ok(lay, mats) && (reinterpret_cast<uintptr_t>(W) & 15) == 0)
    hipLaunchKernelGGL(k_trsm<true>, dim3(G), dim3(256), 0, s, lay, mats, W, info, J, nI, G);
  else
    hipLaunchKernelGGL(k_trsm<false>, dim3(G), dim3(256), 0, s, lay, mats, W, info, J, nI, G);
  return hipGetLastError();
}

}  // namespace plk
