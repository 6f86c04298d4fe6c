// Blocked Cholesky V = L L^T and its log-determinant (Step 2 of Section 3.3),
// left-looking over block columns of width T, batched over omega.
//
// Step J of the factorisation:
//   k_gemm_col : C_IJ -= L_I,0:J L_J,0:J^T for every tile row I >= J (MFMA)
//   k_potrf    : C_JJ = L_JJ L_JJ^T, log|V| += 2 sum log L_jj,
//                W_J = L_JJ^{-1} (triangular inverse), register-blocked, FP64
//   k_trsm     : L_IJ = C_IJ W_J^T for I > J (MFMA)
// With the packed bordered layout the right-hand sides are extra tile rows
// under V, so the same steps produce Z = L^{-1}[Y'|X] (Step 3) and, in the
// final tile, minus the cross products (y,X)^T V^{-1} (y,X) (Step 4).
//
// Two forms share these kernels:
//   FP64  : every tile in FP64, FP64 MFMA.
//   mixed : the factor is stored in FP32 and off-diagonal updates and panel
//           solves use FP32 MFMA; each diagonal tile is updated with FP64
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

#include "common.h"

namespace plk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// ---- MFMA flavours -------------------------------------------------------------
template <typename TC> struct MF;
template <> struct MF<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result column (within a 16x16 block) of accumulator item e in lane group lg
  static __device__ __forceinline__ int col(int lg, int e) { return lg + 4 * e; }
};
template <> struct MF<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int lg, int e) { return 4 * lg + e; }
};

// ---- 16-byte pieces of a column of a panel ---------------------------------------
template <typename TS> struct Piece;
template <> struct Piece<double> {
  typedef dbl2 type;
  static constexpr int N = 2;
};
template <> struct Piece<float> {
  typedef flt4 type;
  static constexpr int N = 4;
};

template <typename TS, bool VEC>
__device__ __forceinline__ typename Piece<TS>::type fetch_piece(const TS* __restrict__ P, int64_t ld,
                                                                int rows, int k, int kmax, int row) {
  typedef typename Piece<TS>::type V;
  constexpr int N = Piece<TS>::N;
  V v;
#pragma unroll
  for (int e = 0; e < N; ++e) v[e] = (TS)0;
  if (k < kmax) {
    const TS* p = P + (int64_t)k * ld + row;
    if (VEC && row + N - 1 < rows) {
      v = *reinterpret_cast<const V*>(p);
    } else {
#pragma unroll
      for (int e = 0; e < N; ++e)
        if (row + e < rows) v[e] = p[e];
    }
  }
  return v;
}

// ---- workgroup GEMM core: acc += A[0:128, 0:kmax] B[0:128, 0:kmax]^T ----------
// 256 threads = 4 waves in a 2x2 grid, each owning a 64x64 quarter of the
// 128x128 result as 4x4 MFMA blocks.  The k range is consumed in chunks of
// KC = 128 / sizeof(TS) columns (16 KB per operand), double-buffered through
// LDS: every thread fetches 4 + 4 16-byte pieces of the next chunk from
// global memory while the waves run the current chunk's MFMAs, then writes
// them to the other LDS stage; one barrier per chunk.  Rows at or beyond
// arows / brows and columns at or beyond kmax read as zero.  TS is the storage
// type, TC the MFMA type (float storage may be widened to FP64 MFMA).
constexpr int LROW = T + 4;         // LDS stride per k column (elements)
constexpr int GEMM_LDS_BYTES = 2 * 2 * 16 * LROW * 8;

template <typename TS, typename TC, bool VEC>
__device__ __forceinline__ void wg_gemm_nt(typename MF<TC>::acc (&acc)[4][4], TS* lds,
                                           const TS* __restrict__ A, int64_t lda, int arows,
                                           const TS* __restrict__ B, int64_t ldb, int brows,
                                           int kmax, bool do_mfma, int ni, int nj) {
  constexpr int N = Piece<TS>::N;
  constexpr int KC = 128 / (int)sizeof(TS);
  constexpr int PPC = T / N;  // pieces per column
  typedef typename Piece<TS>::type V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  V ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      ra[q] = fetch_piece<TS, VEC>(A, lda, arows, k0 + col, kmax, row);
      rb[q] = fetch_piece<TS, VEC>(B, ldb, brows, k0 + col, kmax, row);
    }
  };
  auto stash = [&](int stage) {
    TS* sa = lds + (stage * 2 + 0) * KC * LROW;
    TS* sb = lds + (stage * 2 + 1) * KC * LROW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      *reinterpret_cast<V*>(sa + col * LROW + row) = ra[q];
      *reinterpret_cast<V*>(sb + col * LROW + row) = rb[q];
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
      const TS* sa = lds + ((c & 1) * 2 + 0) * KC * LROW + 64 * wr + lr;
      const TS* sb = lds + ((c & 1) * 2 + 1) * KC * LROW + 64 * wc + lr;
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        TC a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = (TC)sa[kk * LROW + 16 * i];
          b[i] = (TC)sb[kk * LROW + 16 * i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i < ni) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (j < nj) acc[i][j] = MF<TC>::op(b[j], a[i], acc[i][j]);
          }
        }
      }
    }
    if (more) stash((c + 1) & 1);
    __syncthreads();
  }
}

// FP32 MFMA whose partial sums are flushed into FP64 accumulators every
// FLUSH k-steps (FLUSH * 4 products): the FP32 rounding then only touches short
// partial sums instead of the long running sums that cancel in the Schur
// complements of an ill-conditioned V.  Same LDS pipeline as wg_gemm_nt.
template <int FLUSH>
__device__ __forceinline__ void wg_gemm_nt_f32x64(d4 (&acc)[4][4], float* lds,
                                                  const float* __restrict__ A, int64_t lda,
                                                  int arows, const float* __restrict__ B,
                                                  int64_t ldb, int brows, int kmax, bool do_mfma,
                                                  int ni, int nj) {
  constexpr int N = 4;
  constexpr int KC = 32;
  constexpr int PPC = T / N;
  typedef flt4 V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  V ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      ra[q] = fetch_piece<float, true>(A, lda, arows, k0 + col, kmax, row);
      rb[q] = fetch_piece<float, true>(B, ldb, brows, k0 + col, kmax, row);
    }
  };
  auto stash = [&](int stage) {
    float* sa = lds + (stage * 2 + 0) * KC * LROW;
    float* sb = lds + (stage * 2 + 1) * KC * LROW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      *reinterpret_cast<V*>(sa + col * LROW + row) = ra[q];
      *reinterpret_cast<V*>(sb + col * LROW + row) = rb[q];
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
      const float* sa = lds + ((c & 1) * 2 + 0) * KC * LROW + 64 * wr + lr;
      const float* sb = lds + ((c & 1) * 2 + 1) * KC * LROW + 64 * wc + lr;
      // rolled: only one group's fragments and partial sums are live at a time
#pragma unroll 1
      for (int g = 0; g < KC / 4 / FLUSH; ++g) {
        float a[FLUSH][4], b[FLUSH][4];
#pragma unroll
        for (int s4 = 0; s4 < FLUSH; ++s4) {
          const int kk = 4 * (g * FLUSH + s4) + lk;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a[s4][i] = sa[kk * LROW + 16 * i];
            b[s4][i] = sb[kk * LROW + 16 * i];
          }
        }
        // one block row at a time keeps only 4 FP32 partial blocks live
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i < ni) {
            f4 part[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) part[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (j < nj) part[j] = MF<float>::op(b[s4][j], a[s4][i], part[j]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int e = 0; e < 4; ++e) acc[i][j][e] += (double)part[j][e];
          }
        }
      }
    }
    if (more) stash((c + 1) & 1);
    __syncthreads();
  }
}

template <typename TC>
__device__ __forceinline__ void zero_acc(typename MF<TC>::acc (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[i][j][e] = (TC)0;
}

// Cout[r][c] = (SUB ? Cin[r][c] - acc : acc) for the valid part of a wave's
// 64x64 tile; LAYOUT names the MFMA whose result layout acc follows.
template <typename LAYOUT, bool SUB, typename TI, typename TO, typename ACC>
__device__ __forceinline__ void store64_l(const TI* Cin, int64_t ldin, TO* Cout, int64_t ldout,
                                          const ACC (&acc)[4][4], int arows, int brows, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * i + lr;
    if (r >= arows) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * j + MF<LAYOUT>::col(lg, e);
        if (c < brows) {
          const double v = (double)acc[i][j][e];
          TO* po = Cout + (int64_t)c * ldout + r;
          if (SUB) *po = (TO)((double)Cin[(int64_t)c * ldin + r] - v);
          else *po = (TO)v;
        }
      }
    }
  }
}

template <typename TC, bool SUB, typename TI, typename TO>
__device__ __forceinline__ void store64(const TI* Cin, int64_t ldin, TO* Cout, int64_t ldout,
                                        const typename MF<TC>::acc (&acc)[4][4], int arows,
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
        const int c = 16 * j + MF<TC>::col(lg, e);
        if (c < brows) {
          const double v = (double)acc[i][j][e];
          TO* po = Cout + (int64_t)c * ldout + r;
          if (SUB) *po = (TO)((double)Cin[(int64_t)c * ldin + r] - v);
          else *po = (TO)v;
        }
      }
    }
  }
}

__device__ __forceinline__ int nblk(int rows) { return rows <= 0 ? 0 : min(4, (rows + 15) >> 4); }

// ---- left-looking update of block column J ---------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_col(Lay lay, double* __restrict__ mats,
                                                     const int32_t* __restrict__ info, int J, int nI,
                                                     int G) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  double* lds = reinterpret_cast<double*>(lds_raw);
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
  zero_acc<double>(acc);
  wg_gemm_nt<double, double, VEC>(acc, lds, base + lay.tile_off(I, 0), lay.tile_ld(I), arows,
                                  base + lay.tile_off(J, 0), lay.tile_ld(J), brows, kmax, act, ni,
                                  nj);
  if (act) {
    const int64_t ldc = lay.tile_ld(I);
    double* C = base + lay.tile_off(I, J) + 64 * wr + 64 * wc * ldc;
    store64<double, true>(C, ldc, C, ldc, acc, war, wbr, lane);
  }
}

// Mixed form.  Off-diagonal tiles: FP32 storage, FP32 MFMA whose partial
// sums are accumulated in FP64, subtracted from V's FP64 tile and rounded to
// FP32 once.  The diagonal tile: FP64 MFMA on the FP32 panels, subtracted from
// the FP64 tile of V, written to an FP64 scratch tile for k_potrf.
constexpr int MX_FLUSH = 4;  // FP32 MFMA k-steps (16 products) per FP64 flush (default)

// FP64 flush interval of the mixed update: MX_FLUSH, or 1/2/4/8 from the
// environment variable PLPROF_MX_FLUSH (an accuracy/speed study knob).
static int mx_flush() {
  static int v = [] {
    const char* e = getenv("PLPROF_MX_FLUSH");
    const int f = e ? atoi(e) : MX_FLUSH;
    return (f == 1 || f == 2 || f == 4 || f == 8) ? f : MX_FLUSH;
  }();
  return v;
}
template <bool VEC, int FLUSH>
__global__ __launch_bounds__(256, 2) void k_gemm_col_mx(Lay lay, float* __restrict__ m32,
                                                        const double* __restrict__ m64,
                                                        int64_t m64stride,
                                                        const int32_t* __restrict__ info, int J,
                                                        int nI, int G) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  float* lds = reinterpret_cast<float*>(lds_raw);
  const int wg = xcd_remap(blockIdx.x, G);
  const int k = wg / nI;
  const int I = J + 1 + wg % nI;  // tile rows strictly below the diagonal
  if (info[k] != 0) return;       // uniform for the workgroup
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
  wg_gemm_nt_f32x64<FLUSH>(acc, lds, base + lay.tile_off(I, 0), lay.tile_ld(I), arows,
                           base + lay.tile_off(J, 0), lay.tile_ld(J), brows, kmax, act, ni, nj);
  if (act) {
    const int64_t ldc = lay.tile_ld(I);
    float* C = base + lay.tile_off(I, J) + 64 * wr + 64 * wc * ldc;
    if (I < lay.Nv) {
      // V's own tile from the FP64 copy: the update is subtracted in FP64
      const double* Cin = m64 + (int64_t)k * m64stride + lay.tile_off(I, J) + 64 * wr + 64 * wc * T;
      store64_l<float, true>(Cin, T, C, ldc, acc, war, wbr, lane);
    } else {
      store64_l<float, true>(C, ldc, C, ldc, acc, war, wbr, lane);
    }
  }
}

// Mixed form, diagonal tile J: FP64 MFMA on the FP32 panel, subtracted from V's
// FP64 tile, written to the FP64 scratch tile that k_potrf reads.
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_diag_mx(Lay lay, const float* __restrict__ m32,
                                                         const double* __restrict__ m64,
                                                         int64_t m64stride,
                                                         double* __restrict__ dscratch,
                                                         const int32_t* __restrict__ info, int J) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  float* lds = reinterpret_cast<float*>(lds_raw);
  const int k = blockIdx.x;
  if (info[k] != 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int rows = lay.rows(J);
  const int war = rows - 64 * wr, wbr = rows - 64 * wc;
  const int ni = nblk(war), nj = nblk(wbr);
  const bool act = ni > 0 && nj > 0 && wc <= wr;
  const float* P = m32 + (int64_t)k * lay.mstride + lay.tile_off(J, 0);
  const int kmax = min(J * T, lay.n);
  d4 acc[4][4];
  zero_acc<double>(acc);
  wg_gemm_nt<float, double, VEC>(acc, lds, P, lay.tile_ld(J), rows, P, lay.tile_ld(J), rows, kmax,
                                 act, ni, nj);
  if (act) {
    const double* Cin = m64 + (int64_t)k * m64stride + lay.tile_off(J, J) + 64 * wr + 64 * wc * T;
    double* Cout = dscratch + (int64_t)k * T * T + 64 * wr + 64 * wc * T;
    store64<double, true>(Cin, T, Cout, T, acc, war, wbr, lane);
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

hipError_t launch_gemm_col_mx(const Lay& lay, float* m32, const double* m64, int64_t m64stride,
                              double* dscratch, const int32_t* info, int J, int nI, int K,
                              hipStream_t s) {
  // nI counts the tile rows from J down (the diagonal tile included)
  hipLaunchKernelGGL(k_gemm_diag_mx<true>, dim3(K), dim3(256), 0, s, lay, m32, m64, m64stride,
                     dscratch, info, J);
  if (nI > 1) {
    const int G = K * (nI - 1);
    switch (mx_flush()) {
      case 1:
        hipLaunchKernelGGL((k_gemm_col_mx<true, 1>), dim3(G), dim3(256), 0, s, lay, m32, m64,
                           m64stride, info, J, nI - 1, G);
        break;
      case 4:
        hipLaunchKernelGGL((k_gemm_col_mx<true, 4>), dim3(G), dim3(256), 0, s, lay, m32, m64,
                           m64stride, info, J, nI - 1, G);
        break;
      case 8:
        hipLaunchKernelGGL((k_gemm_col_mx<true, 8>), dim3(G), dim3(256), 0, s, lay, m32, m64,
                           m64stride, info, J, nI - 1, G);
        break;
      default:
        hipLaunchKernelGGL((k_gemm_col_mx<true, 2>), dim3(G), dim3(256), 0, s, lay, m32, m64,
                           m64stride, info, J, nI - 1, G);
    }
  }
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
// MODE 0 (FP64 form): the tile is read from and L written back to the packed
//   matrix, W (FP64) to Wbuf[k].  MODE 1 (mixed form): the tile is read from
//   the FP64 scratch tile, L is not kept, W is written in FP32 to slot J of
//   the omega's inverse table (the back substitution needs every W_J).
template <int MODE>
__global__ __launch_bounds__(256) void k_potrf(Lay lay, double* __restrict__ mats,
                                               double* __restrict__ Wbuf, float* __restrict__ W32,
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
  double* C;
  int64_t ld;
  if (MODE == 0) {
    C = mats + (int64_t)k * lay.mstride + lay.tile_off(J, J);
    ld = lay.tile_ld(J);
  } else {
    C = Wbuf + (int64_t)k * T * T;
    ld = T;
  }
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

  // log|V| contribution, 1/L_jj, and (FP64 form) the factor itself
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
  if (MODE == 0 && low) {
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
  if (MODE == 0) {
    double* W = Wbuf + (int64_t)k * T * T;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        W[c * T + r] = (low && r >= c) ? a[rr][cc] : 0.0;
      }
  } else {
    float* W = W32 + ((int64_t)k * lay.Nv + J) * T * T;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        W[c * T + r] = (low && r >= c) ? (float)a[rr][cc] : 0.0f;
      }
  }
}

hipError_t launch_potrf(const Lay& lay, double* mats, double* W, double* logdet, int32_t* info,
                        int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf<0>, dim3(K), dim3(256), 0, s, lay, mats, W, (float*)nullptr, logdet,
                     info, J);
  return hipGetLastError();
}

hipError_t launch_potrf_mx(const Lay& lay, double* dscratch, float* W32, double* logdet,
                           int32_t* info, int J, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf<1>, dim3(K), dim3(256), 0, s, lay, (double*)nullptr, dscratch, W32,
                     logdet, info, J);
  return hipGetLastError();
}

// ---- panel solve L_IJ = C_IJ W_J^T for the nI tile rows below J -----------
// TS double: W from Wbuf[k]; TS float: W from slot J of the omega's table.
template <typename TS, bool VEC>
__global__ __launch_bounds__(256, 2) void k_trsm(Lay lay, TS* __restrict__ mats,
                                                 const TS* __restrict__ Wbuf,
                                                 const int32_t* __restrict__ info, int J, int nI,
                                                 int G, int64_t wstride) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  TS* lds = reinterpret_cast<TS*>(lds_raw);
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
  TS* Ct = mats + (int64_t)k * lay.mstride + lay.tile_off(I, J);
  const int64_t ldc = lay.tile_ld(I);
  TS* Co = Ct + 64 * wr + 64 * wc * ldc;
  // the core's final barrier orders every read of C_IJ before the overwrite
  if constexpr (sizeof(TS) == 8) {
    d4 acc[4][4];
    zero_acc<double>(acc);
    wg_gemm_nt<TS, TS, VEC>(acc, lds, Ct, ldc, arows, Wbuf + (int64_t)k * wstride, T, brows, brows,
                            act, ni, nj);
    if (act) store64<double, false>(Co, ldc, Co, ldc, acc, war, wbr, lane);
  } else {
    d4 acc[4][4];
    zero_acc<double>(acc);
    wg_gemm_nt_f32x64<MX_FLUSH>(acc, lds, Ct, ldc, arows, Wbuf + (int64_t)k * wstride, T, brows,
                                brows, act, ni, nj);
    if (act) store64_l<float, false>(Co, ldc, Co, ldc, acc, war, wbr, lane);
  }
}

hipError_t launch_trsm(const Lay& lay, double* mats, const double* W, const int32_t* info, int J,
                       int nI, int K, hipStream_t s) {
  const int G = K * nI;
  const int64_t ws = (int64_t)T * T;
  if (vec_ok(lay, mats) && (reinterpret_cast<uintptr_t>(W) & 15) == 0)
    hipLaunchKernelGGL((k_trsm<double, true>), dim3(G), dim3(256), 0, s, lay, mats, W, info, J, nI,
                       G, ws);
  else
    hipLaunchKernelGGL((k_trsm<double, false>), dim3(G), dim3(256), 0, s, lay, mats, W, info, J,
                       nI, G, ws);
  return hipGetLastError();
}

hipError_t launch_trsm_mx(const Lay& lay, float* m32, const float* W32, const int32_t* info, int J,
                          int nI, int K, hipStream_t s) {
  const int G = K * nI;
  const int64_t ws = (int64_t)lay.Nv * T * T;
  hipLaunchKernelGGL((k_trsm<float, true>), dim3(G), dim3(256), 0, s, lay, m32,
                     W32 + (int64_t)J * T * T, info, J, nI, G, ws);
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
__global__ __launch_bounds__(256, 2) void k_qform(Lay lay, const double* __restrict__ m64,
                                                  int64_t stride64, const double* __restrict__ X,
                                                  const double* __restrict__ rhs,
                                                  const int32_t* __restrict__ info,
                                                  double* __restrict__ slots, int refine,
                                                  int ntile, int G) {
  __shared__ __attribute__((aligned(16))) char lds_raw[GEMM_LDS_BYTES];
  double* lds = reinterpret_cast<double*>(lds_raw);
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
  const int TB = lay.TB, q = lay.q;
  const int ri = lay.rows(I), rj = lay.rows(J);
  const double* Xk = X + (int64_t)k * lay.n * TB;
  double* slot = slots + ((int64_t)k * ntile + t) * TB * TB;
  const double* Xi = Xk + (int64_t)I * T * TB;   // x0_I: element (r, a) at r*TB + a
  double* Ys = lds;                              // Y, column-major T x TB, after the core
  if (refine) {
    const int war = ri - 64 * wr, wbr = q - 64 * wc;
    const int ni = nblk(war), nj = nblk(wbr);
    const bool act = ni > 0 && nj > 0;
    d4 acc[4][4];
    zero_acc<double>(acc);
    wg_gemm_nt<double, double, true>(acc, lds, m64 + (int64_t)k * stride64 + lay.tile_off(I, J), T,
                                     ri, Xk + (int64_t)J * T * TB, TB, q, rj, act, ni, nj);
    // the core ends with a barrier: the LDS stages are free for Y
    if (act) store64<double, false>(Ys + 64 * wr + 64 * wc * T, T, Ys + 64 * wr + 64 * wc * T, T,
                                    acc, war, wbr, lane);
    __syncthreads();
  }
  const double* Bi = rhs + (int64_t)I * T * TB;
  for (int pr = tid; pr < TB * TB; pr += 256) {
    const int a = pr / TB, b = pr % TB;
    double v = 0.0;
    if (refine) {
      double mab = 0.0, mba = 0.0, bx = 0.0;
      for (int r = 0; r < ri; ++r) {
        const double xa = Xi[r * TB + a], xb = Xi[r * TB + b];
        mab += xa * Ys[b * T + r];
        mba += xb * Ys[a * T + r];
        if (I == J) bx += Bi[r * TB + a] * xb;
      }
      v = (I > J) ? -(mab + mba) : 2.0 * bx - mab;
    } else if (I == J) {
      for (int r = 0; r < ri; ++r) v += Bi[r * TB + a] * Xi[r * TB + b];
    }
    slot[pr] = v;
  }
}

hipError_t launch_qform(const Lay& lay, const double* m64, int64_t stride64, const double* X,
                        const double* rhs, const int32_t* info, double* slots, int refine, int K,
                        hipStream_t s) {
  const int ntile = lay.Nv * (lay.Nv + 1) / 2;
  const int G = K * ntile;
  hipLaunchKernelGGL(k_qform, dim3(G), dim3(256), 0, s, lay, m64, stride64, X, rhs, info, slots,
                     refine, ntile, G);
  return hipGetLastError();
}

}  // namespace plk
