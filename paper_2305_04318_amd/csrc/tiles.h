// Device building blocks shared by the step kernels and the persistent batch
// kernel: the MFMA GEMM core and the tile tasks of the blocked factorisation.
#pragma once

#include <math.h>

#include <type_traits>

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
// arows / brows and columns at or beyond kmax read as zero.  A wave skips its
// block rows at or beyond ni (16-row blocks holding rows below arows) but
// runs all four block columns: those beyond brows multiply zeros and are
// never stored, which keeps the MFMA stream free of per-block branches (a
// caller whose B has at most 16 NJ rows passes NJ < 4 to skip the rest at
// compile time).  TS is the storage type, TC the MFMA type (float storage may
// be widened to FP64 MFMA).
constexpr int LROW = T + 4;         // LDS stride per k column (elements)
constexpr int GEMM_LDS_BYTES = 2 * 2 * 16 * LROW * 8;

// TRI (the panel solve C W^T, W lower triangular): output block column g
// (16 columns) needs only k < 16 (g + 1).  Wave column wc owns the block
// columns tri_blk(wc, 0..3) = {0, 3, 4, 7} or {1, 2, 5, 6}, 18 nonzero
// 16 x 16 x 16 products each, instead of the halves {0..3} and {4..7} (10
// and 26); per k block m the two columns have 4/4, 3/4, 3/3, 3/2, 2/2, 1/2,
// 1/1, 1/0 blocks still running, so a chunk's barrier waits for at most one
// block more on either side.  tri_blk grows with j, so the blocks that still
// need the k from k0 on are j >= tri_lo(wc, k0): one scalar branch per MFMA.
// Blocks at or beyond brows multiply the zero rows of B and are not stored.
__device__ __forceinline__ int tri_blk(int wc, int j) {
  return wc ? (j < 2 ? j + 1 : j + 3) : (j < 2 ? 3 * j : 3 * j - 2);
}

__device__ __forceinline__ int tri_lo(int wc, int k0) {
  int jlo = 4;
#pragma unroll
  for (int j = 3; j >= 0; --j)
    if (16 * tri_blk(wc, j) + 16 > k0) jlo = j;
  return jlo;
}

template <typename TS, typename TC, bool VEC, int NJ = 4, int DEPTH = 2, bool TRI = false>
__device__ __forceinline__ void wg_gemm_nt(typename MF<TC>::acc (&acc)[4][4], TS* lds,
                                           const TS* __restrict__ A, int64_t lda, int arows,
                                           const TS* __restrict__ B, int64_t ldb, int brows,
                                           int kmax, bool do_mfma, int ni) {
  static_assert(!TRI || DEPTH > 1, "the column map is built into the two-set pipeline");
  constexpr int N = Piece<TS>::N;
  constexpr int KC = 128 / (int)sizeof(TS);
  constexpr int PPC = T / N;  // pieces per column
  typedef typename Piece<TS>::type V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  // per-wave values: keep them in scalar registers so that the block-row
  // guards below are scalar branches, not exec masks
  ni = __builtin_amdgcn_readfirstlane(ni);
  do_mfma = __builtin_amdgcn_readfirstlane((int)do_mfma) != 0;
  if constexpr (DEPTH == 1) {
    // one register set: chunk c + 1 is fetched while chunk c is multiplied
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
              for (int j = 0; j < NJ; ++j) acc[i][j] = MF<TC>::op(b[j], a[i], acc[i][j]);
            }
          }
        }
      }
      if (more) stash((c + 1) & 1);
      __syncthreads();
    }
    return;
  }
  // two register sets: chunk c + 2 is fetched while chunk c is multiplied and
  // chunk c + 1 (fetched a chunk earlier) waits in registers for its LDS stage
  V ra[2][4], rb[2][4];
  // whole-tile panels and a chunk inside kmax need no bounds checks: one
  // scalar branch per chunk instead of per-piece exec masks
  const bool full = VEC && __builtin_amdgcn_readfirstlane((int)(arows >= T && brows >= T)) != 0;
  kmax = __builtin_amdgcn_readfirstlane(kmax);
  auto fetch = [&](int k0, auto setc) {
    constexpr int S = decltype(setc)::value;
    if (full && k0 + KC <= kmax) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int idx = tid + 256 * q;
        const int col = idx / PPC, row = (idx % PPC) * N;
        ra[S][q] = *reinterpret_cast<const V*>(A + (int64_t)(k0 + col) * lda + row);
        rb[S][q] = *reinterpret_cast<const V*>(B + (int64_t)(k0 + col) * ldb + row);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int idx = tid + 256 * q;
        const int col = idx / PPC, row = (idx % PPC) * N;
        ra[S][q] = fetch_piece<TS, VEC>(A, lda, arows, k0 + col, kmax, row);
        rb[S][q] = fetch_piece<TS, VEC>(B, ldb, brows, k0 + col, kmax, row);
      }
    }
  };
  auto stash = [&](auto setc) {
    constexpr int S = decltype(setc)::value;  // register set = LDS stage
    TS* sa = lds + (S * 2 + 0) * KC * LROW;
    TS* sb = lds + (S * 2 + 1) * KC * LROW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      *reinterpret_cast<V*>(sa + col * LROW + row) = ra[S][q];
      *reinterpret_cast<V*>(sb + col * LROW + row) = rb[S][q];
    }
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  fetch(0, S0{});
  if (nchunks > 1) fetch(KC, S1{});
  stash(S0{});
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  // chunk c (even: set/stage 0, odd: 1): fetch c + 2 into its own set, run
  // its MFMAs from LDS stage c & 1, then move chunk c + 1 to the other stage
  // the column map is per wave: scalar registers, scalar branches
  const int wcu = TRI ? __builtin_amdgcn_readfirstlane(wc) : wc;
  auto step = [&](int c, auto setc, auto other) {
    constexpr int S = decltype(setc)::value;
    if (c + 2 < nchunks) fetch((c + 2) * KC, setc);
    const int jlo = TRI ? tri_lo(wcu, c * KC) : 0;
    if (do_mfma && jlo < NJ) {
      const TS* sa = lds + (S * 2 + 0) * KC * LROW + 64 * wr + lr;
      const TS* sb = lds + (S * 2 + 1) * KC * LROW + (TRI ? 0 : 64 * wc) + lr;
      // every block row runs (rows at or beyond arows multiply the zeros the
      // fetch put there and are never stored): a wave with fewer valid rows
      // only occurs in a tile's last row block, beside a full wave that sets
      // the workgroup's pace, and a branch-free MFMA stream schedules better
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        TC a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = (TC)sa[kk * LROW + 16 * i];
          b[i] = (TC)sb[kk * LROW + 16 * (TRI ? tri_blk(wcu, i) : i)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i < ni) {
#pragma unroll
            for (int j = 0; j < NJ; ++j)
              if (!TRI || j >= jlo) acc[i][j] = MF<TC>::op(b[j], a[i], acc[i][j]);
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

// FP32 MFMA whose partial sums are flushed into FP64 accumulators every
// FLUSH k-steps (FLUSH * 4 products): the FP32 rounding then only touches short
// partial sums instead of the long running sums that cancel in the Schur
// complements of an ill-conditioned V.  Same LDS pipeline as wg_gemm_nt.
// HALF (the panel solve, W lower triangular): wave column 0 holds output
// columns 0..63 and needs no products past k = 64, so it skips those chunks
// whole (the pending partials are folded at the end); a per-block map as in
// wg_gemm_nt's TRI makes this core spill.
template <int FLUSH, bool HALF = false>
__device__ __forceinline__ void wg_gemm_nt_f32x64(d4 (&acc)[4][4], float* lds,
                                                  const float* __restrict__ A, int64_t lda,
                                                  int arows, const float* __restrict__ B,
                                                  int64_t ldb, int brows, int kmax, bool do_mfma,
                                                  int ni) {
  constexpr int N = 4;
  constexpr int KC = 32;
  constexpr int PPC = T / N;
  typedef flt4 V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  // per-wave values: keep them in scalar registers so that the block-row
  // guards below are scalar branches, not exec masks
  ni = __builtin_amdgcn_readfirstlane(ni);
  do_mfma = __builtin_amdgcn_readfirstlane((int)do_mfma) != 0;
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
  f4 pp[4];  // FP32 partials of the block row that is folded in next
#pragma unroll
  for (int j = 0; j < 4; ++j) pp[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const int wcu = HALF ? __builtin_amdgcn_readfirstlane(wc) : wc;
  for (int c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) fetch((c + 1) * KC);
    if (do_mfma && (!HALF || wcu == 1 || c * KC < 64)) {
      const float* sa = lds + ((c & 1) * 2 + 0) * KC * LROW + 64 * wr + lr;
      const float* sb = lds + ((c & 1) * 2 + 1) * KC * LROW + 64 * wc + lr;
      // rolled: only one group's fragments and partial sums are live at a time
#pragma unroll 1
      for (int g = 0; g < KC / 4 / FLUSH; ++g) {
        float b[FLUSH][4];
#pragma unroll
        for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
          for (int j = 0; j < 4; ++j) b[s4][j] = sb[(4 * (g * FLUSH + s4) + lk) * LROW + 16 * j];
        // software pipeline over block rows: issue row i's MFMAs, then fold
        // the previous row's FP32 partials into FP64 while they run
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float a[FLUSH];
#pragma unroll
          for (int s4 = 0; s4 < FLUSH; ++s4) a[s4] = sa[(4 * (g * FLUSH + s4) + lk) * LROW + 16 * i];
          f4 pc[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) pc[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
          if (i < ni) {
#pragma unroll
            for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
              for (int j = 0; j < 4; ++j) pc[j] = MF<float>::op(b[s4][j], a[s4], pc[j]);
          }
          const int ip = (i + 3) & 3;
          if (ip < ni) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int e = 0; e < 4; ++e) acc[ip][j][e] += (double)pp[j][e];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) pp[j] = pc[j];
        }
      }
    }
    if (more) stash((c + 1) & 1);
    __syncthreads();
  }
  if (do_mfma && 3 < ni) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[3][j][e] += (double)pp[j][e];
  }
}

// LDS pointers for the direct-to-LDS loads (global_load_lds_dwordx4)
typedef __attribute__((address_space(3))) void lds_void;

// Publish direct-to-LDS loads to the workgroup: wait until at most N of the
// wave's vector-memory loads are outstanding (they complete in order, so the
// older ones have written LDS) and for its LDS accesses, then s_barrier; one
// asm statement with a memory clobber, so the compiler neither moves memory
// accesses across it nor relies on its own waits (__syncthreads' fence does
// not reliably wait for these loads).
template <int N>
__device__ __forceinline__ void vmcnt_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// vmcnt_barrier leaving the requests of `ahead` later chunks (P loads per
// wave each, ahead <= MAXA, uniform) in flight.
template <int P, int MAXA>
__device__ __forceinline__ void vmcnt_barrier_ahead(int ahead) {
  if constexpr (MAXA <= 0) {
    vmcnt_barrier<0>();
  } else {
    if (ahead >= MAXA) vmcnt_barrier<P * MAXA>();
    else vmcnt_barrier_ahead<P, MAXA - 1>(ahead);
  }
}

// FP32 form with direct-to-LDS loads (the fold pipeline of wg_gemm_nt_f32x64,
// two stages as in wg_gemm_nt_dma).  One instruction carries two 128-float
// columns (lanes 0-31 and 32-63, 512 B each), so the columns of a pair are
// stored back to back and pairs F32_PS floats apart; the odd column of a pair
// holds row r at r ^ 32 (the lanes' source rows are swizzled, in 16-byte
// pieces), and with F32_PS = 16 mod 64 the 64 lanes of a fragment read (four
// columns, sixteen rows) touch 64 different banks.  Whole 128-row panels of
// leading dimension T; kmax a multiple of 32.
// SPLIT: the column-split plan of wg_gemm_nt_dma (ni then counts the valid
// block rows): the fold pipeline runs over row pairs, slot row i holding
// block rows 2 i and 2 i + 1 against the wave's block columns 2 w, 2 w + 1.
constexpr int F32_PS = 272;
constexpr int F32_DMA_LDS_BYTES = 2 * 2 * 16 * F32_PS * 4;  // stages x panels x pairs

template <int FLUSH, bool SPLIT = false>
__device__ __forceinline__ void wg_gemm_nt_f32x64_dma(d4 (&acc)[4][4], float* lds,
                                                      const float* __restrict__ A,
                                                      const float* __restrict__ B, int kmax,
                                                      bool do_mfma, int ni) {
  constexpr int KC = 32, NPAIR = KC / 2, STG = 2 * NPAIR * F32_PS, PPW = 2 * NPAIR / 4;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = __builtin_amdgcn_readfirstlane(kmax) / KC;
  if (nchunks <= 0) return;
  ni = __builtin_amdgcn_readfirstlane(ni);
  do_mfma = __builtin_amdgcn_readfirstlane((int)do_mfma) != 0;
  // SPLIT: valid block rows, and slot rows (row pairs) with any of them
  const int nrb = ni;
  if (SPLIT) ni = (nrb + 1) >> 1;
  const int half = lane >> 5;                        // even / odd column of a pair
  const int srow = (4 * (lane & 31)) ^ (32 * half);  // source row of the lane's 16 bytes
  // wave w moves pairs PPW w .. PPW w + PPW - 1 of the chunk's 2 NPAIR (A, then B)
  auto request = [&](int c, int stage) {
#pragma unroll
    for (int h = 0; h < PPW; ++h) {
      const int p = PPW * wave + h;
      const bool isb = p >= NPAIR;
      const int q = p - (isb ? NPAIR : 0);
      const float* src = (isb ? B : A) + (int64_t)(c * KC + 2 * q + half) * T + srow;
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const void*>(src),
          (lds_void*)(lds + stage * STG + (isb ? NPAIR * F32_PS : 0) + q * F32_PS), 16, 0, 0);
    }
  };
  request(0, 0);
  const int lr = lane & 15, lk = lane >> 4;
  // column 4 s + lk of a chunk: pair 2 s + (lk >> 1), half lk & 1
  const int swz = (lk & 1) ? 32 : 0;
  const int colbase = (lk >> 1) * F32_PS + (lk & 1) * 128;
  f4 pp[4];  // FP32 partials of the block row that is folded in next
#pragma unroll
  for (int j = 0; j < 4; ++j) pp[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int c = 0; c < nchunks; ++c) {
    const int stage = c & 1;
    vmcnt_barrier<0>();  // chunk c in LDS; chunk c - 1's stage free
    if (c + 1 < nchunks) request(c + 1, stage ^ 1);
    if (do_mfma) {
      const float* sa = lds + stage * STG + colbase;
      const float* sb = sa + NPAIR * F32_PS;
      // rolled: only one group's fragments and partial sums are live at a time
#pragma unroll 1
      for (int g = 0; g < KC / 4 / FLUSH; ++g) {
        if constexpr (SPLIT) {
          float b[FLUSH][2];
#pragma unroll
          for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              b[s4][j] = sb[2 * (g * FLUSH + s4) * F32_PS + ((32 * wave + 16 * j + lr) ^ swz)];
          // a row pair with one valid block row also multiplies the pair's
          // second (padding) row block, which is never stored
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            f4 pc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) pc[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            if (i < ni) {
              float a[FLUSH][2];
#pragma unroll
              for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                  a[s4][h] = sa[2 * (g * FLUSH + s4) * F32_PS + ((32 * i + 16 * h + lr) ^ swz)];
#pragma unroll
              for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                  pc[j] = MF<float>::op(b[s4][j & 1], a[s4][j >> 1], pc[j]);
            }
            const int ip = (i + 3) & 3;
            if (ip < ni) {
#pragma unroll
              for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[ip][j][e] += (double)pp[j][e];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) pp[j] = pc[j];
          }
          continue;
        }
        float b[FLUSH][4];
#pragma unroll
        for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            b[s4][j] = sb[2 * (g * FLUSH + s4) * F32_PS + ((64 * wc + 16 * j + lr) ^ swz)];
        // software pipeline over block rows: issue row i's MFMAs, then fold
        // the previous row's FP32 partials into FP64 while they run
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float a[FLUSH];
#pragma unroll
          for (int s4 = 0; s4 < FLUSH; ++s4)
            a[s4] = sa[2 * (g * FLUSH + s4) * F32_PS + ((64 * wr + 16 * i + lr) ^ swz)];
          f4 pc[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) pc[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
          if (i < ni) {
#pragma unroll
            for (int s4 = 0; s4 < FLUSH; ++s4)
#pragma unroll
              for (int j = 0; j < 4; ++j) pc[j] = MF<float>::op(b[s4][j], a[s4], pc[j]);
          }
          const int ip = (i + 3) & 3;
          if (ip < ni) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int e = 0; e < 4; ++e) acc[ip][j][e] += (double)pp[j][e];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) pp[j] = pc[j];
        }
      }
    }
  }
  __syncthreads();  // the last stage is read before the caller reuses LDS
  if (do_mfma && 3 < ni) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[3][j][e] += (double)pp[j][e];
  }
}

// acc += C[0:128, 0:128] W[0:128, 0:128]^T in FP64 MFMA from FP32 panels
// staged as in wg_gemm_nt_f32x64_dma (chunks of KC columns, column pairs
// F32_PS floats apart, the odd column's rows swizzled by 32), each fragment
// widened to FP64 on its LDS read: the mixed form's panel solve of a whole
// packed tile, with exact products and FP64 sums (no FP32 partials to fold).
// TRI column map of the FP64 panel solve: the blocks that still need a
// k-step from k0 on are j >= tri_lo(wc, k0).  NST stages as in
// wg_gemm_nt_dma.  Both panels have leading dimension T and 128 rows.
template <int KC, int NST>
constexpr int f32dma_lds_bytes() { return NST * 2 * (KC / 2) * F32_PS * 4; }

template <int KC, int NST>
__device__ __forceinline__ void wg_gemm_nt_f32dma_f64(d4 (&acc)[4][4], float* lds,
                                                      const float* __restrict__ A,
                                                      const float* __restrict__ B, int kmax,
                                                      bool do_mfma) {
  constexpr int NPAIR = KC / 2, STG = 2 * NPAIR * F32_PS, PPW = 2 * NPAIR / 4;
  static_assert(NST >= 2 && NST <= 6, "two to six stages");
  static_assert((KC == 8 || KC % 16 == 0) && (NST - 2) * PPW <= 15,
                "no k block split across chunks; vmcnt holds the chunks in flight");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = __builtin_amdgcn_readfirstlane(kmax) / KC;
  if (nchunks <= 0) return;
  do_mfma = __builtin_amdgcn_readfirstlane((int)do_mfma) != 0;
  const int half = lane >> 5;                        // even / odd column of a pair
  const int srow = (4 * (lane & 31)) ^ (32 * half);  // source row of the lane's 16 bytes
  // wave w moves pairs PPW w .. PPW w + PPW - 1 of the chunk's 2 NPAIR (A, then B)
  auto request = [&](int c, int stage) {
#pragma unroll
    for (int h = 0; h < PPW; ++h) {
      const int p = PPW * wave + h;
      const bool isb = p >= NPAIR;
      const int q = p - (isb ? NPAIR : 0);
      const float* src = (isb ? B : A) + (int64_t)(c * KC + 2 * q + half) * T + srow;
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const void*>(src),
          (lds_void*)(lds + stage * STG + (isb ? NPAIR * F32_PS : 0) + q * F32_PS), 16, 0, 0);
    }
  };
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    if (p < nchunks) request(p, p);
  const int lr = lane & 15, lk = lane >> 4;
  // column 4 s + lk of a chunk: pair 2 s + (lk >> 1), half lk & 1
  const int swz = (lk & 1) ? 32 : 0;
  const int colbase = (lk >> 1) * F32_PS + (lk & 1) * 128;
  int stage = 0;
  for (int c = 0; c < nchunks; ++c) {
    // chunk c in LDS (the requests of the chunks after it may stay in
    // flight); chunk c - 1's stage free
    vmcnt_barrier_ahead<PPW, NST - 2>(min(NST - 2, nchunks - 1 - c));
    if (c + NST - 1 < nchunks) request(c + NST - 1, stage == 0 ? NST - 1 : stage - 1);
    // no chunk straddles a 16-column k block: every k of the chunk has the
    // same block columns
    const int jlo = tri_lo(wc, c * KC);
    if (do_mfma && jlo < 4) {
      const float* sa = lds + stage * STG + colbase;
      const float* sb = sa + NPAIR * F32_PS;
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = (double)sa[2 * s4 * F32_PS + ((64 * wr + 16 * i + lr) ^ swz)];
          b[i] = (double)sb[2 * s4 * F32_PS + ((16 * tri_blk(wc, i) + lr) ^ swz)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j >= jlo) acc[i][j] = MF<double>::op(b[j], a[i], acc[i][j]);
      }
    }
    if (++stage == NST) stage = 0;
  }
  __syncthreads();  // the last stage is read before the caller reuses LDS
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
// 64x64 tile; LAYOUT names the MFMA whose result layout acc follows.  With
// SUB the 16 Cin values of a block row are loaded together, from addresses
// clamped into the valid part, before any of its stores: element by element,
// each load would wait behind the store before it (Cin and Cout may alias),
// 64 dependent HBM round trips per lane instead of 4.  BATCH = false keeps
// the element-by-element form for register-bound callers (the 16 staged
// values per lane would spill there).
template <typename LAYOUT, bool SUB, typename TI, typename TO, typename ACC, bool BATCH = true>
__device__ __forceinline__ void store64_l(const TI* Cin, int64_t ldin, TO* Cout, int64_t ldout,
                                          const ACC (&acc)[4][4], int arows, int brows, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  if constexpr (SUB && BATCH) {
    arows = __builtin_amdgcn_readfirstlane(arows);  // per-wave values
    brows = __builtin_amdgcn_readfirstlane(brows);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (16 * i >= arows) break;
      const int r = 16 * i + lr, rc = min(r, arows - 1);
      double cin[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int cc = min(16 * j + MF<LAYOUT>::col(lg, e), brows - 1);
          cin[j][e] = (double)Cin[(int64_t)cc * ldin + rc];
        }
      if (r >= arows) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 16 * j + MF<LAYOUT>::col(lg, e);
          if (c < brows) Cout[(int64_t)c * ldout + r] = (TO)(cin[j][e] - (double)acc[i][j][e]);
        }
    }
  } else {
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
}

template <typename TC, bool SUB, typename TI, typename TO, bool BATCH = true>
__device__ __forceinline__ void store64(const TI* Cin, int64_t ldin, TO* Cout, int64_t ldout,
                                        const typename MF<TC>::acc (&acc)[4][4], int arows,
                                        int brows, int lane) {
  store64_l<TC, SUB, TI, TO, typename MF<TC>::acc, BATCH>(Cin, ldin, Cout, ldout, acc, arows,
                                                          brows, lane);
}

// C -= the bordered row's tile held by the border wave of the diagonal-tile
// workgroup: block (ib, jb) of the nbr x 8 blocks in acc[2 ib + jb / 4][jb % 4]
// (FP64 MFMA layout); rows below qrows and columns below prows are valid.
// The loads of four blocks are issued together, as in store64_l.
template <typename TO>
__device__ __forceinline__ void sub_store_border(TO* C, int64_t ldc, const d4 (&acc)[4][4],
                                                 int nbr, int qrows, int prows, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  nbr = __builtin_amdgcn_readfirstlane(nbr);
  qrows = __builtin_amdgcn_readfirstlane(qrows);
  prows = __builtin_amdgcn_readfirstlane(prows);
#pragma unroll
  for (int ib = 0; ib < 2; ++ib) {
    if (ib >= nbr || 16 * ib >= qrows) break;
    const int r = 16 * ib + lr, rc = min(r, qrows - 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double cin[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int cc = min(64 * h + 16 * j + MF<double>::col(lg, e), prows - 1);
          cin[j][e] = (double)C[(int64_t)cc * ldc + rc];
        }
      if (r < qrows) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = 64 * h + 16 * j + MF<double>::col(lg, e);
            if (c < prows) C[(int64_t)c * ldc + r] = (TO)(cin[j][e] - acc[2 * ib + h][j][e]);
          }
      }
    }
  }
}

__device__ __forceinline__ int nblk(int rows) { return rows <= 0 ? 0 : min(4, (rows + 15) >> 4); }

// ---- workgroup GEMM core, direct-to-LDS form -------------------------------------
// acc += A[0:128, 0:kmax] B[0:128, 0:kmax]^T for whole 128-row panels with
// leading dimension T (the packed tiles and the inverse buffer: every row of
// every column is allocated).  Same wave grid, chunk width (KC = 16) and LDS
// layout as wg_gemm_nt, but the chunks travel from global memory straight
// into LDS (global_load_lds_dwordx4: lane l carries rows 2l, 2l+1 of one
// column, 1 KB per instruction, the LDS column base set per instruction), so
// no registers stage the prefetch and no LDS stores are issued.  NST stages
// of KC columns: chunk c + NST - 1 is requested right after the barrier that
// publishes chunk c (every wave has then left chunk c - 1, whose stage it
// refills) and lands while chunks c .. c + NST - 2 are multiplied.  Each
// chunk is published by vmcnt_barrier: with two stages every load of the
// wave must be done (only chunk c's are outstanding), with three all but the
// next chunk's.  kmax must be a multiple of KC; every block row is
// multiplied (rows a tile does not hold are never stored).  TRI as in
// wg_gemm_nt.
// SPLIT: the column-split plan for a tile with fewer than 128 valid rows
// (the last tile row): wave w takes block columns 2 w and 2 w + 1 and the
// nrb valid block rows, block (i, j) in acc[i >> 1][2 (i & 1) + j] -- 2 nrb
// blocks on every wave, where the quadrant plan runs 16 blocks on the waves
// of the first wave row whatever the valid rows (a compute unit's waves of
// one index share a SIMD, so those 16 set the tile's time).  With TRI the
// wave's block columns are w and 7 - w, which need 9 k blocks together.
// LR: LDS stride per k column.  The update uses LROW_UPD = 144 (1152 B, 128 B
// mod 256): the four 16-lane groups of a fragment read (k columns kk .. kk + 3)
// then fall on banks 0-31, 32-63, 0-31, 32-63, two conflict-free passes; with
// LROW = 132 (an 8-bank shift per column) groups 0 and 1 overlap.  The panel
// solve keeps LROW, whose smaller stages let three workgroups share a CU.
constexpr int LROW_UPD = 144;
constexpr int UPD_DMA_LDS_BYTES = 2 * 2 * 16 * LROW_UPD * 8;

template <int KC, int NST, int LR = LROW>
constexpr int dma_lds_bytes() { return NST * 2 * KC * LR * 8; }

template <bool TRI, int KC = 16, int NST = 2, bool SPLIT = false, int LR = LROW>
__device__ __forceinline__ void wg_gemm_nt_dma(d4 (&acc)[4][4], double* lds,
                                               const double* __restrict__ A,
                                               const double* __restrict__ B, int kmax,
                                               bool do_mfma, int nrb = 8) {
  constexpr int STG = 2 * KC * LR, CPW = 2 * KC / 4;  // columns per wave and chunk
  static_assert(NST == 2 || NST == 3, "two or three stages");
  static_assert(KC % 8 == 0 && CPW <= 15, "whole k-steps; vmcnt holds one chunk");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = __builtin_amdgcn_readfirstlane(kmax) / KC;
  if (nchunks <= 0) return;
  do_mfma = __builtin_amdgcn_readfirstlane((int)do_mfma) != 0;
  nrb = __builtin_amdgcn_readfirstlane(nrb);
  // wave w moves columns CPW w .. CPW w + CPW - 1 of the chunk's 2 KC (A, then B)
  auto request = [&](int c, int stage) {
#pragma unroll
    for (int h = 0; h < CPW; ++h) {
      const int col = CPW * wave + h;
      const bool isb = col >= KC;
      const double* src = (isb ? B : A) + (int64_t)(c * KC + col - (isb ? KC : 0)) * T + 2 * lane;
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                       (lds_void*)(lds + stage * STG + col * LR),
                                       16, 0, 0);
    }
  };
#pragma unroll
  for (int p = 0; p < NST - 1; ++p)
    if (p < nchunks) request(p, p);
  const int lr = lane & 15, lk = lane >> 4;
  int stage = 0;
  for (int c = 0; c < nchunks; ++c) {
    // chunk c in LDS; chunk c - 1's stage free
    if (NST == 2 || c + 1 == nchunks) vmcnt_barrier<0>();
    else vmcnt_barrier<CPW>();
    if (c + NST - 1 < nchunks) request(c + NST - 1, stage == 0 ? NST - 1 : stage - 1);
    if constexpr (SPLIT) {
      // the wave's two output block columns (TRI: w and 7 - w, 9 nonzero
      // k blocks between them; each runs while its k blocks last)
      const int g0 = TRI ? wave : 2 * wave, g1 = TRI ? 7 - wave : 2 * wave + 1;
      const bool on0 = !TRI || 16 * (g0 + 1) > c * KC, on1 = !TRI || 16 * (g1 + 1) > c * KC;
      const double* sa = lds + stage * STG + lr;
      const double* sb = lds + stage * STG + KC * LR + lr;
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = sa[kk * LR + 16 * i];
        const double b0 = sb[kk * LR + 16 * g0], b1 = sb[kk * LR + 16 * g1];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          if (i < nrb && on0) acc[i >> 1][2 * (i & 1)] = MF<double>::op(b0, a[i], acc[i >> 1][2 * (i & 1)]);
          if (i < nrb && on1) acc[i >> 1][2 * (i & 1) + 1] = MF<double>::op(b1, a[i], acc[i >> 1][2 * (i & 1) + 1]);
        }
      }
      if (++stage == NST) stage = 0;
      continue;
    }
    const int jlo = TRI ? tri_lo(wc, c * KC) : 0;
    if (do_mfma && jlo < 4) {
      const double* sa = lds + stage * STG + 64 * wr + lr;
      const double* sb = lds + stage * STG + KC * LR + (TRI ? 0 : 64 * wc) + lr;
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = sa[kk * LR + 16 * i];
          b[i] = sb[kk * LR + 16 * (TRI ? tri_blk(wc, i) : i)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (!TRI || j >= jlo) acc[i][j] = MF<double>::op(b[j], a[i], acc[i][j]);
      }
    }
    if (++stage == NST) stage = 0;
  }
  __syncthreads();  // the last stage is read before the caller reuses LDS
}

// ---- tile tasks -------------------------------------------------------------------

// Left-looking update of tile (I, J), I >= J: C_IJ -= L_I,0:J L_J,0:J^T (FP64 MFMA).
// DEPTH: chunks of the k range prefetched into registers (2 for the step
// kernels; 1 where the caller is register-bound, the persistent batch kernel).
template <bool VEC, int DEPTH = 2>
__device__ __forceinline__ void dev_gemm_col(const Lay& lay, double* base, int J, int I, double* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  const int war = arows - 64 * wr, wbr = brows - 64 * wc;
  const int ni = nblk(war), nj = nblk(wbr);
  const bool act = ni > 0 && nj > 0 && !(I == J && wc > wr);
  const int kmax = min(J * T, lay.n);
  d4 acc[4][4];
  zero_acc<double>(acc);
  wg_gemm_nt<double, double, VEC, 4, DEPTH>(acc, lds, base + lay.tile_off(I, 0), lay.tile_ld(I), arows,
                                  base + lay.tile_off(J, 0), lay.tile_ld(J), brows, kmax, act, ni);
  if (act) {
    const int64_t ldc = lay.tile_ld(I);
    double* C = base + lay.tile_off(I, J) + 64 * wr + 64 * wc * ldc;
    store64<double, true, double, double, (DEPTH > 1)>(C, ldc, C, ldc, acc, war, wbr, lane);
  }
}

// C -= acc for the column-split plan of wg_gemm_nt_dma (wave w; rows below
// arows, columns below brows valid; leading dimension ldc).  The loads of a
// slot row's four blocks are issued together, as in store64_l.
template <typename LAYOUT = double, typename TI = double, typename TO = double>
__device__ __forceinline__ void sub_store_split(const TI* Cin, int64_t ldin, TO* Cout,
                                                int64_t ldout, const d4 (&acc)[4][4], int w,
                                                int arows, int brows, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  arows = __builtin_amdgcn_readfirstlane(arows);
  brows = __builtin_amdgcn_readfirstlane(brows);
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    if (32 * ii >= arows) break;
    double cin[4][4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int rc = min(16 * (2 * ii + (jj >> 1)) + lr, arows - 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int cc = min(32 * w + 16 * (jj & 1) + MF<LAYOUT>::col(lg, e), brows - 1);
        cin[jj][e] = (double)Cin[(int64_t)cc * ldin + rc];
      }
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = 16 * (2 * ii + (jj >> 1)) + lr;
      if (r >= arows) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 32 * w + 16 * (jj & 1) + MF<LAYOUT>::col(lg, e);
        if (c < brows) Cout[(int64_t)c * ldout + r] = (TO)(cin[jj][e] - acc[ii][jj][e]);
      }
    }
  }
}

// dev_gemm_col on the direct-to-LDS core: tile (I, J) with I < Nv of the
// packed layout (whole T x T tiles; L_I,0:J and L_J,0:J are column-major
// panels of leading dimension T).
__device__ __forceinline__ void dev_gemm_col_dma(const Lay& lay, double* base, int J, int I,
                                                 double* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  if (arows <= 0 || brows <= 0) return;  // a tile past an uneven unit's order (uniform)
  d4 acc[4][4];
  zero_acc<double>(acc);
  const int kmax = min(J * T, lay.n);
  if (arows < T) {
    // the last tile row: column-split plan
    const int nrb = (arows + 15) >> 4;
    wg_gemm_nt_dma<false, 16, 2, true, LROW_UPD>(acc, lds, base + lay.tile_off(I, 0),
                                                 base + lay.tile_off(J, 0), kmax, true, nrb);
    double* C = base + lay.tile_off(I, J);
    sub_store_split(C, T, C, T, acc, wave, arows, brows, lane);
    return;
  }
  const int war = arows - 64 * wr, wbr = brows - 64 * wc;
  const bool act = war > 0 && wbr > 0;
  wg_gemm_nt_dma<false, 16, 2, false, LROW_UPD>(acc, lds, base + lay.tile_off(I, 0),
                                                base + lay.tile_off(J, 0), kmax, act);
  if (act) {
    double* C = base + lay.tile_off(I, J) + 64 * wr + 64 * wc * T;
    store64<double, true, double, double>(C, T, C, T, acc, war, wbr, lane);
  }
}

// Chunks of 8 columns in three stages for the FP64 panel solve (49.5 KB of
// LDS, so three workgroups share a CU).
constexpr int TRSM_KC = 8, TRSM_NST = 3;

// L_IJ = C_IJ W^T (FP64, TRI column map) on the direct-to-LDS core: tile
// (I, J) with I < Nv of the packed layout.
template <int KC, int NST>
__device__ __forceinline__ void dev_trsm_dma(const Lay& lay, double* base, const double* W, int J,
                                             int I, double* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  if (arows <= 0 || brows <= 0) return;  // a tile past an uneven unit's order (uniform)
  const int war = arows - 64 * wr;
  const bool act = war > 0 && 16 * tri_blk(wc, 0) < brows;
  double* Ct = base + lay.tile_off(I, J);
  d4 acc[4][4];
  zero_acc<double>(acc);
  const int lr = lane & 15, lg = lane >> 4;
  if (arows < T) {
    // the last tile row: column-split plan, block columns w and 7 - w
    wg_gemm_nt_dma<true, KC, NST, true>(acc, lds, Ct, W, T, true, (arows + 15) >> 4);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = 16 * i + lr;
      if (r >= arows) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int cb = 16 * (h ? 7 - wave : wave);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = cb + MF<double>::col(lg, e);
          if (c < brows) Ct[(int64_t)c * T + r] = acc[i >> 1][2 * (i & 1) + h][e];
        }
      }
    }
    return;
  }
  // the core's barriers order every read of C_IJ before the overwrite
  wg_gemm_nt_dma<true, KC, NST>(acc, lds, Ct, W, T, act);
  if (!act) return;
  double* Cw = Ct + 64 * wr;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * i + lr;
    if (r >= war) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cb = 16 * tri_blk(wc, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = cb + MF<double>::col(lg, e);
        if (c < brows) Cw[(int64_t)c * T + r] = acc[i][j][e];
      }
    }
  }
}

// Mixed-form panel solve of a whole packed tile (I < Nv), FP32 storage:
// wg_gemm_nt_f32dma_f64 with the TRI column map, L rounded to FP32 once.
constexpr int TRSM_MX_KC = 8, TRSM_MX_NST = 3;

__device__ __forceinline__ void dev_trsm_mx_dma(const Lay& lay, float* base, const float* W,
                                                int J, int I, float* lds) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int war = lay.rows(I) - 64 * wr, brows = lay.rows(J);
  const bool act = war > 0 && 16 * tri_blk(wc, 0) < brows;
  float* Ct = base + lay.tile_off(I, J);
  d4 acc[4][4];
  zero_acc<double>(acc);
  // the core's final barrier orders every read of C_IJ before the overwrite
  wg_gemm_nt_f32dma_f64<TRSM_MX_KC, TRSM_MX_NST>(acc, lds, Ct, W, T, act);
  if (!act) return;
  const int lr = lane & 15, lg = lane >> 4;
  float* Cw = Ct + 64 * wr;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 16 * i + lr;
    if (r >= war) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cb = 16 * tri_blk(wc, j);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = cb + MF<double>::col(lg, e);
        if (c < brows) Cw[(int64_t)c * T + r] = (float)acc[i][j][e];
      }
    }
  }
}

// L_NvJ = C_NvJ W^T for the bordered row's tile (q valid rows of TB = 16 NBR,
// leading dimension TB) without LDS: wave w computes the output block
// columns w and 7 - w (w + 1 and 8 - w nonzero k-blocks of W^T: the same
// count for every wave) over all NBR block rows, with fragments loaded
// straight from global memory (16 lanes read 16 consecutive rows of one
// column), four k-steps per batch of loads; columns at or beyond brows (the
// last block column's padding, which need not hold finite values in C or W)
// read as zero.  One barrier separates the last read of C from the first
// write of L (the waves read columns that others write).  TS float: the mixed form's FP32 storage, widened on the load and
// rounded once on the store (the MFMA is FP64).
template <int NBR, typename TS = double>
__device__ __forceinline__ void dev_trsm_border(const Lay& lay, TS* base, const TS* W, int J) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  TS* C = base + lay.tile_off(lay.Nv, J);
  const int64_t ld = lay.TB;
  const int q = lay.q, brows = lay.rows(J);
  const int g0 = w, g1 = 7 - w;         // g1 > g0: the longer k range
  const int nsteps = 4 * (g1 + 1);      // 4-deep k-steps up to k = 16 (g1 + 1)
  d4 acc[NBR][2];
#pragma unroll
  for (int ib = 0; ib < NBR; ++ib) acc[ib][0] = acc[ib][1] = d4{0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < nsteps; s0 += 4) {
    double a[4][NBR], b[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = 4 * (s0 + u) + lk;
#pragma unroll
      for (int ib = 0; ib < NBR; ++ib)
        a[u][ib] = kk < brows ? (double)C[(int64_t)kk * ld + 16 * ib + lr] : 0.0;
      b[u][0] = kk < brows ? (double)W[(int64_t)kk * T + 16 * g0 + lr] : 0.0;
      b[u][1] = kk < brows ? (double)W[(int64_t)kk * T + 16 * g1 + lr] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool first = 4 * (s0 + u) < 16 * (g0 + 1);  // uniform
#pragma unroll
      for (int ib = 0; ib < NBR; ++ib) {
        if (first) acc[ib][0] = MF<double>::op(b[u][0], a[u][ib], acc[ib][0]);
        acc[ib][1] = MF<double>::op(b[u][1], a[u][ib], acc[ib][1]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int ib = 0; ib < NBR; ++ib) {
    const int r = 16 * ib + lr;
    if (r >= q) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cb = 16 * (h ? g1 : g0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = cb + MF<double>::col(lk, e);
        if (c < brows) C[(int64_t)c * ld + r] = (TS)acc[ib][h][e];
      }
    }
  }
}

// Panel solve of tile (I, J), I > J: L_IJ = C_IJ W^T with W = L_JJ^-1 (ld T).
// The FP64 two-set pipeline (step kernels) uses the TRI column map; the FP32
// form skips the chunks its first wave column does not need (HALF); the
// persistent batch kernel's one-set pipeline keeps the plain halves.  The
// mixed form's whole packed tiles take dev_trsm_mx_dma instead.
template <typename TS, bool VEC, int FLUSH, int DEPTH = 2>
__device__ __forceinline__ void dev_trsm(const Lay& lay, TS* base, const TS* W, int J, int I, TS* lds) {
  constexpr bool TRI = sizeof(TS) == 8 && DEPTH > 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const int arows = lay.rows(I), brows = lay.rows(J);
  const int war = arows - 64 * wr, wbr = brows - 64 * wc;
  const int ni = nblk(war);
  const bool act = ni > 0 && (TRI ? 16 * tri_blk(wc, 0) < brows : wbr > 0);
  TS* Ct = base + lay.tile_off(I, J);
  const int64_t ldc = lay.tile_ld(I);
  d4 acc[4][4];
  zero_acc<double>(acc);
  // the core's final barrier orders every read of C_IJ before the overwrite
  if constexpr (sizeof(TS) == 8) {
    wg_gemm_nt<TS, TS, VEC, 4, DEPTH, TRI>(acc, lds, Ct, ldc, arows, W, T, brows, brows, act, ni);
  } else {
    wg_gemm_nt_f32x64<FLUSH, true>(acc, lds, Ct, ldc, arows, W, T, brows, brows, act, ni);
  }
  if (!act) return;
  if constexpr (TRI) {
    // block (i, j) of the wave is rows 64 wr + 16 i, columns 16 tri_blk(wc, j)
    const int lr = lane & 15, lg = lane >> 4;
    TS* Cw = Ct + 64 * wr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * i + lr;
      if (r >= war) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int cb = 16 * tri_blk(wc, j);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = cb + MF<double>::col(lg, e);
          if (c < brows) Cw[(int64_t)c * ldc + r] = acc[i][j][e];
        }
      }
    }
  } else {
    TS* Co = Ct + 64 * wr + 64 * wc * ldc;
    if constexpr (sizeof(TS) == 8) store64<double, false>(Co, ldc, Co, ldc, acc, war, wbr, lane);
    else store64_l<float, false>(Co, ldc, Co, ldc, acc, war, wbr, lane);
  }
}

// ---- diagonal tile and bordered row of block column J in one workgroup -----------
// The diagonal tile's update is P P^T with P = L_J,0:J, so LDS holds that
// panel once per chunk.  Waves (0,0), (1,0) and (1,1) compute the lower
// quadrants as in wg_gemm_nt.  Wave (0,1), whose quadrant lies above the
// diagonal, computes the bordered row's tile instead: Q P^T with Q the
// bordered rows' panel (NBR = TB / 16 <= 2 block rows) against all 8 block
// columns of P -- 8 NBR MFMA blocks, at most the 16 of a quadrant.  Border
// block (ib, jb) lives in acc[2 ib + jb / 4][jb % 4].  Both roles run one
// MFMA stream, acc[i][j] += B-fragment (i & 1, j) x A-fragment i, with
// per-wave LDS offsets (two separate MFMA streams over the same accumulators
// make the register allocator spill): a quadrant wave reads the same four
// B fragments twice, the border wave two halves of P.  Rows at or beyond
// prows / qrows and columns at or beyond kmax read as zero.
//
// BAL: the balanced plan.  The quadrant plan gives one wave the 16 blocks of
// the lower-left quadrant while the others run 10 (the diagonal quadrants'
// lower blocks) or 8 NBR, and a compute unit's waves of one index share a
// SIMD, so the tile takes as long as 16 blocks on every SIMD.  In the
// balanced plan wave w takes block columns w and 7 - w of the lower
// triangle and their bordered-row blocks: 9 + 2 NBR blocks on every wave,
// in fixed accumulator slots (the guards are uniform):
//   acc[i][j], i < 2 : block (4 i + j, w),    run for 4 i + j >= w
//   acc[2][j]        : block (4 + j, 7 - w),  run for 4 + j >= 7 - w
//   acc[3][j]        : bordered block (j & 1, j < 2 ? w : 7 - w)
// Row blocks at or beyond prows are skipped as well (the last diagonal
// tile).  Blocks above the diagonal are not updated (nothing reads them).
constexpr int LQ = 32 + 4;  // LDS stride per k column of the bordered panel
constexpr int DIAG_LDS_BYTES = 2 * 16 * (LROW + LQ) * 8;
static_assert(DIAG_LDS_BYTES <= GEMM_LDS_BYTES, "the diagonal core shares the GEMM LDS");

template <bool VEC, typename TS = double, bool BAL = false>
__device__ __forceinline__ void wg_gemm_diag_border(d4 (&acc)[4][4], TS* lds,
                                                    const TS* __restrict__ P, int prows,
                                                    const TS* __restrict__ Q, int64_t ldq,
                                                    int qrows, int nbr, int kmax,
                                                    int64_t ldp = T) {
  // TS: storage of the panels (FP64, or FP32 in the mixed form); the MFMA is FP64
  // ldp: leading dimension of P (T in the packed layout)
  constexpr int N = Piece<TS>::N, KC = 128 / (int)sizeof(TS), PPC = T / N;
  constexpr int STAGE = KC * (LROW + LQ);
  typedef typename Piece<TS>::type V;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int nchunks = (kmax + KC - 1) / KC;
  if (nchunks <= 0) return;
  nbr = __builtin_amdgcn_readfirstlane(nbr);
  const bool border_wave = wr == 0 && wc == 1;
  // per-wave MFMA plan (uniform): block rows run, LDS offsets of the A
  // fragments (with their k stride) and of the two B fragment sets
  const int nie = __builtin_amdgcn_readfirstlane(border_wave ? 2 * nbr : nblk(prows - 64 * wr));
  const int astr = border_wave ? LQ : LROW;
  // A fragment i at abase + 16 (i >> ash); B fragment set h at bb0 + h * bdh
  const int abase = border_wave ? KC * LROW : 64 * wr;
  const int ash = border_wave ? 1 : 0;
  const int bb0 = border_wave ? 0 : 64 * wc;
  const int bdh = border_wave ? 64 : 0;
  const int qppc = nbr * 16 / N;  // pieces per column of Q
  const int qpieces = KC * qppc;  // at most 256: at most one per thread
  V rp[2][4], rq[2];
  auto fetch = [&](int k0, auto setc) {
    constexpr int S = decltype(setc)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      rp[S][q] = fetch_piece<TS, VEC>(P, ldp, prows, k0 + col, kmax, row);
    }
    if (tid < qpieces) {
      const int col = tid / qppc, row = (tid % qppc) * N;
      rq[S] = fetch_piece<TS, VEC>(Q, ldq, qrows, k0 + col, kmax, row);
    }
  };
  auto stash = [&](auto setc) {
    constexpr int S = decltype(setc)::value;
    TS* sp = lds + S * STAGE;
    TS* sq = sp + KC * LROW;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + 256 * q;
      const int col = idx / PPC, row = (idx % PPC) * N;
      *reinterpret_cast<V*>(sp + col * LROW + row) = rp[S][q];
    }
    if (tid < qpieces) {
      const int col = tid / qppc, row = (tid % qppc) * N;
      *reinterpret_cast<V*>(sq + col * LQ + row) = rq[S];
    }
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  fetch(0, S0{});
  if (nchunks > 1) fetch(KC, S1{});
  stash(S0{});
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  // balanced plan (uniform): the wave's two block columns, valid row blocks
  const int c0 = wave, c1 = 7 - wave;
  const int nrb = __builtin_amdgcn_readfirstlane((min(prows, T) + 15) >> 4);
  auto step = [&](int c, auto setc, auto other) {
    constexpr int S = decltype(setc)::value;
    if (c + 2 < nchunks) fetch((c + 2) * KC, setc);
    const TS* st = lds + S * STAGE + lr;
    if constexpr (BAL) {
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kk = 4 * s4 + lk;
        double a[8], q[2];
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i] = (double)st[kk * LROW + 16 * i];
        const double b0 = (double)st[kk * LROW + 16 * c0];
        const double b1 = (double)st[kk * LROW + 16 * c1];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) q[ib] = (double)st[KC * LROW + kk * LQ + 16 * ib];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (4 * i + j >= c0 && 4 * i + j < nrb)
              acc[i][j] = MF<double>::op(b0, a[4 * i + j], acc[i][j]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 + j >= c1 && 4 + j < nrb) acc[2][j] = MF<double>::op(b1, a[4 + j], acc[2][j]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((j & 1) < nbr && (j < 2 ? c0 : c1) < nrb)
            acc[3][j] = MF<double>::op(j < 2 ? b0 : b1, q[j & 1], acc[3][j]);
      }
      if (c + 1 < nchunks) stash(other);
      __syncthreads();
      return;
    }
#pragma unroll
    for (int s4 = 0; s4 < KC / 4; ++s4) {
      const int kk = 4 * s4 + lk;
      double a[4], b[2][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (double)st[kk * astr + abase + 16 * (i >> ash)];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[h][j] = (double)st[kk * LROW + bb0 + h * bdh + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < nie) {
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = MF<double>::op(b[i & 1][j], a[i], acc[i][j]);
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

// The balanced plan of wg_gemm_diag_border on direct-to-LDS loads, for the
// packed layout: P = L_J,0:J is a whole-tile panel (leading dimension T) and
// the bordered rows' panel Q (nbr <= 2 block rows, leading dimension
// TB = 16 nbr) is contiguous, so a chunk of KC = 16 of its columns is TB / 8
// pieces of 1 KB.  Per chunk: 16 P columns (four per wave) and the Q pieces
// (waves 0 .. TB / 8 - 1), two stages published as in wg_gemm_nt_dma.  kmax is
// a multiple of 16 (J T).
constexpr int DIAG_DMA_KC = 16;
constexpr int DIAG_DMA_STG = DIAG_DMA_KC * LROW_UPD + DIAG_DMA_KC * 32;  // doubles per stage
static_assert(2 * DIAG_DMA_STG * 8 <= UPD_DMA_LDS_BYTES, "the diagonal core shares the update's LDS");

__device__ __forceinline__ void wg_gemm_diag_dma(d4 (&acc)[4][4], double* lds,
                                                 const double* __restrict__ P, int prows,
                                                 const double* __restrict__ Q, int nbr, int kmax) {
  constexpr int KC = DIAG_DMA_KC, STG = DIAG_DMA_STG, CPW = KC / 4;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nchunks = __builtin_amdgcn_readfirstlane(kmax) / KC;
  if (nchunks <= 0) return;
  nbr = __builtin_amdgcn_readfirstlane(nbr);
  const int tb = 16 * nbr, qpieces = 2 * nbr;  // KC tb doubles = qpieces KB
  auto request = [&](int c, int stage) {
    double* st = lds + stage * STG;
#pragma unroll
    for (int h = 0; h < CPW; ++h) {
      const int col = CPW * wave + h;
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const void*>(P + (int64_t)(c * KC + col) * T + 2 * lane),
          (lds_void*)(st + col * LROW_UPD), 16, 0, 0);
    }
    if (wave < qpieces)
      __builtin_amdgcn_global_load_lds(
          reinterpret_cast<const void*>(Q + (int64_t)c * KC * tb + 128 * wave + 2 * lane),
          (lds_void*)(st + KC * LROW_UPD + 128 * wave), 16, 0, 0);
  };
  request(0, 0);
  const int lr = lane & 15, lk = lane >> 4;
  const int c0 = wave, c1 = 7 - wave;
  const int nrb = __builtin_amdgcn_readfirstlane((min(prows, T) + 15) >> 4);
  for (int c = 0; c < nchunks; ++c) {
    const int stage = c & 1;
    vmcnt_barrier<0>();  // chunk c in LDS; chunk c - 1's stage free
    if (c + 1 < nchunks) request(c + 1, stage ^ 1);
    const double* sp = lds + stage * STG + lr;
    const double* sq = lds + stage * STG + KC * LROW_UPD + lr;
#pragma unroll
    for (int s4 = 0; s4 < KC / 4; ++s4) {
      const int kk = 4 * s4 + lk;
      double a[8], q[2];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = sp[kk * LROW_UPD + 16 * i];
      const double b0 = sp[kk * LROW_UPD + 16 * c0], b1 = sp[kk * LROW_UPD + 16 * c1];
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) q[ib] = sq[kk * tb + 16 * ib];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * i + j >= c0 && 4 * i + j < nrb)
            acc[i][j] = MF<double>::op(b0, a[4 * i + j], acc[i][j]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (4 + j >= c1 && 4 + j < nrb) acc[2][j] = MF<double>::op(b1, a[4 + j], acc[2][j]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if ((j & 1) < nbr && (j < 2 ? c0 : c1) < nrb)
          acc[3][j] = MF<double>::op(j < 2 ? b0 : b1, q[j & 1], acc[3][j]);
    }
  }
  __syncthreads();  // the last stage is read before the caller reuses LDS
}

// C -= acc for the balanced plan of wg_gemm_diag_border (wave w): C the
// diagonal tile (leading dimension ldc, prows valid rows and columns), Cb the
// bordered row's tile (leading dimension ldb, qrows valid rows, nbr block
// rows).  The loads of a slot row's four blocks are issued together, as in
// store64_l.
template <typename TI = double, typename TO = double, typename TBR = double>
__device__ __forceinline__ void sub_store_diag_bal(const TI* Cin, int64_t ldin, TO* Cout,
                                                   int64_t ldout, TBR* Cb, int64_t ldb,
                                                   const d4 (&acc)[4][4], int w, int prows,
                                                   int qrows, int nbr, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  prows = __builtin_amdgcn_readfirstlane(prows);
  qrows = __builtin_amdgcn_readfirstlane(qrows);
  nbr = __builtin_amdgcn_readfirstlane(nbr);
  const int c1 = 7 - w;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double cin[4][4];
    bool ok[4];
    int rb[4], cb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (i < 2) {
        rb[j] = 4 * i + j;
        cb[j] = w;
        ok[j] = rb[j] >= w;
      } else if (i == 2) {
        rb[j] = 4 + j;
        cb[j] = c1;
        ok[j] = rb[j] >= c1;
      } else {
        rb[j] = j & 1;
        cb[j] = j < 2 ? w : c1;
        ok[j] = rb[j] < nbr;
      }
      const int rmax = i < 3 ? prows : qrows;
      ok[j] = ok[j] && 16 * rb[j] < rmax && 16 * cb[j] < prows;
      const int rc = max(min(16 * rb[j] + lr, rmax - 1), 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int cc = max(min(16 * cb[j] + MF<double>::col(lg, e), prows - 1), 0);
        cin[j][e] = 0.0;
        if (ok[j]) {
          if (i < 3) cin[j][e] = (double)Cin[(int64_t)cc * ldin + rc];
          else cin[j][e] = (double)Cb[(int64_t)cc * ldb + rc];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rmax = i < 3 ? prows : qrows;
      const int r = 16 * rb[j] + lr;
      if (!ok[j] || r >= rmax) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * cb[j] + MF<double>::col(lg, e);
        if (c >= prows) continue;
        const double v = cin[j][e] - acc[i][j][e];
        if (i < 3) Cout[(int64_t)c * ldout + r] = (TO)v;
        else Cb[(int64_t)c * ldb + r] = (TBR)v;
      }
    }
  }
}

// C_JJ -= L_J,0:J L_J,0:J^T and, when `border` (TB <= 32), the bordered row's
// tile C_NvJ -= L_Nv,0:J L_J,0:J^T, in one workgroup (balanced plan; VEC:
// direct-to-LDS loads, wg_gemm_diag_dma; else wg_gemm_diag_border).  Packed
// layout, 0 < J < Nv.
template <bool VEC>
__device__ __forceinline__ void dev_gemm_diag_border(const Lay& lay, double* base, int J,
                                                     bool border, double* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int prows = lay.rows(J);
  const int qrows = border ? lay.q : 0;
  const int nbr = border ? lay.TB / 16 : 0;
  const int kmax = min(J * T, lay.n);
  if (prows <= 0 || kmax <= 0) return;
  d4 acc[4][4];
  zero_acc<double>(acc);
  if constexpr (VEC)  // packed layout, J < Nv: kmax = J T
    wg_gemm_diag_dma(acc, lds, base + lay.tile_off(J, 0), prows, base + lay.tile_off(lay.Nv, 0),
                     nbr, kmax);
  else
    wg_gemm_diag_border<VEC, double, true>(acc, lds, base + lay.tile_off(J, 0), prows,
                                           base + lay.tile_off(lay.Nv, 0), lay.TB, qrows, nbr,
                                           kmax);
  double* C = base + lay.tile_off(J, J);
  sub_store_diag_bal(C, T, C, T, base + lay.tile_off(lay.Nv, J), lay.TB, acc, wave, prows, qrows,
                     nbr, lane);
}

// Diagonal tile J: factor and invert, register-blocked.
// Thread t owns the 8x8 block (rows 8*(t/16).., columns 8*(t%16)..) of the
// unit-padded tile; LDS only broadcasts one column (and one row) per step, with
// two alternating buffers so that a single barrier separates the steps.
//  factor (right-looking): publish column j unscaled; every owner of a lower
//    block updates a_rc -= a_rj a_cj / a_jj for c > j; owners of column j
//    scale it by 1/sqrt(a_jj).
//  inverse (in place, W = L^-1 row by row): at step m scale W's row m by
//    1/L_mm (it then holds its final values), publish it and L's column m;
//    W_rc -= L_rm W_mc for r > m, c < m; W_rm = -L_rm / L_mm; W_mm = 1/L_mm.
// C (leading dimension ld) holds the tile's lower triangle.  MODE 0: L is
// written back to C and W (FP64, ld T) to Wd.  MODE 1: C is read only and W is
// written in FP32 to W32.  MODE 2: as MODE 1, and L is rounded to FP32 into
// L32 (leading dimension ld32).  log|V| is added to *logdet_k; a non-positive
// pivot sets *info_k and returns (uniformly).  smem: at least 5*T + 256
// doubles.
constexpr int POTRF_SMEM_DOUBLES = 5 * T + 256;

template <int MODE>
__device__ __forceinline__ void dev_potrf(const Lay& lay, double* C, int64_t ld, double* Wd,
                                          float* W32, double* logdet_k, int32_t* info_k, int J,
                                          double* smem, float* L32 = nullptr, int64_t ld32 = 0) {
  double (*bc0)[T] = reinterpret_cast<double (*)[T]>(smem);
  double (*bc1)[T] = reinterpret_cast<double (*)[T]>(smem + 2 * T);
  double* dinv = smem + 4 * T;
  double* red = smem + 5 * T;
  const int tid = threadIdx.x, bi = tid >> 4, bj = tid & 15;
  const bool low = bi >= bj;
  const int nv = lay.rows(J);
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
        if (tid == 0) *info_k = J * T + j + 1;
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
  if (MODE == 2 && low) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        if (r < nv && c < nv && r >= c) L32[(int64_t)c * ld32 + r] = (float)a[rr][cc];
      }
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) *logdet_k += 2.0 * red[0];

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
    double* W = Wd;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        W[c * T + r] = (low && r >= c) ? a[rr][cc] : 0.0;
      }
  } else {
    float* W = W32;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        W[c * T + r] = (low && r >= c) ? (float)a[rr][cc] : 0.0f;
      }
  }
}

// ---- diagonal tile, 2 x 2 blocked: factor and invert -----------------------------
// The tile (identity-padded beyond nv) splits into 64 x 64 blocks
//   [A11 .  ]   [L11  0 ] [L11^T L21^T]        W = L^-1 = [W11  0 ]
//   [A21 A22] = [L21 L22] [ 0    L22^T],                  [W21 W22]
// with L21 = A21 W11^T, L22 L22^T = A22 - L21 L21^T, W21 = -W22 (L21 W11).
// Each diagonal block is factored and inverted by one wave alone in registers
// (wave64_chol_inv: lane (bi, bj) owns the 8 x 8 block at rows 8 bi, columns
// 8 bj; one column or row is broadcast through LDS per step; the wave's LDS
// operations complete in order, so no barrier is needed).  The three
// off-diagonal products run on FP64 MFMA, wave w taking block row or column
// w, operands in LDS.  256 threads; results, outputs and failure semantics as
// dev_potrf (the first non-positive pivot sets *info_k; the workgroup then
// returns uniformly).  smem: at least POTRF_BLK_SMEM_DOUBLES.
constexpr int PB_LS = 65;  // LDS column stride of a 64 x 64 block
constexpr int POTRF_BLK_SMEM_DOUBLES = 2 * 64 * PB_LS + 64 + 8;

// LDS hand-off between the lanes of one wave: its LDS operations execute in
// order, so only the compiler has to be kept from moving or forwarding
// accesses across this point (a wavefront-scope fence).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// 1 / sqrt(d) for d > 0: the hardware estimate (v_rsq_f64) refined by two
// Newton-Raphson steps y <- y (3 - d y^2) / 2, each squaring the relative
// error: a few ulps, with a short dependent chain (the correctly rounded
// division and square root take about 30 dependent instructions).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y;
}

// Factor (and then invert) the 64 x 64 block held in a[8][8] by the 64 lanes
// of one wave.  nvb: valid order of the block (rows at or beyond it are the
// identity).  On return a holds W = L^-1 (lower, garbage above the diagonal)
// and Lout receives L through put_l(r, c, v) for every valid r >= c; sl gets
// the sum of log L_jj over valid j.  Returns the first failing column + 1
// (0: success).  colbuf and rowbuf hold two 64-double buffers each, dinv 64.
//
// Both sweeps look one step ahead, so that a step's latency chain (LDS
// round trip, reciprocal square root) runs under the previous step's bulk
// arithmetic: step j first updates column j + 1 (8 of the lane's 64 FMAs),
// publishes it to the other buffer and reads the next pivot from its owner
// lane, and only then runs its other 56 FMAs.  The inverse does the same
// with row m + 1 of W, which step m completes and scales before its bulk
// update (L's columns do not change during the inverse, so column m + 1 is
// published at the start of step m).
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename PutL>
__device__ __forceinline__ int wave64_chol_inv(double (&a)[8][8], int nvb, double* colbuf,
                                               double* rowbuf, double* dinv, double& sl,
                                               PutL put_l) {
  const int lane = threadIdx.x & 63, bi = lane >> 3, bj = lane & 7;
  const bool low = bi >= bj;
  // ---- factor, right-looking: column j unscaled in colbuf[j & 1]
  if (bj == 0) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) colbuf[8 * bi + rr] = a[rr][0];
  }
  wave_lds_sync();
  double d = lane_bcast(a[0][0], 0);  // the pivot, from its owner lane
  for (int jb = 0; jb < 8; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int j = 8 * jb + jj;
      const double* cb = colbuf + 64 * (jj & 1);
      double cr[8], cc8[8];
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) cr[rr] = cb[8 * bi + rr];
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) cc8[c8] = cb[8 * bj + c8];
      if (!(d > 0.0)) return j + 1;
      const double rs = rsqrt_nr(d);  // 1 / L_jj
      if (lane == 0) dinv[j] = rs;
      const int cn = (jj + 1) & 7;  // lane column of column j + 1
      const int jbn = jj == 7 ? jb + 1 : jb;
      const bool more = j + 1 < 64;
      if (low && bj >= jb) {
        const double invd = rs * rs;
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) cr[rr] *= invd;
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) cc8[c8] = (bj > jb || c8 > jj) ? cc8[c8] : 0.0;
        // column j + 1 first, then its publication
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) a[rr][cn] = fma(-cr[rr], cc8[cn], a[rr][cn]);
        if (more && bj == jbn) {
          double* nb = colbuf + 64 * ((jj + 1) & 1);
#pragma unroll
          for (int rr = 0; rr < 8; ++rr) nb[8 * bi + rr] = a[rr][cn];
        }
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
#pragma unroll
          for (int c8 = 0; c8 < 8; ++c8)
            if (c8 != cn) a[rr][c8] = fma(-cr[rr], cc8[c8], a[rr][c8]);
        if (bj == jb) {
#pragma unroll
          for (int rr = 0; rr < 8; ++rr)
            if (bi > jb || rr >= jj) a[rr][jj] *= rs;
        }
      }
      if (more) d = lane_bcast(a[cn][cn], 9 * jbn);
      wave_lds_sync();  // keeps this step's LDS accesses before the next step's
    }
  }
  // L is final (dinv holds 1 / L_jj): hand it out, log L_jj
  sl = 0.0;
  if (low) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        if (r < nvb && c < nvb && r >= c) put_l(r, c, a[rr][cc]);
      }
  }
  if (bi == bj) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
      if (8 * bi + rr < nvb) sl += log(a[rr][rr]);
  }
  // ---- inverse, row by row: L's column m in colbuf[m & 1], W's final row m
  // (columns below m) in rowbuf[m & 1]; row 0 has no such columns
  if (low && bj == 0) {
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) colbuf[8 * bi + rr] = a[rr][0];
  }
  wave_lds_sync();
  for (int mb = 0; mb < 8; ++mb) {
#pragma unroll
    for (int mm = 0; mm < 8; ++mm) {
      const int m = 8 * mb + mm;
      const int rn = (mm + 1) & 7;  // lane row of row m + 1
      const int mbn = mm == 7 ? mb + 1 : mb;
      const bool more = m + 1 < 64;
      const int p = mm & 1;
      double lr[8], wv[8];
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) lr[rr] = colbuf[64 * p + 8 * bi + rr];
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) wv[c8] = rowbuf[64 * p + 8 * bj + c8];
      const double wmm = dinv[m];
      const double wn = more ? dinv[m + 1] : 0.0;
      // L's column m + 1, unchanged since the factorisation
      if (more && low && bj == mbn) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) colbuf[64 * (1 - p) + 8 * bi + rr] = a[rr][rn];
      }
      if (low && bi >= mb && bj <= mb) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) lr[rr] = (bi > mb || rr > mm) ? lr[rr] : 0.0;
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) wv[c8] = (bj < mb || c8 < mm) ? wv[c8] : 0.0;
        // row m + 1 first: its update by row m, W_{m+1,m}, its scaling and
        // publication
#pragma unroll
        for (int c8 = 0; c8 < 8; ++c8) a[rn][c8] = fma(-lr[rn], wv[c8], a[rn][c8]);
        if (bj == mb && (bi > mb || rn > mm)) a[rn][mm] = -lr[rn] * wmm;
        if (more && bi == mbn) {
          double* nb = rowbuf + 64 * (1 - p);
#pragma unroll
          for (int c8 = 0; c8 < 8; ++c8) {
            if (bj < mbn || c8 < rn) a[rn][c8] *= wn;
            nb[8 * bj + c8] = a[rn][c8];
          }
        }
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
          if (rr == rn) continue;
#pragma unroll
          for (int c8 = 0; c8 < 8; ++c8) a[rr][c8] = fma(-lr[rr], wv[c8], a[rr][c8]);
        }
        if (bj == mb) {
#pragma unroll
          for (int rr = 0; rr < 8; ++rr)
            if (rr != rn && (bi > mb || rr > mm)) a[rr][mm] = -lr[rr] * wmm;
          if (bi == mb) a[mm][mm] = wmm;
        }
      }
      wave_lds_sync();
    }
  }
  return 0;
}

template <int MODE>
__device__ __forceinline__ void dev_potrf_blk(const Lay& lay, double* C, int64_t ld, double* Wd,
                                              float* W32, double* logdet_k, int32_t* info_k,
                                              int J, double* smem, float* L32 = nullptr,
                                              int64_t ld32 = 0) {
  double* P = smem;                  // W11, then X^T = (L21 W11)^T
  double* Q = smem + 64 * PB_LS;     // L21, then A22 - L21 L21^T, then W22
  // the one-wave sweeps' buffers live in Q, which holds nothing then (the
  // first sweep precedes L21; the second starts by loading A22' from it)
  double* colbuf = Q;        // two buffers
  double* rowbuf = Q + 128;  // two buffers
  double* dinv = Q + 256;
  double* red = smem + 2 * 64 * PB_LS;
  volatile int* flag = reinterpret_cast<volatile int*>(red + 64);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int nv = lay.rows(J);
  // the wave that factors the diagonal blocks varies with the workgroup index
  // (differently for neighbours 1 and 256 apart), so that co-resident
  // workgroups are likely to run their serial phases on different SIMDs
  const int ws = (int)((blockIdx.x + (blockIdx.x >> 8)) & 3);
  // element (r, c) of the identity-padded tile, r >= c
  auto tile = [&](int r, int c) -> double {
    if (r < nv && c < nv) return C[(int64_t)c * ld + r];
    return r == c ? 1.0 : 0.0;
  };
  auto put_w = [&](int r, int c, double v) {
    if (MODE == 0) Wd[c * T + r] = v;
    else W32[c * T + r] = (float)v;
  };
  auto put_l = [&](int r, int c, double v) {  // r, c < nv, r >= c
    if (MODE == 0) C[(int64_t)c * ld + r] = v;
    if (MODE == 2) L32[(int64_t)c * ld32 + r] = (float)v;
  };
  double sl_total = 0.0;

  // ---- A11 = L11 L11^T, W11 (wave ws) -> P
  if (w == ws) {
    if (lane == 0) *flag = 0;  // read by every wave after the next barrier
    const int bi = lane >> 3, bj = lane & 7;
    double a[8][8];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        a[rr][cc] = r >= c ? tile(r, c) : 0.0;
      }
    double sl;
    const int bad = wave64_chol_inv(a, min(nv, 64), colbuf, rowbuf, dinv, sl,
                                    [&](int r, int c, double v) { put_l(r, c, v); });
    if (bad) {
      if (lane == 0) {
        *info_k = J * T + bad;
        *flag = 1;
      }
    } else {
      sl_total = sl;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr)
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const int r = 8 * bi + rr, c = 8 * bj + cc;
          const double v = (bi >= bj && r >= c) ? a[rr][cc] : 0.0;
          P[c * PB_LS + r] = v;
          put_w(r, c, v);
        }
    }
  }
  __syncthreads();
  if (*flag) return;

  // ---- L21 = A21 W11^T (wave w: block row w) -> Q and the output
  {
    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    const int R = 64 + 16 * w + lr;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int kk = 4 * s + lk;
      const double av = (R < nv && kk < nv) ? C[(int64_t)kk * ld + R] : 0.0;
#pragma unroll
      for (int j = s >> 2; j < 4; ++j)  // W11 row 16 j + lr is zero past column 16 j + 15
        acc[j] = MF<double>::op(P[kk * PB_LS + 16 * j + lr], av, acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * j + MF<double>::col(lk, e), r = 16 * w + lr;
        Q[c * PB_LS + r] = acc[j][e];
        if (64 + r < nv && c < nv) put_l(64 + r, c, acc[j][e]);
      }
  }
  __syncthreads();

  // ---- X^T = W11^T L21^T (wave w: block row w of X^T), then into P
  {
    d4 acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
    for (int s = 4 * w; s < 16; ++s) {  // W11 column 16 w + lr is zero above row 16 w
      const int kk = 4 * s + lk;
      const double av = P[(16 * w + lr) * PB_LS + kk];
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] = MF<double>::op(Q[kk * PB_LS + 16 * m + lr], av, acc[m]);
    }
    __syncthreads();  // every read of W11 done
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) P[(16 * m + MF<double>::col(lk, e)) * PB_LS + 16 * w + lr] = acc[m][e];
  }

  // ---- A22 - L21 L21^T (wave w: block row w, blocks j <= w) -> Q
  {
    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int kk = 4 * s + lk;
      const double av = Q[kk * PB_LS + 16 * w + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (j <= w) acc[j] = MF<double>::op(Q[kk * PB_LS + 16 * j + lr], av, acc[j]);
    }
    __syncthreads();  // every read of L21 done
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j > w) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 16 * j + MF<double>::col(lk, e), r = 16 * w + lr;
        Q[c * PB_LS + r] = r >= c ? tile(64 + r, 64 + c) - acc[j][e] : 0.0;
      }
    }
  }
  __syncthreads();

  // ---- A22' = L22 L22^T, W22 (wave ws) -> Q
  if (w == ws) {
    const int bi = lane >> 3, bj = lane & 7;
    double a[8][8];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr)
#pragma unroll
      for (int cc = 0; cc < 8; ++cc) {
        const int r = 8 * bi + rr, c = 8 * bj + cc;
        a[rr][cc] = r >= c ? Q[c * PB_LS + r] : 0.0;
      }
    double sl;
    const int bad = wave64_chol_inv(a, max(nv - 64, 0), colbuf, rowbuf, dinv, sl,
                                    [&](int r, int c, double v) { put_l(64 + r, 64 + c, v); });
    if (bad) {
      if (lane == 0) {
        *info_k = J * T + 64 + bad;
        *flag = 1;
      }
    } else {
      sl_total += sl;
#pragma unroll
      for (int rr = 0; rr < 8; ++rr)
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const int r = 8 * bi + rr, c = 8 * bj + cc;
          const double v = (bi >= bj && r >= c) ? a[rr][cc] : 0.0;
          Q[c * PB_LS + r] = v;
          put_w(64 + r, 64 + c, v);
        }
      // log|V| of the tile: 2 sum log L_jj over both blocks
      red[lane] = sl_total;
      wave_lds_sync();
      if (lane == 0) {
        double t = 0.0;
        for (int i = 0; i < 64; ++i) t += red[i];
        *logdet_k += 2.0 * t;
      }
    }
  }
  __syncthreads();
  if (*flag) return;

  // ---- W21 = -W22 X (wave w: block column w); W12 = 0
  {
    d4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int kk = 4 * s + lk;
      const double bv = P[kk * PB_LS + 16 * w + lr];  // X^T row 16 w + lr, column kk
#pragma unroll
      for (int i = s >> 2; i < 4; ++i)  // W22 row block i is zero past column 16 i + 15
        acc[i] = MF<double>::op(bv, Q[kk * PB_LS + 16 * i + lr], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * i + lr, c = 16 * w + MF<double>::col(lk, e);  // acc[i]: (W22 X) block (i, w)
        put_w(64 + r, c, -acc[i][e]);
      }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int idx = 64 * t + lane;  // 1024 zeros of block column w of W12
      put_w(idx & 63, 64 + 16 * w + (idx >> 6), 0.0);
    }
  }
}

}  // namespace plk
