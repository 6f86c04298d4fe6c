// Internal declarations shared by the plprof HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/plprof.h"

namespace plk {

// Tile edge of the blocked factorisation and of the covariance builder.
constexpr int T = 128;
// Chebyshev tables of rho(sqrt w), w = x^2 = 8 kappa d^2, per
// omega: pieces uniform in the mantissa of w, PB per binade [2^e, 2^(e+1)),
// for the NBIN binades from 2^W_E_LO up, NC coefficients per piece.
constexpr int W_E_LO = -20;        // w < 2^-20 (x < ~1e-3): direct quadrature
constexpr int NBIN = 44;           // binades tabulated: w < 2^24 (x < 4096)
constexpr int PB = 4;              // pieces per binade
constexpr int NC = 10;             // coefficients per piece
constexpr int NPIECE = NBIN * PB;
constexpr int TABLE = NPIECE * NC; // doubles per omega

// Per-omega constants, computed on the host once per call.
struct MaternParams {
  double inv_phix, inv_phiy;   // 1/phi_X, 1/phi_Y
  double cosA, sinA;           // rotation by phi_A
  double k8;                   // 8 kappa (w = 8 kappa d^2)
  double nugget;               // nu^2
  double kappa;
  double log_norm;             // log(2^(1-kappa) / Gamma(kappa))
  double w_hi;                 // rho underflows for w >= w_hi
  double pad[3];
};

// Host: the constants of omega = (phi_X, kappa, nu^2, phi_R, phi_A).
MaternParams make_matern_params(const double* om);

// One omega of an uneven batch pass (datasets of different n in one launch):
// its dataset's order, the dataset's index (Jacobian, y check), its
// locations (n x 2), the element offset of its right-hand sides (n x TB) in
// the batch's array, and its omega index in the records (record om M + m).
struct UnitInfo {
  int32_t n;
  int32_t ds;
  const double* locs;
  int64_t rhs;
  int64_t om;
};

// Addressing of the per-omega matrices.
//  kind 0: packed lower tiles, each T x T column-major, tile (I,J) of the V
//          part at (I(I+1)/2 + J) T^2; below them a bordered tile row of
//          height TB holding the right-hand sides as rows (tile (Nv,J) is
//          TB x T, the final tile (Nv,Nv) TB x TB).  A row panel I (tiles
//          (I,0..I-1)) is then one contiguous column-major block.
//  kind 1: plain column-major n x n with leading dimension ld.
struct Lay {
  int kind;
  int Nv;        // tile rows covering the n rows of V
  int n;         // order of V
  int q;         // bordered rows (right-hand sides), 0 for kind 1
  int TB;        // height of the bordered tile row (q rounded up to 16)
  int pad;
  int64_t ld;      // kind 1 leading dimension
  int64_t mstride; // elements per matrix
  // uneven batches: per-omega data of the pass, null otherwise.  n is then
  // the unit's own order inside a kernel (lay_of) and every unit shares Nv.
  const UnitInfo* units;

  __host__ __device__ int64_t tile_off(int I, int J) const {
    if (kind == 1) return (int64_t)J * T * ld + (int64_t)I * T;
    if (I < Nv) return ((int64_t)I * (I + 1) / 2 + J) * (int64_t)(T * T);
    return (int64_t)Nv * (Nv + 1) / 2 * (T * T) + (int64_t)J * TB * T;
  }
  __host__ __device__ int64_t tile_ld(int I) const {
    if (kind == 1) return ld;
    return I < Nv ? T : TB;
  }
  __host__ __device__ int rows(int I) const {
    if (I < Nv) { int r = n - I * T; return r < T ? r : T; }
    return q;
  }
};

// The layout of omega k of a launch: its own order n in an uneven batch.
__device__ __forceinline__ Lay lay_of(const Lay& lay, int k) {
  Lay L = lay;
  if (lay.units) L.n = lay.units[k].n;
  return L;
}

// Elements per omega of the mixed form's x0 (rows of TB values, Nv T rows).
__host__ __device__ inline int64_t x0_stride(const Lay& lay) {
  return (int64_t)lay.Nv * T * lay.TB;
}

__host__ inline int64_t packed_stride(int Nv, int TB) {
  return (int64_t)Nv * (Nv + 1) / 2 * (T * T) + (int64_t)Nv * TB * T + (int64_t)TB * TB;
}

// Workgroup index remapped so that consecutive logical indices share an XCD
// (hardware dispatches consecutive workgroups round-robin over the 8 XCDs,
// each with its own L2).  Bijective for any grid size.
__device__ inline int xcd_remap(int wg, int G) {
  const int nx = 8;
  int per = G / nx, rem = G % nx;
  int x = wg % nx, i = wg / nx;
  return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Stream-ordered copy of a small host array (the caller may reuse it at once).
hipError_t stage_h2d(void* dst, const void* src, size_t bytes, hipStream_t s);

// ---- launch wrappers (defined in the .hip files) --------------------------
hipError_t launch_cheb_tables(const MaternParams* mp, double* nodes, double* tables,
                              int K, hipStream_t s);
// flag_ws: scratch of at least 4 bytes per tile per omega (the pass's table
// nodes, dead once the tables are built), or null; with it the elements that
// need the quadrature go to a second, short launch (see matern.hip)
hipError_t launch_matern_packed(const Lay& lay, double* mats, const double* locs,
                                const MaternParams* mp, const double* tables, int K,
                                hipStream_t s, uint8_t* flag_ws = nullptr);
hipError_t launch_matern_colmajor(double* V, int64_t ld, int n, const double* locs,
                                  const MaternParams* mp, const double* tables, int K,
                                  hipStream_t s);
hipError_t launch_matern_colmajor_f32(float* V, int64_t ld, int n, const double* locs,
                                      const MaternParams* mp, const double* tables, int K,
                                      hipStream_t s);
hipError_t launch_potrf(const Lay& lay, double* mats, double* W, double* logdet,
                        int32_t* info, int J, int K, hipStream_t s);
hipError_t launch_trsm(const Lay& lay, double* mats, const double* W, const int32_t* info,
                       int J, int nI, int K, hipStream_t s);
hipError_t launch_gemm_col(const Lay& lay, double* mats, const int32_t* info, int J, int nI,
                           int K, hipStream_t s);
hipError_t launch_col_update(const Lay& lay, double* mats, const int32_t* info, int J, int K,
                             hipStream_t s);
// the bordered row's own TB x TB block (TB <= 32) after the last block column
hipError_t launch_border_block(const Lay& lay, double* mats, const int32_t* info, int K,
                               hipStream_t s);
hipError_t launch_fill(double* p, double v, int64_t count, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t s);
hipError_t launch_boxcox_rhs(const double* y, const double* X, const double* lam, int n,
                             int p, int M, double* rhs, double* jac, int32_t* flags,
                             hipStream_t s);
hipError_t launch_border_init(const Lay& lay, double* mats, const double* rhs, int K,
                              hipStream_t s);
// mixed form: red[k red_stride + b TB + a] = -(1/2) sum over the omega's lower
// tiles of the refined slots (a, b) + (b, a)
hipError_t launch_slot_reduce(const Lay& lay, const double* slots, double* red,
                              int64_t red_stride, int K, hipStream_t s);
// sred: null (FP64: the Schur tile of the factor) or the reduced slots
hipError_t launch_finalize(const Lay& lay, const double* mats, const double* sred,
                           int64_t sred_stride, const double* logdet, const int32_t* info, const double* jac,
                           const int32_t* flags, const double* lam, int n, int p, int M, int K,
                           pl_result* out, double* beta, double* xvi, hipStream_t s);
// mixed form
hipError_t launch_matern_mixed(const Lay& lay, double* m64, int64_t stride64, float* m32,
                               const double* locs, const MaternParams* mp, const double* tables,
                               int K, hipStream_t s, uint8_t* flag_ws = nullptr);
hipError_t launch_border_init_f32(const Lay& lay, float* mats, const double* rhs, int K,
                                  hipStream_t s);
constexpr int MX_FLUSH = 4;  // default FP32 MFMA k-steps per FP64 fold of the mixed update
hipError_t launch_gemm_col_mx(const Lay& lay, float* m32, const double* m64, int64_t m64stride,
                              double* dscratch, const int32_t* info, int J, int nI, int K,
                              int flush, hipStream_t s);
hipError_t launch_potrf_mx(const Lay& lay, double* dscratch, float* W32, double* logdet,
                           int32_t* info, int J, int K, hipStream_t s);
hipError_t launch_trsm_mx(const Lay& lay, float* m32, const float* W32, const int32_t* info, int J,
                          int nI, int K, hipStream_t s);
// mixed form on a plain column-major FP32 matrix (kind 1): the update of
// block column J (diagonal tile in FP64 into dscratch, the nI - 1 tiles below
// it in FP32 MFMA with FP64 folds, in place), the diagonal factor (L_JJ
// rounded into the matrix, W_J in FP32 to W32[k], one T x T slot per omega)
// and the panel solve of the nI - 1 tiles below J
hipError_t launch_col_update_mx_plain(const Lay& lay, float* m32, double* dscratch,
                                      const int32_t* info, int J, int K, int flush,
                                      hipStream_t s);
hipError_t launch_potrf_mx_plain(const Lay& lay, float* m32, double* dscratch, float* W32,
                                 double* logdet, int32_t* info, int J, int K, hipStream_t s);
hipError_t launch_trsm_mx_plain(const Lay& lay, float* m32, const float* W32,
                                const int32_t* info, int J, int K, hipStream_t s);
hipError_t launch_backsolve(const Lay& lay, const float* m32, const float* W32,
                            const int32_t* info, double* X, int K, hipStream_t s);
hipError_t launch_qform(const Lay& lay, const double* m64, int64_t stride64, const double* X,
                        const double* rhs, const int32_t* info, double* slots, int refine, int K,
                        hipStream_t s);
hipError_t launch_mark_fallback(pl_result* out, int M, hipStream_t s);

// ---- one device pass of Step 3 over omega points sharing a layout ----------------
struct PassBufs {
  double* mats;                  // FP64: packed bordered matrices
  double* W;                     // FP64: W_J per omega
  float* m32;                    // mixed: FP32 packed factor
  double* m64;                   // mixed: FP64 copy of V
  float* W32;                    // mixed: every W_J in FP32
  double* dscr;                  // mixed: FP64 diagonal tile / reduced slots
  double* x0;                    // mixed: x0 = V^-1 [Y'|X]
  double* slots;                 // mixed: refined cross-product slots
  double* logdet;
  int32_t* info;
  size_t bytes;                  // bytes carved
};
struct PassArgs {
  Lay lay;                       // lay.units set for an uneven batch
  bool mixed;
  int flush, refine;
  const double* locs;            // the dataset's (or the batch's) locations
  const double* rhs;             // its Box-Cox right-hand sides (n x TB)
  const MaternParams* mp;        // this pass's omega constants and tables
  const double* tables;
  uint8_t* flag_ws;              // the pass's table nodes, reused by the covariance build, or null
  const double* jac;
  const int32_t* yflags;
  const double* lam;             // device, M values
  int p, M;
  pl_result* out;                // records of the pass's first omega (batch: all records)
  double* beta;
  double* xvx;
  int32_t* info_out;             // per-omega info copy, or null
};
PassBufs carve_pass(char* base, const Lay& lay, bool mixed, int64_t kc);
size_t pass_bytes(const Lay& lay, bool mixed, int64_t kc);
hipError_t run_pass(const PassArgs& a, const PassBufs& b, int kk, hipStream_t s);
// Suspends (pause = true) or resumes the per-kernel-class event timing;
// returns whether it was on before the call.
bool profiling_pause(bool pause);

// Tuning cache (tune.hip): kind 0 pl_autotune, 1 pl_batch_autotune; a hit
// writes the stored choice into opts.
bool tune_cache_find(int kind, int64_t n, int64_t units, int64_t q, double tol, pl_opts* opts);
void tune_cache_put(int kind, int64_t n, int64_t units, int64_t q, double tol, const pl_opts& o,
                    double ms);
Lay packed_layout(int64_t n, int64_t q);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int n, hipStream_t s);

}  // namespace plk
