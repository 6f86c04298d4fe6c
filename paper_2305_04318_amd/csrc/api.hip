// C-ABI entry points: argument checks, per-omega constants, workspace
// carving and the kernel sequence of Step 3 (Section 3.3).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"

using namespace plk;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Carve {
  char* base;
  size_t off = 0;
  template <class P>
  P* take(size_t bytes) {
    P* p = reinterpret_cast<P*>(base + off);
    off += align_up(bytes);
    return p;
  }
};

bool omega_ok(const double* om) {
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(om[i])) return false;
  return om[0] > 0.0 && om[1] >= PL_MIN_SHAPE && om[1] <= PL_MAX_SHAPE && om[2] >= 0.0 &&
         om[3] > 0.0;
}

}  // namespace

Lay plk::packed_layout(int64_t n, int64_t q) {
  Lay lay{};
  lay.kind = 0;
  lay.n = (int)n;
  lay.Nv = (int)((n + T - 1) / T);
  lay.q = (int)q;
  lay.TB = (int)((q + 15) / 16 * 16);
  lay.mstride = packed_stride(lay.Nv, lay.TB);
  return lay;
}

namespace {

size_t per_omega_bytes(const Lay& lay) {
  return align_up(lay.mstride * sizeof(double)) + align_up((size_t)T * T * sizeof(double)) +
         2 * ALIGN;
}

// mixed form: FP32 packed factor (with the bordered row), FP64 copy of V,
// the FP32 inverses of every diagonal tile, an FP64 scratch tile, x0 and the
// per-tile-row cross-product slots
int64_t v_stride64(const Lay& lay) { return (int64_t)lay.Nv * (lay.Nv + 1) / 2 * T * T; }

size_t per_omega_bytes_mixed(const Lay& lay) {
  return align_up(lay.mstride * sizeof(float)) + align_up(v_stride64(lay) * sizeof(double)) +
         align_up((size_t)lay.Nv * T * T * sizeof(float)) + align_up((size_t)T * T * sizeof(double)) +
         align_up((size_t)x0_stride(lay) * sizeof(double)) +
         align_up((size_t)lay.Nv * (lay.Nv + 1) / 2 * lay.TB * lay.TB * sizeof(double)) + 2 * ALIGN;
}

size_t fixed_bytes(int64_t n, int64_t K, int64_t M, const Lay& lay) {
  size_t b = 0;
  b += align_up(K * sizeof(MaternParams));
  b += 2 * align_up((size_t)K * TABLE * sizeof(double));
  b += align_up(M * sizeof(double));
  b += align_up((size_t)n * lay.TB * sizeof(double));
  b += align_up(sizeof(double)) + align_up(sizeof(int32_t));
  b += align_up(K * sizeof(int32_t));  // per-omega info of the whole call
  return b;
}

#define PL_CHECK(call)                        \
  do {                                        \
    hipError_t _e = (call);                   \
    if (_e != hipSuccess) return PL_E_HIP;    \
  } while (0)

// ---- optional per-kernel-class timing with HIP events -----------------------
struct ProfRec {
  int cls;
  double flops;
  hipEvent_t a, b;
};
struct Prof {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Prof g_prof;
bool g_prof_paused_on = false;  // timing was on when paused

// Runs `launch`, bracketed by events on stream s when profiling is on.
template <class F>
hipError_t timed(int cls, double flops, hipStream_t s, F&& launch) {
  if (!g_prof.on) return launch();
  hipEvent_t a = g_prof.get(), b = g_prof.get();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  g_prof.recs.push_back({cls, flops, a, b});
  return hipSuccess;
}

// Algorithmic flops of one left-looking column update (lower triangle only).
double gemm_col_flops(const Lay& lay, int J, int nI) {
  const double kk = std::min<double>((double)J * T, lay.n);
  const double cj = lay.rows(J);
  double f = 0.0;
  for (int I = J; I < J + nI; ++I) {
    const double ri = lay.rows(I);
    f += (I == J) ? ri * (ri + 1.0) * kk : 2.0 * ri * cj * kk;
  }
  return f;
}

}  // namespace

bool plk::profiling_pause(bool pause) {
  const bool was = pause ? g_prof.on : g_prof_paused_on;
  if (pause) {
    g_prof_paused_on = g_prof.on;
    g_prof.on = false;
  } else {
    g_prof.on = g_prof_paused_on;
    g_prof_paused_on = false;
  }
  return was;
}

// Per-pass buffers for kc omega points of layout lay, carved from base.
PassBufs plk::carve_pass(char* base, const Lay& lay, bool mixed, int64_t kc) {
  Carve cv{base};
  PassBufs b{};
  if (!mixed) {
    b.mats = cv.take<double>((size_t)kc * lay.mstride * sizeof(double));
    b.W = cv.take<double>((size_t)kc * T * T * sizeof(double));
  } else {
    b.m32 = cv.take<float>((size_t)kc * lay.mstride * sizeof(float));
    b.m64 = cv.take<double>((size_t)kc * v_stride64(lay) * sizeof(double));
    b.W32 = cv.take<float>((size_t)kc * lay.Nv * T * T * sizeof(float));
    b.dscr = cv.take<double>((size_t)kc * T * T * sizeof(double));
    b.x0 = cv.take<double>((size_t)kc * x0_stride(lay) * sizeof(double));
    b.slots = cv.take<double>((size_t)kc * lay.Nv * (lay.Nv + 1) / 2 * lay.TB * lay.TB *
                              sizeof(double));
  }
  b.logdet = cv.take<double>((size_t)kc * sizeof(double));
  b.info = cv.take<int32_t>((size_t)kc * sizeof(int32_t));
  b.bytes = cv.off;
  return b;
}

size_t plk::pass_bytes(const Lay& lay, bool mixed, int64_t kc) {
  return (size_t)kc * (mixed ? per_omega_bytes_mixed(lay) : per_omega_bytes(lay));
}

// Steps 1-8 of Section 3.3 for kk omega points sharing one layout: the
// bordered right-hand sides, the covariance tiles, the bordered blocked
// Cholesky (FP64, or the mixed form with its back substitution and refined
// cross products), the p x p stage.  Records go to a.out (omega k at
// a.out + k M, or at its UnitInfo index in an uneven batch).
hipError_t plk::run_pass(const PassArgs& a, const PassBufs& b, int kk, hipStream_t s) {
  const Lay& lay = a.lay;
  hipError_t e = timed(PL_KC_OTHER, 0.0, s, [&] {
    hipError_t r = a.mixed ? launch_border_init_f32(lay, b.m32, a.rhs, kk, s)
                           : launch_border_init(lay, b.mats, a.rhs, kk, s);
    if (r == hipSuccess) r = launch_fill(b.logdet, 0.0, kk, s);
    if (r == hipSuccess) r = launch_fill_i32(b.info, 0, kk, s);
    return r;
  });
  if (e != hipSuccess) return e;
  e = timed(PL_KC_MATERN, 0.0, s, [&] {
    return a.mixed ? launch_matern_mixed(lay, b.m64, v_stride64(lay), b.m32, a.locs, a.mp,
                                         a.tables, kk, s, a.flag_ws)
                   : launch_matern_packed(lay, b.mats, a.locs, a.mp, a.tables, kk, s, a.flag_ws);
  });
  if (e != hipSuccess) return e;
  if (!a.mixed) {
    // per block column: the update of every tile of the column (the bordered
    // row folded into the diagonal tile's workgroup), the diagonal tile's
    // factor and inverse, the panel solve; the bordered row's own block
    // closes the factorisation
    for (int J = 0; J <= lay.Nv; ++J) {
      if (J < lay.Nv) {
        if (J > 0) {
          e = timed(PL_KC_GEMM, kk * gemm_col_flops(lay, J, lay.Nv - J + 1), s,
                    [&] { return launch_col_update(lay, b.mats, b.info, J, kk, s); });
          if (e != hipSuccess) return e;
        }
        e = timed(PL_KC_POTRF, 0.0, s,
                  [&] { return launch_potrf(lay, b.mats, b.W, b.logdet, b.info, J, kk, s); });
        if (e != hipSuccess) return e;
        e = timed(PL_KC_TRSM, 0.0, s,
                  [&] { return launch_trsm(lay, b.mats, b.W, b.info, J, lay.Nv - J, kk, s); });
        if (e != hipSuccess) return e;
      } else {
        e = timed(PL_KC_GEMM, kk * gemm_col_flops(lay, J, 1), s, [&] {
          return lay.TB <= 32 ? launch_border_block(lay, b.mats, b.info, kk, s)
                              : launch_gemm_col(lay, b.mats, b.info, J, 1, kk, s);
        });
        if (e != hipSuccess) return e;
      }
    }
  } else {
    for (int J = 0; J < lay.Nv; ++J) {
      // J = 0 has no update: the diagonal kernel then copies V's FP64 tile
      const int nI = (J == 0) ? 1 : lay.Nv - J + 1;
      e = timed(PL_KC_GEMM, kk * gemm_col_flops(lay, J, nI), s, [&] {
        return launch_gemm_col_mx(lay, b.m32, b.m64, v_stride64(lay), b.dscr, b.info, J, nI, kk,
                                  a.flush, s);
      });
      if (e != hipSuccess) return e;
      e = timed(PL_KC_POTRF, 0.0, s,
                [&] { return launch_potrf_mx(lay, b.dscr, b.W32, b.logdet, b.info, J, kk, s); });
      if (e != hipSuccess) return e;
      e = timed(PL_KC_TRSM, 0.0, s,
                [&] { return launch_trsm_mx(lay, b.m32, b.W32, b.info, J, lay.Nv - J, kk, s); });
      if (e != hipSuccess) return e;
    }
    e = timed(PL_KC_OTHER, 0.0, s, [&] {
      hipError_t r = launch_backsolve(lay, b.m32, b.W32, b.info, b.x0, kk, s);
      if (r == hipSuccess)
        r = launch_qform(lay, b.m64, v_stride64(lay), b.x0, a.rhs, b.info, b.slots, a.refine, kk,
                         s);
      return r;
    });
    if (e != hipSuccess) return e;
  }
  return timed(PL_KC_OTHER, 0.0, s, [&] {
    hipError_t r = hipSuccess;
    if (a.mixed) r = launch_slot_reduce(lay, b.slots, b.dscr, (int64_t)T * T, kk, s);
    if (r == hipSuccess)
      r = launch_finalize(lay, b.mats, a.mixed ? b.dscr : nullptr, (int64_t)T * T, b.logdet,
                          b.info, a.jac, a.yflags, a.lam, lay.n, a.p, a.M, kk, a.out, a.beta,
                          a.xvx, s);
    if (r == hipSuccess && a.info_out) r = launch_copy_i32(b.info, a.info_out, kk, s);
    return r;
  });
}

// Constants for one omega = (phi_X, kappa, nu^2, phi_R, phi_A); phi_Y = phi_X / phi_R.
MaternParams plk::make_matern_params(const double* om) {
  MaternParams P{};
  const double phix = om[0], kappa = om[1], nug = om[2], ratio = om[3], ang = om[4];
  P.inv_phix = 1.0 / phix;
  P.inv_phiy = ratio / phix;
  P.cosA = cos(ang);
  P.sinA = sin(ang);
  P.k8 = 8.0 * kappa;
  P.nugget = nug;
  P.kappa = kappa;
  P.log_norm = (1.0 - kappa) * M_LN2 - lgamma(kappa);
  // x_hi: beyond it rho < exp(-745) (below the smallest double).  From the
  // large-argument form log rho ~ log_norm + 0.5 log(pi/2) + (kappa-1/2) log x - x,
  // solved by fixed-point iteration, then widened for the neglected terms;
  // capped at the table's end (rho there is far below exp(-745) for every
  // admissible shape).
  const double C = P.log_norm + 0.5 * log(M_PI / 2.0) + 760.0;
  double x = std::max(C, 10.0);
  for (int i = 0; i < 60; ++i) x = std::max(10.0, C + (kappa - 0.5) * log(x));
  const double x_hi = 1.1 * x + 50.0;
  P.w_hi = std::min(x_hi * x_hi, ldexp(1.0, W_E_LO + NBIN));
  return P;
}

// Host-to-device copy of a small host array ordered on the stream: the bytes
// are copied into a heap buffer that a host callback on the stream frees once
// the copy has consumed it, so the caller may reuse its array at once.
hipError_t plk::stage_h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  char* hold = new char[bytes];
  memcpy(hold, src, bytes);
  hipError_t e = hipMemcpyAsync(dst, hold, bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    delete[] hold;
    return e;
  }
  return hipLaunchHostFunc(s, [](void* p) { delete[] static_cast<char*>(p); }, hold);
}

extern "C" {

const char* pl_version(void) { return "plprof 0.1 (gfx950)"; }

const char* pl_error_string(int code) {
  if (code == PL_OK) return "ok";
  if (code < 0) return "invalid argument";
  switch (code) {
    case PL_E_HIP: return "HIP runtime error";
    case PL_E_WORKSPACE: return "workspace too small";
    case PL_E_UNSUPPORTED: return "unsupported size";
    case PL_E_SCRATCH: return "one omega of this problem does not fit the fixed scratch array";
    default: return "unknown error";
  }
}

int pl_matern_workspace_size(int64_t K, size_t* bytes) {
  if (K < 1) return -1;
  if (!bytes) return -2;
  *bytes = align_up(K * sizeof(MaternParams)) + 2 * align_up((size_t)K * TABLE * sizeof(double));
  return PL_OK;
}

int pl_matern_cov(const double* locs, int64_t n, const double* omega, int64_t K, int dtype,
                  void* V, int64_t ld, void* work, size_t work_bytes, void* stream) {
  if (!locs) return -1;
  if (n < 1 || n > (1 << 30)) return -2;
  if (!omega) return -3;
  if (K < 1 || K > (1 << 24)) return -4;
  for (int64_t k = 0; k < K; ++k)
    if (!omega_ok(omega + 5 * k)) return -3;
  if (dtype != PL_F64 && dtype != PL_F32) return -5;
  if (!V) return -6;
  if (ld < n) return -7;
  if (!work) return -8;
  size_t need = 0;
  pl_matern_workspace_size(K, &need);
  if (work_bytes < need) return -9;
  hipStream_t s = (hipStream_t)stream;
  std::vector<MaternParams> hp(K);
  for (int64_t k = 0; k < K; ++k) hp[k] = make_matern_params(omega + 5 * k);
  Carve cv{(char*)work};
  MaternParams* mp = cv.take<MaternParams>(K * sizeof(MaternParams));
  double* nodes = cv.take<double>((size_t)K * TABLE * sizeof(double));
  double* tables = cv.take<double>((size_t)K * TABLE * sizeof(double));
  if (stage_h2d(mp, hp.data(), K * sizeof(MaternParams), s) != hipSuccess) return PL_E_HIP;
  PL_CHECK(timed(PL_KC_TABLES, 0.0, s, [&] { return launch_cheb_tables(mp, nodes, tables, (int)K, s); }));
  PL_CHECK(timed(PL_KC_MATERN, 0.0, s, [&] {
    return dtype == PL_F64
               ? launch_matern_colmajor((double*)V, ld, (int)n, locs, mp, tables, (int)K, s)
               : launch_matern_colmajor_f32((float*)V, ld, (int)n, locs, mp, tables, (int)K, s);
  }));
  return PL_OK;
}

int pl_chol_workspace_size(int64_t K, int precision, size_t* bytes) {
  if (K < 1 || K > (1 << 24)) return -1;
  if (precision != PL_FP64 && precision != PL_MIXED) return -2;
  if (!bytes) return -3;
  // FP64: W_J (FP64) per omega; mixed: the FP64 diagonal tile and W_J in FP32
  *bytes = align_up((size_t)K * T * T * sizeof(double));
  if (precision == PL_MIXED) *bytes += align_up((size_t)K * T * T * sizeof(float));
  return PL_OK;
}

int pl_chol_batched(void* V, int64_t n, int64_t K, int64_t ld, int precision, double* logdet,
                    int32_t* info, void* work, size_t work_bytes, void* stream) {
  const bool mixed = precision == PL_MIXED;
  if (!V || (mixed && (reinterpret_cast<uintptr_t>(V) & 15) != 0)) return -1;
  if (n < 1 || n > (1 << 30)) return -2;
  if (K < 1 || K > (1 << 24)) return -3;
  if (ld < n || (mixed && ld % 4 != 0)) return -4;
  if (precision != PL_FP64 && precision != PL_MIXED) return -5;
  if (!logdet) return -6;
  if (!info) return -7;
  if (!work) return -8;
  size_t need = 0;
  pl_chol_workspace_size(K, precision, &need);
  if (work_bytes < need) return -9;
  hipStream_t s = (hipStream_t)stream;
  Lay lay{};
  lay.kind = 1;
  lay.n = (int)n;
  lay.Nv = (int)((n + T - 1) / T);
  lay.ld = ld;
  lay.mstride = ld * n;
  PL_CHECK(launch_fill(logdet, 0.0, K, s));
  PL_CHECK(launch_fill_i32(info, 0, K, s));
  if (mixed) {
    // FP32 factor: off-diagonal updates and panel solves on FP32 MFMA with
    // FP64 folds; each diagonal tile updated in FP64 into dscr and factored
    // in FP64 (log|V| in FP64), L_JJ rounded into the matrix
    float* V32 = (float*)V;
    double* dscr = (double*)work;
    float* W32 = (float*)((char*)work + align_up((size_t)K * T * T * sizeof(double)));
    for (int J = 0; J < lay.Nv; ++J) {
      PL_CHECK(timed(PL_KC_GEMM, J > 0 ? K * gemm_col_flops(lay, J, lay.Nv - J) : 0.0, s, [&] {
        return launch_col_update_mx_plain(lay, V32, dscr, info, J, (int)K, MX_FLUSH, s);
      }));
      PL_CHECK(timed(PL_KC_POTRF, 0.0, s, [&] {
        return launch_potrf_mx_plain(lay, V32, dscr, W32, logdet, info, J, (int)K, s);
      }));
      if (lay.Nv - J - 1 > 0)
        PL_CHECK(timed(PL_KC_TRSM, 0.0, s,
                       [&] { return launch_trsm_mx_plain(lay, V32, W32, info, J, (int)K, s); }));
    }
    return PL_OK;
  }
  double* W = (double*)work;
  double* V64 = (double*)V;
  for (int J = 0; J < lay.Nv; ++J) {
    if (J > 0)
      PL_CHECK(timed(PL_KC_GEMM, K * gemm_col_flops(lay, J, lay.Nv - J), s,
                     [&] { return launch_gemm_col(lay, V64, info, J, lay.Nv - J, (int)K, s); }));
    PL_CHECK(timed(PL_KC_POTRF, 0.0, s,
                   [&] { return launch_potrf(lay, V64, W, logdet, info, J, (int)K, s); }));
    if (lay.Nv - J - 1 > 0)
      PL_CHECK(timed(PL_KC_TRSM, 0.0, s,
                     [&] { return launch_trsm(lay, V64, W, info, J, lay.Nv - J - 1, (int)K, s); }));
  }
  return PL_OK;
}

int pl_workspace_size(int64_t n, int64_t p, int64_t K, int64_t M, const pl_opts* opts,
                      size_t* bytes) {
  if (n < 2 || n > (1 << 30)) return -1;
  if (p < 1 || p >= n || p > PL_MAX_P) return -2;
  if (K < 1 || K > (1 << 24)) return -3;
  if (M < 1 || M > PL_MAX_M) return -4;
  if (!bytes) return -6;
  if (opts && opts->precision != PL_FP64 && opts->precision != PL_MIXED) return -5;
  const bool mixed = opts && opts->precision == PL_MIXED;
  if (mixed && M + p > PL_MAX_Q_MIXED) return PL_E_UNSUPPORTED;
  const Lay lay = packed_layout(n, M + p);
  int64_t kc = K;
  if (opts && opts->chunk > 0) kc = std::min<int64_t>(kc, opts->chunk);
  *bytes = fixed_bytes(n, K, M, lay) + (size_t)kc * (mixed ? per_omega_bytes_mixed(lay)
                                                           : per_omega_bytes(lay));
  return PL_OK;
}

int pl_profile_loglik(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
                      const double* omega, int64_t K, const double* lambda, int64_t M,
                      pl_result* out, double* beta_hat, double* xvx_inv, const pl_opts* opts,
                      void* work, size_t work_bytes, void* stream) {
  if (!locs) return -1;
  if (!y) return -2;
  if (!X) return -3;
  if (n < 2 || n > (1 << 30)) return -4;
  if (p < 1 || p >= n || p > PL_MAX_P) return -5;
  if (!omega) return -6;
  if (K < 1 || K > (1 << 24)) return -7;
  for (int64_t k = 0; k < K; ++k)
    if (!omega_ok(omega + 5 * k)) return -6;
  if (!lambda) return -8;
  for (int64_t m = 0; m < M && m < PL_MAX_M; ++m)
    if (!std::isfinite(lambda[m])) return -8;
  if (M < 1 || M > PL_MAX_M) return -9;
  if (!out) return -10;
  int precision = PL_FP64, refine = 1, flags = 0, flush = MX_FLUSH;
  int64_t chunk = 0;
  if (opts) {
    precision = opts->precision;
    chunk = opts->chunk;
    refine = opts->refine;
    flags = opts->flags;
    if (opts->flush != 0) flush = opts->flush;
    if (precision != PL_FP64 && precision != PL_MIXED) return -13;
    if (chunk < 0 || refine < 0 || refine > 1) return -13;
    if (flush != 1 && flush != 2 && flush != 4) return -13;
  }
  const bool mixed = precision == PL_MIXED;
  if (mixed && M + p > PL_MAX_Q_MIXED) return PL_E_UNSUPPORTED;
  if (!work) return -14;
  hipStream_t s = (hipStream_t)stream;

  const Lay lay = packed_layout(n, M + p);
  const size_t fixed = fixed_bytes(n, K, M, lay);
  const size_t per = mixed ? per_omega_bytes_mixed(lay) : per_omega_bytes(lay);
  if (work_bytes < fixed + per) return -15;
  int64_t kc = (int64_t)((work_bytes - fixed) / per);
  kc = std::min<int64_t>(kc, K);
  if (chunk > 0) kc = std::min<int64_t>(kc, chunk);

  Carve cv{(char*)work};
  MaternParams* mp = cv.take<MaternParams>(K * sizeof(MaternParams));
  double* nodes = cv.take<double>((size_t)K * TABLE * sizeof(double));
  double* tables = cv.take<double>((size_t)K * TABLE * sizeof(double));
  double* lam_d = cv.take<double>(M * sizeof(double));
  double* rhs = cv.take<double>((size_t)n * lay.TB * sizeof(double));
  double* jac = cv.take<double>(sizeof(double));
  int32_t* yflags = cv.take<int32_t>(sizeof(int32_t));
  int32_t* info_all = cv.take<int32_t>(K * sizeof(int32_t));
  const PassBufs pb = carve_pass(cv.base + cv.off, lay, mixed, kc);

  std::vector<MaternParams> hp(K);
  for (int64_t k = 0; k < K; ++k) hp[k] = make_matern_params(omega + 5 * k);
  if (stage_h2d(mp, hp.data(), K * sizeof(MaternParams), s) != hipSuccess ||
      stage_h2d(lam_d, lambda, M * sizeof(double), s) != hipSuccess)
    return PL_E_HIP;

  PL_CHECK(timed(PL_KC_TABLES, 0.0, s, [&] { return launch_cheb_tables(mp, nodes, tables, (int)K, s); }));
  PL_CHECK(timed(PL_KC_OTHER, 0.0, s, [&] {
    return launch_boxcox_rhs(y, X, lam_d, (int)n, (int)p, (int)M, rhs, jac, yflags, s);
  }));

  PassArgs pa{};
  pa.lay = lay;
  pa.mixed = mixed;
  pa.flush = flush;
  pa.refine = refine;
  pa.locs = locs;
  pa.rhs = rhs;
  pa.jac = jac;
  pa.yflags = yflags;
  pa.lam = lam_d;
  pa.p = (int)p;
  pa.M = (int)M;
  for (int64_t c0 = 0; c0 < K; c0 += kc) {
    const int kk = (int)std::min<int64_t>(kc, K - c0);
    pa.mp = mp + c0;
    pa.tables = tables + c0 * TABLE;
    pa.flag_ws = reinterpret_cast<uint8_t*>(nodes + c0 * TABLE);
    pa.out = out + c0 * M;
    pa.beta = beta_hat ? beta_hat + c0 * M * p : nullptr;
    pa.xvx = xvx_inv ? xvx_inv + c0 * p * p : nullptr;
    pa.info_out = info_all + c0;
    PL_CHECK(run_pass(pa, pb, kk, s));
  }

  if (mixed && !(flags & PL_OPT_NO_FALLBACK)) {
    // Points whose FP32 factorisation broke down are redone with the FP64 form
    // into their own records, then flagged.
    std::vector<int32_t> hinfo(K);
    if (hipMemcpyAsync(hinfo.data(), info_all, K * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PL_E_HIP;
    pl_opts o64{};
    o64.precision = PL_FP64;
    o64.chunk = 1;
    for (int64_t k = 0; k < K; ++k) {
      if (hinfo[k] > 0) {
        const int rc = pl_profile_loglik(locs, y, X, n, p, omega + 5 * k, 1, lambda, M,
                                         out + k * M, beta_hat ? beta_hat + k * M * p : nullptr,
                                         xvx_inv ? xvx_inv + k * p * p : nullptr, &o64, work,
                                         work_bytes, stream);
        if (rc != PL_OK) return rc;
        PL_CHECK(launch_mark_fallback(out + k * M, (int)M, s));
      }
    }
  }
  return PL_OK;
}

// ---- autotuner ------------------------------------------------------------------
namespace {
constexpr int TUNE_SAMPLE = 64;
constexpr int TUNE_NCAND = 4;
const int kTuneFlush[TUNE_NCAND] = {0, 4, 2, 1};  // 0: the FP64 form

size_t tune_records_bytes(int64_t S, int64_t M) { return align_up((size_t)S * M * sizeof(pl_result)); }

size_t tune_call_bytes(int64_t n, int64_t p, int64_t S, int64_t M, bool with_mixed) {
  size_t b64 = 0, bmx = 0;
  pl_opts o{};
  o.precision = PL_FP64;
  if (pl_workspace_size(n, p, S, M, &o, &b64) != PL_OK) return 0;
  if (with_mixed) {
    o.precision = PL_MIXED;
    if (pl_workspace_size(n, p, S, M, &o, &bmx) != PL_OK) return 0;
  }
  return std::max(b64, bmx);
}
}  // namespace

int pl_autotune_workspace_size(int64_t n, int64_t p, int64_t K, int64_t M, int64_t sample,
                               size_t* bytes) {
  if (n < 2 || n > (1 << 30)) return -1;
  if (p < 1 || p >= n || p > PL_MAX_P) return -2;
  if (K < 1 || K > (1 << 24)) return -3;
  if (M < 1 || M > PL_MAX_M) return -4;
  if (sample < 0) return -5;
  if (!bytes) return -6;
  const int64_t S = std::min<int64_t>(K, sample > 0 ? sample : TUNE_SAMPLE);
  *bytes = tune_call_bytes(n, p, S, M, M + p <= PL_MAX_Q_MIXED) + 2 * tune_records_bytes(S, M);
  return PL_OK;
}

int pl_autotune(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
                const double* omega, int64_t K, const double* lambda, int64_t M, int64_t sample,
                double tol, pl_opts* opts, double* report, void* work, size_t work_bytes,
                void* stream) {
  if (!locs) return -1;
  if (!y) return -2;
  if (!X) return -3;
  if (n < 2 || n > (1 << 30)) return -4;
  if (p < 1 || p >= n || p > PL_MAX_P) return -5;
  if (!omega) return -6;
  if (K < 1 || K > (1 << 24)) return -7;
  for (int64_t k = 0; k < K; ++k)
    if (!omega_ok(omega + 5 * k)) return -6;
  if (!lambda) return -8;
  if (M < 1 || M > PL_MAX_M) return -9;
  for (int64_t m = 0; m < M; ++m)
    if (!std::isfinite(lambda[m])) return -8;
  if (sample < 0) return -10;
  if (!std::isfinite(tol) || tol < 0.0) return -11;
  if (!opts) return -12;
  if (!work) return -14;
  if (tune_cache_find(0, n, 0, M + p, tol, opts)) {
    if (report)
      for (int c = 0; c < 2 * TUNE_NCAND; ++c) report[c] = -2.0;  // cached: nothing timed
    return PL_OK;
  }
  const int64_t S = std::min<int64_t>(K, sample > 0 ? sample : TUNE_SAMPLE);
  const bool with_mixed = M + p <= PL_MAX_Q_MIXED;
  const size_t call_bytes = tune_call_bytes(n, p, S, M, with_mixed);
  const size_t rec_bytes = tune_records_bytes(S, M);
  if (call_bytes == 0 || work_bytes < call_bytes + 2 * rec_bytes) return -15;
  hipStream_t s = (hipStream_t)stream;
  pl_result* rec_ref = reinterpret_cast<pl_result*>((char*)work + call_bytes);
  pl_result* rec_c = reinterpret_cast<pl_result*>((char*)work + call_bytes + rec_bytes);

  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return PL_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return PL_E_HIP;
  }
  std::vector<pl_result> href((size_t)S * M), hc((size_t)S * M);
  double ms_per[TUNE_NCAND], err[TUNE_NCAND];
  int rc = PL_OK;
  for (int c = 0; c < TUNE_NCAND && rc == PL_OK; ++c) {
    ms_per[c] = -1.0;
    err[c] = -1.0;
    if (c > 0 && !with_mixed) continue;
    pl_opts o = *opts;
    o.precision = c == 0 ? PL_FP64 : PL_MIXED;
    o.flush = kTuneFlush[c];
    pl_result* dst = c == 0 ? rec_ref : rec_c;
    // one untimed call (first use of the kernels), then two timed
    rc = pl_profile_loglik(locs, y, X, n, p, omega, S, lambda, M, dst, nullptr, nullptr, &o,
                           work, call_bytes, stream);
    if (rc != PL_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) { rc = PL_E_HIP; break; }
    for (int r = 0; r < 2 && rc == PL_OK; ++r)
      rc = pl_profile_loglik(locs, y, X, n, p, omega, S, lambda, M, dst, nullptr, nullptr, &o,
                             work, call_bytes, stream);
    if (rc != PL_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = PL_E_HIP;
      break;
    }
    ms_per[c] = ms / 2.0 / (double)S;
    std::vector<pl_result>& h = c == 0 ? href : hc;
    if (hipMemcpy(h.data(), dst, (size_t)S * M * sizeof(pl_result), hipMemcpyDeviceToHost) !=
        hipSuccess) {
      rc = PL_E_HIP;
      break;
    }
    if (c == 0) {
      err[c] = 0.0;
      continue;
    }
    // largest |delta loglik| over records that FP64 evaluated; a record that is
    // finite in one form only disqualifies the candidate
    double e = 0.0;
    for (size_t i = 0; i < href.size(); ++i) {
      const double a = href[i].loglik, b = hc[i].loglik;
      if (std::isfinite(a) != std::isfinite(b)) {
        e = INFINITY;
        break;
      }
      if (std::isfinite(a)) e = std::max(e, fabs(a - b));
    }
    err[c] = e;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != PL_OK) return rc;
  int best = 0;
  for (int c = 1; c < TUNE_NCAND; ++c)
    if (ms_per[c] >= 0.0 && err[c] >= 0.0 && err[c] <= tol && ms_per[c] < ms_per[best]) best = c;
  opts->precision = best == 0 ? PL_FP64 : PL_MIXED;
  opts->flush = kTuneFlush[best];
  tune_cache_put(0, n, 0, M + p, tol, *opts, ms_per[best] * S);
  if (report) {
    for (int c = 0; c < TUNE_NCAND; ++c) {
      report[c] = ms_per[c];
      report[TUNE_NCAND + c] = err[c];
    }
  }
  return PL_OK;
}

int pl_profiling_enable(int on) {
  for (auto& r : g_prof.recs) {
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.recs.clear();
  g_prof.on = on != 0;
  return PL_OK;
}

int pl_profiling_read(double* ms, double* alg_flops, int64_t* launches, int nclass) {
  if (nclass < 1 || nclass > PL_KC_COUNT) return -1;
  if (!ms) return -2;
  if (!alg_flops) return -3;
  if (!launches) return -4;
  for (int c = 0; c < nclass; ++c) {
    ms[c] = 0.0;
    alg_flops[c] = 0.0;
    launches[c] = 0;
  }
  for (auto& r : g_prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return PL_E_HIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return PL_E_HIP;
    if (r.cls < nclass) {
      ms[r.cls] += t;
      alg_flops[r.cls] += r.flops;
      launches[r.cls] += 1;
    }
  }
  return PL_OK;
}

}  // extern "C"
