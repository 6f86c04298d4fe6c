// Maximum-likelihood estimates of (omega, lambda) by numerical maximisation of
// the profile likelihood (Step 1 of the method, Section 3.1), and the internal
// parametrisation of Step 2 (Section 3.2, "Reparameterization").  Host code
// driving pl_profile_loglik: every likelihood is evaluated on the device.
//
// The maximiser is a batched compass (coordinate pattern) search: each
// iteration evaluates the +-h neighbours along every free coordinate of every
// start in ONE pl_profile_loglik call, so a launch carries 10 x starts points
// instead of the one point per launch of a sequential quasi-Newton method.
// lambda is maximised over the columns of the same call (the M Box-Cox values
// share one factorisation of V), then refined on a fine grid around the best
// value, and omega is polished once more at that grid.
//
// Search coordinates (all unconstrained):
//   s0 = gamma1 = log phi_X + log phi_Y,  s1 = log kappa,  s2 = log nu^2,
//   s3 = gamma2 = sqrt(phi_X/phi_Y - 1) cos(2 phi_A),
//   s4 = gamma3 = sqrt(phi_X/phi_Y - 1) sin(2 phi_A),
// the internal parametrisation of Step 2 with log kappa for the shape and
// log nu^2 for the nugget (both positive).
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

// A model with ratio phi_X/phi_Y < 1 is the model with the axes exchanged:
// phi_X' = phi_Y = phi_X/ratio, ratio' = 1/ratio, angle' = angle + pi/2.
void canonical(const double* om, double& phix, double& ratio, double& angle) {
  phix = om[0];
  ratio = om[3];
  angle = om[4];
  if (ratio < 1.0) {
    phix = om[0] / ratio;
    ratio = 1.0 / ratio;
    angle = om[4] + 0.5 * M_PI;
  }
}

void aniso_to(const double* om, double& g1, double& g2, double& g3) {
  double phix, ratio, angle;
  canonical(om, phix, ratio, angle);
  const double r = sqrt(ratio - 1.0);
  g1 = 2.0 * log(phix) - log(ratio);  // log phi_X + log phi_Y
  g2 = r * cos(2.0 * angle);
  g3 = r * sin(2.0 * angle);
}

// phi_X, ratio, angle from (gamma1, gamma2, gamma3); angle in (-pi/2, pi/2]
void aniso_from(double g1, double g2, double g3, double* om) {
  const double ratio = 1.0 + g2 * g2 + g3 * g3;
  om[0] = exp(0.5 * (g1 + log(ratio)));
  om[3] = ratio;
  om[4] = 0.5 * atan2(g3, g2);
}

void to_search(const double* om, double* s) {
  aniso_to(om, s[0], s[3], s[4]);
  s[1] = log(om[1]);
  s[2] = log(om[2]);
}

void from_search(const double* s, double* om) {
  aniso_from(s[0], s[3], s[4], om);
  om[1] = std::min(PL_MAX_SHAPE, std::max(PL_MIN_SHAPE, exp(s[1])));
  om[2] = exp(s[2]);
}

inline bool usable(int32_t info) { return info == 0 || info == PL_INFO_FALLBACK; }

constexpr int NS = 5;          // search coordinates
constexpr double H0 = 0.5;     // initial step
constexpr double HMAX = 2.0;   // largest step

struct Evaluator {
  const double *locs, *y, *X;
  int64_t n, p;
  int reml;
  const pl_opts* opts;
  void* work;
  size_t ws;  // bytes of work given to pl_profile_loglik
  pl_result* rec_d;
  std::vector<pl_result> rec_h;
  hipStream_t stream;
  const double* omega0;  // starts: a held shape or nugget keeps its value exactly
  int32_t fixed;

  void natural(const double* s, int64_t start, double* om) const {
    from_search(s, om);
    if (fixed & 2) om[1] = omega0[NS * start + 1];
    if (fixed & 4) om[2] = omega0[NS * start + 2];
  }

  // value of every candidate (search coordinates; candidate k belongs to
  // start owner[k]) = max over the lambda set of the (restricted) profile
  // log-likelihood; -inf when no record is usable
  int operator()(const std::vector<double>& s, const std::vector<int64_t>& owner,
                 const double* lam, int64_t Ml, std::vector<double>& val,
                 std::vector<double>& lamv) {
    const int64_t kc = (int64_t)s.size() / NS;
    std::vector<double> om(NS * kc);
    for (int64_t k = 0; k < kc; ++k) natural(&s[NS * k], owner[k], &om[NS * k]);
    const int r = pl_profile_loglik(locs, y, X, n, p, om.data(), kc, lam, Ml, rec_d, nullptr,
                                    nullptr, opts, work, ws, stream);
    if (r == -13) return -18;  // the caller's options
    if (r != PL_OK) return r;
    if (hipMemcpyAsync(rec_h.data(), rec_d, (size_t)kc * Ml * sizeof(pl_result),
                       hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return PL_E_HIP;
    val.assign(kc, -INFINITY);
    lamv.assign(kc, NAN);
    for (int64_t k = 0; k < kc; ++k)
      for (int64_t m = 0; m < Ml; ++m) {
        const pl_result& q = rec_h[k * Ml + m];
        const double v = reml ? q.loglik_reml : q.loglik;
        if (usable(q.info) && v > val[k]) {
          val[k] = v;
          lamv[k] = lam[m];
        }
      }
    return PL_OK;
  }
};

// Compass search from every start in x (starts x NS); f and lam hold the
// starts' current values.  Returns the iterations used in *its.
int compass(Evaluator& ev, std::vector<double>& x, const std::vector<int64_t>& ids,
            std::vector<double>& f, std::vector<double>& lam, double h0,
            const double* lamset, int64_t Ml, int32_t fixed, double tol, int max_iter,
            int* its) {
  const int64_t starts = (int64_t)f.size();
  std::vector<double> h(NS * starts, h0);
  std::vector<double> cand, val, lamv;
  std::vector<int64_t> owner, start_of, first(starts), count(starts);
  int it = 0;
  for (; it < max_iter; ++it) {
    cand.clear();
    owner.clear();
    start_of.clear();
    for (int64_t st = 0; st < starts; ++st) {
      first[st] = (int64_t)owner.size();
      count[st] = 0;
      double hmax = 0.0;
      for (int i = 0; i < NS; ++i)
        if (!(fixed & (1 << i))) hmax = std::max(hmax, h[NS * st + i]);
      if (hmax < tol || !isfinite(f[st])) continue;  // converged, or no usable start
      for (int i = 0; i < NS; ++i) {
        if (fixed & (1 << i)) continue;
        for (int sg = -1; sg <= 1; sg += 2) {
          for (int j = 0; j < NS; ++j)
            cand.push_back(x[NS * st + j] + (j == i ? sg * h[NS * st + i] : 0.0));
          owner.push_back(st);
          start_of.push_back(ids[st]);
          ++count[st];
        }
      }
    }
    if (owner.empty()) break;
    const int rc = ev(cand, start_of, lamset, Ml, val, lamv);
    if (rc != PL_OK) return rc;
    for (int64_t st = 0; st < starts; ++st) {
      if (count[st] == 0) continue;
      int64_t best = -1;
      for (int64_t c = first[st]; c < first[st] + count[st]; ++c)
        if (val[c] > f[st] && (best < 0 || val[c] > val[best])) best = c;
      if (best >= 0) {
        // move; a successful direction doubles its step
        for (int j = 0; j < NS; ++j) {
          if (cand[NS * best + j] != x[NS * st + j])
            h[NS * st + j] = std::min(HMAX, 2.0 * h[NS * st + j]);
          x[NS * st + j] = cand[NS * best + j];
        }
        f[st] = val[best];
        lam[st] = lamv[best];
      } else {
        for (int j = 0; j < NS; ++j) h[NS * st + j] *= 0.5;
      }
    }
  }
  *its += it;
  return PL_OK;
}

int64_t fine_columns(int64_t p, const pl_opts* opts) {
  // the mixed form carries at most PL_MAX_Q_MIXED bordered columns (M + p)
  if (opts && opts->precision == PL_MIXED) return std::min<int64_t>(PL_MAX_M, PL_MAX_Q_MIXED - p);
  return PL_MAX_M;
}

}  // namespace

extern "C" {

int pl_to_internal(const double* omega, int64_t K, int shape_transform, double* internal) {
  if (!omega) return -1;
  if (K < 1) return -2;
  if (shape_transform != 0 && shape_transform != 1) return -3;
  if (!internal) return -4;
  for (int64_t k = 0; k < K; ++k) {
    const double* om = omega + NS * k;
    for (int i = 0; i < NS; ++i)
      if (!isfinite(om[i])) return -1;
    if (!(om[0] > 0.0) || !(om[1] > 0.0) || !(om[2] >= 0.0) || !(om[3] > 0.0)) return -1;
  }
  for (int64_t k = 0; k < K; ++k) {
    const double* om = omega + NS * k;
    double* w = internal + NS * k;
    aniso_to(om, w[0], w[3], w[4]);
    w[1] = shape_transform == 0 ? log(om[1]) : 1.0 / sqrt(om[1]);
    w[2] = sqrt(om[2]);
  }
  return PL_OK;
}

int pl_from_internal(const double* internal, int64_t K, int shape_transform, double* omega) {
  if (!internal) return -1;
  if (K < 1) return -2;
  if (shape_transform != 0 && shape_transform != 1) return -3;
  if (!omega) return -4;
  for (int64_t k = 0; k < K; ++k) {
    const double* w = internal + NS * k;
    for (int i = 0; i < NS; ++i)
      if (!isfinite(w[i])) return -1;
    if (shape_transform == 1 && !(w[1] > 0.0)) return -1;
  }
  for (int64_t k = 0; k < K; ++k) {
    const double* w = internal + NS * k;
    double* om = omega + NS * k;
    aniso_from(w[0], w[3], w[4], om);
    om[1] = shape_transform == 0 ? exp(w[1]) : 1.0 / (w[1] * w[1]);
    om[2] = w[2] * fabs(w[2]);  // a negative nu maps to a negative nugget
  }
  return PL_OK;
}

int pl_mle_workspace_size(int64_t n, int64_t p, int64_t starts, int64_t M, const pl_opts* opts,
                          size_t* bytes) {
  if (starts < 1 || starts > PL_MLE_MAX_STARTS) return -3;
  if (M < 1 || M > PL_MAX_M) return -4;
  if (!bytes) return -6;
  const int64_t Kc = starts * 2 * NS;
  const int64_t Mw = std::max<int64_t>(M, std::max<int64_t>(1, fine_columns(p, opts)));
  size_t ws = 0;
  const int rc = pl_workspace_size(n, p, Kc, Mw, opts, &ws);
  if (rc != PL_OK) return rc;
  *bytes = ((ws + 255) / 256) * 256 + (size_t)Kc * Mw * sizeof(pl_result);
  return PL_OK;
}

int pl_mle(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
           const double* omega0, int64_t starts, const double* lambda, int64_t M,
           int32_t fixed_mask, int32_t reml, double tol, int32_t max_iter, double* omega_hat,
           double* lambda_hat, double* loglik_hat, int32_t* iterations, const pl_opts* opts,
           void* work, size_t work_bytes, void* stream) {
  if (!locs) return -1;
  if (!y) return -2;
  if (!X) return -3;
  if (n < 2) return -4;
  if (p < 1 || p >= n || p > PL_MAX_P) return -5;
  if (!omega0) return -6;
  if (starts < 1 || starts > PL_MLE_MAX_STARTS) return -7;
  for (int64_t s = 0; s < NS * starts; ++s)
    if (!isfinite(omega0[s])) return -6;
  for (int64_t s = 0; s < starts; ++s) {
    const double* om = omega0 + NS * s;
    if (!(om[0] > 0.0) || !(om[1] >= PL_MIN_SHAPE) || !(om[1] <= PL_MAX_SHAPE) ||
        !(om[2] > 0.0) || !(om[3] > 0.0))
      return -6;
  }
  if (!lambda) return -8;
  if (M < 1 || M > PL_MAX_M) return -9;
  for (int64_t m = 0; m < M; ++m)
    if (!isfinite(lambda[m])) return -8;
  if (fixed_mask < 0 || fixed_mask >= (1 << NS)) return -10;
  if (reml != 0 && reml != 1) return -11;
  if (!(tol > 0.0) || !(tol < H0)) return -12;
  if (max_iter < 1) return -13;
  if (!omega_hat) return -14;
  if (!lambda_hat) return -15;
  if (!loglik_hat) return -16;
  if (!work) return -19;
  size_t need = 0;
  int rc = pl_mle_workspace_size(n, p, starts, M, opts, &need);
  if (rc == -1) return -4;
  if (rc == -5) return -18;
  if (rc != PL_OK) return rc;
  if (work_bytes < need) return -20;

  const int64_t Kc = starts * 2 * NS;
  const int64_t Mf = fine_columns(p, opts);
  const int64_t Mw = std::max<int64_t>(M, std::max<int64_t>(1, Mf));
  Evaluator ev;
  ev.locs = locs;
  ev.y = y;
  ev.X = X;
  ev.n = n;
  ev.p = p;
  ev.reml = reml;
  ev.opts = opts;
  ev.work = work;
  rc = pl_workspace_size(n, p, Kc, Mw, opts, &ev.ws);
  if (rc != PL_OK) return rc;
  ev.rec_d = reinterpret_cast<pl_result*>((char*)work + ((ev.ws + 255) / 256) * 256);
  ev.rec_h.resize((size_t)Kc * Mw);
  ev.stream = (hipStream_t)stream;
  ev.omega0 = omega0;
  ev.fixed = fixed_mask;

  // phase 1: every start on the caller's lambda values
  std::vector<double> x(NS * starts), f, lam;
  std::vector<int64_t> ids(starts);
  for (int64_t s = 0; s < starts; ++s) {
    to_search(omega0 + NS * s, &x[NS * s]);
    ids[s] = s;
  }
  rc = ev(x, ids, lambda, M, f, lam);
  if (rc != PL_OK) return rc;
  int its = 0;
  rc = compass(ev, x, ids, f, lam, H0, lambda, M, fixed_mask, tol, max_iter, &its);
  if (rc != PL_OK) return rc;
  int64_t b = 0;
  for (int64_t s = 1; s < starts; ++s)
    if (f[s] > f[b]) b = s;
  if (!isfinite(f[b])) return PL_E_UNSUPPORTED;  // no start had a usable record
  std::vector<double> xb(x.begin() + NS * b, x.begin() + NS * b + NS);
  std::vector<double> fb{f[b]}, lb{lam[b]};
  const std::vector<int64_t> idb{b};

  // phase 2: lambda on Mf values -- the phase-1 value and Mf - 1 evenly
  // spaced ones between its neighbouring caller values (+-0.5 beyond the ends
  // of the caller's range) -- then omega polished on that set
  if (Mf >= 3) {
    double lo = -INFINITY, hi = INFINITY;
    for (int64_t m = 0; m < M; ++m) {
      if (lambda[m] < lb[0]) lo = std::max(lo, lambda[m]);
      if (lambda[m] > lb[0]) hi = std::min(hi, lambda[m]);
    }
    if (!isfinite(lo)) lo = lb[0] - 0.5;
    if (!isfinite(hi)) hi = lb[0] + 0.5;
    std::vector<double> fine(Mf);
    for (int64_t m = 0; m + 1 < Mf; ++m)
      fine[m] = lo + (hi - lo) * (double)m / (double)(Mf - 2);
    fine[Mf - 1] = lb[0];
    std::sort(fine.begin(), fine.end());
    std::vector<double> v, lv;
    rc = ev(xb, idb, fine.data(), Mf, v, lv);
    if (rc != PL_OK) return rc;
    if (isfinite(v[0])) {
      fb[0] = v[0];  // >= the phase-1 value up to rounding: lb[0] is in the set
      lb[0] = lv[0];
    }
    rc = compass(ev, xb, idb, fb, lb, std::min(H0, 16.0 * tol), fine.data(), Mf, fixed_mask,
                 tol, max_iter, &its);
    if (rc != PL_OK) return rc;
  }
  ev.natural(xb.data(), b, omega_hat);
  *lambda_hat = lb[0];
  *loglik_hat = fb[0];
  if (iterations) *iterations = its;
  return PL_OK;
}

}  // extern "C"
