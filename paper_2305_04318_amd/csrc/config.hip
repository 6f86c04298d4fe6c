// Representative parameter points (Step 2 of the method, Section 3.2):
// a numerical Hessian of the profile log-likelihood in the internal
// parameters, evaluated in one batched likelihood call; the eigen-repair of
// minus the Hessian; points spread over the unit sphere (maximin) and mapped
// onto the ellipsoids of chi-square contour levels; the Box-Cox grid from the
// one-dimensional quadratic approximation in lambda; the nugget repair.
// Host code; the likelihoods come from pl_profile_loglik on the device.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

constexpr int NS = 5;

// ---- chi-square quantiles ------------------------------------------------
// Regularised incomplete gamma functions: the power series of the lower
// function for x < a + 1 and the continued fraction of the upper function
// otherwise (Abramowitz & Stegun 6.5.29 and 6.5.31), the continued fraction
// evaluated by the modified Lentz method.
double gamma_p_series(double a, double x) {
  double term = 1.0 / a, sum = term;
  for (int k = 1; k < 1000; ++k) {
    term *= x / (a + k);
    sum += term;
    if (fabs(term) < 1e-17 * fabs(sum)) break;
  }
  return sum * exp(-x + a * log(x) - lgamma(a));
}

double gamma_q_fraction(double a, double x) {
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int k = 1; k < 1000; ++k) {
    const double an = -k * (k - a);
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < tiny) d = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return exp(-x + a * log(x) - lgamma(a)) * h;
}

// upper tail Q(a, x) = Gamma(a, x) / Gamma(a)
double gamma_q(double a, double x) {
  if (x <= 0.0) return 1.0;
  if (x < a + 1.0) return 1.0 - gamma_p_series(a, x);
  return gamma_q_fraction(a, x);
}

// q with Pr(chi^2_dof > q) = upper, by bisection on the monotone tail
double chisq_upper_quantile(int dof, double upper) {
  const double a = 0.5 * dof;
  double lo = 0.0, hi = 1.0;
  while (gamma_q(a, 0.5 * hi) > upper) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (gamma_q(a, 0.5 * mid) > upper) lo = mid;
    else hi = mid;
    if (hi - lo <= 1e-15 * hi) break;
  }
  return 0.5 * (lo + hi);
}

// ---- symmetric eigen-decomposition -----------------------------------------
// Cyclic Jacobi rotations (Golub & Van Loan, Section 8.5) on a d x d
// symmetric matrix (row-major).  w: eigenvalues ascending; V (row-major):
// column j is the eigenvector of w[j], normalised so that its entry of
// largest magnitude (the first such on ties) is positive.
void jacobi_eigh(int d, const double* A0, double* w, double* V) {
  std::vector<double> A(A0, A0 + d * d);
  for (int i = 0; i < d * d; ++i) V[i] = 0.0;
  for (int i = 0; i < d; ++i) V[i * d + i] = 1.0;
  double scale = 0.0;
  for (int i = 0; i < d * d; ++i) scale = std::max(scale, fabs(A[i]));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < d; ++i)
      for (int j = i + 1; j < d; ++j) off = std::max(off, fabs(A[i * d + j]));
    if (off <= 1e-300 || off <= 1e-17 * scale) break;
    for (int p = 0; p < d; ++p)
      for (int q = p + 1; q < d; ++q) {
        const double apq = A[p * d + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * d + q] - A[p * d + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < d; ++k) {  // columns p, q of A
          const double akp = A[k * d + p], akq = A[k * d + q];
          A[k * d + p] = c * akp - s * akq;
          A[k * d + q] = s * akp + c * akq;
        }
        for (int k = 0; k < d; ++k) {  // rows p, q of A
          const double apk = A[p * d + k], aqk = A[q * d + k];
          A[p * d + k] = c * apk - s * aqk;
          A[q * d + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < d; ++k) {
          const double vkp = V[k * d + p], vkq = V[k * d + q];
          V[k * d + p] = c * vkp - s * vkq;
          V[k * d + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> ord(d);
  for (int i = 0; i < d; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return A[a * d + a] < A[b * d + b]; });
  std::vector<double> Vs(d * d);
  for (int j = 0; j < d; ++j) {
    const int c = ord[j];
    w[j] = A[c * d + c];
    int big = 0;
    for (int k = 1; k < d; ++k)
      if (fabs(V[k * d + c]) > fabs(V[big * d + c])) big = k;
    const double sg = V[big * d + c] < 0.0 ? -1.0 : 1.0;
    for (int k = 0; k < d; ++k) Vs[k * d + j] = sg * V[k * d + c];
  }
  std::copy(Vs.begin(), Vs.end(), V);
}

// ---- internal parameters ----------------------------------------------------
// natural omega for the likelihood: gamma1, gamma2, gamma3 by their
// definitions, the shape by the chosen transform, nugget = nu^2
void internal_to_natural_eval(const double* w, int st, double* om) {
  const double ratio = 1.0 + w[3] * w[3] + w[4] * w[4];
  om[0] = exp(0.5 * (w[0] + log(ratio)));
  om[1] = st == 0 ? exp(w[1]) : 1.0 / (w[1] * w[1]);
  om[2] = w[2] * w[2];
  om[3] = ratio;
  om[4] = 0.5 * atan2(w[4], w[3]);
}

inline bool usable(int32_t info) { return info == 0 || info == PL_INFO_FALLBACK; }

// the coordinates varied: all five, or all but the shape
int free_coords(int fix_shape, int* idx) {
  int d = 0;
  for (int i = 0; i < NS; ++i)
    if (!(fix_shape && i == 1)) idx[d++] = i;
  return d;
}

}  // namespace

extern "C" {

int pl_chisq_quantile(int dof, double upper, double* q) {
  if (dof < 1 || dof > 1000) return -1;
  if (!(upper > 0.0) || !(upper < 1.0)) return -2;
  if (!q) return -3;
  *q = chisq_upper_quantile(dof, upper);
  return PL_OK;
}

int pl_sphere_points(int d, int64_t npts, const double* init, int iters, double* out,
                     double* min_dist) {
  if (d < 2 || d > 16) return -1;
  if (npts < 2 || npts > 100000) return -2;
  if (!init) return -3;
  if (iters < 0) return -4;
  if (!out) return -5;
  std::vector<double> x(init, init + d * npts);
  for (int64_t i = 0; i < npts; ++i) {
    double nr = 0.0;
    for (int k = 0; k < d; ++k) nr += x[i * d + k] * x[i * d + k];
    nr = sqrt(nr);
    if (!(nr > 0.0) || !isfinite(nr)) return -3;
    for (int k = 0; k < d; ++k) x[i * d + k] /= nr;
  }
  auto closest = [&](const std::vector<double>& y) {
    double m = INFINITY;
    for (int64_t i = 0; i < npts; ++i)
      for (int64_t j = i + 1; j < npts; ++j) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
          const double t = y[i * d + k] - y[j * d + k];
          s += t * t;
        }
        m = std::min(m, s);
      }
    return sqrt(m);
  };
  // repulsion: each point moves along the tangential part of sum_j
  // (x_i - x_j) / |x_i - x_j|^(S+2) (the gradient of a Riesz S-energy, whose
  // minimisers approach the maximin arrangement as S grows) by a step that is
  // a shrinking fraction of the current closest distance; the arrangement
  // with the largest closest distance is kept
  constexpr double ETA = 0.3;  // S = 8: weight |x_i - x_j|^-10
  std::vector<double> best = x, F(d * npts);
  double dmin = closest(x), bmin = dmin;
  for (int it = 0; it < iters; ++it) {
    for (int64_t i = 0; i < npts; ++i) {
      double* f = &F[i * d];
      for (int k = 0; k < d; ++k) f[k] = 0.0;
      for (int64_t j = 0; j < npts; ++j) {
        if (j == i) continue;
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
          const double t = x[i * d + k] - x[j * d + k];
          r2 += t * t;
        }
        if (r2 <= 0.0) continue;  // coincident points: no direction
        const double inv = 1.0 / r2, inv2 = inv * inv;
        const double wgt = inv2 * inv2 * inv;
        for (int k = 0; k < d; ++k) f[k] += wgt * (x[i * d + k] - x[j * d + k]);
      }
      double radial = 0.0;
      for (int k = 0; k < d; ++k) radial += f[k] * x[i * d + k];
      double nf = 0.0;
      for (int k = 0; k < d; ++k) {
        f[k] -= radial * x[i * d + k];
        nf += f[k] * f[k];
      }
      nf = sqrt(nf);
      const double step = nf > 0.0 ? ETA * dmin * (1.0 - (double)it / iters) / nf : 0.0;
      for (int k = 0; k < d; ++k) f[k] *= step;
    }
    for (int64_t i = 0; i < npts; ++i) {
      double nr = 0.0;
      for (int k = 0; k < d; ++k) {
        x[i * d + k] += F[i * d + k];
        nr += x[i * d + k] * x[i * d + k];
      }
      nr = sqrt(nr);
      for (int k = 0; k < d; ++k) x[i * d + k] /= nr;
    }
    dmin = closest(x);
    if (dmin > bmin) {
      bmin = dmin;
      best = x;
    }
  }
  std::copy(best.begin(), best.end(), out);
  if (min_dist) *min_dist = bmin;
  return PL_OK;
}

int pl_hessian_workspace_size(int64_t n, int64_t p, const pl_opts* opts, size_t* bytes) {
  if (!bytes) return -4;
  size_t ws = 0;
  const int rc = pl_workspace_size(n, p, PL_HESS_POINTS, 3, opts, &ws);
  if (rc == -5) return -3;
  if (rc != PL_OK) return rc;
  *bytes = ((ws + 255) / 256) * 256 + (size_t)PL_HESS_POINTS * 3 * sizeof(pl_result);
  return PL_OK;
}

int pl_hessian(const double* locs, const double* y, const double* X, int64_t n, int64_t p,
               const double* omega_hat, double lambda_hat, int shape_transform, int fix_shape,
               double delta, double* hess, double* lambda_curv, double* loglik_center,
               const pl_opts* opts, void* work, size_t work_bytes, void* stream) {
  if (!locs) return -1;
  if (!y) return -2;
  if (!X) return -3;
  if (n < 2) return -4;
  if (p < 1 || p >= n || p > PL_MAX_P) return -5;
  if (!omega_hat) return -6;
  for (int i = 0; i < NS; ++i)
    if (!isfinite(omega_hat[i])) return -6;
  if (!(omega_hat[0] > 0.0) || !(omega_hat[1] > 0.0) || !(omega_hat[2] > 0.0) ||
      !(omega_hat[3] > 0.0))
    return -6;
  if (!isfinite(lambda_hat)) return -7;
  if (shape_transform != 0 && shape_transform != 1) return -8;
  if (fix_shape != 0 && fix_shape != 1) return -9;
  if (!(delta > 0.0) || !(delta <= 1.0)) return -10;
  if (!hess) return -11;
  if (!work) return -15;
  size_t need = 0;
  int rc = pl_hessian_workspace_size(n, p, opts, &need);
  if (rc == -1) return -4;
  if (rc == -3) return -14;
  if (rc != PL_OK) return rc;
  if (work_bytes < need) return -16;

  int idx[NS];
  const int d = free_coords(fix_shape, idx);
  double w0[NS];
  if (pl_to_internal(omega_hat, 1, shape_transform, w0) != PL_OK) return -6;
  const double* w0p = w0;
  // stencil: centre; +-delta along each coordinate; (+-delta, +-delta) on
  // each pair -- 1 + 2d + 2d(d-1) points (51 for d = 5, 33 for d = 4)
  std::vector<double> pts;
  auto add = [&](int i, double si, int j, double sj) {
    double w[NS];
    for (int k = 0; k < NS; ++k) w[k] = w0p[k];
    if (i >= 0) w[idx[i]] += si * delta;
    if (j >= 0) w[idx[j]] += sj * delta;
    double om[NS];
    internal_to_natural_eval(w, shape_transform, om);
    if (fix_shape) om[1] = omega_hat[1];  // held exactly
    for (int k = 0; k < NS; ++k) pts.push_back(om[k]);
  };
  add(-1, 0, -1, 0);
  for (int i = 0; i < d; ++i) {
    add(i, 1.0, -1, 0);
    add(i, -1.0, -1, 0);
  }
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j) {
      add(i, 1.0, j, 1.0);
      add(i, 1.0, j, -1.0);
      add(i, -1.0, j, 1.0);
      add(i, -1.0, j, -1.0);
    }
  const int64_t K = (int64_t)pts.size() / NS;
  for (int64_t k = 0; k < K; ++k) {
    const double sh = pts[NS * k + 1];
    if (!(sh >= PL_MIN_SHAPE && sh <= PL_MAX_SHAPE)) return PL_E_UNSUPPORTED;
  }
  const double lam[3] = {lambda_hat - delta, lambda_hat, lambda_hat + delta};
  size_t ws = 0;
  pl_workspace_size(n, p, PL_HESS_POINTS, 3, opts, &ws);
  pl_result* rec_d = reinterpret_cast<pl_result*>((char*)work + ((ws + 255) / 256) * 256);
  rc = pl_profile_loglik(locs, y, X, n, p, pts.data(), K, lam, 3, rec_d, nullptr, nullptr, opts,
                         work, ws, stream);
  if (rc == -13) return -14;
  if (rc != PL_OK) return rc;
  std::vector<pl_result> rec(K * 3);
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(rec.data(), rec_d, rec.size() * sizeof(pl_result), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return PL_E_HIP;
  for (const pl_result& r : rec)
    if (!usable(r.info)) return PL_E_UNSUPPORTED;
  auto f = [&](int64_t k, int m) { return rec[k * 3 + m].loglik; };
  const double f0 = f(0, 1), h2 = delta * delta;
  for (int i = 0; i < d; ++i) hess[i * d + i] = (f(1 + 2 * i, 1) - 2.0 * f0 + f(2 + 2 * i, 1)) / h2;
  int64_t k = 1 + 2 * d;
  for (int i = 0; i < d; ++i)
    for (int j = i + 1; j < d; ++j, k += 4) {
      const double v = (f(k, 1) - f(k + 1, 1) - f(k + 2, 1) + f(k + 3, 1)) / (4.0 * h2);
      hess[i * d + j] = hess[j * d + i] = v;
    }
  if (lambda_curv) *lambda_curv = (f(0, 0) - 2.0 * f0 + f(0, 2)) / h2;
  if (loglik_center) *loglik_center = f0;
  return PL_OK;
}

int pl_config_points(const double* omega_hat, int shape_transform, int fix_shape,
                     const double* hess, const double* alpha, int64_t nlev, const double* sphere,
                     int64_t npts, const double* uniforms, double* omega_out, double* eigvals,
                     int64_t* nugget_repaired) {
  if (!omega_hat) return -1;
  if (shape_transform != 0 && shape_transform != 1) return -2;
  if (fix_shape != 0 && fix_shape != 1) return -3;
  if (!hess) return -4;
  if (!alpha) return -5;
  if (nlev < 1 || nlev > 1024) return -6;
  for (int64_t l = 0; l < nlev; ++l)
    if (!(alpha[l] > 0.0 && alpha[l] < 1.0)) return -5;
  if (!sphere) return -7;
  if (npts < 1 || npts > 1000000) return -8;
  if (!uniforms) return -9;
  if (!omega_out) return -10;
  double w0[NS];
  if (pl_to_internal(omega_hat, 1, shape_transform, w0) != PL_OK) return -1;
  int idx[NS];
  const int d = free_coords(fix_shape, idx);
  for (int i = 0; i < d * d; ++i)
    if (!isfinite(hess[i])) return -4;
  // minus the Hessian, symmetrised
  double A[NS * NS], D[NS], E[NS * NS];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) A[i * d + j] = -0.5 * (hess[i * d + j] + hess[j * d + i]);
  jacobi_eigh(d, A, D, E);
  // repair: negative eigenvalues -> absolute values; when the largest
  // exceeds 100, every eigenvalue below 0.1 -> 0.1
  double dmax = 0.0;
  for (int i = 0; i < d; ++i) {
    D[i] = fabs(D[i]);
    dmax = std::max(dmax, D[i]);
  }
  if (dmax > 100.0)
    for (int i = 0; i < d; ++i) D[i] = std::max(D[i], 0.1);
  for (int i = 0; i < d; ++i)
    if (!(D[i] > 0.0)) return PL_E_UNSUPPORTED;  // a flat direction: no ellipsoid
  if (eigvals) {
    for (int i = 0; i < d; ++i) eigvals[i] = D[i];
    std::sort(eigvals, eigvals + d);
  }
  // x' = w0 + sqrt(q) E D^(-1/2) x on every level (upper-tail probability alpha)
  int64_t negatives = 0;
  for (int64_t l = 0; l < nlev; ++l) {
    const double rq = sqrt(chisq_upper_quantile(d, alpha[l]));
    for (int64_t t = 0; t < npts; ++t) {
      const double* x = sphere + t * d;
      double w[NS];
      for (int k = 0; k < NS; ++k) w[k] = w0[k];
      for (int i = 0; i < d; ++i) {
        double v = 0.0;
        for (int j = 0; j < d; ++j) v += E[i * d + j] * x[j] / sqrt(D[j]);
        w[idx[i]] += rq * v;
      }
      const int64_t o = l * npts + t;
      double* om = omega_out + NS * o;
      const double ratio = 1.0 + w[3] * w[3] + w[4] * w[4];
      om[0] = exp(0.5 * (w[0] + log(ratio)));
      if (fix_shape) om[1] = omega_hat[1];
      else if (shape_transform == 0) om[1] = exp(w[1]);
      else om[1] = w[1] > 0.0 ? 1.0 / (w[1] * w[1]) : PL_MAX_SHAPE;
      om[1] = std::min(PL_MAX_SHAPE, std::max(PL_MIN_SHAPE, om[1]));
      om[3] = ratio;
      om[4] = 0.5 * atan2(w[4], w[3]);
      if (w[2] >= 0.0) {
        om[2] = w[2] * w[2];
      } else {
        // a negative nugget: alternately 0 and a uniform draw on (0, 2)
        om[2] = (negatives % 2 == 0) ? 0.0 : 2.0 * uniforms[o];
        ++negatives;
      }
    }
  }
  if (nugget_repaired) *nugget_repaired = negatives;
  return PL_OK;
}

int pl_lambda_grid(double lambda_hat, double lambda_curv, double tail, int64_t m, double* out) {
  if (!isfinite(lambda_hat)) return -1;
  if (!isfinite(lambda_curv) || lambda_curv == 0.0) return -2;
  if (!(tail > 0.0 && tail < 0.5)) return -3;
  if (m < 2 || m > PL_MAX_M) return -4;
  if (!out) return -5;
  // normal quantile from the chi-square one: z_(1-tail)^2 = chi^2_1 upper 2 tail
  const double z = sqrt(chisq_upper_quantile(1, 2.0 * tail));
  const double half = z / sqrt(fabs(lambda_curv));
  for (int64_t i = 0; i < m; ++i)
    out[i] = lambda_hat - half + 2.0 * half * (double)i / (double)(m - 1);
  return PL_OK;
}

}  // extern "C"
