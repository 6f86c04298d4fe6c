// Univariate profile likelihoods of the correlation parameters and of lambda
// from the evaluated points, and their likelihood intervals (Step 4 of the
// method; Section 3.6, "Profile likelihood for correlation parameters";
// Section 2's likelihood-based interval).  Host code: a few thousand points.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace {

inline bool usable(int32_t info) { return info == 0 || info == PL_INFO_FALLBACK; }

struct Pt {
  double x, y;
};

// Upper convex hull of points sorted by x with distinct x (monotone chain):
// a point is dropped when it lies on or below the segment joining its
// neighbours on the hull.
std::vector<Pt> upper_hull(const std::vector<Pt>& p) {
  std::vector<Pt> h;
  for (const Pt& q : p) {
    while (h.size() >= 2) {
      const Pt& a = h[h.size() - 2];
      const Pt& b = h[h.size() - 1];
      // cross((b - a), (q - a)) >= 0: b is not above the chord a-q
      const double cr = (b.x - a.x) * (q.y - a.y) - (b.y - a.y) * (q.x - a.x);
      if (cr >= 0.0) h.pop_back();
      else break;
    }
    h.push_back(q);
  }
  return h;
}

}  // namespace

extern "C" int pl_profile_param(const pl_result* rec, int64_t K, int64_t M, const double* omega,
                                const double* lambda, int which, double drop, double* curve_x,
                                double* curve_y, int64_t* npts, double* interval,
                                int32_t* open_ends) {
  if (!rec) return -1;
  if (K < 1 || K > (1 << 24)) return -2;
  if (M < 1 || M > PL_MAX_M) return -3;
  if (!omega && which != 5) return -4;
  if (!lambda && which == 5) return -5;
  if (which < 0 || which > 5) return -6;
  if (!(drop > 0.0) || !isfinite(drop)) return -7;
  if (!curve_x) return -8;
  if (!curve_y) return -9;
  if (!npts) return -10;
  if (!interval) return -11;
  // point cloud: (theta_k, max_m l) for a correlation parameter, (lambda_m,
  // max_k l) for lambda; equal abscissae keep their largest likelihood
  std::vector<Pt> pts;
  if (which == 5) {
    for (int64_t m = 0; m < M; ++m) {
      double best = -INFINITY;
      for (int64_t k = 0; k < K; ++k) {
        const pl_result& r = rec[k * M + m];
        if (usable(r.info) && r.loglik > best) best = r.loglik;
      }
      if (isfinite(best) && isfinite(lambda[m])) pts.push_back({lambda[m], best});
    }
  } else {
    for (int64_t k = 0; k < K; ++k) {
      double best = -INFINITY;
      for (int64_t m = 0; m < M; ++m) {
        const pl_result& r = rec[k * M + m];
        if (usable(r.info) && r.loglik > best) best = r.loglik;
      }
      const double x = omega[5 * k + which];
      if (isfinite(best) && isfinite(x)) pts.push_back({x, best});
    }
  }
  *npts = 0;
  if (open_ends) *open_ends = 0;
  if (pts.empty()) {
    interval[0] = interval[1] = interval[2] = NAN;
    return PL_OK;
  }
  std::sort(pts.begin(), pts.end(), [](const Pt& a, const Pt& b) {
    return a.x < b.x || (a.x == b.x && a.y > b.y);
  });
  std::vector<Pt> uniq;
  for (const Pt& q : pts)
    if (uniq.empty() || q.x != uniq.back().x) uniq.push_back(q);
  // lambda: interpolation of all points; correlation parameters: the hull
  const std::vector<Pt> c = (which == 5) ? uniq : upper_hull(uniq);
  const int64_t nc = (int64_t)c.size();
  for (int64_t i = 0; i < nc; ++i) {
    curve_x[i] = c[i].x;
    curve_y[i] = c[i].y;
  }
  *npts = nc;
  // likelihood interval: where the piecewise-linear curve stays within
  // `drop` of its maximum; an end that never drops is reported at the last
  // vertex and flagged open
  int64_t im = 0;
  for (int64_t i = 1; i < nc; ++i)
    if (c[i].y > c[im].y) im = i;
  const double thr = c[im].y - drop;
  double lo = c[0].x, hi = c[nc - 1].x;
  int32_t open = 3;
  for (int64_t i = im; i > 0; --i) {
    if (c[i - 1].y < thr) {
      const double f = (c[i].y - thr) / (c[i].y - c[i - 1].y);
      lo = c[i].x - f * (c[i].x - c[i - 1].x);
      open &= ~1;
      break;
    }
  }
  for (int64_t i = im; i + 1 < nc; ++i) {
    if (c[i + 1].y < thr) {
      const double f = (c[i].y - thr) / (c[i].y - c[i + 1].y);
      hi = c[i].x + f * (c[i + 1].x - c[i].x);
      open &= ~2;
      break;
    }
  }
  interval[0] = c[im].x;
  interval[1] = lo;
  interval[2] = hi;
  if (open_ends) *open_ends = open;
  return PL_OK;
}
