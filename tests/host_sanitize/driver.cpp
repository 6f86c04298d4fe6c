// Host-only exercise of the library's host code, built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host side (device code is not built):
// argument checks of every entry point, workspace sizing, the persistent-batch
// planner, the Step 2 configuration code, the internal parameters and the
// Step 4 profile extraction.  No call reaches the device.  Exit status 0 when
// every check holds; a sanitizer report aborts the program.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <unistd.h>

#include <vector>

#include "plprof.h"

static int failures = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

// deterministic pseudo-random numbers (xorshift64*)
static uint64_t rs = 0x9E3779B97F4A7C15ull;
static double urand() {
  rs ^= rs >> 12;
  rs ^= rs << 25;
  rs ^= rs >> 27;
  return (double)((rs * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}
static double nrand() {
  const double u = urand() + 1e-300, v = urand();
  return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

static void workspace_sizes() {
  size_t b = 0;
  pl_opts o{};
  for (int prec = 0; prec < 2; ++prec) {
    o.precision = prec;
    for (int64_t n : {2, 3, 127, 128, 129, 2000, 8000})
      for (int64_t M : {1, 8, 28}) {
        const int rc = pl_workspace_size(n, 1, 5, M, &o, &b);
        CHECK(rc == 0 || (prec == 1 && rc == PL_E_UNSUPPORTED) || n <= 1);
      }
  }
  CHECK(pl_workspace_size(1, 1, 1, 1, nullptr, &b) == -1);
  CHECK(pl_matern_workspace_size(3, &b) == 0 && b > 0);
  CHECK(pl_chol_workspace_size(3, PL_MIXED, &b) == 0 && b > 0);
  CHECK(pl_chol_workspace_size(3, 7, &b) == -2);
  CHECK(pl_mle_workspace_size(500, 2, 12, 4, nullptr, &b) == 0);
  CHECK(pl_hessian_workspace_size(500, 2, nullptr, &b) == 0);
  CHECK(pl_curves_workspace_size(3, 4, 10, 10, &b) == 0);
  CHECK(pl_autotune_workspace_size(500, 2, 64, 4, 64, &b) == 0);
  // entry points that must return before any device work
  double om[5] = {1.0, 1.0, 0.1, 1.0, 0.0}, lam[2] = {0.0, 1.0};
  CHECK(pl_profile_loglik(nullptr, nullptr, nullptr, 10, 1, om, 1, lam, 2, nullptr, nullptr,
                          nullptr, nullptr, nullptr, 0, nullptr) == -1);
  CHECK(pl_profile_loglik_noalloc((double*)8, (double*)8, (double*)8, 9000, 2, om, 1, lam, 2,
                                  (pl_result*)8, nullptr, nullptr, nullptr, nullptr) == PL_E_SCRATCH);
  CHECK(pl_matern_cov((double*)8, 10, om, 1, 5, (void*)8, 10, (void*)8, 1 << 20, nullptr) == -5);
  CHECK(pl_chol_batched((void*)8, 10, 1, 12, PL_MIXED, (double*)8, (int32_t*)8, (void*)8, 1 << 20,
                        nullptr) == -1);
}

static void batch_planner() {
  // datasets of uneven size; device pointers are never dereferenced here
  std::vector<std::vector<double>> oms;
  std::vector<pl_dataset> ds;
  const int D = 37;
  for (int d = 0; d < D; ++d) {
    const int K = 1 + d % 5;
    std::vector<double> om;
    for (int k = 0; k < K; ++k) {
      om.insert(om.end(), {0.2 + urand(), 0.5 + 3 * urand(), 0.1, 1.0, 0.0});
    }
    oms.push_back(om);
  }
  for (int d = 0; d < D; ++d) {
    pl_dataset s{};
    s.locs = (const double*)16;
    s.y = (const double*)16;
    s.X = (const double*)16;
    s.n = 3 + (int64_t)(urand() * 700);
    s.omega = oms[d].data();
    s.K = (int64_t)oms[d].size() / 5;
    ds.push_back(s);
  }
  double lam[3] = {0.0, 0.5, 1.0};
  for (int64_t slabs : {0, 1, 3, 64}) {
    pl_opts o{};
    o.chunk = slabs;
    o.flags = PL_OPT_BATCH_PERSISTENT;
    pl_batch* b = nullptr;
    CHECK(pl_batch_create(ds.data(), D, 2, lam, 3, &o, &b) == 0 && b);
    int64_t units = 0, tasks = 0, ns = 0;
    size_t ws = 0;
    CHECK(pl_batch_stats(b, &units, &tasks, &ns) == 0 && units > 0 && tasks > units);
    CHECK(pl_batch_workspace_size(b, &ws) == 0 && ws > 0);
    pl_batch_destroy(b);
  }
  // the size-bucketed schedule, both forms, several pass sizes and streams
  for (int prec = 0; prec < 2; ++prec)
    for (int64_t chunk : {0, 1, 5}) {
      pl_opts o{};
      o.precision = prec;
      o.chunk = chunk;
      o.lanes = (int32_t)(1 + chunk % 4);
      pl_batch* b = nullptr;
      CHECK(pl_batch_create(ds.data(), D, 2, lam, 3, &o, &b) == 0 && b);
      int64_t units = 0, passes = 0, lanes = 0;
      size_t ws = 0;
      CHECK(pl_batch_stats(b, &units, &passes, &lanes) == 0 && units > 0 && passes >= 1 &&
            lanes == o.lanes);
      CHECK(pl_batch_workspace_size(b, &ws) == 0 && ws > 0);
      pl_batch_destroy(b);
    }
  pl_batch* b = nullptr;
  CHECK(pl_batch_create(ds.data(), 0, 2, lam, 3, nullptr, &b) == -2);
  ds[3].n = 1;
  CHECK(pl_batch_create(ds.data(), D, 2, lam, 3, nullptr, &b) == -1);
  pl_opts mx{};
  mx.precision = 9;
  ds[3].n = 50;
  CHECK(pl_batch_create(ds.data(), D, 2, lam, 3, &mx, &b) == -6);
}

static void step2_and_params() {
  // internal parameters: round trip, including ratios below 1
  const int K = 64;
  std::vector<double> om(5 * K), in(5 * K), back(5 * K);
  for (int k = 0; k < K; ++k) {
    om[5 * k + 0] = 0.1 + 3 * urand();
    om[5 * k + 1] = 0.2 + 5 * urand();
    om[5 * k + 2] = 0.01 + urand();
    om[5 * k + 3] = 0.3 + 4 * urand();
    om[5 * k + 4] = 3.14159 * (urand() - 0.5);
  }
  for (int st = 0; st < 2; ++st) {
    CHECK(pl_to_internal(om.data(), K, st, in.data()) == 0);
    CHECK(pl_from_internal(in.data(), K, st, back.data()) == 0);
  }
  // configuration points from a negative definite Hessian
  double H[25] = {0};
  for (int i = 0; i < 5; ++i) {
    H[6 * i] = -(1.0 + i);
    if (i) H[5 * i + i - 1] = H[5 * (i - 1) + i] = 0.2;
  }
  const double omh[5] = {1.0, 1.5, 0.2, 2.0, 0.5};
  const int npts = 40, nlev = 3;
  std::vector<double> init(npts * 5), sph(npts * 5), unif(nlev * npts), out(nlev * npts * 5);
  for (double& v : init) v = nrand();
  for (double& v : unif) v = urand();
  double md = 0.0;
  CHECK(pl_sphere_points(5, npts, init.data(), 50, sph.data(), &md) == 0 && md > 0.0);
  const double alpha[nlev] = {0.5, 0.1, 0.01};
  double ev[5];
  int64_t rep = 0;
  for (int st = 0; st < 2; ++st)
    CHECK(pl_config_points(omh, st, 0, H, alpha, nlev, sph.data(), npts, unif.data(), out.data(),
                           ev, &rep) == 0);
  CHECK(pl_config_points(omh, 0, 1, H, alpha, nlev, sph.data(), npts, unif.data(), out.data(),
                         ev, &rep) == 0);
  double q = 0.0;
  CHECK(pl_chisq_quantile(2, 0.05, &q) == 0 && fabs(q + 2.0 * log(0.05)) < 1e-9);
  double grid[30];
  CHECK(pl_lambda_grid(0.4, -50.0, 0.01, 30, grid) == 0 && grid[0] < grid[29]);
}

static void step4_extraction() {
  const int K = 300, M = 4;
  std::vector<pl_result> rec(K * M);
  std::vector<double> om(5 * K);
  const double lam[M] = {0.0, 0.3, 0.6, 1.0};
  for (int k = 0; k < K; ++k) {
    om[5 * k + 0] = 0.5 + 2 * urand();
    om[5 * k + 1] = 0.5 + 2 * urand();
    om[5 * k + 2] = 0.1 + urand();
    om[5 * k + 3] = 1.0 + urand();
    om[5 * k + 4] = urand();
    for (int m = 0; m < M; ++m) {
      pl_result& r = rec[k * M + m];
      r = pl_result{};
      const double x = om[5 * k + 0] - 1.3;
      r.loglik = -100.0 - 4.0 * x * x - (lam[m] - 0.4) * (lam[m] - 0.4) + 0.01 * nrand();
      r.info = (k % 37 == 5) ? 3 : 0;
    }
  }
  std::vector<double> cx(K + M), cy(K + M);
  for (int which = 0; which <= 5; ++which) {
    int64_t np = 0;
    double iv[3];
    int32_t open = 0;
    CHECK(pl_profile_param(rec.data(), K, M, om.data(), lam, which, 1.92, cx.data(), cy.data(),
                           &np, iv, &open) == 0);
    CHECK(np >= 1 && np <= K);
  }
}

static void tuning_cache() {
  char path[] = "/tmp/plprof_tune_XXXXXX";
  const int fd = mkstemp(path);
  CHECK(fd >= 0);
  if (fd < 0) return;
  close(fd);
  CHECK(pl_tune_cache_set(path) == 0);
  pl_opts o{};
  o.precision = PL_MIXED;
  o.flush = 2;
  o.lanes = 4;
  CHECK(pl_tune_store("gfx950", 0, 2000, 0, 12, 1e-3, &o, 1.0) == 0);
  CHECK(pl_tune_store("gfx950", 1, 1500, 32768, 4, 1e-3, &o, 2.0) == 0);
  pl_opts g{};
  CHECK(pl_tune_lookup("gfx950", 0, 1500, 0, 12, 1e-3, &g) == 0 && g.flush == 2);
  CHECK(pl_tune_lookup("gfx950", 0, 4000, 0, 12, 1e-3, &g) == PL_TUNE_MISS);
  CHECK(pl_tune_cache_set(path) == 0);  // reload
  int64_t entries = 0;
  CHECK(pl_tune_cache_stats(&entries, nullptr, nullptr) == 0 && entries == 2);
  CHECK(pl_tune_cache_set(nullptr) == 0);
  unlink(path);
}

int main() {
  tuning_cache();
  workspace_sizes();
  batch_planner();
  step2_and_params();
  step4_extraction();
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("host checks passed\n");
  return 0;
}
