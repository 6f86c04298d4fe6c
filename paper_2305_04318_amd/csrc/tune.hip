// Autotuning of the uneven batch and the persisted tuning cache.
//
// pl_batch_autotune times candidate plans of pl_batch_create on the caller's
// datasets -- the size-bucketed schedule with several stream counts and pass
// sizes, the persistent kernel, the mixed form with two FP32 partial-sum
// depths -- and keeps the fastest whose records stay within the caller's
// log-likelihood budget of the FP64 records.  The paper sets its launch
// sizes (omega points per iteration, global and local work sizes, local
// cache) by hand for each dataset (Section 4); here they are measured.
//
// Choices of pl_autotune and pl_batch_autotune are kept per (device
// architecture, kind, size bucket, right-hand sides, budget) in a process-wide
// table, persisted to a text file when one is set (pl_tune_cache_set): one
// line per choice, appended, the last line of a key winning on reload.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

using namespace plk;

namespace {

struct TuneKey {
  std::string arch;
  int kind;        // 0 pl_autotune, 1 pl_batch_autotune
  int nb, ub, q;   // floor(log2 n) (largest n of a batch), floor(log2 units) (batch), M + p
  std::string tol; // budget, printed with %.6g
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, kind, nb, ub, q, tol) < std::tie(o.arch, o.kind, o.nb, o.ub, o.q, o.tol);
  }
};

struct TuneVal {
  int precision, flush, flags, lanes;
  int64_t chunk;
  double ms;
};

std::mutex g_mu;
std::map<TuneKey, TuneVal> g_table;
std::string g_path;
bool g_enabled = false;  // the autotuners consult and fill the table
int64_t g_hits = 0, g_misses = 0;

int ilog2(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

std::string tol_str(double tol) {
  char buf[64];
  snprintf(buf, sizeof buf, "%.6g", tol);
  return buf;
}

// Architecture name of the current device (the part before any ':').
bool current_arch(std::string& arch) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return false;
  arch = prop.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch.resize(c);
  return !arch.empty();
}

bool load_file(const std::string& path) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return true;  // created on the first store
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char arch[128], tol[64];
    TuneKey k;
    TuneVal v;
    long long chunk = 0;
    if (sscanf(line,
               "v1 %127s %d %d %d %d %63s precision=%d flush=%d chunk=%lld lanes=%d flags=%d "
               "ms=%lf",
               arch, &k.kind, &k.nb, &k.ub, &k.q, tol, &v.precision, &v.flush, &chunk, &v.lanes,
               &v.flags, &v.ms) != 12)
      continue;  // not a tuning line
    k.arch = arch;
    k.tol = tol;
    v.chunk = chunk;
    g_table[k] = v;
  }
  fclose(f);
  return true;
}

bool append_file(const TuneKey& k, const TuneVal& v) {
  if (g_path.empty()) return true;
  FILE* f = fopen(g_path.c_str(), "a");
  if (!f) return false;
  fprintf(f, "v1 %s %d %d %d %d %s precision=%d flush=%d chunk=%lld lanes=%d flags=%d ms=%.6g\n",
          k.arch.c_str(), k.kind, k.nb, k.ub, k.q, k.tol.c_str(), v.precision, v.flush,
          (long long)v.chunk, v.lanes, v.flags, v.ms);
  return fclose(f) == 0;
}

TuneKey make_key(const std::string& arch, int kind, int64_t n, int64_t units, int64_t q,
                 double tol) {
  return TuneKey{arch, kind, ilog2(n), kind == 1 ? ilog2(units) : 0, (int)q, tol_str(tol)};
}

void apply(const TuneVal& v, pl_opts* o) {
  o->precision = v.precision;
  o->flush = v.flush;
  o->chunk = v.chunk;
  o->lanes = v.lanes;
  o->flags = (o->flags & ~PL_OPT_BATCH_PERSISTENT) | (v.flags & PL_OPT_BATCH_PERSISTENT);
}

}  // namespace

// ---- library-internal access for pl_autotune -----------------------------------------
bool plk::tune_cache_find(int kind, int64_t n, int64_t units, int64_t q, double tol,
                          pl_opts* opts) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_enabled) return false;
  }
  std::string arch;
  if (!current_arch(arch)) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(make_key(arch, kind, n, units, q, tol));
  if (it == g_table.end()) {
    ++g_misses;
    return false;
  }
  ++g_hits;
  apply(it->second, opts);
  return true;
}

void plk::tune_cache_put(int kind, int64_t n, int64_t units, int64_t q, double tol,
                         const pl_opts& o, double ms) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_enabled) return;
  }
  std::string arch;
  if (!current_arch(arch)) return;
  const TuneKey k = make_key(arch, kind, n, units, q, tol);
  const TuneVal v{o.precision, o.flush, o.flags & PL_OPT_BATCH_PERSISTENT, o.lanes, o.chunk, ms};
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[k] = v;
  (void)append_file(k, v);
}

extern "C" {

int pl_tune_cache_set(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_hits = g_misses = 0;
  g_enabled = path != nullptr;
  g_path = (path && path[0]) ? path : "";
  if (g_path.empty()) return PL_OK;
  FILE* probe = fopen(g_path.c_str(), "a");  // the file must be writable
  if (!probe) {
    g_path.clear();
    g_enabled = false;
    return -1;
  }
  fclose(probe);
  return load_file(g_path) ? PL_OK : -1;
}

int pl_tune_store(const char* arch, int kind, int64_t n, int64_t units, int64_t q, double tol,
                  const pl_opts* opts, double ms) {
  if (kind != 0 && kind != 1) return -2;
  if (n < 2) return -3;
  if (kind == 1 && units < 1) return -4;
  if (q < 2 || q > PL_MAX_P + PL_MAX_M) return -5;
  if (!std::isfinite(tol) || tol < 0.0) return -6;
  if (!opts) return -7;
  std::string a;
  if (arch && arch[0]) a = arch;
  else if (!current_arch(a)) return PL_E_HIP;
  const TuneKey k = make_key(a, kind, n, units, q, tol);
  const TuneVal v{opts->precision, opts->flush, opts->flags & PL_OPT_BATCH_PERSISTENT,
                  opts->lanes, opts->chunk, ms};
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[k] = v;
  return append_file(k, v) ? PL_OK : -1;
}

int pl_tune_lookup(const char* arch, int kind, int64_t n, int64_t units, int64_t q, double tol,
                   pl_opts* opts) {
  if (kind != 0 && kind != 1) return -2;
  if (n < 2) return -3;
  if (kind == 1 && units < 1) return -4;
  if (q < 2 || q > PL_MAX_P + PL_MAX_M) return -5;
  if (!std::isfinite(tol) || tol < 0.0) return -6;
  if (!opts) return -7;
  std::string a;
  if (arch && arch[0]) a = arch;
  else if (!current_arch(a)) return PL_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(make_key(a, kind, n, units, q, tol));
  if (it == g_table.end()) {
    ++g_misses;
    return PL_TUNE_MISS;
  }
  ++g_hits;
  apply(it->second, opts);
  return PL_OK;
}

int pl_tune_cache_stats(int64_t* entries, int64_t* hits, int64_t* misses) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (entries) *entries = (int64_t)g_table.size();
  if (hits) *hits = g_hits;
  if (misses) *misses = g_misses;
  return PL_OK;
}

}  // extern "C"

// ---- pl_batch_autotune --------------------------------------------------------------
namespace {

struct BatchCand {
  int precision, flush, lanes, flags;
  int64_t chunk;
};
// FP64 size-bucketed with 2, 4, 8 streams and the default pass size, 4
// streams with passes of at most 256 units, the persistent kernel; the mixed
// form (4 streams) with 16- and 8-product FP32 partial sums
const BatchCand kBatchCand[] = {
    {PL_FP64, 0, 2, 0, 0},  {PL_FP64, 0, 4, 0, 0},  {PL_FP64, 0, 8, 0, 0},
    {PL_FP64, 0, 4, 0, 256}, {PL_FP64, 0, 0, PL_OPT_BATCH_PERSISTENT, 0},
    {PL_MIXED, 4, 4, 0, 0}, {PL_MIXED, 2, 4, 0, 0}};
constexpr int NBC = sizeof(kBatchCand) / sizeof(kBatchCand[0]);

size_t rec_bytes(int64_t U, int64_t M) { return ((size_t)U * M * sizeof(pl_result) + 255) / 256 * 256; }

}  // namespace

extern "C" {

int pl_batch_autotune_workspace_size(const pl_dataset* datasets, int64_t D, int64_t p,
                                     const double* lambda, int64_t M, size_t* bytes) {
  if (!bytes) return -6;
  size_t need = 0;
  int64_t U = 0;
  for (int c = 0; c < NBC; ++c) {
    if (kBatchCand[c].precision == PL_MIXED && M + p > PL_MAX_Q_MIXED) continue;
    pl_opts o{};
    o.precision = kBatchCand[c].precision;
    o.flush = kBatchCand[c].flush;
    o.lanes = kBatchCand[c].lanes;
    o.chunk = kBatchCand[c].chunk;
    o.flags = kBatchCand[c].flags;
    pl_batch* b = nullptr;
    const int rc = pl_batch_create(datasets, D, p, lambda, M, &o, &b);
    if (rc != PL_OK) return rc;
    size_t w = 0;
    pl_batch_workspace_size(b, &w);
    pl_batch_stats(b, &U, nullptr, nullptr);
    pl_batch_destroy(b);
    need = std::max(need, w);
  }
  *bytes = need + 2 * rec_bytes(U, M);
  return PL_OK;
}

int pl_batch_autotune(const pl_dataset* datasets, int64_t D, int64_t p, const double* lambda,
                      int64_t M, double tol, pl_opts* opts, double* report, void* work,
                      size_t work_bytes, void* stream) {
  if (!std::isfinite(tol) || tol < 0.0) return -6;
  if (!opts) return -7;
  if (!work) return -9;
  size_t need = 0;
  int rc = pl_batch_autotune_workspace_size(datasets, D, p, lambda, M, &need);
  if (rc != PL_OK) return rc;
  if (work_bytes < need) return -10;
  int64_t nmax = 0, U = 0;
  for (int64_t d = 0; d < D; ++d) {
    nmax = std::max(nmax, datasets[d].n);
    U += datasets[d].K;
  }
  if (tune_cache_find(1, nmax, U, M + p, tol, opts)) {
    if (report)
      for (int c = 0; c < 2 * NBC; ++c) report[c] = -2.0;  // a cached choice: nothing timed
    return PL_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t rb = rec_bytes(U, M);
  const size_t wb = work_bytes - 2 * rb;
  pl_result* rec_ref = reinterpret_cast<pl_result*>((char*)work + wb);
  pl_result* rec_c = reinterpret_cast<pl_result*>((char*)work + wb + rb);
  std::vector<pl_result> href((size_t)U * M), hc((size_t)U * M);
  double ms[NBC], err[NBC];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return PL_E_HIP;
  }
  for (int c = 0; c < NBC && rc == PL_OK; ++c) {
    ms[c] = err[c] = -1.0;
    const BatchCand& bc = kBatchCand[c];
    if (bc.precision == PL_MIXED && M + p > PL_MAX_Q_MIXED) continue;
    pl_opts o = *opts;
    o.precision = bc.precision;
    o.flush = bc.flush;
    o.lanes = bc.lanes;
    o.chunk = bc.chunk;
    o.flags = (o.flags & ~PL_OPT_BATCH_PERSISTENT) | bc.flags;
    pl_batch* b = nullptr;
    if ((rc = pl_batch_create(datasets, D, p, lambda, M, &o, &b)) != PL_OK) break;
    pl_result* dst = c == 0 ? rec_ref : rec_c;
    // the first run captures the graph; then two timed replays
    rc = pl_batch_run(b, dst, nullptr, work, wb, stream);
    float t = 0.0f;
    if (rc == PL_OK && hipEventRecord(e0, s) != hipSuccess) rc = PL_E_HIP;
    for (int r = 0; r < 2 && rc == PL_OK; ++r) rc = pl_batch_run(b, dst, nullptr, work, wb, stream);
    if (rc == PL_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      rc = PL_E_HIP;
    int32_t derr = 0;
    if (rc == PL_OK && (rc = pl_batch_error(b, work, &derr)) == PL_OK && derr != 0) t = -1.0f;
    pl_batch_destroy(b);
    if (rc != PL_OK) break;
    std::vector<pl_result>& h = c == 0 ? href : hc;
    if (hipMemcpy(h.data(), dst, (size_t)U * M * sizeof(pl_result), hipMemcpyDeviceToHost) !=
        hipSuccess) {
      rc = PL_E_HIP;
      break;
    }
    ms[c] = t < 0.0f ? -1.0 : t / 2.0;
    double e = 0.0;
    for (size_t i = 0; c > 0 && i < href.size(); ++i) {
      const double a = href[i].loglik, v = hc[i].loglik;
      if (std::isfinite(a) != std::isfinite(v)) {
        e = INFINITY;
        break;
      }
      if (std::isfinite(a)) e = std::max(e, fabs(a - v));
    }
    err[c] = e;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PL_OK) return rc;
  int best = -1;
  for (int c = 0; c < NBC; ++c)
    if (ms[c] >= 0.0 && err[c] >= 0.0 && err[c] <= tol && (best < 0 || ms[c] < ms[best])) best = c;
  if (best < 0) return PL_E_UNSUPPORTED;
  const BatchCand& bc = kBatchCand[best];
  opts->precision = bc.precision;
  opts->flush = bc.flush;
  opts->lanes = bc.lanes;
  opts->chunk = bc.chunk;
  opts->flags = (opts->flags & ~PL_OPT_BATCH_PERSISTENT) | bc.flags;
  tune_cache_put(1, nmax, U, M + p, tol, *opts, ms[best]);
  if (report)
    for (int c = 0; c < NBC; ++c) {
      report[c] = ms[c];
      report[NBC + c] = err[c];
    }
  return PL_OK;
}

}  // extern "C"
