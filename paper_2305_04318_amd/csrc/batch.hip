// Many independent datasets of uneven size, evaluated by one graph launch.
//
// Every (dataset d, omega k) pair is a unit: Step 3 of Section 3.3 for one V.
// Two schedules share the plan interface.
//
// Size-bucketed (the default; FP64 or mixed).  Units are grouped by their
// number of tile rows Nv; a group's units run through the same step kernels
// as pl_profile_loglik in passes of many units at once, each unit with its
// own order n, locations and right-hand sides (UnitInfo), so one launch of
// a step kernel covers the units of one pass whatever their datasets.  The
// passes are spread over a few streams (largest first, to the least loaded
// stream); each stream reuses its own workspace region pass after pass.
// The whole sequence -- omega tables, Box-Cox right-hand sides of every
// dataset, then every stream's passes, forked from and joined back to the
// caller's stream -- is captured once into a HIP graph and replayed.
//
// Persistent (FP64, on request).  A unit's work is cut into tile tasks
// grouped in phases that must run in order (bordering + covariance tiles;
// then, per block column J, the left-looking updates, the diagonal factor,
// the panel solves; the final Schur tile; the p x p stage).  The host lists
// all tasks so that every task depends only on tasks listed before it; one
// persistent kernel (grid = the number of resident workgroups) pops tasks
// from an atomic queue, waits until its unit has completed the earlier
// phases (a per-unit completion counter), runs the task and counts it done.
// A task popped earlier is held by a running workgroup whose own
// dependencies were listed earlier still, so the queue drains.  Units
// recycle a pool of matrix slabs: a unit's first phase also waits for the
// previous user of its slab.  Every wait is bounded by wall time (the
// device's constant-rate counter): a wait that outlives its limit sets an
// error flag, after which every wait returns at once and every task skips
// its work, so the kernel always drains and terminates.
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "finalize_dev.h"
#include "matern_dev.h"
#include "tiles.h"

namespace plk {

enum : int16_t { TK_BORDER = 0, TK_MATERN = 1, TK_GEMM = 2, TK_POTRF = 3, TK_TRSM = 4, TK_FINAL = 5 };

struct BTask {
  int32_t unit;
  int16_t type;
  int16_t I;
  int16_t J;
  int16_t first;  // 1 for tasks of the unit's first phase (slab hand-over)
  int32_t wait;   // tasks of the unit that must be done before this one
};

struct BDataset {
  const double* locs;
  const double* y;
  const double* X;
  int32_t n;
  int32_t om_off;   // first global omega index of the dataset
  int64_t rhs_off;  // offset of its right-hand-side rows (elements)
};

struct BUnit {
  int32_t d;
  int32_t om;          // global omega index (params, tables, records)
  int32_t Nv;
  int32_t slab;
  int32_t pred;        // previous unit on the same slab, or -1
  int32_t pred_total;  // task count of pred
};

struct BatchArgs {
  const BTask* tasks;
  int32_t ntasks;
  int32_t* head;
  int32_t* done;
  int32_t* err;
  const BUnit* units;
  const BDataset* ds;
  const MaternParams* mp;
  const double* tables;
  const double* rhs;
  const double* jac;
  const int32_t* yflags;
  const double* lam;
  double* slabs;
  int64_t slab_stride;  // elements per slab
  int64_t w_off;        // offset of the W tile inside a slab
  double* logdet;
  int32_t* info;
  int32_t p, M, q, TB;
  pl_result* out;
  double* beta;
  int64_t wait_ticks;  // limit of one wait, in ticks of the constant-rate counter
};

// Waits until *ctr >= v.  Gives up when the error flag is set, or when the
// wait has lasted wait_ticks of wall time (it then sets the flag).  Returns
// whether the count was reached.
__device__ __forceinline__ bool wait_ge(int32_t* ctr, int32_t v, int32_t* err, int64_t wait_ticks) {
  const int64_t t0 = wall_clock64();
  for (;;) {
    if (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= v) return true;
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (wall_clock64() - t0 > wait_ticks) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__device__ __forceinline__ Lay unit_lay(const BDataset& d, int Nv, int q, int TB) {
  Lay lay{};
  lay.kind = 0;
  lay.n = d.n;
  lay.Nv = Nv;
  lay.q = q;
  lay.TB = TB;
  lay.mstride = 0;  // slabs are addressed explicitly
  return lay;
}

// The task bodies as calls of their own: inlined into one switch they share
// one register allocation, and the largest (the factorisation) makes the
// others spill inside their k-loops.
__device__ __noinline__ void task_gemm(const Lay& lay, double* base, int I, int J, double* smem) {
  // the step kernels' bodies: direct-to-LDS loads (no staging registers),
  // the balanced plans; the bordered row's tiles (I = Nv, its own block at
  // J = Nv included) keep the register-staged core (their panel has TB rows)
  if (I < lay.Nv && I == J) dev_gemm_diag_border<true>(lay, base, J, false, smem);
  else if (I < lay.Nv) dev_gemm_col_dma(lay, base, J, I, smem);
  else dev_gemm_col<true, 1>(lay, base, J, I, smem);
}

__device__ __noinline__ void task_trsm(const Lay& lay, double* base, const double* W, int I, int J,
                                       double* smem) {
  if (I < lay.Nv) {
    dev_trsm_dma<TRSM_KC, TRSM_NST>(lay, base, W, J, I, smem);
    return;
  }
  switch (lay.TB) {  // the bordered row's tile
    case 16: dev_trsm_border<1>(lay, base, W, J); break;
    case 32: dev_trsm_border<2>(lay, base, W, J); break;
    case 48: dev_trsm_border<3>(lay, base, W, J); break;
    case 64: dev_trsm_border<4>(lay, base, W, J); break;
    default: dev_trsm<double, true, 1, 1>(lay, base, W, J, I, smem); break;
  }
}

__device__ __noinline__ void task_potrf(const Lay& lay, double* base, double* W, double* logdet_k,
                                        int32_t* info_k, int J, double* smem) {
  dev_potrf<0>(lay, base + lay.tile_off(J, J), lay.tile_ld(J), W, nullptr, logdet_k, info_k, J,
               smem);
}

__global__ __launch_bounds__(256, 2) void k_batch_persistent(BatchArgs a) {
  __shared__ __attribute__((aligned(16)))
  char smem_raw[UPD_DMA_LDS_BYTES > GEMM_LDS_BYTES ? UPD_DMA_LDS_BYTES : GEMM_LDS_BYTES];
  static_assert((TABLE + 2 * T) * 8 <= GEMM_LDS_BYTES, "covariance task staging");
  static_assert(POTRF_SMEM_DOUBLES * 8 <= GEMM_LDS_BYTES, "factorisation task staging");
  static_assert(FIN_SMEM_DOUBLES * 8 <= GEMM_LDS_BYTES, "finalize task staging");
  __shared__ int32_t s_task, s_ok;
  double* smem = reinterpret_cast<double*>(smem_raw);
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(a.head, 1);
    __syncthreads();
    const int32_t t = s_task;
    if (t >= a.ntasks) break;  // uniform: every workgroup leaves once the queue is empty
    const BTask tk = a.tasks[t];
    const BUnit u = a.units[tk.unit];
    if (threadIdx.x == 0) {
      bool ok = wait_ge(a.done + tk.unit, tk.wait, a.err, a.wait_ticks);
      if (ok && tk.first && u.pred >= 0) ok = wait_ge(a.done + u.pred, u.pred_total, a.err, a.wait_ticks);
      __threadfence();  // acquire: the unit's earlier tasks' stores are visible
      s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    // after a wait gave up (here or anywhere) the task only counts itself done
    const bool run = s_ok != 0;
    const BDataset d = a.ds[u.d];
    const Lay lay = unit_lay(d, u.Nv, a.q, a.TB);
    double* base = a.slabs + (int64_t)u.slab * a.slab_stride;
    double* W = base + a.w_off;
    const bool failed = a.info[tk.unit] != 0;
    if (run) switch (tk.type) {
      case TK_BORDER: {
        const int64_t nrhs = (int64_t)d.n * a.TB;
        const double* rhs = a.rhs + d.rhs_off;
        double* bp = base + lay.tile_off(u.Nv, 0);
        for (int64_t e = threadIdx.x; e < nrhs; e += blockDim.x) bp[e] = rhs[e];
        double* st = base + lay.tile_off(u.Nv, u.Nv);
        for (int e = threadIdx.x; e < a.TB * a.TB; e += blockDim.x) st[e] = 0.0;
        break;
      }
      case TK_MATERN:
        dev_matern_tile<0>(lay, a.mp[u.om], a.tables + (int64_t)u.om * TABLE, d.locs, tk.I, tk.J,
                           base + lay.tile_off(tk.I, tk.J), lay.tile_ld(tk.I), nullptr, smem);
        break;
      case TK_GEMM:
        if (!failed) task_gemm(lay, base, tk.I, tk.J, smem);
        break;
      case TK_POTRF:
        if (!failed) task_potrf(lay, base, W, a.logdet + tk.unit, a.info + tk.unit, tk.J, smem);
        break;
      case TK_TRSM:
        if (!failed) task_trsm(lay, base, W, tk.I, tk.J, smem);
        break;
      default: {  // TK_FINAL
        const int64_t rec = (int64_t)u.om * a.M;
        dev_finalize(base + lay.tile_off(u.Nv, u.Nv), a.TB, a.logdet[tk.unit], a.info[tk.unit],
                     a.jac[u.d], a.yflags[u.d] != 0, a.lam, d.n, a.p, a.M, a.out + rec,
                     a.beta ? a.beta + rec * a.p : nullptr, nullptr, smem);
        break;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();  // release: this task's stores before the count
      __hip_atomic_fetch_add(a.done + tk.unit, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Box-Cox right-hand sides and Jacobian of every dataset: one workgroup per
// dataset (fixed summation order for the Jacobian).
__global__ __launch_bounds__(256) void k_batch_boxcox(const BDataset* __restrict__ ds,
                                                      const double* __restrict__ lam, int p, int M,
                                                      int TB, double* __restrict__ rhs,
                                                      double* __restrict__ jac,
                                                      int32_t* __restrict__ yflags) {
  __shared__ double red[256];
  __shared__ int bad;
  const BDataset d = ds[blockIdx.x];
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double s = 0.0;
  int lbad = 0;
  double* r = rhs + d.rhs_off;
  for (int i = threadIdx.x; i < d.n; i += blockDim.x) {
    const double yi = d.y[i];
    if (!(yi > 0.0) || !isfinite(yi)) lbad = 1;
    const double ly = log(yi);
    if (!lbad) s += ly;
    for (int a = 0; a < TB; ++a) {
      double v = 0.0;
      if (a < M) {
        const double l = lam[a];
        v = (l == 0.0) ? ly : expm1(l * ly) / l;
      } else if (a < M + p) {
        v = d.X[(int64_t)(a - M) * d.n + i];
      }
      r[(int64_t)i * TB + a] = v;
    }
  }
  red[threadIdx.x] = s;
  if (lbad) atomicOr(&bad, 1);
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    jac[blockIdx.x] = red[0];
    yflags[blockIdx.x] = bad;
  }
}

__global__ void k_zero_i32(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace plk

using namespace plk;

// ---- host side -------------------------------------------------------------------
// One pass of the size-bucketed schedule: units [u0, u0 + cnt) of the sorted
// unit list (one group, so one Nv), run on stream `lane`.
struct BPass {
  int32_t u0, cnt, lane, nmax;
  double cost;
};

struct pl_batch {
  // inputs (host copies)
  std::vector<BDataset> ds;
  std::vector<BUnit> units;
  std::vector<BTask> tasks;
  std::vector<MaternParams> params;
  std::vector<double> lam;
  std::vector<double> omega;     // natural omega of every unit, record order (K x 5)
  int32_t p = 0, M = 0, q = 0, TB = 0;
  bool persistent = false, mixed = false, fallback = true;
  int32_t flush = MX_FLUSH, refine = 1;
  int32_t wait_us = 0;  // persistent: limit of one task wait
  int64_t n_omega = 0, nslabs = 0, slab_stride = 0, w_off = 0;
  // size-bucketed schedule: units sorted by Nv (descending), their records
  std::vector<UnitInfo> uinfo;   // sorted order; locs pointers, rhs offsets, record index
  std::vector<int32_t> order;    // sorted position -> record (unit) index
  std::vector<BPass> passes;
  int32_t lanes = 0;
  size_t region = 0;             // workspace bytes of one stream
  // workspace layout (bytes)
  size_t off_tasks, off_units, off_ds, off_mp, off_nodes, off_tables, off_lam, off_rhs, off_jac,
      off_yflags, off_done, off_ctl, off_logdet, off_info, off_slabs, off_uinfo, off_lanes, total;
  int64_t rhs_elems = 0;
  // graph state
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> lane_s;
  std::vector<hipEvent_t> ev;
  hipGraphExec_t exec = nullptr;
  void* g_work = nullptr;
  pl_result* g_out = nullptr;
  double* g_beta = nullptr;
  int grid = 0;
};

namespace {

constexpr size_t BALIGN = 256;
inline size_t balign(size_t x) { return (x + BALIGN - 1) / BALIGN * BALIGN; }
constexpr size_t PASS_BYTES = (size_t)4 << 30;  // default workspace of one pass
constexpr int DEFAULT_LANES = 4;

bool omega_ok_b(const double* om) {
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(om[i])) return false;
  return om[0] > 0.0 && om[1] >= PL_MIN_SHAPE && om[1] <= PL_MAX_SHAPE && om[2] >= 0.0 &&
         om[3] > 0.0;
}


// Tasks of one unit, phase by phase.
void unit_phases(int Nv, std::vector<std::vector<BTask>>& ph) {
  ph.clear();
  std::vector<BTask> p0;
  p0.push_back({0, TK_BORDER, 0, 0, 1, 0});
  for (int I = 0; I < Nv; ++I)
    for (int J = 0; J <= I; ++J) p0.push_back({0, TK_MATERN, (int16_t)I, (int16_t)J, 1, 0});
  ph.push_back(p0);
  for (int J = 0; J <= Nv; ++J) {
    if (J > 0) {
      std::vector<BTask> g;
      for (int I = J; I <= Nv; ++I) g.push_back({0, TK_GEMM, (int16_t)I, (int16_t)J, 0, 0});
      ph.push_back(g);
    }
    if (J < Nv) {
      ph.push_back({{0, TK_POTRF, (int16_t)J, (int16_t)J, 0, 0}});
      std::vector<BTask> tr;
      for (int I = J + 1; I <= Nv; ++I) tr.push_back({0, TK_TRSM, (int16_t)I, (int16_t)J, 0, 0});
      ph.push_back(tr);
    }
  }
  ph.push_back({{0, TK_FINAL, 0, 0, 0, 0}});
}

// Every wait must be met by tasks listed earlier (so the queue drains).
bool validate(const std::vector<BTask>& tasks, const std::vector<BUnit>& units,
              const std::vector<int32_t>& total) {
  std::vector<int32_t> seen(units.size(), 0);
  for (const BTask& t : tasks) {
    if (t.unit < 0 || t.unit >= (int)units.size()) return false;
    if (t.wait > seen[t.unit]) return false;
    const BUnit& u = units[t.unit];
    if (t.first && u.pred >= 0) {
      if (u.pred_total != total[u.pred] || seen[u.pred] != total[u.pred]) return false;
    }
    seen[t.unit]++;
  }
  for (size_t u = 0; u < units.size(); ++u)
    if (seen[u] != total[u]) return false;
  return true;
}

// Persistent schedule: slab pool, task list, workspace layout.
int plan_persistent(pl_batch* b, int64_t chunk, int maxNv) {
  const int64_t U = (int64_t)b->units.size(), D = (int64_t)b->ds.size();
  // slab pool: one slab holds the largest unit's packed matrix and its W tile
  const int64_t mat = packed_stride(maxNv, b->TB);
  b->w_off = (mat + 31) / 32 * 32;
  b->slab_stride = b->w_off + (int64_t)T * T;
  int64_t S = chunk > 0 ? chunk : std::min<int64_t>(U, 2048);
  b->nslabs = std::max<int64_t>(1, std::min(S, U));

  // order units by decreasing size (largest first), waves of nslabs units;
  // alternate the slab order between waves so that the largest units of a wave
  // take the slabs freed first by the smallest units of the previous wave
  std::vector<int32_t> order(U);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return b->units[x].Nv > b->units[y].Nv; });
  std::vector<int32_t> total(U, 0);
  std::vector<std::vector<BTask>> ph;
  std::vector<std::vector<std::vector<BTask>>> unit_ph(U);
  for (int64_t u = 0; u < U; ++u) {
    unit_phases(b->units[u].Nv, ph);
    // waits: a task waits for all tasks of earlier phases of its unit
    int32_t before = 0;
    for (auto& v : ph) {
      for (auto& t : v) {
        t.unit = (int32_t)u;
        t.wait = before;
      }
      before += (int32_t)v.size();
    }
    total[u] = before;
    unit_ph[u] = ph;
  }
  std::vector<int32_t> slab_user(b->nslabs, -1);
  for (int64_t w0 = 0, wave = 0; w0 < U; w0 += b->nslabs, ++wave) {
    const int64_t w1 = std::min<int64_t>(U, w0 + b->nslabs);
    for (int64_t i = w0; i < w1; ++i) {
      const int32_t u = order[i];
      const int64_t pos = i - w0;
      const int32_t slab = (int32_t)((wave % 2 == 0) ? pos : (b->nslabs - 1 - pos));
      b->units[u].slab = slab;
      b->units[u].pred = slab_user[slab];
      b->units[u].pred_total = slab_user[slab] >= 0 ? total[slab_user[slab]] : 0;
      slab_user[slab] = u;
    }
    size_t maxph = 0;
    for (int64_t i = w0; i < w1; ++i) maxph = std::max(maxph, unit_ph[order[i]].size());
    for (size_t f = 0; f < maxph; ++f)
      for (int64_t i = w0; i < w1; ++i) {
        const auto& up = unit_ph[order[i]];
        if (f < up.size())
          for (const BTask& t : up[f]) b->tasks.push_back(t);
      }
  }
  if (b->tasks.size() > (size_t)INT32_MAX || !validate(b->tasks, b->units, total))
    return PL_E_UNSUPPORTED;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += balign(bytes);
    return o;
  };
  b->off_tasks = take(b->tasks.size() * sizeof(BTask));
  b->off_units = take(U * sizeof(BUnit));
  b->off_ds = take(D * sizeof(BDataset));
  b->off_mp = take(b->n_omega * sizeof(MaternParams));
  b->off_nodes = take((size_t)b->n_omega * TABLE * sizeof(double));
  b->off_tables = take((size_t)b->n_omega * TABLE * sizeof(double));
  b->off_lam = take(b->M * sizeof(double));
  b->off_rhs = take((size_t)b->rhs_elems * sizeof(double));
  b->off_jac = take(D * sizeof(double));
  b->off_yflags = take(D * sizeof(int32_t));
  b->off_done = take(U * sizeof(int32_t));
  b->off_ctl = take(2 * sizeof(int32_t));
  b->off_logdet = take(U * sizeof(double));
  b->off_info = take(U * sizeof(int32_t));
  b->off_slabs = take((size_t)b->nslabs * b->slab_stride * sizeof(double));
  b->total = off;
  return PL_OK;
}

// Size-bucketed schedule: groups by Nv, passes, streams, workspace layout.
int plan_bucketed(pl_batch* b, int64_t chunk, int lanes) {
  const int64_t U = (int64_t)b->units.size(), D = (int64_t)b->ds.size();
  std::vector<int32_t>& order = b->order;
  order.resize(U);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return b->units[x].Nv > b->units[y].Nv; });
  b->uinfo.resize(U);
  for (int64_t i = 0; i < U; ++i) {
    const BUnit& u = b->units[order[i]];
    const BDataset& d = b->ds[u.d];
    b->uinfo[i] = UnitInfo{d.n, u.d, d.locs, d.rhs_off, (int64_t)u.om};
  }
  // passes: a group's units in chunks that fit the pass budget
  b->lanes = std::max(1, lanes);
  size_t region = 0;
  for (int64_t g0 = 0; g0 < U;) {
    const int Nv = b->units[order[g0]].Nv;
    int64_t g1 = g0;
    while (g1 < U && b->units[order[g1]].Nv == Nv) ++g1;
    const Lay lay = packed_layout((int64_t)Nv * T, b->q);
    const size_t per = pass_bytes(lay, b->mixed, 1);
    int64_t cap = chunk > 0 ? chunk : std::max<int64_t>(1, (int64_t)(PASS_BYTES / per));
    cap = std::min<int64_t>(cap, 1 << 20);
    const int64_t cnt = g1 - g0, np = (cnt + cap - 1) / cap;
    for (int64_t j = 0; j < np; ++j) {
      const int64_t a = g0 + cnt * j / np, e = g0 + cnt * (j + 1) / np;
      BPass ps{(int32_t)a, (int32_t)(e - a), 0, 0, 0.0};
      for (int64_t i = a; i < e; ++i) {
        const double n = b->uinfo[i].n;
        ps.nmax = std::max<int32_t>(ps.nmax, b->uinfo[i].n);
        ps.cost += n * n * n / 3.0 + 2e3 * n * n;  // factorisation and covariance build
      }
      ps.cost += 3.0 * Nv * 5e9;                     // launch latencies of the pass
      region = std::max(region, pass_bytes(lay, b->mixed, e - a));
      b->passes.push_back(ps);
    }
    g0 = g1;
  }
  // largest passes first, each to the least loaded stream
  std::vector<int32_t> po(b->passes.size());
  std::iota(po.begin(), po.end(), 0);
  std::stable_sort(po.begin(), po.end(),
                   [&](int32_t x, int32_t y) { return b->passes[x].cost > b->passes[y].cost; });
  std::vector<double> load(b->lanes, 0.0);
  std::vector<BPass> sorted;
  for (int32_t i : po) {
    BPass ps = b->passes[i];
    ps.lane = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
    load[ps.lane] += ps.cost;
    sorted.push_back(ps);
  }
  b->passes = sorted;
  // a mixed-form breakdown is redone in FP64 in stream 0's region afterwards
  if (b->mixed) {
    int nbig = 0;
    for (const BDataset& d : b->ds) nbig = std::max(nbig, d.n);
    pl_opts o{};
    o.precision = PL_FP64;
    size_t fb = 0;
    if (pl_workspace_size(nbig, b->p, 1, b->M, &o, &fb) != PL_OK) return PL_E_UNSUPPORTED;
    region = std::max(region, fb);
  }
  b->region = balign(region);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += balign(bytes);
    return o;
  };
  b->off_ds = take(D * sizeof(BDataset));
  b->off_mp = take(U * sizeof(MaternParams));
  b->off_nodes = take((size_t)U * TABLE * sizeof(double));
  b->off_tables = take((size_t)U * TABLE * sizeof(double));
  b->off_lam = take(b->M * sizeof(double));
  b->off_rhs = take((size_t)b->rhs_elems * sizeof(double));
  b->off_jac = take(D * sizeof(double));
  b->off_yflags = take(D * sizeof(int32_t));
  b->off_uinfo = take(U * sizeof(UnitInfo));
  b->off_info = take(U * sizeof(int32_t));
  b->off_lanes = take((size_t)b->lanes * b->region);
  b->total = off;
  return PL_OK;
}

}  // namespace

extern "C" {

int pl_batch_create(const pl_dataset* datasets, int64_t D, int64_t p, const double* lambda,
                    int64_t M, const pl_opts* opts, pl_batch** plan) {
  if (!datasets) return -1;
  if (D < 1 || D > (1 << 22)) return -2;
  if (p < 1 || p > PL_MAX_P) return -3;
  if (!lambda) return -4;
  if (M < 1 || M > PL_MAX_M) return -5;
  for (int64_t m = 0; m < M; ++m)
    if (!std::isfinite(lambda[m])) return -4;
  const bool persistent = opts && (opts->flags & PL_OPT_BATCH_PERSISTENT);
  const bool mixed = opts && opts->precision == PL_MIXED;
  if (opts) {
    if (opts->precision != PL_FP64 && opts->precision != PL_MIXED) return -6;
    if (opts->chunk < 0 || opts->wait_us < 0 || opts->lanes < 0 || opts->lanes > 16) return -6;
    if (opts->refine < 0 || opts->refine > 1) return -6;
    if (opts->flush != 0 && opts->flush != 1 && opts->flush != 2 && opts->flush != 4) return -6;
    if (persistent && mixed) return -6;  // the persistent kernel carries FP64 tasks only
  }
  if (!plan) return -7;
  if (mixed && M + p > PL_MAX_Q_MIXED) return PL_E_UNSUPPORTED;
  pl_batch* b = new pl_batch();
  b->p = (int32_t)p;
  b->M = (int32_t)M;
  b->q = (int32_t)(M + p);
  b->TB = (int32_t)((b->q + 15) / 16 * 16);
  b->lam.assign(lambda, lambda + M);
  b->persistent = persistent;
  b->mixed = mixed;
  if (opts) {
    b->refine = opts->refine;
    b->fallback = !(opts->flags & PL_OPT_NO_FALLBACK);
    if (opts->flush) b->flush = opts->flush;
  }
  b->wait_us = (opts && opts->wait_us > 0) ? opts->wait_us : PL_BATCH_WAIT_US;
  int64_t rhs_off = 0, om = 0;
  int maxNv = 0;
  for (int64_t d = 0; d < D; ++d) {
    const pl_dataset& s = datasets[d];
    // tile indices are int16_t in the persistent task list: at most 32767 tile rows
    if (!s.locs || !s.y || !s.X || s.n < 2 || s.n <= p || s.n > (int64_t)32767 * T || !s.omega ||
        s.K < 1 || s.K > (1 << 24)) {
      delete b;
      return -1;
    }
    for (int64_t k = 0; k < s.K; ++k)
      if (!omega_ok_b(s.omega + 5 * k)) {
        delete b;
        return -1;
      }
    BDataset bd{s.locs, s.y, s.X, (int32_t)s.n, (int32_t)om, rhs_off};
    b->ds.push_back(bd);
    const int Nv = (int)((s.n + T - 1) / T);
    maxNv = std::max(maxNv, Nv);
    for (int64_t k = 0; k < s.K; ++k) {
      b->params.push_back(make_matern_params(s.omega + 5 * k));
      b->units.push_back({(int32_t)d, (int32_t)(om + k), Nv, 0, -1, 0});
      b->omega.insert(b->omega.end(), s.omega + 5 * k, s.omega + 5 * k + 5);
    }
    om += s.K;
    rhs_off += s.n * b->TB;
    if (om > INT32_MAX / 2) {
      delete b;
      return -2;
    }
  }
  b->n_omega = om;
  b->rhs_elems = rhs_off;
  const int rc = persistent
                     ? plan_persistent(b, opts ? opts->chunk : 0, maxNv)
                     : plan_bucketed(b, opts ? opts->chunk : 0,
                                     (opts && opts->lanes > 0) ? opts->lanes : DEFAULT_LANES);
  if (rc != PL_OK) {
    delete b;
    return rc;
  }
  *plan = b;
  return PL_OK;
}

int pl_batch_workspace_size(const pl_batch* plan, size_t* bytes) {
  if (!plan) return -1;
  if (!bytes) return -2;
  *bytes = plan->total;
  return PL_OK;
}

int pl_batch_stats(const pl_batch* plan, int64_t* units, int64_t* tasks, int64_t* slabs) {
  if (!plan) return -1;
  if (units) *units = (int64_t)plan->units.size();
  if (tasks) *tasks = plan->persistent ? (int64_t)plan->tasks.size() : (int64_t)plan->passes.size();
  if (slabs) *slabs = plan->persistent ? plan->nslabs : plan->lanes;
  return PL_OK;
}

namespace {

// Capture of the persistent schedule's launch sequence (after the upload).
hipError_t capture_persistent(pl_batch* b, char* w, pl_result* out, double* beta_hat) {
  int dev = 0, cus = 0, per_cu = 0, clock_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      clock_khz <= 0 ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent, 256, 0) !=
          hipSuccess)
    return hipErrorUnknown;
  b->grid = std::max(1, cus * std::max(1, per_cu));
  const int64_t U = (int64_t)b->units.size(), D = (int64_t)b->ds.size();
  BatchArgs a{};
  a.tasks = (const BTask*)(w + b->off_tasks);
  a.ntasks = (int32_t)b->tasks.size();
  a.head = (int32_t*)(w + b->off_ctl);
  a.err = (int32_t*)(w + b->off_ctl) + 1;
  a.done = (int32_t*)(w + b->off_done);
  a.units = (const BUnit*)(w + b->off_units);
  a.ds = (const BDataset*)(w + b->off_ds);
  a.mp = (const MaternParams*)(w + b->off_mp);
  a.tables = (const double*)(w + b->off_tables);
  a.rhs = (const double*)(w + b->off_rhs);
  a.jac = (const double*)(w + b->off_jac);
  a.yflags = (const int32_t*)(w + b->off_yflags);
  a.lam = (const double*)(w + b->off_lam);
  a.slabs = (double*)(w + b->off_slabs);
  a.slab_stride = b->slab_stride;
  a.w_off = b->w_off;
  a.logdet = (double*)(w + b->off_logdet);
  a.info = (int32_t*)(w + b->off_info);
  a.p = b->p;
  a.M = b->M;
  a.q = b->q;
  a.TB = b->TB;
  a.out = out;
  a.beta = beta_hat;
  a.wait_ticks = (int64_t)b->wait_us * clock_khz / 1000;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, b->cap, a.done, U);
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, b->cap, a.info, U);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(256), 0, b->cap, a.head, (int64_t)2);
  (void)launch_fill(a.logdet, 0.0, U, b->cap);
  (void)launch_cheb_tables(a.mp, (double*)(w + b->off_nodes), (double*)a.tables, (int)b->n_omega,
                           b->cap);
  hipLaunchKernelGGL(k_batch_boxcox, dim3((unsigned)D), dim3(256), 0, b->cap, a.ds, a.lam, b->p,
                     b->M, b->TB, (double*)a.rhs, (double*)a.jac, (int32_t*)a.yflags);
  hipLaunchKernelGGL(k_batch_persistent, dim3(b->grid), dim3(256), 0, b->cap, a);
  return hipGetLastError();
}

// Capture of the size-bucketed schedule: prologue on the capture stream, the
// passes on the stream lanes forked from it, joined back at the end.
hipError_t capture_bucketed(pl_batch* b, char* w, pl_result* out, double* beta_hat) {
  const int64_t U = (int64_t)b->units.size(), D = (int64_t)b->ds.size();
  const BDataset* ds = (const BDataset*)(w + b->off_ds);
  const MaternParams* mp = (const MaternParams*)(w + b->off_mp);
  double* tables = (double*)(w + b->off_tables);
  double* rhs = (double*)(w + b->off_rhs);
  double* jac = (double*)(w + b->off_jac);
  int32_t* yflags = (int32_t*)(w + b->off_yflags);
  const double* lam = (const double*)(w + b->off_lam);
  const UnitInfo* ui = (const UnitInfo*)(w + b->off_uinfo);
  int32_t* info = (int32_t*)(w + b->off_info);
  hipError_t e = launch_cheb_tables(mp, (double*)(w + b->off_nodes), tables, (int)U, b->cap);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_boxcox, dim3((unsigned)D), dim3(256), 0, b->cap, ds, lam, b->p, b->M,
                     b->TB, rhs, jac, yflags);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(b->ev[0], b->cap)) != hipSuccess) return e;
  for (int l = 0; l < b->lanes; ++l)
    if ((e = hipStreamWaitEvent(b->lane_s[l], b->ev[0], 0)) != hipSuccess) return e;
  PassArgs pa{};
  pa.mixed = b->mixed;
  pa.flush = b->flush;
  pa.refine = b->refine;
  pa.locs = nullptr;  // each unit's own (UnitInfo)
  pa.rhs = rhs;
  pa.jac = jac;
  pa.yflags = yflags;
  pa.lam = lam;
  pa.p = b->p;
  pa.M = b->M;
  pa.out = out;
  pa.beta = beta_hat;
  pa.xvx = nullptr;
  for (const BPass& ps : b->passes) {
    pa.lay = packed_layout(ps.nmax, b->q);
    pa.lay.units = ui + ps.u0;
    pa.mp = mp + ps.u0;
    pa.tables = tables + (int64_t)ps.u0 * TABLE;
    pa.flag_ws = reinterpret_cast<uint8_t*>(w + b->off_nodes) + (size_t)ps.u0 * TABLE * sizeof(double);
    pa.info_out = info + ps.u0;
    const PassBufs pb = carve_pass(w + b->off_lanes + (size_t)ps.lane * b->region, pa.lay,
                                   b->mixed, ps.cnt);
    if ((e = run_pass(pa, pb, ps.cnt, b->lane_s[ps.lane])) != hipSuccess) return e;
  }
  for (int l = 0; l < b->lanes; ++l) {
    if ((e = hipEventRecord(b->ev[1 + l], b->lane_s[l])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(b->cap, b->ev[1 + l], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

int pl_batch_run(pl_batch* b, pl_result* out, double* beta_hat, void* work, size_t work_bytes,
                 void* stream) {
  if (!b) return -1;
  if (!out) return -2;
  if (!work) return -4;
  if (work_bytes < b->total) return -5;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)work;
  const bool rebuild = !b->exec || b->g_work != work || b->g_out != out || b->g_beta != beta_hat;
  if (rebuild) {
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
      return PL_E_HIP;
    if (!b->persistent && b->lane_s.empty()) {
      b->lane_s.assign(b->lanes, nullptr);
      b->ev.assign(b->lanes + 1, nullptr);
      for (auto& ls : b->lane_s)
        if (hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) != hipSuccess) return PL_E_HIP;
      for (auto& ev : b->ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return PL_E_HIP;
    }
    // the plan's tables go to the workspace once (outside the graph)
    auto up = [&](size_t off, const void* src, size_t bytes) {
      return bytes == 0 ? hipSuccess
                        : hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, b->cap);
    };
    std::vector<MaternParams> mps;
    if (!b->persistent) {  // parameters in the sorted unit order
      mps.resize(b->order.size());
      for (size_t i = 0; i < b->order.size(); ++i) mps[i] = b->params[b->order[i]];
    }
    const std::vector<MaternParams>& mpv = b->persistent ? b->params : mps;
    if ((b->persistent &&
         (up(b->off_tasks, b->tasks.data(), b->tasks.size() * sizeof(BTask)) != hipSuccess ||
          up(b->off_units, b->units.data(), b->units.size() * sizeof(BUnit)) != hipSuccess)) ||
        (!b->persistent &&
         up(b->off_uinfo, b->uinfo.data(), b->uinfo.size() * sizeof(UnitInfo)) != hipSuccess) ||
        up(b->off_ds, b->ds.data(), b->ds.size() * sizeof(BDataset)) != hipSuccess ||
        up(b->off_mp, mpv.data(), mpv.size() * sizeof(MaternParams)) != hipSuccess ||
        up(b->off_lam, b->lam.data(), b->lam.size() * sizeof(double)) != hipSuccess ||
        hipStreamSynchronize(b->cap) != hipSuccess)
      return PL_E_HIP;
    // per-kernel-class event timing is not recorded inside the graph
    (void)profiling_pause(true);
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)profiling_pause(false);
      return PL_E_HIP;
    }
    const hipError_t le = b->persistent ? capture_persistent(b, w, out, beta_hat)
                                        : capture_bucketed(b, w, out, beta_hat);
    const hipError_t ce = hipStreamEndCapture(b->cap, &graph);
    (void)profiling_pause(false);
    if (le != hipSuccess || ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return PL_E_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return PL_E_HIP;
    b->g_work = work;
    b->g_out = out;
    b->g_beta = beta_hat;
  }
  if (hipGraphLaunch(b->exec, s) != hipSuccess) return PL_E_HIP;
  if (b->mixed && b->fallback) {
    // units whose FP32 factorisation broke down: redone with the FP64 form
    // (their dataset alone) into their own records, then flagged
    const size_t U = b->units.size();
    std::vector<int32_t> hinfo(U);
    if (hipMemcpyAsync(hinfo.data(), w + b->off_info, U * sizeof(int32_t), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PL_E_HIP;
    pl_opts o64{};
    o64.precision = PL_FP64;
    o64.chunk = 1;
    for (size_t i = 0; i < U; ++i) {
      if (hinfo[i] <= 0) continue;
      const BUnit& u = b->units[b->order[i]];
      const BDataset& d = b->ds[u.d];
      const int rc = pl_profile_loglik(d.locs, d.y, d.X, d.n, b->p, &b->omega[5 * (size_t)u.om], 1,
                                       b->lam.data(), b->M, out + (int64_t)u.om * b->M,
                                       beta_hat ? beta_hat + (int64_t)u.om * b->M * b->p : nullptr,
                                       nullptr, &o64, w + b->off_lanes, b->region, stream);
      if (rc != PL_OK) return rc;
      if (launch_mark_fallback(out + (int64_t)u.om * b->M, b->M, s) != hipSuccess) return PL_E_HIP;
    }
  }
  return PL_OK;
}

int pl_batch_error(const pl_batch* b, void* work, int32_t* err) {
  if (!b) return -1;
  if (!work) return -2;
  if (!err) return -3;
  *err = 0;
  if (!b->persistent) return PL_OK;  // no waits in the size-bucketed schedule
  if (hipMemcpy(err, (char*)work + b->off_ctl + sizeof(int32_t), sizeof(int32_t),
                hipMemcpyDeviceToHost) != hipSuccess)
    return PL_E_HIP;
  return PL_OK;
}

void pl_batch_destroy(pl_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (auto ls : b->lane_s)
    if (ls) (void)hipStreamDestroy(ls);
  for (auto ev : b->ev)
    if (ev) (void)hipEventDestroy(ev);
  delete b;
}

}  // extern "C"
