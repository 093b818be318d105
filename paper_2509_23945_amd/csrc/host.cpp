// Host side of libtnmc: the C ABI of include/tnmc.h.  Owns the lattice state
// on the device, the per-task workspace (environments and R factors of every
// slice task of a half-sweep), builds the task lists of the even/odd
// half-sweeps and launches the contraction and sampling kernels on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "nn_internal.h"
#include "tnmc.h"
#include "tnmc_internal.h"

using tnmc::TaskDesc;


namespace {

// Host wall time of an entry point that reports statistics, from entry to
// return (such calls synchronise before they return).
struct CallClock {
  tnmc_stats* st;
  std::chrono::steady_clock::time_point t0;
  explicit CallClock(tnmc_stats* s) : st(s), t0(std::chrono::steady_clock::now()) {}
  ~CallClock() {
    if (st) st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};


thread_local std::string g_last_error;

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return (e_ == hipErrorOutOfMemory) ? TNMC_ERR_OOM : TNMC_ERR_DEVICE;            \
    }                                                                                 \
  } while (0)

constexpr int kLxMax = 64;
constexpr int kLyMax = 64;
// Philox sweep counters of TNMCMC-2 sweeps: sweep + 3 * 2^56 (slice directions
// use + 1 and + 2 times 2^56), so no uniform is shared with other updates.
constexpr uint64_t kSuperspinStride = 3ull << 56;

}  // namespace

struct tnmc_lattice {
  int Lx = 0, Ly = 0, Lz = 0, d = 2, chi = 1, chi_max = 4, precision = TNMC_FP64;
  int n_cand = 1;           // candidates per environment in sweeps
  int n_chains = 0, n_instances = 0, n_pairs = 0, record_capacity = 0;
  int64_t n_recorded = 0;
  uint64_t seed = 0;
  std::vector<int> chain_instance;
  std::vector<double> beta;
  std::vector<uint64_t> chain_key;
  std::vector<int> pairs;
  uint64_t J_hash = 0;      // FNV-1a of the couplings given at init (checkpoints are tied to them)
  float* dJ = nullptr;
  int8_t* dspins = nullptr;
  int* dpa = nullptr;
  int* dpb = nullptr;
  const float** dJc = nullptr;
  int8_t** dSc = nullptr;
  double* dErec = nullptr;
  double* dMrec = nullptr;
  double* dqrec = nullptr;
  double* dscal = nullptr;
  // learned proposal: per-(chain, z) running counts of its proposals
  // ([n_chains][Lz], kCounterStride long longs apart) and the frozen
  // tensor-network fallback flags (1 = that layer uses the TN proposal)
  long long* dnncnt = nullptr;
  std::vector<int8_t> nn_fallback;
  // slice-direction views (index 1: y-slices, 2: x-slices): the lattice with
  // permuted axes and coupling components, built on first use
  tnmc_lattice* view[3] = {nullptr, nullptr, nullptr};
  size_t sites() const { return (size_t)Lx * Ly * Lz; }
  const float* J_of(int c) const { return dJ + (size_t)chain_instance[c] * 3 * sites(); }
  int8_t* spins_of(int c) const { return dspins + (size_t)c * sites(); }
};

namespace {

// Grow-only device buffers shared by all lattices of the process.
struct Workspace {
  std::mutex mu;
  double* env = nullptr;
  size_t env_cap = 0;
  double* rscr = nullptr;
  size_t rscr_cap = 0;
  int* ints = nullptr;
  size_t ints_cap = 0;
  double* dbl = nullptr;
  size_t dbl_cap = 0;
  long long* counters = nullptr;
  size_t counters_cap = 0;
  TaskDesc* tasks = nullptr;
  size_t tasks_cap = 0;
  int8_t* bytes = nullptr;
  size_t bytes_cap = 0;
  double* gscr = nullptr;     // full contraction tile layout in global memory, per task (retry path)
  size_t gscr_cap = 0;
  TaskDesc* nn_tasks = nullptr;   // descriptors of the learned-proposal tasks of a sweep
  size_t nn_tasks_cap = 0;
  TaskDesc* tune_tasks = nullptr;   // descriptors of the layout trials
  size_t tune_tasks_cap = 0;
  long long* graph_state = nullptr;   // graph replays: [0] sweep counter, [1 + l] record slot of lattice l
  size_t graph_state_cap = 0;
  hipStream_t capture = nullptr;      // private stream on which sweeps are captured (default priority)
  // Device-side end of the last call that used this workspace, on whatever
  // stream it ran: the next call's stream waits for it, so calls made on
  // different streams never overwrite descriptors or workspace that kernels
  // of an earlier call still read.
  hipEvent_t done = nullptr;
  bool done_recorded = false;
};
Workspace g_ws;

// Orders one workspace-using call after the previous one (whatever stream
// either ran on) and marks its own end.  Taken with g_ws.mu held.
struct WsOrder {
  hipStream_t s;
  explicit WsOrder(hipStream_t st) : s(st) {
    if (!g_ws.done && hipEventCreateWithFlags(&g_ws.done, hipEventDisableTiming) != hipSuccess) g_ws.done = nullptr;
    if (g_ws.done && g_ws.done_recorded) (void)hipStreamWaitEvent(s, g_ws.done, 0);
  }
  ~WsOrder() {
    if (g_ws.done && hipEventRecord(g_ws.done, s) == hipSuccess) g_ws.done_recorded = true;
  }
};

template <typename T>
tnmc_status grow(T*& p, size_t& cap, size_t need) {
  if (need <= cap) return TNMC_OK;
  if (p) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(p));
    p = nullptr;
    cap = 0;
  }
  size_t n = std::max(need, (size_t)1);
  HIP_TRY(hipMalloc((void**)&p, n * sizeof(T)));
  cap = n;
  return TNMC_OK;
}

// Relative cut-off of the rank-revealing factorisations: 1e-15 for FP64
// environments, 1e-6 for FP32 ones, or 10^-g_rank_cut_exp for both when that is
// set (an ablation knob, tnmc_debug_set(3, k)).
int g_rank_cut_exp = 0;
double rank_tol_for(int precision) {
  if (g_rank_cut_exp > 0) return std::pow(10.0, -(double)g_rank_cut_exp);
  return (precision == TNMC_FP32) ? tnmc::kRankTolF32 : tnmc::kRankTolF64;
}

struct Task {
  tnmc_lattice* lat;
  int chain;
  int z;
  int key = 0;     // launch class: tasks of different keys never share a launch; lower keys first
  int super = 0;   // 1: TNMCMC-2 composite layer (z, z + 1) of superspins, d = 4
};

// States per site of a task's layer.
int task_d(const Task& t) { return t.super ? 4 : t.lat->d; }

// Builds the device descriptors of `tasks` at descriptor slot `slot0`, laid out
// in the shared workspace, grouped by kernel instantiation.
struct Plan {
  std::vector<TaskDesc> desc;
  std::vector<int> order;   // desc[k] runs tasks[order[k]]
  struct Group {
    int d, chi_max, first, count, lx_max, ly_max, key, precision;
  };
  std::vector<Group> groups;
};

// Relative cost of one slice task, for longest-first ordering: the
// contraction does Lx Ly factorisations of (d chi)-sized tiles; a layer with
// one held neighbour (z = 0 or Lz - 1) sees a weaker field, and its boundary
// states need larger bonds (about twice the work).
double task_cost(const Task& t) {
  const auto* L = t.lat;
  const double dc = (double)task_d(t) * L->chi;
  const bool edge = (L->Lz > 1) && (t.z == 0 || t.z == L->Lz - 1);
  return (double)L->Lx * L->Ly * dc * dc * dc * (edge ? 2.0 : 1.0);
}

tnmc_status make_plan(const std::vector<Task>& tasks, Plan& plan) {
  // order by instantiation so that each group is a contiguous launch, and
  // within a group longest task first: workgroups are dispatched in index
  // order, so the long tasks start in the first wave of the grid
  std::vector<int> order(tasks.size());
  for (size_t i = 0; i < tasks.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const auto* la = tasks[a].lat;
    const auto* lb = tasks[b].lat;
    if (tasks[a].key != tasks[b].key) return tasks[a].key < tasks[b].key;
    if (task_d(tasks[a]) != task_d(tasks[b])) return task_d(tasks[a]) < task_d(tasks[b]);
    if (la->chi_max != lb->chi_max) return la->chi_max < lb->chi_max;
    if (la->precision != lb->precision) return la->precision < lb->precision;
    return task_cost(tasks[a]) > task_cost(tasks[b]);
  });
  // Tasks of different keys (the two parities of a sweep) run in launches
  // strictly in key order, and a task's workspace is dead once its sampler
  // launch has run, so each key's tasks lay their workspace out from the
  // start of the buffers again: the buffers hold the largest key's share.
  size_t env_need = 0, rscr_need = 0, int_need = 0, dbl_need = 0, gscr_need = 0;
  {
    size_t e = 0, r = 0, in = 0, db = 0, g = 0;
    for (size_t k = 0; k < order.size(); ++k) {
      const auto* L = tasks[order[k]].lat;
      const int d = task_d(tasks[order[k]]);
      if (k > 0 && tasks[order[k]].key != tasks[order[k - 1]].key) e = r = in = db = g = 0;
      if (tnmc::contract_uses_global(d, L->chi_max))
        g += tnmc::pad256_doubles(tnmc::contract_lds_bytes(d, L->chi_max) / sizeof(double));
      e += tnmc::pad256_doubles(tnmc::env_doubles(L->Lx, L->Ly, d, L->chi_max, L->precision));
      r += tnmc::pad256_doubles(tnmc::rscr_doubles(L->Lx, d, L->chi_max));
      in += tnmc::pad256_ints((size_t)L->Ly * L->Lx + 1);
      db += tnmc::pad256_doubles((size_t)L->Ly);
      env_need = std::max(env_need, e);
      rscr_need = std::max(rscr_need, r);
      int_need = std::max(int_need, in);
      dbl_need = std::max(dbl_need, db);
      gscr_need = std::max(gscr_need, g);
    }
  }
  if (grow(g_ws.env, g_ws.env_cap, env_need) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.rscr, g_ws.rscr_cap, rscr_need) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.ints, g_ws.ints_cap, int_need) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.dbl, g_ws.dbl_cap, dbl_need) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.gscr, g_ws.gscr_cap, gscr_need) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.counters, g_ws.counters_cap, tnmc::kCounterStride * tasks.size()) != TNMC_OK) return TNMC_ERR_OOM;
  plan.desc.clear();
  plan.groups.clear();
  plan.order = order;
  size_t eo = 0, ro = 0, io = 0, dof = 0, go = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    const Task& tk = tasks[order[k]];
    const auto* L = tk.lat;
    const int d = task_d(tk);
    if (k > 0 && tk.key != tasks[order[k - 1]].key) eo = ro = io = dof = go = 0;
    TaskDesc t;
    std::memset(&t, 0, sizeof(t));
    t.J = L->J_of(tk.chain);
    t.spins = L->spins_of(tk.chain);
    t.env = g_ws.env + eo;
    t.rscr = g_ws.rscr + ro;
    t.gscr = tnmc::contract_uses_global(d, L->chi_max) ? g_ws.gscr + go : nullptr;
    t.bond = g_ws.ints + io;
    t.status = g_ws.ints + io + (size_t)L->Ly * L->Lx;
    t.logscale = g_ws.dbl + dof;
    t.counters = g_ws.counters + tnmc::kCounterStride * k;
    t.beta = L->beta[tk.chain];
    t.rank_tol = rank_tol_for(L->precision);
    t.key0 = L->seed;
    t.key1 = L->chain_key[tk.chain];
    t.Lx = L->Lx;
    t.Ly = L->Ly;
    t.Lz = L->Lz;
    t.z = tk.z;
    t.chi = L->chi;
    t.d = d;
    t.chi_max = L->chi_max;
    t.write_back = 1;
    t.n_cand = L->n_cand;
    eo += tnmc::pad256_doubles(tnmc::env_doubles(L->Lx, L->Ly, d, L->chi_max, L->precision));
    if (tnmc::contract_uses_global(d, L->chi_max))
      go += tnmc::pad256_doubles(tnmc::contract_lds_bytes(d, L->chi_max) / sizeof(double));
    ro += tnmc::pad256_doubles(tnmc::rscr_doubles(L->Lx, d, L->chi_max));
    io += tnmc::pad256_ints((size_t)L->Ly * L->Lx + 1);
    dof += tnmc::pad256_doubles((size_t)L->Ly);
    if (plan.groups.empty() || plan.groups.back().d != d || plan.groups.back().chi_max != L->chi_max ||
        plan.groups.back().key != tk.key || plan.groups.back().precision != L->precision) {
      plan.groups.push_back({d, L->chi_max, (int)k, 0, 0, 0, tk.key, L->precision});
    }
    plan.groups.back().count += 1;
    plan.groups.back().lx_max = std::max(plan.groups.back().lx_max, L->Lx);
    plan.groups.back().ly_max = std::max(plan.groups.back().ly_max, L->Ly);
    plan.desc.push_back(t);
  }
  return TNMC_OK;
}

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> c_ev, s_ev;   // start/stop pairs
  ~Timer() {
    for (auto e : c_ev) (void)hipEventDestroy(e);
    for (auto e : s_ev) (void)hipEventDestroy(e);
  }
  tnmc_status mark(std::vector<hipEvent_t>& v, hipStream_t s) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    v.push_back(e);
    HIP_TRY(hipEventRecord(e, s));
    return TNMC_OK;
  }
};

tnmc::ContractCfg contract_cfg(const Plan::Group& g);   // the autotuner's choice for a launch group (below)

// Launch the contraction and sampling kernels of a plan whose descriptors are at dtasks.
tnmc_status launch_plan(const Plan& plan, const TaskDesc* dtasks, uint64_t sweep, hipStream_t s, Timer* tm,
                        tnmc_stats* st) {
  for (const auto& g : plan.groups) {
    if (tm && tm->on && tm->mark(tm->c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
    HIP_TRY(tnmc::launch_contract(dtasks + g.first, g.count, g.d, g.chi_max, g.precision, contract_cfg(g), s));
    if (tm && tm->on && tm->mark(tm->c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
    if (st) st->contract_launches += 1;
  }
  for (const auto& g : plan.groups) {
    if (tm && tm->on && tm->mark(tm->s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
    HIP_TRY(tnmc::launch_sample(dtasks + g.first, g.count, g.d, g.chi_max, g.precision, g.lx_max, g.ly_max, sweep,
                                s));
    if (tm && tm->on && tm->mark(tm->s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
    if (st) st->sample_launches += 1;
  }
  return TNMC_OK;
}

std::vector<Task> half_sweep_tasks(tnmc_lattice* const* lats, int n_lats, int parity) {
  std::vector<Task> v;
  for (int l = 0; l < n_lats; ++l)
    for (int c = 0; c < lats[l]->n_chains; ++c)
      for (int z = parity; z < lats[l]->Lz; z += 2) v.push_back({lats[l], c, z});
  return v;
}

tnmc_status check_lats(tnmc_lattice* const* lats, int n_lats) {
  if (!lats || n_lats < 1) return TNMC_ERR_ARG;
  for (int i = 0; i < n_lats; ++i)
    if (!lats[i]) return TNMC_ERR_ARG;
  return TNMC_OK;
}

tnmc_status read_counters(size_t n_tasks, tnmc_stats* st) {
  const int K = tnmc::kCounterStride;
  std::vector<long long> c(K * n_tasks);
  HIP_TRY(hipMemcpy(c.data(), g_ws.counters, c.size() * sizeof(long long), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < n_tasks; ++i) {
    st->proposed += c[K * i];
    st->accepted += c[K * i + 1];
    st->numeric_faults += c[K * i + 2];
    st->contract_flops += (double)c[K * i + 3];
    st->contract_retries += c[K * i + 4];
  }
  return TNMC_OK;
}

tnmc_status finish_timer(Timer& tm, tnmc_stats* st) {
  if (!tm.on || !st) return TNMC_OK;
  auto sum = [](std::vector<hipEvent_t>& v, double& acc) -> tnmc_status {
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
      HIP_TRY(hipEventSynchronize(v[i + 1]));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, v[i], v[i + 1]));
      acc += ms;
    }
    return TNMC_OK;
  };
  tnmc_status r = sum(tm.c_ev, st->contract_ms);
  if (r != TNMC_OK) return r;
  return sum(tm.s_ev, st->sample_ms);
}

// Autotuner of the contraction (batching).  A class of slice tasks is keyed
// by (d, chi_max, storage precision, row length, row count, tasks in the
// launch).  Its candidates are the product engines (vector ALU, matrix cores)
// times, where the class has a compact layout (two tasks per CU, with a
// full-layout redo of the tasks that outgrow it), the two tile layouts.
// Every candidate is a correct contraction; they agree within the parity bar
// of the storage precision (not bit for bit, so pin them for bit-for-bit
// reproducible runs across processes).  Before the second sweep of a class,
// the contraction of that sweep's tasks runs once per candidate untimed (a
// kernel's first launch also loads its code), then three times per candidate
// timed with HIP events (descriptors without counters, so the statistics see
// only the real launch, which follows and rewrites the same workspace); the
// candidate of the smallest median is kept for the process.  The first sweep
// from a prepared (often random) configuration meets larger ranks than the
// chain sees afterwards and would bias the choice.
struct TuneResult {
  tnmc::ContractCfg cfg;
  double ms[2][2] = {{-1.0, -1.0}, {-1.0, -1.0}};   // median ms per [engine][layout], -1: not a candidate
};
using TuneKey = std::tuple<int, int, int, int, int, int>;
std::map<TuneKey, TuneResult> g_tune;
std::map<TuneKey, int> g_tune_seen;   // sweeps run per class before its trial
TuneKey g_tune_last{};                // most recent key tuned (reported by tnmc_layout_choice)
bool g_tune_any = false;
bool g_autotune = true;
int g_pin_layout = -1, g_pin_engine = -1;   // -1: tuned; 0 / 1: fixed by tnmc_autotune_pin
bool g_nn_pairing = true;   // two learned-proposal tasks per workgroup where a launch allows it

TuneKey tune_key(const Plan::Group& g) {
  return std::make_tuple(g.d, g.chi_max, g.precision, g.lx_max, g.ly_max, g.count);
}

// Configuration used for a launch group: the pins, then the tuned choice,
// then the defaults (compact layout where it exists, vector-ALU products).
tnmc::ContractCfg contract_cfg(const Plan::Group& g) {
  tnmc::ContractCfg c;
  auto it = g_tune.find(tune_key(g));
  if (it != g_tune.end()) c = it->second.cfg;
  if (g_pin_layout >= 0) c.full = g_pin_layout;
  if (g_pin_engine >= 0) c.mfma = g_pin_engine;
  return c;
}

tnmc_status time_launch(const TaskDesc* dt, const Plan::Group& g, tnmc::ContractCfg cfg, hipStream_t s, double* ms) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    HIP_TRY(e);
  }
  e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = tnmc::launch_contract(dt, g.count, g.d, g.chi_max, g.precision, cfg, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(e);
  *ms = t;
  return TNMC_OK;
}

// Trials for the classes of the plan that have run one sweep already (every
// class of the plan with force, replacing earlier choices).
tnmc_status autotune_groups(const Plan& plan, hipStream_t s, bool force = false) {
  if (!g_autotune) return TNMC_OK;
  std::set<TuneKey> done;
  for (const auto& g : plan.groups) {
    const TuneKey key = tune_key(g);
    if (force) {
      if (done.count(key)) continue;
      done.insert(key);
      g_tune.erase(key);
    } else if (g_tune.count(key) || g_tune_seen[key] < 1) {
      continue;
    }
    std::vector<tnmc::ContractCfg> cands;
    for (int mf : {0, 1})
      for (int full : {0, 1}) {
        if (full && !tnmc::contract_has_compact(g.d, g.chi_max)) continue;
        if ((g_pin_layout >= 0 && full != g_pin_layout && tnmc::contract_has_compact(g.d, g.chi_max)) ||
            (g_pin_engine >= 0 && mf != g_pin_engine))
          continue;
        tnmc::ContractCfg c;
        c.full = full;
        c.mfma = mf;
        cands.push_back(c);
      }
    TuneResult r;
    r.cfg = contract_cfg(g);
    if (cands.size() > 1) {
      std::vector<TaskDesc> trial(plan.desc.begin() + g.first, plan.desc.begin() + g.first + g.count);
      for (auto& t : trial) {
        t.counters = nullptr;
        t.record = nullptr;
      }
      if (grow(g_ws.tune_tasks, g_ws.tune_tasks_cap, trial.size()) != TNMC_OK) return TNMC_ERR_OOM;
      HIP_TRY(hipMemcpyAsync(g_ws.tune_tasks, trial.data(), trial.size() * sizeof(TaskDesc), hipMemcpyHostToDevice,
                             s));
      HIP_TRY(hipStreamSynchronize(s));
      for (const auto& c : cands) HIP_TRY(tnmc::launch_contract(g_ws.tune_tasks, g.count, g.d, g.chi_max, g.precision, c, s));
      HIP_TRY(hipStreamSynchronize(s));
      double best = 1e300;
      for (const auto& c : cands) {
        double t[3];
        for (double& ti : t) {
          tnmc_status st = time_launch(g_ws.tune_tasks, g, c, s, &ti);
          if (st != TNMC_OK) return st;
        }
        std::sort(t, t + 3);
        r.ms[c.mfma][c.full] = t[1];
        if (t[1] < best) {
          best = t[1];
          r.cfg = c;
        }
      }
    }
    g_tune[key] = r;
    g_tune_last = key;
    g_tune_any = true;
  }
  return TNMC_OK;
}

// One task run with optional forced layer; used by propose / logq.
tnmc_status run_single(tnmc_lattice* lat, int chain, int z, uint64_t sweep, const int8_t* force_in,
                       int8_t* s_new_out, double* rec_host, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_ws.mu);
  WsOrder order(s);
  g_last_error.clear();
  std::vector<Task> tasks{{lat, chain, z}};
  Plan plan;
  tnmc_status r = make_plan(tasks, plan);
  if (r != TNMC_OK) return r;
  const size_t plane = (size_t)lat->Lx * lat->Ly;
  if (grow(g_ws.bytes, g_ws.bytes_cap, 2 * plane) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.tasks, g_ws.tasks_cap, (size_t)1) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.dbl, g_ws.dbl_cap, (size_t)lat->Ly + 8) != TNMC_OK) return TNMC_ERR_OOM;
  double* drec = g_ws.dbl + lat->Ly;   // after this task's logscale
  plan.desc[0].logscale = g_ws.dbl;
  plan.desc[0].record = drec;
  plan.desc[0].counters = nullptr;
  plan.desc[0].write_back = 0;
  plan.desc[0].n_cand = 1;   // a single proposal
  plan.desc[0].s_new_out = g_ws.bytes;
  if (force_in) {
    HIP_TRY(hipMemcpyAsync(g_ws.bytes + plane, force_in, plane, hipMemcpyDefault, s));   // host or device
    plan.desc[0].force_new = g_ws.bytes + plane;
  }
  HIP_TRY(hipMemcpyAsync(g_ws.tasks, plan.desc.data(), sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // host buffers above are released on return
  r = launch_plan(plan, g_ws.tasks, sweep, s, nullptr, nullptr);
  if (r != TNMC_OK) return r;
  if (s_new_out) HIP_TRY(hipMemcpyAsync(s_new_out, g_ws.bytes, plane, hipMemcpyDefault, s));   // host or device
  HIP_TRY(hipMemcpyAsync(rec_host, drec, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return TNMC_OK;
}

double qr_flops(double m, double n) {   // Householder, R only: min(m, n) reflections
  double f = 0.0;
  const int r = (int)std::min(m, n);
  for (int k = 0; k < r; ++k) f += 4.0 * (m - k) * (n - k - 1) + 3.0 * (m - k);
  return f;
}
double svd_flops(double m, double n) {  // Golub-Reinsch, singular values and right vectors
  const double a = std::max(m, n), b = std::min(m, n);
  return 4.0 * a * b * b + 8.0 * b * b * b;
}

}  // namespace

extern "C" {

const char* tnmc_status_string(tnmc_status s) {
  switch (s) {
    case TNMC_OK: return "ok";
    case TNMC_ERR_ARG: return "invalid argument";
    case TNMC_ERR_OOM: return "device out of memory";
    case TNMC_ERR_DEVICE: return "HIP error";
    case TNMC_ERR_NUMERIC: return "numeric fault";
    case TNMC_ERR_UNSUPPORTED: return "unsupported configuration";
    case TNMC_ERR_IO: return "checkpoint file error";
  }
  return "unknown status";
}

const char* tnmc_last_error(void) { return g_last_error.c_str(); }

tnmc_status tnmc_mh_accept(double logq_old, double logq_new, double beta, double dE, double u, int32_t* accepted) {
  if (!accepted || !(u > 0.0 && u < 1.0) || !std::isfinite(beta)) return TNMC_ERR_ARG;
  const double lr = logq_old - logq_new - beta * dE;
  *accepted = (u < std::exp(std::min(0.0, lr))) ? 1 : 0;
  return TNMC_OK;
}

tnmc_status tnmc_lattice_init(const tnmc_lattice_desc* ds, tnmc_lattice** out) {
  if (!ds || !out) return TNMC_ERR_ARG;
  if (ds->Lx < 1 || ds->Ly < 1 || ds->Lz < 1 || ds->Lx > kLxMax || ds->Ly > kLyMax) return TNMC_ERR_ARG;
  if (ds->d != 2 && ds->d != 3) return TNMC_ERR_ARG;
  if (ds->chi < 1 || ds->n_chains < 1 || ds->n_instances < 1 || !ds->J || !ds->beta || !ds->spins)
    return TNMC_ERR_ARG;
  if (ds->n_pairs < 0 || (ds->n_pairs > 0 && !ds->pairs) || ds->record_capacity < 0) return TNMC_ERR_ARG;
  if (ds->precision != TNMC_FP64 && ds->precision != TNMC_FP32) return TNMC_ERR_UNSUPPORTED;
  if (ds->n_candidates < 0 || ds->n_candidates > 64) return TNMC_ERR_ARG;
  const int cm = tnmc::chi_bucket(ds->chi);
  if (cm == 0 || !tnmc::contract_supported(ds->d, cm)) return TNMC_ERR_UNSUPPORTED;
  // the sampler keeps a row of right environments and two site tiles in LDS
  if (tnmc::sample_lds_bytes(ds->d, cm, ds->Lx, ds->Ly) > 160 * 1024) return TNMC_ERR_UNSUPPORTED;
  for (int c = 0; c < ds->n_chains; ++c) {
    const int inst = ds->chain_instance ? ds->chain_instance[c] : c % ds->n_instances;
    if (inst < 0 || inst >= ds->n_instances) return TNMC_ERR_ARG;
    if (!(ds->beta[c] >= 0.0) || !std::isfinite(ds->beta[c])) return TNMC_ERR_ARG;
  }
  for (int p = 0; p < 2 * ds->n_pairs; ++p)
    if (ds->pairs[p] < 0 || ds->pairs[p] >= ds->n_chains) return TNMC_ERR_ARG;
  const size_t n = (size_t)ds->Lx * ds->Ly * ds->Lz;
  for (size_t i = 0; i < n * ds->n_chains; ++i) {
    const int v = ds->spins[i];
    if (ds->d == 2 ? (v != 1 && v != -1) : (v < 0 || v >= ds->d)) return TNMC_ERR_ARG;
  }
  auto* L = new tnmc_lattice();
  L->Lx = ds->Lx;
  L->Ly = ds->Ly;
  L->Lz = ds->Lz;
  L->d = ds->d;
  L->chi = ds->chi;
  L->chi_max = cm;
  L->precision = ds->precision;
  L->n_cand = ds->n_candidates > 0 ? ds->n_candidates : 1;
  L->n_chains = ds->n_chains;
  L->n_instances = ds->n_instances;
  L->n_pairs = ds->n_pairs;
  L->record_capacity = ds->record_capacity;
  L->seed = ds->seed;
  L->chain_instance.resize(ds->n_chains);
  L->beta.assign(ds->beta, ds->beta + ds->n_chains);
  L->chain_key.resize(ds->n_chains);
  for (int c = 0; c < ds->n_chains; ++c) {
    L->chain_instance[c] = ds->chain_instance ? ds->chain_instance[c] : c % ds->n_instances;
    L->chain_key[c] = ds->chain_key ? ds->chain_key[c] : (uint64_t)c;
  }
  L->pairs.assign(ds->pairs, ds->pairs + 2 * ds->n_pairs);
  auto fail = [&](tnmc_status r) {
    tnmc_lattice_free(L);
    return r;
  };
#define INIT_TRY(expr)                                                   \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess) {                                              \
      g_last_error = std::string(#expr) + ": " + hipGetErrorString(e_);  \
      return fail(e_ == hipErrorOutOfMemory ? TNMC_ERR_OOM : TNMC_ERR_DEVICE); \
    }                                                                    \
  } while (0)
  {
    uint64_t h = 1469598103934665603ull;
    const unsigned char* p = reinterpret_cast<const unsigned char*>(ds->J);
    for (size_t i = 0; i < (size_t)ds->n_instances * 3 * n * sizeof(float); ++i) h = (h ^ p[i]) * 1099511628211ull;
    L->J_hash = h;
  }
  (void)tnmc::device_cus();   // the one device query of the launch rules, made here, outside any capture
  INIT_TRY(hipMalloc((void**)&L->dJ, (size_t)ds->n_instances * 3 * n * sizeof(float)));
  INIT_TRY(hipMemcpy(L->dJ, ds->J, (size_t)ds->n_instances * 3 * n * sizeof(float), hipMemcpyHostToDevice));
  INIT_TRY(hipMalloc((void**)&L->dspins, (size_t)ds->n_chains * n));
  INIT_TRY(hipMemcpy(L->dspins, ds->spins, (size_t)ds->n_chains * n, hipMemcpyHostToDevice));
  std::vector<const float*> jc(ds->n_chains);
  std::vector<int8_t*> sc(ds->n_chains);
  for (int c = 0; c < ds->n_chains; ++c) {
    jc[c] = L->J_of(c);
    sc[c] = L->spins_of(c);
  }
  INIT_TRY(hipMalloc((void**)&L->dJc, ds->n_chains * sizeof(float*)));
  INIT_TRY(hipMemcpy(L->dJc, jc.data(), ds->n_chains * sizeof(float*), hipMemcpyHostToDevice));
  INIT_TRY(hipMalloc((void**)&L->dSc, ds->n_chains * sizeof(int8_t*)));
  INIT_TRY(hipMemcpy(L->dSc, sc.data(), ds->n_chains * sizeof(int8_t*), hipMemcpyHostToDevice));
  if (ds->n_pairs > 0) {
    std::vector<int> pa(ds->n_pairs), pb(ds->n_pairs);
    for (int p = 0; p < ds->n_pairs; ++p) {
      pa[p] = ds->pairs[2 * p];
      pb[p] = ds->pairs[2 * p + 1];
    }
    INIT_TRY(hipMalloc((void**)&L->dpa, ds->n_pairs * sizeof(int)));
    INIT_TRY(hipMemcpy(L->dpa, pa.data(), ds->n_pairs * sizeof(int), hipMemcpyHostToDevice));
    INIT_TRY(hipMalloc((void**)&L->dpb, ds->n_pairs * sizeof(int)));
    INIT_TRY(hipMemcpy(L->dpb, pb.data(), ds->n_pairs * sizeof(int), hipMemcpyHostToDevice));
  }
  const size_t cap = std::max(1, ds->record_capacity);
  INIT_TRY(hipMalloc((void**)&L->dErec, cap * ds->n_chains * sizeof(double)));
  INIT_TRY(hipMalloc((void**)&L->dMrec, cap * ds->n_chains * sizeof(double)));
  INIT_TRY(hipMalloc((void**)&L->dqrec, cap * std::max(1, ds->n_pairs) * sizeof(double)));
  INIT_TRY(hipMalloc((void**)&L->dscal, 8 * sizeof(double)));
#undef INIT_TRY
  *out = L;
  return TNMC_OK;
}

tnmc_status tnmc_lattice_free(tnmc_lattice* L) {
  if (!L) return TNMC_ERR_ARG;
  (void)hipDeviceSynchronize();
  for (tnmc_lattice* v : L->view)
    if (v) tnmc_lattice_free(v);
  void* ptrs[] = {L->dJ, L->dspins, L->dpa, L->dpb, (void*)L->dJc, (void*)L->dSc,
                  L->dErec, L->dMrec, L->dqrec, L->dscal, (void*)L->dnncnt};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete L;
  return TNMC_OK;
}

tnmc_status tnmc_slice_propose(tnmc_lattice* lat, int32_t chain, int32_t z, uint64_t sweep, int8_t* s_new,
                               double* logq_new, double* logq_old, double* dE, void* stream) {
  if (!lat || chain < 0 || chain >= lat->n_chains || z < 0 || z >= lat->Lz) return TNMC_ERR_ARG;
  if (!s_new || !logq_new || !logq_old || !dE) return TNMC_ERR_ARG;
  double rec[5];
  tnmc_status r = run_single(lat, chain, z, sweep, nullptr, s_new, rec, (hipStream_t)stream);
  if (r != TNMC_OK) return r;
  *logq_new = rec[0];
  *logq_old = rec[1];
  *dE = rec[2];
  if (rec[4] != 0.0 || !std::isfinite(rec[0]) || !std::isfinite(rec[1])) {
    g_last_error = "numeric fault bits " + std::to_string((int)rec[4]) +
                   " (1-2: new path, 4-8: current path, 16-64: contraction)";
    return TNMC_ERR_NUMERIC;
  }
  return TNMC_OK;
}

tnmc_status tnmc_slice_logq(tnmc_lattice* lat, int32_t chain, int32_t z, const int8_t* s, double* logq,
                            void* stream) {
  if (!lat || chain < 0 || chain >= lat->n_chains || z < 0 || z >= lat->Lz || !s || !logq) return TNMC_ERR_ARG;
  const size_t plane = (size_t)lat->Lx * lat->Ly;
  for (size_t i = 0; i < plane; ++i) {
    const int v = s[i];
    if (lat->d == 2 ? (v != 1 && v != -1) : (v < 0 || v >= lat->d)) return TNMC_ERR_ARG;
  }
  double rec[5];
  tnmc_status r = run_single(lat, chain, z, 0, s, nullptr, rec, (hipStream_t)stream);
  if (r != TNMC_OK) return r;
  *logq = rec[0];
  if (!std::isfinite(rec[0])) return TNMC_ERR_NUMERIC;
  return TNMC_OK;
}

tnmc_status tnmc_half_sweep(tnmc_lattice* const* lats, int32_t n_lats, int32_t parity, uint64_t sweep,
                            double* trace, tnmc_stats* stats, void* stream) {
  CallClock clock(stats);
  if (check_lats(lats, n_lats) != TNMC_OK || (parity != 0 && parity != 1)) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  hipStream_t s = (hipStream_t)stream;
  WsOrder order(s);
  auto tasks = half_sweep_tasks(lats, n_lats, parity);
  Plan plan;
  tnmc_status r = make_plan(tasks, plan);
  if (r != TNMC_OK) return r;
  // trace order is the task order (lattice, chain, z); descriptor k runs task plan.order[k]
  for (size_t k = 0; k < plan.desc.size(); ++k) {
    plan.desc[k].record = trace ? trace + 5 * (size_t)plan.order[k] : nullptr;
  }
  if (grow(g_ws.tasks, g_ws.tasks_cap, plan.desc.size()) != TNMC_OK) return TNMC_ERR_OOM;
  HIP_TRY(hipMemcpyAsync(g_ws.tasks, plan.desc.data(), plan.desc.size() * sizeof(TaskDesc),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) HIP_TRY(hipMemsetAsync(g_ws.counters, 0, tnmc::kCounterStride * tasks.size() * sizeof(long long), s));
  Timer tm;
  tm.on = (stats != nullptr);
  r = launch_plan(plan, g_ws.tasks, sweep, s, &tm, stats);
  if (r != TNMC_OK) return r;
  if (stats) {
    HIP_TRY(hipStreamSynchronize(s));
    r = read_counters(tasks.size(), stats);
    if (r != TNMC_OK) return r;
    r = finish_timer(tm, stats);
    if (r != TNMC_OK) return r;
  }
  return TNMC_OK;
}

// Streams of the sweep schedule besides the caller's (default priority,
// created on first use).
tnmc_status tnmc_sweep(tnmc_lattice* const* lats, int32_t n_lats, int32_t n_sweeps, uint64_t sweep_offset,
                       int32_t record, int32_t time_kernels, tnmc_stats* stats, void* stream) {
  CallClock clock(stats);
  if (check_lats(lats, n_lats) != TNMC_OK || n_sweeps < 0) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  hipStream_t s = (hipStream_t)stream;
  WsOrder order(s);
  // Every task of a parity with a workspace of its own (the two parities
  // share the buffers); one launch pair (contraction, sampler) per (parity,
  // d, chi_max), longest task first, all on the caller's stream.  Launches
  // are kept strictly in order (no two kernels of a sweep run at the same
  // time), which the shared workspace relies on.
  std::vector<Task> tasks;
  for (int p : {0, 1})
    for (Task t : half_sweep_tasks(lats, n_lats, p)) {
      t.key = p;
      tasks.push_back(t);
    }
  Plan plan;
  tnmc_status r = make_plan(tasks, plan);
  if (r != TNMC_OK) return r;
  const size_t n_tasks = plan.desc.size();
  if (grow(g_ws.counters, g_ws.counters_cap, tnmc::kCounterStride * n_tasks) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.tasks, g_ws.tasks_cap, n_tasks) != TNMC_OK) return TNMC_ERR_OOM;
  for (size_t k = 0; k < n_tasks; ++k) plan.desc[k].counters = g_ws.counters + tnmc::kCounterStride * k;
  HIP_TRY(hipMemcpyAsync(g_ws.tasks, plan.desc.data(), n_tasks * sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // plan.desc is released on return
  HIP_TRY(hipMemsetAsync(g_ws.counters, 0, tnmc::kCounterStride * n_tasks * sizeof(long long), s));

  Timer tm;
  tm.on = (time_kernels != 0 && stats != nullptr);
  for (int t = 0; t < n_sweeps; ++t) {
    const uint64_t sw = sweep_offset + (uint64_t)t;
    r = autotune_groups(plan, s);
    if (r != TNMC_OK) return r;
    for (const auto& g : plan.groups) {
      const TaskDesc* dt = g_ws.tasks + g.first;
      if (tm.on && tm.mark(tm.c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      HIP_TRY(tnmc::launch_contract(dt, g.count, g.d, g.chi_max, g.precision, contract_cfg(g), s));
      if (tm.on && tm.mark(tm.c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      HIP_TRY(tnmc::launch_sample(dt, g.count, g.d, g.chi_max, g.precision, g.lx_max, g.ly_max, sw, s));
      if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      if (stats) {
        stats->contract_launches += 1;
        stats->sample_launches += 1;
      }
    }
    {
      std::set<TuneKey> swept;
      for (const auto& g : plan.groups) swept.insert(tune_key(g));
      for (const auto& k : swept) g_tune_seen[k] += 1;
    }
    if (record) {
      for (int l = 0; l < n_lats; ++l) {
        tnmc_lattice* L = lats[l];
        if (L->n_recorded >= L->record_capacity) continue;
        const int64_t i = L->n_recorded++;
        HIP_TRY(tnmc::launch_observables(L->dJc, L->dSc, L->n_chains, L->dpa, L->dpb, L->n_pairs, L->Lx, L->Ly,
                                         L->Lz, L->d, L->dErec + i * L->n_chains, L->dMrec + i * L->n_chains,
                                         L->dqrec + i * std::max(1, L->n_pairs), s));
      }
    }
  }
  if (stats) {
    HIP_TRY(hipStreamSynchronize(s));
    r = read_counters(n_tasks, stats);
    if (r != TNMC_OK) return r;
    r = finish_timer(tm, stats);
    if (r != TNMC_OK) return r;
  }
  return TNMC_OK;
}

tnmc_status tnmc_sweep_superspin(tnmc_lattice* const* lats, int32_t n_lats, int32_t n_sweeps, uint64_t sweep_offset,
                                 int32_t record, int32_t time_kernels, double* trace, tnmc_stats* stats,
                                 void* stream) {
  CallClock clock(stats);
  if (check_lats(lats, n_lats) != TNMC_OK || n_sweeps < 0) return TNMC_ERR_ARG;
  for (int l = 0; l < n_lats; ++l) {
    const tnmc_lattice* L = lats[l];
    if (L->d != 2 || L->Lz < 2 || L->chi_max > 8 || !tnmc::contract_supported(4, L->chi_max) ||
        tnmc::sample_lds_bytes(4, L->chi_max, L->Lx, L->Ly) > 160 * 1024)
      return TNMC_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_ws.mu);
  hipStream_t s = (hipStream_t)stream;
  WsOrder order(s);
  // composite layers z0 = 0 .. Lz - 2 in three phases (z0 mod 3): the
  // composites of a phase share no layer they update nor one they hold, so
  // each phase is one launch pair per (precision, chi_max), strictly in order
  std::vector<Task> tasks;
  for (int p = 0; p < 3; ++p)
    for (int l = 0; l < n_lats; ++l)
      for (int c = 0; c < lats[l]->n_chains; ++c)
        for (int z0 = p; z0 + 1 < lats[l]->Lz; z0 += 3) {
          Task t{lats[l], c, z0};
          t.key = p;
          t.super = 1;
          tasks.push_back(t);
        }
  Plan plan;
  tnmc_status r = make_plan(tasks, plan);
  if (r != TNMC_OK) return r;
  const size_t n_tasks = plan.desc.size();
  if (grow(g_ws.counters, g_ws.counters_cap, tnmc::kCounterStride * n_tasks) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.tasks, g_ws.tasks_cap, n_tasks) != TNMC_OK) return TNMC_ERR_OOM;
  for (size_t k = 0; k < n_tasks; ++k) {
    plan.desc[k].counters = g_ws.counters + tnmc::kCounterStride * k;
    plan.desc[k].n_cand = 1;   // one candidate per composite update
    plan.desc[k].record = trace ? trace + 5 * (size_t)plan.order[k] : nullptr;
  }
  HIP_TRY(hipMemcpyAsync(g_ws.tasks, plan.desc.data(), n_tasks * sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemsetAsync(g_ws.counters, 0, tnmc::kCounterStride * n_tasks * sizeof(long long), s));
  Timer tm;
  tm.on = (time_kernels != 0 && stats != nullptr);
  for (int t = 0; t < n_sweeps; ++t) {
    const uint64_t sw = sweep_offset + (uint64_t)t + kSuperspinStride;
    for (const auto& g : plan.groups) {
      const TaskDesc* dt = g_ws.tasks + g.first;
      if (tm.on && tm.mark(tm.c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      HIP_TRY(tnmc::launch_contract(dt, g.count, g.d, g.chi_max, g.precision, contract_cfg(g), s));
      if (tm.on && tm.mark(tm.c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      HIP_TRY(tnmc::launch_sample(dt, g.count, g.d, g.chi_max, g.precision, g.lx_max, g.ly_max, sw, s));
      if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
      if (stats) {
        stats->contract_launches += 1;
        stats->sample_launches += 1;
      }
    }
    if (record) {
      for (int l = 0; l < n_lats; ++l) {
        tnmc_lattice* L = lats[l];
        if (L->n_recorded >= L->record_capacity) continue;
        const int64_t i = L->n_recorded++;
        HIP_TRY(tnmc::launch_observables(L->dJc, L->dSc, L->n_chains, L->dpa, L->dpb, L->n_pairs, L->Lx, L->Ly,
                                         L->Lz, L->d, L->dErec + i * L->n_chains, L->dMrec + i * L->n_chains,
                                         L->dqrec + i * std::max(1, L->n_pairs), s));
      }
    }
  }
  if (stats) {
    HIP_TRY(hipStreamSynchronize(s));
    r = read_counters(n_tasks, stats);
    if (r != TNMC_OK) return r;
    r = finish_timer(tm, stats);
    if (r != TNMC_OK) return r;
  }
  return TNMC_OK;
}

tnmc_status tnmc_sweep_graph(tnmc_lattice* const* lats, int32_t n_lats, int32_t n_sweeps, uint64_t sweep_offset,
                             int32_t record, tnmc_stats* stats, void* stream) {
  CallClock clock(stats);
  if (check_lats(lats, n_lats) != TNMC_OK || n_sweeps < 0) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  hipStream_t s = (hipStream_t)stream;
  WsOrder order(s);
  if (n_sweeps == 0) return TNMC_OK;
  std::vector<Task> tasks;
  for (int p : {0, 1})
    for (Task t : half_sweep_tasks(lats, n_lats, p)) {
      t.key = p;
      tasks.push_back(t);
    }
  Plan plan;
  tnmc_status r = make_plan(tasks, plan);
  if (r != TNMC_OK) return r;
  const size_t n_tasks = plan.desc.size();
  if (grow(g_ws.counters, g_ws.counters_cap, tnmc::kCounterStride * n_tasks) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.tasks, g_ws.tasks_cap, n_tasks) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.graph_state, g_ws.graph_state_cap, (size_t)n_lats + 1) != TNMC_OK) return TNMC_ERR_OOM;
  for (size_t k = 0; k < n_tasks; ++k) plan.desc[k].counters = g_ws.counters + tnmc::kCounterStride * k;
  std::vector<long long> state(n_lats + 1);
  state[0] = (long long)sweep_offset;
  for (int l = 0; l < n_lats; ++l) state[1 + l] = lats[l]->n_recorded;
  // everything the replays read is set up on the caller's stream, outside the graph
  HIP_TRY(hipMemcpyAsync(g_ws.tasks, plan.desc.data(), n_tasks * sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(g_ws.graph_state, state.data(), state.size() * sizeof(long long), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(g_ws.counters, 0, tnmc::kCounterStride * n_tasks * sizeof(long long), s));
  HIP_TRY(hipStreamSynchronize(s));   // plan.desc and state are released on return
  if (!g_ws.capture) HIP_TRY(hipStreamCreateWithFlags(&g_ws.capture, hipStreamNonBlocking));
  // one sweep: the launch pairs of both parities, the observables, and the
  // advance of the device-resident sweep counter and record slots
  auto* sweep_dev = reinterpret_cast<unsigned long long*>(g_ws.graph_state);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct GraphGuard {
    hipGraph_t& g;
    hipGraphExec_t& e;
    ~GraphGuard() {
      if (e) (void)hipGraphExecDestroy(e);
      if (g) (void)hipGraphDestroy(g);
    }
  } guard{graph, exec};
  HIP_TRY(hipStreamBeginCapture(g_ws.capture, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (const auto& g : plan.groups) {
    const TaskDesc* dt = g_ws.tasks + g.first;
    if (e == hipSuccess) e = tnmc::launch_contract(dt, g.count, g.d, g.chi_max, g.precision, contract_cfg(g), g_ws.capture);
    if (e == hipSuccess)
      e = tnmc::launch_sample(dt, g.count, g.d, g.chi_max, g.precision, g.lx_max, g.ly_max, 0, g_ws.capture, sweep_dev);
  }
  if (record) {
    for (int l = 0; l < n_lats && e == hipSuccess; ++l) {
      tnmc_lattice* L = lats[l];
      e = tnmc::launch_observables(L->dJc, L->dSc, L->n_chains, L->dpa, L->dpb, L->n_pairs, L->Lx, L->Ly, L->Lz, L->d,
                                   L->dErec, L->dMrec, L->dqrec, g_ws.capture, g_ws.graph_state + 1 + l,
                                   L->record_capacity);
    }
  }
  if (e == hipSuccess) e = tnmc::launch_graph_advance(sweep_dev, g_ws.graph_state + 1, n_lats, g_ws.capture);
  const hipError_t e_end = hipStreamEndCapture(g_ws.capture, &graph);
  HIP_TRY(e);
  HIP_TRY(e_end);
  HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  for (int t = 0; t < n_sweeps; ++t) HIP_TRY(hipGraphLaunch(exec, s));
  if (record)
    for (int l = 0; l < n_lats; ++l)
      lats[l]->n_recorded = std::min<int64_t>(lats[l]->n_recorded + n_sweeps, lats[l]->record_capacity);
  if (stats) {
    stats->contract_launches += (int64_t)n_sweeps * (int64_t)plan.groups.size();
    stats->sample_launches += (int64_t)n_sweeps * (int64_t)plan.groups.size();
    HIP_TRY(hipStreamSynchronize(s));
    r = read_counters(n_tasks, stats);
    if (r != TNMC_OK) return r;
  }
  return TNMC_OK;
}

tnmc_status tnmc_autotune_now(tnmc_lattice* const* lats, int32_t n_lats, void* stream) {
  if (check_lats(lats, n_lats) != TNMC_OK) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  hipStream_t s = (hipStream_t)stream;
  WsOrder order(s);
  std::vector<Task> tasks;
  for (int p : {0, 1})
    for (Task t : half_sweep_tasks(lats, n_lats, p)) {
      t.key = p;
      tasks.push_back(t);
    }
  Plan plan;
  tnmc_status r = make_plan(tasks, plan);
  if (r != TNMC_OK) return r;
  return autotune_groups(plan, s, true);
}

tnmc_status tnmc_debug_set(int32_t what, int32_t value) {
  if (what < 0 || what > 4) return TNMC_ERR_ARG;
  if (what == 3 ? (value < 0 || value > 15) : (value != 0 && value != 1)) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  if (what == 3) {
    g_rank_cut_exp = value;
  } else if (what == 0) {
    tnmc::set_force_retry(value);
  } else if (what == 4) {
    tnmc::set_force_narrow(value);
  } else if (what == 2) {
    g_nn_pairing = value != 0;
  } else {
    // autotuner off: forget its choices and run the defaults (or the pins)
    g_autotune = value != 0;
    if (!g_autotune) {
      g_tune.clear();
      g_tune_seen.clear();
      g_tune_any = false;
    }
  }
  return TNMC_OK;
}

// The most recent tuned class with this (d, chi bucket, precision), if any.
const TuneResult* find_tuned(int d, int chi, int precision) {
  const int cm = tnmc::chi_bucket(chi);
  const TuneResult* r = nullptr;
  if (g_tune_any && std::get<0>(g_tune_last) == d && std::get<1>(g_tune_last) == cm &&
      std::get<2>(g_tune_last) == precision)
    return &g_tune.at(g_tune_last);
  for (const auto& kv : g_tune)
    if (std::get<0>(kv.first) == d && std::get<1>(kv.first) == cm && std::get<2>(kv.first) == precision)
      r = &kv.second;
  return r;
}

tnmc_status tnmc_layout_choice(int32_t d, int32_t chi, int32_t precision, int32_t* layout, double* ms_compact,
                               double* ms_full) {
  if (!layout || (d != 2 && d != 3) || chi < 1) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  *layout = -1;
  if (ms_compact) *ms_compact = 0.0;
  if (ms_full) *ms_full = 0.0;
  const TuneResult* r = find_tuned(d, chi, precision);
  if (!r || !tnmc::contract_has_compact(d, tnmc::chi_bucket(chi))) return TNMC_OK;
  *layout = r->cfg.full;
  if (ms_compact) *ms_compact = r->ms[r->cfg.mfma][0];
  if (ms_full) *ms_full = r->ms[r->cfg.mfma][1];
  return TNMC_OK;
}

tnmc_status tnmc_autotune_choice(int32_t d, int32_t chi, int32_t precision, int32_t* layout, int32_t* engine,
                                 double* ms) {
  if (!layout || !engine || (d != 2 && d != 3) || chi < 1) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  *layout = -1;
  *engine = -1;
  if (ms)
    for (int i = 0; i < 4; ++i) ms[i] = -1.0;
  const TuneResult* r = find_tuned(d, chi, precision);
  if (!r) return TNMC_OK;
  *layout = r->cfg.full;
  *engine = r->cfg.mfma;
  if (ms)
    for (int e = 0; e < 2; ++e)
      for (int l = 0; l < 2; ++l) ms[2 * e + l] = r->ms[e][l];
  return TNMC_OK;
}

tnmc_status tnmc_autotune_pin(int32_t layout, int32_t engine) {
  if (layout < -1 || layout > 1 || engine < -1 || engine > 1) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  g_pin_layout = layout;
  g_pin_engine = engine;
  g_tune.clear();   // choices made under other pins are dropped
  g_tune_seen.clear();
  g_tune_any = false;
  return TNMC_OK;
}

tnmc_status tnmc_debug_workspace(int32_t what, void* out, int64_t bytes) {
  if (!out || bytes < 0) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  const void* src = nullptr;
  size_t cap = 0;
  switch (what) {
    case 0: src = g_ws.env; cap = g_ws.env_cap * sizeof(double); break;
    case 1: src = g_ws.ints; cap = g_ws.ints_cap * sizeof(int); break;
    case 2: src = g_ws.ints; cap = g_ws.ints_cap * sizeof(int); break;
    case 3: src = g_ws.rscr; cap = g_ws.rscr_cap * sizeof(double); break;
    case 4: src = g_ws.dbl; cap = g_ws.dbl_cap * sizeof(double); break;
    default: return TNMC_ERR_ARG;
  }
  if (!src) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, src, std::min((size_t)bytes, cap), hipMemcpyDeviceToHost));
  return TNMC_OK;
}

tnmc_status tnmc_get_spins(tnmc_lattice* L, int32_t chain, int8_t* out) {
  if (!L || !out || chain < 0 || chain >= L->n_chains) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, L->spins_of(chain), L->sites(), hipMemcpyDeviceToHost));
  return TNMC_OK;
}

tnmc_status tnmc_set_spins(tnmc_lattice* L, int32_t chain, const int8_t* in) {
  if (!L || !in || chain < 0 || chain >= L->n_chains) return TNMC_ERR_ARG;
  for (size_t i = 0; i < L->sites(); ++i) {
    const int v = in[i];
    if (L->d == 2 ? (v != 1 && v != -1) : (v < 0 || v >= L->d)) return TNMC_ERR_ARG;
  }
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(L->spins_of(chain), in, L->sites(), hipMemcpyHostToDevice));
  return TNMC_OK;
}

tnmc_status tnmc_energy(tnmc_lattice* L, int32_t chain, double* E) {
  if (!L || !E || chain < 0 || chain >= L->n_chains) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(tnmc::launch_energy(L->J_of(chain), L->spins_of(chain), L->Lx, L->Ly, L->Lz, L->d, L->dscal, 0));
  HIP_TRY(hipMemcpy(E, L->dscal, sizeof(double), hipMemcpyDeviceToHost));
  return TNMC_OK;
}

tnmc_status tnmc_timeseries(tnmc_lattice* L, double* E, double* M, double* q, int64_t* n) {
  if (!L || !n) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  const int64_t k = L->n_recorded;
  if (E && k) HIP_TRY(hipMemcpy(E, L->dErec, k * L->n_chains * sizeof(double), hipMemcpyDeviceToHost));
  if (M && k) HIP_TRY(hipMemcpy(M, L->dMrec, k * L->n_chains * sizeof(double), hipMemcpyDeviceToHost));
  if (q && k && L->n_pairs > 0)
    HIP_TRY(hipMemcpy(q, L->dqrec, k * L->n_pairs * sizeof(double), hipMemcpyDeviceToHost));
  *n = k;
  return TNMC_OK;
}

tnmc_status tnmc_timeseries_reset(tnmc_lattice* L) {
  if (!L) return TNMC_ERR_ARG;
  L->n_recorded = 0;
  return TNMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ allocation-free proposal
// Static device scratch of the allocation-free entry point: the workspace of
// one slice task (descriptor, environments, R factors, global tile scratch,
// bond dimensions, log scales, record, drawn layer).  Each GPU the library
// runs on holds its own copy for the life of the process.  In host code the
// array's name is only a stand-in: its device address comes from
// hipGetSymbolAddress, once per device.
namespace {

constexpr size_t kStaticScratchBytes = (size_t)24 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch (looked up on the first call on it).
tnmc_status static_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    g_last_error = "device index beyond the static scratch table";
    return TNMC_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      g_last_error = "hipGetSymbolAddress returned no address for the static scratch";
      return TNMC_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TNMC_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

tnmc_status tnmc_slice_propose_static(tnmc_lattice* lat, int32_t chain, int32_t z, uint64_t sweep, int8_t* s_new,
                                      double* logq_new, double* logq_old, double* dE, void* stream) {
  if (!lat || chain < 0 || chain >= lat->n_chains || z < 0 || z >= lat->Lz) return TNMC_ERR_ARG;
  if (!s_new || !logq_new || !logq_old || !dE) return TNMC_ERR_ARG;
  g_last_error.clear();
  const int Lx = lat->Lx, Ly = lat->Ly, d = lat->d, cm = lat->chi_max;
  const size_t plane = (size_t)Lx * Ly;
  // scratch layout, every region on a 256-byte boundary
  const bool glob = tnmc::contract_uses_global(d, cm);
  const size_t o_desc = 0;
  const size_t o_env = o_desc + align256(sizeof(TaskDesc));
  const size_t o_rscr = o_env + align256(tnmc::env_doubles(Lx, Ly, d, cm, lat->precision) * sizeof(double));
  const size_t o_gscr = o_rscr + align256(tnmc::rscr_doubles(Lx, d, cm) * sizeof(double));
  const size_t o_ints = o_gscr + (glob ? align256(tnmc::contract_lds_bytes(d, cm)) : 0);
  const size_t o_dbl = o_ints + align256((plane + 1) * sizeof(int));
  const size_t o_bytes = o_dbl + align256(((size_t)Ly + 5) * sizeof(double));
  const size_t need = o_bytes + align256(plane);
  if (need > kStaticScratchBytes) {
    g_last_error = "tnmc_slice_propose_static: this layer needs " + std::to_string(need) +
                   " bytes of workspace, more than the " + std::to_string(kStaticScratchBytes) +
                   " bytes of static scratch";
    return TNMC_ERR_ARG;
  }
  void* base = nullptr;
  tnmc_status r = static_scratch(&base);
  if (r != TNMC_OK) return r;
  unsigned char* sb = static_cast<unsigned char*>(base);
  TaskDesc t;
  std::memset(&t, 0, sizeof(t));
  t.J = lat->J_of(chain);
  t.spins = lat->spins_of(chain);
  t.env = sb + o_env;
  t.rscr = reinterpret_cast<double*>(sb + o_rscr);
  t.gscr = glob ? reinterpret_cast<double*>(sb + o_gscr) : nullptr;
  t.bond = reinterpret_cast<int*>(sb + o_ints);
  t.status = t.bond + plane;
  t.logscale = reinterpret_cast<double*>(sb + o_dbl);
  t.record = t.logscale + Ly;
  t.s_new_out = reinterpret_cast<int8_t*>(sb + o_bytes);
  t.counters = nullptr;
  t.force_new = nullptr;
  t.beta = lat->beta[chain];
  t.rank_tol = rank_tol_for(lat->precision);
  t.key0 = lat->seed;
  t.key1 = lat->chain_key[chain];
  t.Lx = Lx;
  t.Ly = Ly;
  t.Lz = lat->Lz;
  t.z = z;
  t.chi = lat->chi;
  t.d = d;
  t.chi_max = cm;
  t.write_back = 0;
  hipStream_t s = (hipStream_t)stream;
  TaskDesc* dt = reinterpret_cast<TaskDesc*>(sb + o_desc);
  // the descriptor is copied from this frame: wait for the copy before
  // returning (and before the kernels read it, which stream order gives)
  HIP_TRY(hipMemcpyAsync(dt, &t, sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  {
    tnmc::ContractCfg cfg;   // the pins, else the defaults (a single task is not tuned)
    if (g_pin_layout >= 0) cfg.full = g_pin_layout;
    if (g_pin_engine >= 0) cfg.mfma = g_pin_engine;
    HIP_TRY(tnmc::launch_contract(dt, 1, d, cm, lat->precision, cfg, s));
  }
  HIP_TRY(tnmc::launch_sample(dt, 1, d, cm, lat->precision, Lx, Ly, sweep, s));
  double rec[5];
  HIP_TRY(hipMemcpyAsync(s_new, t.s_new_out, plane, hipMemcpyDefault, s));   // host or device
  HIP_TRY(hipMemcpyAsync(rec, t.record, sizeof(rec), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *logq_new = rec[0];
  *logq_old = rec[1];
  *dE = rec[2];
  if (rec[4] != 0.0 || !std::isfinite(rec[0]) || !std::isfinite(rec[1])) {
    g_last_error = "numeric fault bits " + std::to_string((int)rec[4]) +
                   " (1-2: new path, 4-8: current path, 16-64: contraction)";
    return TNMC_ERR_NUMERIC;
  }
  return TNMC_OK;
}

tnmc_status tnmc_flop_model(int32_t Lx, int32_t Ly, int32_t d, int32_t chi, double* contract_flops,
                            double* sample_flops) {
  if (Lx < 1 || Ly < 1 || (d != 2 && d != 3) || chi < 1) return TNMC_ERR_ARG;
  // bond dimensions of the environments: exact caps min(d^(x+1), d^(Lx-1-x), chi)
  auto cap = [&](int x) -> double {   // right bond of site x (x < Lx-1)
    double a = 1.0, b = 1.0;
    for (int i = 0; i <= x && a < 1e9; ++i) a *= d;
    for (int i = 0; i < Lx - 1 - x && b < 1e9; ++i) b *= d;
    return std::min<double>(std::min(a, b), chi);
  };
  double total = 0.0;
  // rows below the top: E_{Ly-2} is built from the trivial E_{Ly-1} (bonds 1),
  // every other row from a chi-capped environment
  for (int y = Ly - 1; y >= 1; --y) {
    const bool trivial = (y == Ly - 1);
    auto bnd = [&](int x) -> double { return (x < 0 || x >= Lx - 1 || trivial) ? 1.0 : cap(x); };
    // left sweep
    double rR = 1.0;
    std::vector<double> rrows(Lx, 1.0);
    for (int x = 0; x < Lx - 1; ++x) {
      const double cl = bnd(x - 1), cr = bnd(x);
      const double m = rR * d, n = cr * d;
      total += 2.0 * rR * d * cr * cl;   // M = G (R~ A)
      total += qr_flops(m, n);
      rR = std::min(m, n);
      rrows[x] = rR;
    }
    // right sweep
    double k = 1.0;
    for (int x = Lx - 1; x >= 1; --x) {
      const double cl = bnd(x - 1), cr = bnd(x);
      const double rr = rrows[x - 1];
      const double nC = d * k;
      total += 2.0 * d * cl * cr * k;            // AT
      total += 2.0 * rr * d * cl * k;            // Z
      total += 2.0 * rr * d * d * k;             // C
      if (rr > nC) total += qr_flops(rr, nC);    // C is tall: QR first
      total += svd_flops(std::min(rr, nC), nC);
      const double kx = std::min<double>(chi, std::min(rr, nC));
      total += 2.0 * kx * d * d * k;             // V~
      total += 2.0 * cl * d * kx * k;            // Y
      total += 2.0 * cl * d * d * kx;            // T
      k = kx;
    }
  }
  if (contract_flops) *contract_flops = total;
  total = 0.0;
  // sampling: two paths, right environments and draws over every row
  for (int y = 0; y < Ly; ++y) {
    for (int x = 0; x < Lx; ++x) {
      const double cl = (x > 0 && y < Ly - 1) ? cap(x - 1) : 1.0;
      const double cr = (x < Lx - 1 && y < Ly - 1) ? cap(x) : 1.0;
      total += 2.0 * (2.0 * d * cl * cr + 2.0 * d * cl * cr);
    }
  }
  if (sample_flops) *sample_flops = total;
  return TNMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ learned proposal

struct tnmc_nn {
  float* theta = nullptr;   // FP32 master parameters, the flat layout of include/tnmc.h
  uint16_t* wbf = nullptr;  // their BF16 roundings, which every evaluation of the network uses
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* grad = nullptr;
  int64_t step = 0;         // Adam steps taken
  // batch buffers (grow-only)
  size_t cap_elems = 0;     // n * Ly * Lx of the buffers below
  float* act = nullptr;     // 5 * 32 * elems
  float* gbuf = nullptr;    // 2 * 32 * elems
  float* logit = nullptr;   // elems
  float* glogit = nullptr;  // elems
  double* logq = nullptr;   // n
  size_t cap_n = 0;
  float* part = nullptr;    // kNnWeightParts * (32*32*9 + 32)
};

namespace {

// Normal deviates for the default initialisation (splitmix64 + Box-Muller).
struct InitRng {
  uint64_t x;
  uint64_t next() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((double)(next() >> 11) + 0.5) * 0x1p-53; }
  double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(6.283185307179586 * uniform()); }
};

tnmc_status nn_batch(tnmc_nn* nn, const float* cond, const int8_t* s, int n, int Lx, int Ly, tnmc::NnBatch& B) {
  const size_t elems = (size_t)n * Lx * Ly;
  if (elems > nn->cap_elems) {
    HIP_TRY(hipDeviceSynchronize());
    float* bufs[] = {nn->act, nn->gbuf, nn->logit, nn->glogit};
    for (float* p : bufs)
      if (p) HIP_TRY(hipFree(p));
    nn->act = nn->gbuf = nn->logit = nn->glogit = nullptr;
    nn->cap_elems = 0;
    HIP_TRY(hipMalloc((void**)&nn->act, 5 * tnmc::kNnChannels * elems * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&nn->gbuf, 2 * tnmc::kNnChannels * elems * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&nn->logit, elems * sizeof(float)));
    HIP_TRY(hipMalloc((void**)&nn->glogit, elems * sizeof(float)));
    nn->cap_elems = elems;
  }
  if ((size_t)n > nn->cap_n) {
    HIP_TRY(hipDeviceSynchronize());
    if (nn->logq) HIP_TRY(hipFree(nn->logq));
    nn->logq = nullptr;
    HIP_TRY(hipMalloc((void**)&nn->logq, (size_t)n * sizeof(double)));
    nn->cap_n = n;
  }
  if (!nn->part)
    HIP_TRY(hipMalloc((void**)&nn->part, (size_t)tnmc::kNnWeightParts * (32 * 32 * 9 + 32) * sizeof(float)));
  B.n = n;
  B.Lx = Lx;
  B.Ly = Ly;
  B.cond = cond;
  B.s = s;
  for (int l = 0; l < 5; ++l) B.act[l] = nn->act + (size_t)l * tnmc::kNnChannels * elems;
  B.g[0] = nn->gbuf;
  B.g[1] = nn->gbuf + (size_t)tnmc::kNnChannels * elems;
  B.logit = nn->logit;
  B.glogit = nn->glogit;
  B.logq = nn->logq;
  B.part = nn->part;
  return TNMC_OK;
}

constexpr size_t kNnStaticLds = 64;   // the sampler's static LDS (log q and fault slots), rounded up

bool nn_shape_ok(int n, int Lx, int Ly) {
  return n >= 1 && Lx >= 1 && Ly >= 1 && Lx <= tnmc::kNnLxMax && Ly <= kLyMax;
}

// The learned proposal runs on Ising lattices whose sampler fits in a CU's LDS.
tnmc_status nn_lattice_ok(const tnmc_lattice* L) {
  if (L->d != 2) return TNMC_ERR_UNSUPPORTED;
  if (tnmc::nn_sample_lds_bytes(L->Lx, L->Ly) + kNnStaticLds > 160 * 1024) return TNMC_ERR_UNSUPPORTED;
  return TNMC_OK;
}

tnmc_status nn_counters(tnmc_lattice* L) {
  if (L->dnncnt) return TNMC_OK;
  const size_t n = (size_t)L->n_chains * L->Lz * tnmc::kCounterStride;
  HIP_TRY(hipMalloc((void**)&L->dnncnt, n * sizeof(long long)));
  HIP_TRY(hipMemset(L->dnncnt, 0, n * sizeof(long long)));
  L->nn_fallback.assign((size_t)L->n_chains * L->Lz, 0);
  return TNMC_OK;
}

TaskDesc nn_task(tnmc_lattice* L, int chain, int z) {
  TaskDesc t;
  std::memset(&t, 0, sizeof(t));
  t.J = L->J_of(chain);
  t.spins = L->spins_of(chain);
  t.beta = L->beta[chain];
  t.key0 = L->seed;
  t.key1 = L->chain_key[chain];
  t.Lx = L->Lx;
  t.Ly = L->Ly;
  t.Lz = L->Lz;
  t.z = z;
  t.d = L->d;
  t.chi = L->chi;
  t.chi_max = L->chi_max;
  t.write_back = 1;
  return t;
}

tnmc_status nn_single(tnmc_lattice* lat, tnmc_nn* nn, int chain, int z, uint64_t sweep, const int8_t* force_in,
                      int8_t* s_new_out, double* rec_host, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_ws.mu);
  WsOrder order(s);
  g_last_error.clear();
  const size_t plane = (size_t)lat->Lx * lat->Ly;
  if (grow(g_ws.bytes, g_ws.bytes_cap, 2 * plane) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.nn_tasks, g_ws.nn_tasks_cap, (size_t)1) != TNMC_OK) return TNMC_ERR_OOM;
  if (grow(g_ws.dbl, g_ws.dbl_cap, (size_t)8) != TNMC_OK) return TNMC_ERR_OOM;
  TaskDesc t = nn_task(lat, chain, z);
  t.record = g_ws.dbl;
  t.write_back = 0;
  t.s_new_out = g_ws.bytes;
  if (force_in) {
    HIP_TRY(hipMemcpyAsync(g_ws.bytes + plane, force_in, plane, hipMemcpyDefault, s));   // host or device
    t.force_new = g_ws.bytes + plane;
  }
  HIP_TRY(hipMemcpyAsync(g_ws.nn_tasks, &t, sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // the host copies above are released on return
  HIP_TRY(tnmc::launch_nn_sample(g_ws.nn_tasks, 1, nn->wbf, lat->Lx, lat->Ly, sweep, s));
  if (s_new_out) HIP_TRY(hipMemcpyAsync(s_new_out, g_ws.bytes, plane, hipMemcpyDefault, s));   // host or device
  HIP_TRY(hipMemcpyAsync(rec_host, g_ws.dbl, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return TNMC_OK;
}

}  // namespace

extern "C" {

tnmc_status tnmc_nn_create(const float* params, uint64_t seed, tnmc_nn** out) {
  if (!out) return TNMC_ERR_ARG;
  std::vector<float> h(tnmc::kNnParams);
  if (params) {
    std::memcpy(h.data(), params, h.size() * sizeof(float));
  } else {
    // W ~ N(0, 2 / (9 c_in)), b = 0
    InitRng rng{seed};
    const int cin[6] = {5, 32, 32, 32, 32, 32}, cout[6] = {32, 32, 32, 32, 32, 1};
    size_t o = 0;
    for (int l = 0; l < 6; ++l) {
      const double sd = std::sqrt(2.0 / (9.0 * cin[l]));
      for (int i = 0; i < cout[l] * cin[l] * 9; ++i) h[o++] = (float)(sd * rng.normal());
      for (int i = 0; i < cout[l]; ++i) h[o++] = 0.0f;
    }
  }
  for (float x : h)
    if (!std::isfinite(x)) return TNMC_ERR_ARG;
  auto* nn = new tnmc_nn();
  auto fail = [&](hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    tnmc_nn_free(nn);
    return e == hipErrorOutOfMemory ? TNMC_ERR_OOM : TNMC_ERR_DEVICE;
  };
  const size_t bytes = tnmc::kNnParams * sizeof(float);
  float** bufs[] = {&nn->theta, &nn->m, &nn->v, &nn->grad};
  for (float** b : bufs) {
    hipError_t e = hipMalloc((void**)b, bytes);
    if (e != hipSuccess) return fail(e, "hipMalloc");
    e = hipMemset(*b, 0, bytes);
    if (e != hipSuccess) return fail(e, "hipMemset");
  }
  hipError_t e = hipMalloc((void**)&nn->wbf, tnmc::kNnParams * sizeof(uint16_t));
  if (e != hipSuccess) return fail(e, "hipMalloc");
  e = hipMemcpy(nn->theta, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(e, "hipMemcpy");
  e = tnmc::nn_round_bf16(nn->theta, nn->wbf, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail(e, "BF16 parameters");
  *out = nn;
  return TNMC_OK;
}

tnmc_status tnmc_nn_free(tnmc_nn* nn) {
  if (!nn) return TNMC_ERR_ARG;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {nn->theta, nn->wbf, nn->m, nn->v, nn->grad, nn->act, nn->gbuf, nn->logit, nn->glogit, nn->logq, nn->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete nn;
  return TNMC_OK;
}

tnmc_status tnmc_nn_get_params(tnmc_nn* nn, float* out) {
  if (!nn || !out) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, nn->theta, tnmc::kNnParams * sizeof(float), hipMemcpyDeviceToHost));
  return TNMC_OK;
}

tnmc_status tnmc_nn_set_params(tnmc_nn* nn, const float* in) {
  if (!nn || !in) return TNMC_ERR_ARG;
  for (int i = 0; i < tnmc::kNnParams; ++i)
    if (!std::isfinite(in[i])) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(nn->theta, in, tnmc::kNnParams * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(tnmc::nn_round_bf16(nn->theta, nn->wbf, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemset(nn->m, 0, tnmc::kNnParams * sizeof(float)));
  HIP_TRY(hipMemset(nn->v, 0, tnmc::kNnParams * sizeof(float)));
  nn->step = 0;
  return TNMC_OK;
}

tnmc_status tnmc_nn_logq(tnmc_nn* nn, const float* cond, const int8_t* s, int32_t n, int32_t Lx, int32_t Ly,
                         double* logq, void* stream) {
  if (!nn || !cond || !s || !logq || !nn_shape_ok(n, Lx, Ly)) return TNMC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  tnmc::NnBatch B;
  tnmc_status r = nn_batch(nn, cond, s, n, Lx, Ly, B);
  if (r != TNMC_OK) return r;
  HIP_TRY(tnmc::nn_forward(B, nn->wbf, st));
  HIP_TRY(hipMemcpyAsync(logq, B.logq, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st));
  return TNMC_OK;
}

tnmc_status tnmc_nn_loss_grad(tnmc_nn* nn, const float* cond, const int8_t* s, int32_t n, int32_t Lx, int32_t Ly,
                              double* loss, float* grad, void* stream) {
  if (!nn || !cond || !s || !loss || !nn_shape_ok(n, Lx, Ly)) return TNMC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  tnmc::NnBatch B;
  tnmc_status r = nn_batch(nn, cond, s, n, Lx, Ly, B);
  if (r != TNMC_OK) return r;
  HIP_TRY(tnmc::nn_forward(B, nn->wbf, st));
  HIP_TRY(tnmc::nn_backward(B, nn->wbf, nn->grad, st));
  if (grad) HIP_TRY(hipMemcpyAsync(grad, nn->grad, tnmc::kNnParams * sizeof(float), hipMemcpyDeviceToDevice, st));
  std::vector<double> lq(n);
  HIP_TRY(hipMemcpyAsync(lq.data(), B.logq, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double acc = 0.0;
  for (double v : lq) acc -= v;
  *loss = acc / n;
  return std::isfinite(*loss) ? TNMC_OK : TNMC_ERR_NUMERIC;
}

tnmc_status tnmc_nn_adam_step(tnmc_nn* nn, const float* grad, double lr, void* stream) {
  if (!nn || !grad || !(lr > 0.0) || !std::isfinite(lr)) return TNMC_ERR_ARG;
  nn->step += 1;
  HIP_TRY(tnmc::nn_adam(nn->theta, nn->wbf, nn->m, nn->v, grad, nn->step, lr, (hipStream_t)stream));
  return TNMC_OK;
}

tnmc_status tnmc_nn_train(tnmc_nn* nn, const float* cond, const int8_t* s, int64_t n, int32_t Lx, int32_t Ly,
                          int32_t epochs, int32_t batch, double lr, double* last_loss, void* stream) {
  if (!nn || !cond || !s || n < 1 || epochs < 0 || batch < 1 || !(lr > 0.0) || !std::isfinite(lr)) return TNMC_ERR_ARG;
  if (!nn_shape_ok(batch, Lx, Ly)) return TNMC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const size_t plane = (size_t)Lx * Ly;
  tnmc::NnBatch B;
  int last_n = 0;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; i += batch) {
      const int bn = (int)std::min<int64_t>(batch, n - i);
      tnmc_status r = nn_batch(nn, cond + (size_t)i * tnmc::kNnCond * plane, s + (size_t)i * plane, bn, Lx, Ly, B);
      if (r != TNMC_OK) return r;
      HIP_TRY(tnmc::nn_forward(B, nn->wbf, st));
      HIP_TRY(tnmc::nn_backward(B, nn->wbf, nn->grad, st));
      nn->step += 1;
      HIP_TRY(tnmc::nn_adam(nn->theta, nn->wbf, nn->m, nn->v, nn->grad, nn->step, lr, st));
      last_n = bn;
    }
  }
  if (last_loss) {
    *last_loss = std::nan("");
    if (last_n > 0) {
      std::vector<double> lq(last_n);
      HIP_TRY(hipMemcpyAsync(lq.data(), nn->logq, (size_t)last_n * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double acc = 0.0;
      for (double v : lq) acc -= v;
      *last_loss = acc / last_n;
      if (!std::isfinite(*last_loss)) return TNMC_ERR_NUMERIC;
    }
  }
  return TNMC_OK;
}

tnmc_status tnmc_nn_dataset(tnmc_lattice* lat, float* cond, int8_t* s, void* stream) {
  if (!lat || !cond || !s) return TNMC_ERR_ARG;
  if (lat->d != 2) return TNMC_ERR_UNSUPPORTED;
  HIP_TRY(tnmc::launch_nn_dataset(lat->dJc, lat->dSc, lat->n_chains, lat->Lx, lat->Ly, lat->Lz, cond, s,
                                  (hipStream_t)stream));
  return TNMC_OK;
}

tnmc_status tnmc_nn_slice_propose(tnmc_lattice* lat, tnmc_nn* nn, int32_t chain, int32_t z, uint64_t sweep,
                                  int8_t* s_new, double* logq_new, double* logq_old, double* dE, void* stream) {
  if (!lat || !nn || chain < 0 || chain >= lat->n_chains || z < 0 || z >= lat->Lz) return TNMC_ERR_ARG;
  if (!s_new || !logq_new || !logq_old || !dE) return TNMC_ERR_ARG;
  tnmc_status r = nn_lattice_ok(lat);
  if (r != TNMC_OK) return r;
  double rec[5];
  r = nn_single(lat, nn, chain, z, sweep, nullptr, s_new, rec, (hipStream_t)stream);
  if (r != TNMC_OK) return r;
  *logq_new = rec[0];
  *logq_old = rec[1];
  *dE = rec[2];
  if (rec[4] != 0.0 || !std::isfinite(rec[0]) || !std::isfinite(rec[1])) {
    g_last_error = "non-finite logit (fault bits " + std::to_string((int)rec[4]) + ")";
    return TNMC_ERR_NUMERIC;
  }
  return TNMC_OK;
}

tnmc_status tnmc_nn_slice_logq(tnmc_lattice* lat, tnmc_nn* nn, int32_t chain, int32_t z, const int8_t* s,
                               double* logq, void* stream) {
  if (!lat || !nn || chain < 0 || chain >= lat->n_chains || z < 0 || z >= lat->Lz || !s || !logq)
    return TNMC_ERR_ARG;
  tnmc_status r = nn_lattice_ok(lat);
  if (r != TNMC_OK) return r;
  const size_t plane = (size_t)lat->Lx * lat->Ly;
  for (size_t i = 0; i < plane; ++i)
    if (s[i] != 1 && s[i] != -1) return TNMC_ERR_ARG;
  double rec[5];
  r = nn_single(lat, nn, chain, z, 0, s, nullptr, rec, (hipStream_t)stream);
  if (r != TNMC_OK) return r;
  *logq = rec[0];
  return std::isfinite(rec[0]) && rec[4] == 0.0 ? TNMC_OK : TNMC_ERR_NUMERIC;
}

tnmc_status tnmc_nn_sweep(tnmc_lattice* const* lats, int32_t n_lats, tnmc_nn* nn, int32_t n_sweeps,
                          uint64_t sweep_offset, int32_t record, int32_t time_kernels, tnmc_stats* stats,
                          void* stream) {
  CallClock clock(stats);
  if (check_lats(lats, n_lats) != TNMC_OK || !nn || n_sweeps < 0) return TNMC_ERR_ARG;
  for (int l = 0; l < n_lats; ++l) {
    tnmc_status r = nn_lattice_ok(lats[l]);
    if (r != TNMC_OK) return r;
  }
  std::lock_guard<std::mutex> lk(g_ws.mu);
  hipStream_t s = (hipStream_t)stream;
  WsOrder order(s);
  for (int l = 0; l < n_lats; ++l) {
    tnmc_status r = nn_counters(lats[l]);
    if (r != TNMC_OK) return r;
  }
  // learned-proposal tasks per parity, and the layers frozen to the TN proposal
  std::vector<TaskDesc> nd[2];
  int lxm[2] = {1, 1}, lym[2] = {1, 1};
  std::vector<Task> tn_tasks;
  for (int p : {0, 1})
    for (Task t : half_sweep_tasks(lats, n_lats, p)) {
      tnmc_lattice* L = t.lat;
      const size_t slot = (size_t)t.chain * L->Lz + t.z;
      if (L->nn_fallback[slot]) {
        t.key = p;
        tn_tasks.push_back(t);
      } else {
        TaskDesc d = nn_task(L, t.chain, t.z);
        d.counters = L->dnncnt + tnmc::kCounterStride * slot;
        nd[p].push_back(d);
        lxm[p] = std::max(lxm[p], L->Lx);
        lym[p] = std::max(lym[p], L->Ly);
      }
    }
  for (int p : {0, 1})   // lattices of different shapes share one launch per parity
    if (!nd[p].empty() && tnmc::nn_sample_lds_bytes(lxm[p], lym[p]) + kNnStaticLds > 160 * 1024)
      return TNMC_ERR_UNSUPPORTED;
  // Two tasks per workgroup share the weights in LDS, which halves the rounds
  // of a launch with more tasks than CUs; only where every task of the
  // launch has one layer shape (both halves of a workgroup then pass the
  // same barriers) and their count is even.
  bool paired[2] = {false, false};
  for (int p : {0, 1}) {
    bool one_shape = true;
    for (const auto& d : nd[p]) one_shape = one_shape && d.Lx == nd[p][0].Lx && d.Ly == nd[p][0].Ly;
    paired[p] = g_nn_pairing && one_shape && nd[p].size() > 256 && nd[p].size() % 2 == 0 &&
                tnmc::nn_sample_lds_bytes(lxm[p], lym[p], 2) + kNnStaticLds <= 160 * 1024;
  }
  const size_t n_nn = nd[0].size() + nd[1].size();
  if (grow(g_ws.nn_tasks, g_ws.nn_tasks_cap, std::max<size_t>(n_nn, 1)) != TNMC_OK) return TNMC_ERR_OOM;
  if (!nd[0].empty())
    HIP_TRY(hipMemcpyAsync(g_ws.nn_tasks, nd[0].data(), nd[0].size() * sizeof(TaskDesc), hipMemcpyHostToDevice, s));
  if (!nd[1].empty())
    HIP_TRY(hipMemcpyAsync(g_ws.nn_tasks + nd[0].size(), nd[1].data(), nd[1].size() * sizeof(TaskDesc),
                           hipMemcpyHostToDevice, s));
  Plan plan;
  size_t n_tn = 0;
  if (!tn_tasks.empty()) {
    tnmc_status r = make_plan(tn_tasks, plan);
    if (r != TNMC_OK) return r;
    n_tn = plan.desc.size();
    if (grow(g_ws.tasks, g_ws.tasks_cap, n_tn) != TNMC_OK) return TNMC_ERR_OOM;
    HIP_TRY(hipMemcpyAsync(g_ws.tasks, plan.desc.data(), n_tn * sizeof(TaskDesc), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(g_ws.counters, 0, tnmc::kCounterStride * n_tn * sizeof(long long), s));
  }
  // counts before the sweeps, to report this call's proposals
  std::vector<std::vector<long long>> before(n_lats);
  if (stats) {
    for (int l = 0; l < n_lats; ++l) {
      before[l].resize((size_t)lats[l]->n_chains * lats[l]->Lz * tnmc::kCounterStride);
      HIP_TRY(hipMemcpyAsync(before[l].data(), lats[l]->dnncnt, before[l].size() * sizeof(long long),
                             hipMemcpyDeviceToHost, s));
    }
  }
  HIP_TRY(hipStreamSynchronize(s));   // host descriptors are released on return
  Timer tm;
  tm.on = (time_kernels != 0 && stats != nullptr);
  for (int t = 0; t < n_sweeps; ++t) {
    const uint64_t sw = sweep_offset + (uint64_t)t;
    for (int p : {0, 1}) {
      if (!nd[p].empty()) {
        if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
        HIP_TRY(tnmc::launch_nn_sample(g_ws.nn_tasks + (p ? nd[0].size() : 0), (int)nd[p].size(), nn->wbf, lxm[p],
                                       lym[p], sw, s, paired[p]));
        if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
        if (stats) stats->sample_launches += 1;
      }
      for (const auto& g : plan.groups) {
        if (g.key != p) continue;
        const TaskDesc* dt = g_ws.tasks + g.first;
        if (tm.on && tm.mark(tm.c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
        HIP_TRY(tnmc::launch_contract(dt, g.count, g.d, g.chi_max, g.precision, contract_cfg(g), s));
        if (tm.on && tm.mark(tm.c_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
        if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
        HIP_TRY(tnmc::launch_sample(dt, g.count, g.d, g.chi_max, g.precision, g.lx_max, g.ly_max, sw, s));
        if (tm.on && tm.mark(tm.s_ev, s) != TNMC_OK) return TNMC_ERR_DEVICE;
        if (stats) {
          stats->contract_launches += 1;
          stats->sample_launches += 1;
        }
      }
    }
    if (record) {
      for (int l = 0; l < n_lats; ++l) {
        tnmc_lattice* L = lats[l];
        if (L->n_recorded >= L->record_capacity) continue;
        const int64_t i = L->n_recorded++;
        HIP_TRY(tnmc::launch_observables(L->dJc, L->dSc, L->n_chains, L->dpa, L->dpb, L->n_pairs, L->Lx, L->Ly,
                                         L->Lz, L->d, L->dErec + i * L->n_chains, L->dMrec + i * L->n_chains,
                                         L->dqrec + i * std::max(1, L->n_pairs), s));
      }
    }
  }
  if (stats) stats->nn_fallbacks += (int64_t)tn_tasks.size() * n_sweeps;
  if (stats) {
    HIP_TRY(hipStreamSynchronize(s));
    for (int l = 0; l < n_lats; ++l) {
      std::vector<long long> after(before[l].size());
      HIP_TRY(hipMemcpy(after.data(), lats[l]->dnncnt, after.size() * sizeof(long long), hipMemcpyDeviceToHost));
      for (size_t k = 0; k < after.size(); k += tnmc::kCounterStride) {
        stats->proposed += after[k] - before[l][k];
        stats->accepted += after[k + 1] - before[l][k + 1];
        stats->numeric_faults += after[k + 2] - before[l][k + 2];
      }
    }
    if (n_tn) {
      tnmc_status r = read_counters(n_tn, stats);
      if (r != TNMC_OK) return r;
    }
    tnmc_status r = finish_timer(tm, stats);
    if (r != TNMC_OK) return r;
  }
  return TNMC_OK;
}

tnmc_status tnmc_nn_counts(tnmc_lattice* lat, int64_t* proposed, int64_t* accepted) {
  if (!lat) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  tnmc_status r = nn_counters(lat);
  if (r != TNMC_OK) return r;
  const size_t n = (size_t)lat->n_chains * lat->Lz;
  std::vector<long long> c(n * tnmc::kCounterStride);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(c.data(), lat->dnncnt, c.size() * sizeof(long long), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < n; ++i) {
    if (proposed) proposed[i] = c[i * tnmc::kCounterStride];
    if (accepted) accepted[i] = c[i * tnmc::kCounterStride + 1];
  }
  return TNMC_OK;
}

tnmc_status tnmc_nn_counts_reset(tnmc_lattice* lat) {
  if (!lat) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  tnmc_status r = nn_counters(lat);
  if (r != TNMC_OK) return r;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemset(lat->dnncnt, 0, (size_t)lat->n_chains * lat->Lz * tnmc::kCounterStride * sizeof(long long)));
  return TNMC_OK;
}

tnmc_status tnmc_nn_set_fallback(tnmc_lattice* lat, const int8_t* flags) {
  if (!lat) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  tnmc_status r = nn_counters(lat);
  if (r != TNMC_OK) return r;
  const size_t n = (size_t)lat->n_chains * lat->Lz;
  if (flags) {
    for (size_t i = 0; i < n; ++i)
      if (flags[i] != 0 && flags[i] != 1) return TNMC_ERR_ARG;
    lat->nn_fallback.assign(flags, flags + n);
  } else {
    lat->nn_fallback.assign(n, 0);
  }
  return TNMC_OK;
}

tnmc_status tnmc_nn_get_fallback(tnmc_lattice* lat, int8_t* flags) {
  if (!lat || !flags) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  tnmc_status r = nn_counters(lat);
  if (r != TNMC_OK) return r;
  std::memcpy(flags, lat->nn_fallback.data(), lat->nn_fallback.size());
  return TNMC_OK;
}

tnmc_status tnmc_nn_calibrate_fallback(tnmc_lattice* lat, double threshold, int32_t* n_fallback) {
  if (!lat || !(threshold >= 0.0) || !(threshold <= 1.0)) return TNMC_ERR_ARG;
  const size_t n = (size_t)lat->n_chains * lat->Lz;
  std::vector<int64_t> prop(n), acc(n);
  tnmc_status r = tnmc_nn_counts(lat, prop.data(), acc.data());
  if (r != TNMC_OK) return r;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  int cnt = 0;
  for (size_t i = 0; i < n; ++i) {
    // a layer never proposed keeps its current kernel
    if (prop[i] > 0) lat->nn_fallback[i] = ((double)acc[i] < threshold * (double)prop[i]) ? 1 : 0;
    cnt += lat->nn_fallback[i];
  }
  if (n_fallback) *n_fallback = cnt;
  return TNMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ checkpoints

namespace {

constexpr char kCkptMagic[8] = {'T', 'N', 'M', 'C', 'C', 'K', 'P', '1'};

struct CkptHeader {
  char magic[8];
  int32_t Lx, Ly, Lz, d, chi, precision, n_chains, n_instances, n_pairs, record_capacity;
  uint64_t seed, J_hash, next_sweep;
  int64_t n_recorded;
  int32_t has_nn, pad;
};

struct File {
  FILE* f = nullptr;
  ~File() {
    if (f) fclose(f);
  }
};

tnmc_status io_fail(const std::string& what) {
  g_last_error = what;
  return TNMC_ERR_IO;
}

}  // namespace

extern "C" {

tnmc_status tnmc_get_couplings(tnmc_lattice* L, float* out) {
  if (!L || !out) return TNMC_ERR_ARG;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(out, L->dJ, (size_t)L->n_instances * 3 * L->sites() * sizeof(float), hipMemcpyDeviceToHost));
  return TNMC_OK;
}

tnmc_status tnmc_checkpoint_save(tnmc_lattice* L, uint64_t next_sweep, const char* path) {
  if (!L || !path) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  HIP_TRY(hipDeviceSynchronize());
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kCkptMagic, 8);
  h.Lx = L->Lx; h.Ly = L->Ly; h.Lz = L->Lz; h.d = L->d; h.chi = L->chi; h.precision = L->precision;
  h.n_chains = L->n_chains; h.n_instances = L->n_instances; h.n_pairs = L->n_pairs;
  h.record_capacity = L->record_capacity;
  h.seed = L->seed; h.J_hash = L->J_hash; h.next_sweep = next_sweep; h.n_recorded = L->n_recorded;
  h.has_nn = L->dnncnt ? 1 : 0;
  const size_t nc = L->n_chains, k = (size_t)L->n_recorded, np = L->n_pairs;
  std::vector<double> E(k * nc), M(k * nc), q(k * np);
  std::vector<int8_t> spins(nc * L->sites());
  if (k) {
    HIP_TRY(hipMemcpy(E.data(), L->dErec, E.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(M.data(), L->dMrec, M.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (np) HIP_TRY(hipMemcpy(q.data(), L->dqrec, q.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  HIP_TRY(hipMemcpy(spins.data(), L->dspins, spins.size(), hipMemcpyDeviceToHost));
  std::vector<long long> cnt;
  if (h.has_nn) {
    cnt.resize(nc * L->Lz * tnmc::kCounterStride);
    HIP_TRY(hipMemcpy(cnt.data(), L->dnncnt, cnt.size() * sizeof(long long), hipMemcpyDeviceToHost));
  }
  File f;
  f.f = fopen(path, "wb");
  if (!f.f) return io_fail(std::string("cannot open ") + path + " for writing");
  bool ok = fwrite(&h, sizeof(h), 1, f.f) == 1;
  ok = ok && fwrite(L->chain_key.data(), sizeof(uint64_t), nc, f.f) == nc;
  ok = ok && fwrite(L->beta.data(), sizeof(double), nc, f.f) == nc;
  ok = ok && fwrite(L->chain_instance.data(), sizeof(int), nc, f.f) == nc;
  ok = ok && (np == 0 || fwrite(L->pairs.data(), sizeof(int), 2 * np, f.f) == 2 * np);
  ok = ok && (k == 0 || fwrite(E.data(), sizeof(double), E.size(), f.f) == E.size());
  ok = ok && (k == 0 || fwrite(M.data(), sizeof(double), M.size(), f.f) == M.size());
  ok = ok && (k * np == 0 || fwrite(q.data(), sizeof(double), q.size(), f.f) == q.size());
  ok = ok && fwrite(spins.data(), 1, spins.size(), f.f) == spins.size();
  if (h.has_nn) {
    ok = ok && fwrite(L->nn_fallback.data(), 1, L->nn_fallback.size(), f.f) == L->nn_fallback.size();
    ok = ok && fwrite(cnt.data(), sizeof(long long), cnt.size(), f.f) == cnt.size();
  }
  ok = ok && fflush(f.f) == 0;
  if (!ok) return io_fail(std::string("short write to ") + path);
  return TNMC_OK;
}

tnmc_status tnmc_checkpoint_load(tnmc_lattice* L, const char* path, uint64_t* next_sweep) {
  if (!L || !path) return TNMC_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_ws.mu);
  File f;
  f.f = fopen(path, "rb");
  if (!f.f) return io_fail(std::string("cannot open ") + path);
  CkptHeader h;
  if (fread(&h, sizeof(h), 1, f.f) != 1 || std::memcmp(h.magic, kCkptMagic, 8) != 0)
    return io_fail(std::string(path) + " is not a checkpoint");
  if (h.Lx != L->Lx || h.Ly != L->Ly || h.Lz != L->Lz || h.d != L->d || h.chi != L->chi ||
      h.precision != L->precision || h.n_chains != L->n_chains || h.n_instances != L->n_instances ||
      h.n_pairs != L->n_pairs || h.seed != L->seed || h.J_hash != L->J_hash)
    return io_fail("checkpoint belongs to another lattice (shape, chi, precision, chains, seed or couplings differ)");
  if (h.n_recorded < 0 || h.n_recorded > L->record_capacity)
    return io_fail("checkpoint holds more recorded sweeps than this lattice's record capacity");
  const size_t nc = L->n_chains, k = (size_t)h.n_recorded, np = L->n_pairs;
  std::vector<uint64_t> keys(nc);
  std::vector<double> beta(nc), E(k * nc), M(k * nc), q(k * np);
  std::vector<int> inst(nc), pairs(2 * np);
  std::vector<int8_t> spins(nc * L->sites());
  bool ok = fread(keys.data(), sizeof(uint64_t), nc, f.f) == nc;
  ok = ok && fread(beta.data(), sizeof(double), nc, f.f) == nc;
  ok = ok && fread(inst.data(), sizeof(int), nc, f.f) == nc;
  ok = ok && (np == 0 || fread(pairs.data(), sizeof(int), 2 * np, f.f) == 2 * np);
  if (!ok || keys != L->chain_key || beta != L->beta || inst != L->chain_instance || pairs != L->pairs)
    return io_fail("checkpoint belongs to another lattice (chain keys, betas, instances or pairs differ)");
  ok = (k == 0 || fread(E.data(), sizeof(double), E.size(), f.f) == E.size());
  ok = ok && (k == 0 || fread(M.data(), sizeof(double), M.size(), f.f) == M.size());
  ok = ok && (k * np == 0 || fread(q.data(), sizeof(double), q.size(), f.f) == q.size());
  ok = ok && fread(spins.data(), 1, spins.size(), f.f) == spins.size();
  std::vector<int8_t> flags;
  std::vector<long long> cnt;
  if (ok && h.has_nn) {
    flags.resize(nc * L->Lz);
    cnt.resize(nc * L->Lz * tnmc::kCounterStride);
    ok = fread(flags.data(), 1, flags.size(), f.f) == flags.size();
    ok = ok && fread(cnt.data(), sizeof(long long), cnt.size(), f.f) == cnt.size();
  }
  if (!ok) return io_fail(std::string(path) + " is truncated");
  for (int8_t v : spins)
    if (L->d == 2 ? (v != 1 && v != -1) : (v < 0 || v >= L->d)) return io_fail("checkpoint holds invalid spins");
  for (int8_t v : flags)
    if (v != 0 && v != 1) return io_fail("checkpoint holds invalid fallback flags");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(L->dspins, spins.data(), spins.size(), hipMemcpyHostToDevice));
  if (k) {
    HIP_TRY(hipMemcpy(L->dErec, E.data(), E.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(L->dMrec, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice));
    if (np) HIP_TRY(hipMemcpy(L->dqrec, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  L->n_recorded = h.n_recorded;
  if (h.has_nn) {
    tnmc_status r = nn_counters(L);
    if (r != TNMC_OK) return r;
    L->nn_fallback = flags;
    HIP_TRY(hipMemcpy(L->dnncnt, cnt.data(), cnt.size() * sizeof(long long), hipMemcpyHostToDevice));
  }
  if (next_sweep) *next_sweep = h.next_sweep;
  return TNMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------ slice directions

namespace tnmc {
hipError_t launch_permute_spins(int8_t* const* lat_spins, int8_t* const* view_spins, int n_chains, int Lx, int Ly,
                                int Lz, int dir, int to_view, hipStream_t s);
}

namespace {

constexpr uint64_t kDirectionStride = 1ull << 56;

// The lattice seen with slices perpendicular to axis dir (1: y, 2: x) as
// z-slices: dir 1 maps site (z, y, x) to (y, z, x) with bond components
// (x, z, y), dir 2 maps it to (x, z, y) with components (y, z, x).
tnmc_status make_view(tnmc_lattice* L, int dir, tnmc_lattice** out) {
  const int Lx = L->Lx, Ly = L->Ly, Lz = L->Lz;
  const int nx = (dir == 1) ? Lx : Ly, ny = Lz, nz = (dir == 1) ? Ly : Lx;
  if (nx > kLxMax || ny > kLyMax) return TNMC_ERR_UNSUPPORTED;
  if (tnmc::sample_lds_bytes(L->d, L->chi_max, nx, ny) > 160 * 1024) return TNMC_ERR_UNSUPPORTED;
  const size_t n = L->sites();
  std::vector<float> J((size_t)L->n_instances * 3 * n), Jp(J.size());
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(J.data(), L->dJ, J.size() * sizeof(float), hipMemcpyDeviceToHost));
  const int comp[2][3] = {{0, 2, 1}, {1, 2, 0}};   // source component of the view's x-, y- and z-bonds
  for (int i = 0; i < L->n_instances; ++i)
    for (int c = 0; c < 3; ++c) {
      const float* src = J.data() + ((size_t)i * 3 + comp[dir - 1][c]) * n;
      float* dst = Jp.data() + ((size_t)i * 3 + c) * n;
      for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < Ly; ++y)
          for (int x = 0; x < Lx; ++x) {
            const size_t j = (dir == 1) ? ((size_t)y * Lz + z) * Lx + x : ((size_t)x * Lz + z) * Ly + y;
            dst[j] = src[((size_t)z * Ly + y) * Lx + x];
          }
    }
  auto* V = new tnmc_lattice();
  V->Lx = nx;
  V->Ly = ny;
  V->Lz = nz;
  V->d = L->d;
  V->chi = L->chi;
  V->chi_max = L->chi_max;
  V->precision = L->precision;
  V->n_cand = L->n_cand;
  V->n_chains = L->n_chains;
  V->n_instances = L->n_instances;
  V->seed = L->seed;
  V->chain_instance = L->chain_instance;
  V->beta = L->beta;
  V->chain_key = L->chain_key;
  auto fail = [&](hipError_t e) {
    g_last_error = std::string("slice-direction view: ") + hipGetErrorString(e);
    tnmc_lattice_free(V);
    return e == hipErrorOutOfMemory ? TNMC_ERR_OOM : TNMC_ERR_DEVICE;
  };
  hipError_t e;
  if ((e = hipMalloc((void**)&V->dJ, Jp.size() * sizeof(float))) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(V->dJ, Jp.data(), Jp.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  if ((e = hipMalloc((void**)&V->dspins, (size_t)L->n_chains * n)) != hipSuccess) return fail(e);
  std::vector<const float*> jc(L->n_chains);
  std::vector<int8_t*> sc(L->n_chains);
  for (int c = 0; c < L->n_chains; ++c) {
    jc[c] = V->J_of(c);
    sc[c] = V->spins_of(c);
  }
  if ((e = hipMalloc((void**)&V->dJc, L->n_chains * sizeof(float*))) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(V->dJc, jc.data(), L->n_chains * sizeof(float*), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  if ((e = hipMalloc((void**)&V->dSc, L->n_chains * sizeof(int8_t*))) != hipSuccess) return fail(e);
  if ((e = hipMemcpy(V->dSc, sc.data(), L->n_chains * sizeof(int8_t*), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  *out = V;
  return TNMC_OK;
}

}  // namespace

extern "C" {

tnmc_status tnmc_sweep_direction(tnmc_lattice* const* lats, int32_t n_lats, int32_t direction, int32_t n_sweeps,
                                 uint64_t sweep_offset, int32_t record, int32_t time_kernels, tnmc_stats* stats,
                                 void* stream) {
  if (direction == 0) return tnmc_sweep(lats, n_lats, n_sweeps, sweep_offset, record, time_kernels, stats, stream);
  CallClock clock(stats);
  if (check_lats(lats, n_lats) != TNMC_OK || n_sweeps < 0 || direction < 0 || direction > 2) return TNMC_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  std::vector<tnmc_lattice*> views(n_lats);
  for (int l = 0; l < n_lats; ++l) {
    tnmc_lattice* L = lats[l];
    if (!L->view[direction]) {
      tnmc_status r = make_view(L, direction, &L->view[direction]);
      if (r != TNMC_OK) return r;
    }
    views[l] = L->view[direction];
  }
  for (int t = 0; t < n_sweeps; ++t) {
    for (int l = 0; l < n_lats; ++l)
      HIP_TRY(tnmc::launch_permute_spins(lats[l]->dSc, views[l]->dSc, lats[l]->n_chains, lats[l]->Lx, lats[l]->Ly,
                                         lats[l]->Lz, direction, 1, s));
    tnmc_status r = tnmc_sweep(views.data(), n_lats, 1, sweep_offset + (uint64_t)t + direction * kDirectionStride, 0,
                               time_kernels, stats, stream);
    if (r != TNMC_OK) return r;
    for (int l = 0; l < n_lats; ++l) {
      tnmc_lattice* L = lats[l];
      HIP_TRY(tnmc::launch_permute_spins(L->dSc, views[l]->dSc, L->n_chains, L->Lx, L->Ly, L->Lz, direction, 0, s));
      if (record && L->n_recorded < L->record_capacity) {
        const int64_t i = L->n_recorded++;
        HIP_TRY(tnmc::launch_observables(L->dJc, L->dSc, L->n_chains, L->dpa, L->dpb, L->n_pairs, L->Lx, L->Ly,
                                         L->Lz, L->d, L->dErec + i * L->n_chains, L->dMrec + i * L->n_chains,
                                         L->dqrec + i * std::max(1, L->n_pairs), s));
      }
    }
  }
  return TNMC_OK;
}

}  // extern "C"
