// Internal declarations shared by the HIP kernels and the host side of libtnmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnmc {

constexpr int kCounters = 5;   // per-task counters, see TaskDesc::counters
constexpr int kCounterStride = 32;   // long longs between the counters of consecutive tasks (256 B)

// Per-task workspace regions start on 256-byte boundaries, so that no cache
// line holds data of two tasks (tasks of concurrent launches run on different
// XCDs, whose L2 caches are not coherent with each other within a launch).
inline size_t pad256_ints(size_t n) { return (n + 63) & ~(size_t)63; }
inline size_t pad256_doubles(size_t n) { return (n + 31) & ~(size_t)31; }

// Storage precision of the environments (same values as TNMC_FP64 / TNMC_FP32).
constexpr int kPrecF64 = 0;
constexpr int kPrecF32 = 1;

// Relative cut-off of the rank-revealing factorisations: directions whose
// weight is below this fraction of the largest one are dropped.  FP64 storage:
// such directions are zero at FP64 resolution.  (Gram-Schmidt residuals of
// dependent rows sit at ~eps sqrt(n), slightly above this, so the right-sweep
// LQ may keep a few rounding-level directions; its rank is bounded by the left
// factor's and they are harmless.)  FP32 storage: the stored environments
// carry relative rounding of 2^-24, so directions below ~1e-7 are rounding
// noise; the cut sits a decade above it.
constexpr double kRankTolF64 = 1e-15;
constexpr double kRankTolF32 = 1e-6;

// One slice task: layer z of one chain.  Everything a kernel needs, with
// device pointers into the lattice state and into the per-task workspace.
struct TaskDesc {
  const float* J;          // couplings of the chain's instance [3][Lz][Ly][Lx]
  int8_t* spins;           // chain configuration [Lz][Ly][Lx]
  void* env;               // environments [Ly][Lx][d][chi_max][chi_max], double or float
  double* rscr;            // R factors of the left sweep [Lx][(d chi_max)^2]
  int* bond;               // right bond dimension of every environment site [Ly][Lx]
  double* logscale;        // log of the removed scale of every environment [Ly]
  int* status;             // contraction fault bits of this task (0 = ok); a compact launch that leaves the
                           // task unfinished writes 8 | fault bits << 4 | row to resume at << 8
  long long* counters;     // per-task running totals {proposed, accepted, faults, contraction flops,
                           //  contractions redone with the full LDS layout}
  const int8_t* force_new; // if set: evaluate this layer instead of sampling [Ly][Lx]
  int8_t* s_new_out;       // if set: copy of the proposed layer [Ly][Lx]
  double* record;          // if set: {logq_new, logq_old, dE, accepted, fault}
  double* gscr;            // global scratch for the full contraction tile layout, where it exceeds a CU's LDS
  double beta;
  double rank_tol;         // kRankTolF64 or kRankTolF32
  uint64_t key0, key1;     // Philox key
  int Lx, Ly, Lz, z, chi, d;
  int chi_max;             // storage stride of the environment tensors
  int write_back;          // apply the MH decision to spins
  int n_cand;              // candidates drawn from the environments and chained by MH (<= 1: one)
};

// Per-task workspace sizes (doubles / ints) for a (Lx, Ly, d, chi_max) task;
// FP32 environments take half the doubles (rounded up).
inline size_t env_doubles(int Lx, int Ly, int d, int chi_max, int precision = kPrecF64) {
  const size_t n = (size_t)Ly * Lx * d * chi_max * chi_max;
  return precision == kPrecF32 ? (n + 1) / 2 : n;
}
inline size_t rscr_doubles(int Lx, int d, int chi_max) {
  return (size_t)Lx * (size_t)(d * chi_max) * (d * chi_max);
}

// How the slice tasks of one (d, chi_max, precision) class are contracted:
// the tile layout (full = 1 runs a class that has the compact two-per-CU
// layout with the full one-per-CU layout instead) and the engine of the
// products M, AT, C and Y (mfma = 1: matrix cores, FP64 or FP32 operands as
// the environments are stored; 0: FP64 on the vector ALU).  Every choice is a
// correct contraction; they agree within the FP64 parity bar (FP64 storage)
// or the reduced-precision one (FP32 storage).
struct ContractCfg {
  int full = 0;
  int mfma = 0;
};

// Kernel launchers (return hipError_t of the launch).
hipError_t launch_contract(const TaskDesc* tasks, int n_tasks, int d, int chi_max, int precision, ContractCfg cfg,
                           hipStream_t s);
hipError_t launch_contract_f64(const TaskDesc* tasks, int n_tasks, int d, int chi_max, int full, hipStream_t s);
hipError_t launch_contract_f64_mf(const TaskDesc* tasks, int n_tasks, int d, int chi_max, int full, hipStream_t s);
hipError_t launch_contract_f32(const TaskDesc* tasks, int n_tasks, int d, int chi_max, int full, hipStream_t s);
hipError_t launch_contract_f32_mf(const TaskDesc* tasks, int n_tasks, int d, int chi_max, int full, hipStream_t s);
bool contract_has_compact(int d, int chi_max);
// sweep_dev (may be null): the sweep counter in device memory, read by the
// kernel instead of sweep (graph replays).
hipError_t launch_sample(const TaskDesc* tasks, int n_tasks, int d, int chi_max, int precision, int Lx_max,
                         int Ly_max, uint64_t sweep, hipStream_t s, const unsigned long long* sweep_dev = nullptr);
hipError_t launch_energy(const float* J, const int8_t* spins, int Lx, int Ly, int Lz, int d,
                         double* out, hipStream_t s);
hipError_t launch_observables(const float* const* Jc, int8_t* const* spins, int n_chains,
                              const int* pair_a, const int* pair_b, int n_pairs, int Lx, int Ly,
                              int Lz, int d, double* E_out, double* M_out, double* q_out,
                              hipStream_t s, const long long* slot_dev = nullptr, long long capacity = 0);
// slot_dev (may be null): the record slot in device memory (graph replays); the
// outputs are then E_out + slot * n_chains etc., and slots >= capacity are dropped.
hipError_t launch_graph_advance(unsigned long long* sweep, long long* slots, int n_slots, hipStream_t s);
bool contract_supported(int d, int chi_max);
bool contract_uses_global(int d, int chi_max);   // tiles in the per-task global scratch (gscr)
size_t contract_lds_bytes(int d, int chi_max);
size_t sample_lds_bytes(int d, int chi_max, int Lx, int Ly);   // static + dynamic LDS of a sampler workgroup
void set_force_retry(int on);   // test hook: every compact-layout task takes the retry path
void set_force_narrow(int on);  // test hook: full-layout launches take the narrow (two per CU) variant at any size
// Compute units of the current device (queried on the first call, 256 on
// MI355X); lattice creation makes that call, so no later launch queries the
// device, not even under graph capture.
int device_cus();
int chi_bucket(int chi);   // storage chi_max used for a requested chi (0 if unsupported)

}  // namespace tnmc
