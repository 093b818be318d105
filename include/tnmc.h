/*
 * tnmc.h - C ABI of the MI355X TNMCMC-1 slice-proposal library (libtnmc.so).
 *
 * Method: Tensor Network Markov Chain Monte Carlo, arXiv 2509.23945.  A layer
 * (z-slice) of a 3D lattice with quenched couplings is resampled given its two
 * neighbouring layers (SM S2.A, TNMCMC-1): the layer's 2D tensor network, with
 * the neighbours acting as an external field, is contracted by boundary MPS with
 * truncation to bond dimension chi (SM S1.B), a new layer is drawn site by site
 * with its exact log-probability log q (main text "TNMCMC"; SM S1.C), q of the
 * current layer is evaluated by teacher forcing (SM Alg. 2), and the move is
 * accepted by Metropolis-Hastings (main text Eq. 1).
 *
 * Conventions shared by every call:
 *  - Lattices have free boundaries.  Couplings are float32 J[3][Lz][Ly][Lx]:
 *    component 0 couples (x,y,z)-(x+1,y,z), 1 couples (x,y,z)-(x,y+1,z),
 *    2 couples (x,y,z)-(x,y,z+1); bonds leaving the lattice must be 0.
 *  - Ising (d=2): spins int8 +1/-1, energy -sum J s s'.  Potts (d=3): states
 *    int8 0/1/2, energy -sum J delta(s,s').  Spins are [Lz][Ly][Lx] per chain.
 *  - Random numbers: Philox4x64-10 with key (seed, chain_key) and counter
 *    (draw, z, sweep, purpose); purpose 0 = site draws (draw = y*Lx+x),
 *    purpose 1 = the MH uniform; U = ((w0 >> 11) + 0.5) * 2^-53.
 *  - All device work is stream-ordered on the hip_stream argument (a
 *    hipStream_t, NULL = default stream).  Calls that return host data
 *    synchronise that stream.  A handle is used by one host thread at a time.
 *  - Every call returns a tnmc_status; on TNMC_ERR_ARG nothing is changed.
 */
#ifndef TNMC_H
#define TNMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TNMC_OK = 0,
  TNMC_ERR_ARG = -1,         /* invalid shape, pointer or parameter */
  TNMC_ERR_OOM = -2,         /* device allocation failed */
  TNMC_ERR_DEVICE = -3,      /* a HIP call failed (message: tnmc_last_error) */
  TNMC_ERR_NUMERIC = -4,     /* non-finite result in a proposal */
  TNMC_ERR_UNSUPPORTED = -5, /* (d, chi, precision) combination not built */
  TNMC_ERR_IO = -6           /* checkpoint file unreadable / unwritable, or of another lattice */
} tnmc_status;

enum { TNMC_FP64 = 0, TNMC_FP32 = 1 };   /* storage precision of the boundary-MPS environments */

typedef struct tnmc_lattice tnmc_lattice;  /* opaque; owns the device state it allocates */

/* A batch of chains on lattices of one shape (Lx, Ly, Lz, d) and bond
 * dimension chi.  Chains may have different couplings (instances) and
 * different inverse temperatures.  All pointers are HOST pointers, copied at
 * init and not retained. */
typedef struct {
  int32_t Lx, Ly, Lz;           /* 1 <= Lx, Ly; 1 <= Lz */
  int32_t d;                    /* 2 (Ising / EA) or 3 (Potts) */
  int32_t chi;                  /* boundary-MPS bond dimension, >= 1 */
  int32_t precision;            /* TNMC_FP64, or TNMC_FP32: the reduced-precision form.  The
                                   environments are stored in FP32 and the rank-revealing
                                   factorisations cut at 1e-6 relative (FP32 resolution) instead
                                   of 1e-15; the factorisations, log q, dE and the MH test stay
                                   FP64, the products run in FP64 on the vector ALU or with FP32
                                   operands on the matrix cores (the autotuner's choice).  The
                                   proposal q changes (log q typically by ~1e-6 relative, more
                                   where the dropped directions carry a layer's weight, as for
                                   near-ordered layers of an ordered ferromagnet); the chain's
                                   stationary law does not: q(old) and q(new) come from the same
                                   environments (SM S2.A, MH of main text Eq. 1). */
  int32_t n_chains;             /* >= 1 */
  int32_t n_instances;          /* >= 1, number of coupling sets */
  const float* J;               /* [n_instances][3][Lz][Ly][Lx] */
  const int32_t* chain_instance;/* [n_chains] in [0, n_instances); NULL: chain c -> c % n_instances */
  const double* beta;           /* [n_chains], >= 0 */
  const int8_t* spins;          /* [n_chains][Lz][Ly][Lx] initial configuration */
  uint64_t seed;                /* Philox key word 0 */
  const uint64_t* chain_key;    /* [n_chains] Philox key word 1; NULL: chain index */
  int32_t n_pairs;              /* replica pairs for the overlap q, >= 0 */
  const int32_t* pairs;         /* [n_pairs][2] chain indices (same instance) */
  int32_t record_capacity;      /* sweeps of observables kept on the device */
  int32_t n_candidates;         /* 0 or 1: one proposal per layer update; K in 2..64: sweeps draw K
                                   candidates from each layer's environments and chain K
                                   independence-MH steps (main text, "TNMCMC": a batch of candidates
                                   from the same approximate distribution, one kept); candidate k
                                   uses Philox purposes 2k (sites) and 2k + 1 (MH).  Single-task
                                   calls (propose, logq) always draw one. */
} tnmc_lattice_desc;

/* Allocate the device state of a batch of chains (SM Alg. 2 inputs: L, {J},
 * chi, beta, initial configuration).  *out receives the handle. */
tnmc_status tnmc_lattice_init(const tnmc_lattice_desc* desc, tnmc_lattice** out);
tnmc_status tnmc_lattice_free(tnmc_lattice* lat);

/* One TNMCMC-1 proposal for layer z of chain `chain` (SM Alg. 2, SampleLayer):
 * builds the layer network from the held layers z-1, z+1, contracts it by
 * boundary MPS to chi, draws a new layer with the site uniforms of counter
 * (., z, sweep, 0), and evaluates q of the current layer by teacher forcing.
 * The state is not changed.  Outputs: s_new [Ly][Lx] int8, a HOST or DEVICE
 * pointer (the copy takes its direction from unified addressing), and, at HOST
 * pointers, natural-log q of the new and current layer and dE = E(new) - E(current).
 * Returns TNMC_ERR_NUMERIC if either path hit a non-positive or non-finite
 * total site weight (the outputs are still written). */
tnmc_status tnmc_slice_propose(tnmc_lattice* lat, int32_t chain, int32_t z, uint64_t sweep,
                               int8_t* s_new, double* logq_new, double* logq_old, double* dE,
                               void* hip_stream);

/* As tnmc_slice_propose, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): this call makes no device allocation of any kind.  The slice
 * task's workspace lives in a static device array of 24 MiB that each GPU the
 * library runs on holds until the process ends; layers whose workspace
 * (environments of Ly*Lx*d*chi_max^2 values, R factors, tiles) does not fit
 * it return TNMC_ERR_ARG with the sizes in tnmc_last_error (FP64 Ising layers
 * up to 32x32 at chi <= 32 fit).  Results equal tnmc_slice_propose's.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other host threads, or other streams before this call has returned) race
 * and must not be made.  Outputs as for tnmc_slice_propose; the call
 * synchronises hip_stream. */
tnmc_status tnmc_slice_propose_static(tnmc_lattice* lat, int32_t chain, int32_t z, uint64_t sweep,
                                      int8_t* s_new, double* logq_new, double* logq_old, double* dE,
                                      void* hip_stream);

/* log q of an arbitrary configuration s [Ly][Lx] (HOST or DEVICE) of layer z given the
 * current held layers (SM S1.C: product of the conditionals along the
 * sampling order, with the spins projected on their states). */
tnmc_status tnmc_slice_logq(tnmc_lattice* lat, int32_t chain, int32_t z, const int8_t* s,
                            double* logq, void* hip_stream);

/* Metropolis-Hastings decision of main text Eq. 1 for an independence
 * proposal: *accepted = u < exp(min(0, logq_old - logq_new - beta*dE)),
 * with 0 < u < 1.  Pure host function. */
tnmc_status tnmc_mh_accept(double logq_old, double logq_new, double beta, double dE, double u,
                           int32_t* accepted);

typedef struct {
  int64_t proposed, accepted, numeric_faults;
  double contract_ms;           /* summed duration of the contraction launches (HIP events) */
  double sample_ms;             /* summed duration of the sampling/MH launches */
  double contract_flops;        /* algorithmic FP64 flops of the contractions (textbook counts of
                                   the QR, SVD and GEMM steps at the bond dimensions used) */
  int64_t contract_launches, sample_launches;
  int64_t contract_retries;     /* slice tasks whose left-sweep rank outgrew the compact LDS layout
                                   (two workgroups per CU) and were contracted again with the full one */
  double seconds;               /* host wall time of the call, entry to return (a call given stats
                                   synchronises hip_stream before it returns) */
  int64_t nn_fallbacks;         /* tnmc_nn_sweep: layer updates proposed by the tensor-network fallback */
} tnmc_stats;

/* n_sweeps sweeps of every chain of every lattice in lats[0..n_lats-1]
 * (SM S2.A: all even layers with the odd ones held, then all odd layers; one
 * sweep updates every layer once).  Sweep t uses Philox sweep counter
 * sweep_offset + t.  With record != 0 the energy, magnetisation and pair
 * overlaps after each sweep are appended to each lattice's device record.
 * stats (may be NULL) accumulates counts; with time_kernels != 0 it also
 * receives the summed kernel durations measured with HIP events on
 * hip_stream (the call then synchronises). */
tnmc_status tnmc_sweep(tnmc_lattice* const* lats, int32_t n_lats, int32_t n_sweeps,
                       uint64_t sweep_offset, int32_t record, int32_t time_kernels,
                       tnmc_stats* stats, void* hip_stream);

/* TNMCMC-2 sweeps (SM S2.B, coarse-graining with superspins): layers z0 and
 * z0 + 1 of an Ising lattice (d = 2) are merged into one composite layer of
 * 4-state superspins u = u_a + 2 u_b (u_a, u_b the 0/1 states of layers z0 and
 * z0 + 1).  The composite's 2D network carries both sublayers' in-plane bonds,
 * and its on-site term holds the bond between the two layers and the fields of
 * the held layers z0 - 1 and z0 + 2; it is contracted, sampled and accepted
 * like a TNMCMC-1 layer (main text, Methods: boundary-MPS contraction, exact
 * sampling of the approximate distribution, Metropolis-Hastings with its log q).
 * One sweep updates the composites z0 = 0 .. Lz - 2 in three phases (z0 mod 3),
 * a launch pair per phase, each phase's composites sharing no layer they update
 * or hold.  Philox counters use the sweep index sweep_offset + t + 3 * 2^56,
 * so they never meet those of tnmc_sweep.  Requires d = 2, Lz >= 2,
 * chi_max <= 8 (4 or 8 after rounding up) and a sampler footprint within a
 * CU's LDS; anything else returns TNMC_ERR_UNSUPPORTED without touching device
 * memory (TNMC_ERR_ARG for invalid handles or n_sweeps < 0).  trace is a
 * DEVICE pointer or NULL: 5 doubles per composite task (log q of the
 * proposal, log q of the current composite, dE, accepted, numeric fault), tasks
 * ordered by phase, then lattice, chain and z0, rewritten by every sweep; record, time_kernels, stats and hip_stream mean what
 * they mean for tnmc_sweep.  The composite contraction uses the vector-ALU
 * engine and the full tile layout only. */
tnmc_status tnmc_sweep_superspin(tnmc_lattice* const* lats, int32_t n_lats, int32_t n_sweeps, uint64_t sweep_offset,
                                 int32_t record, int32_t time_kernels, double* trace, tnmc_stats* stats,
                                 void* hip_stream);

/* As tnmc_sweep (without kernel timing), with one sweep captured once into a
 * HIP graph (the contraction and sampler launches of both parities, the
 * observables, and the advance of a device-resident sweep counter and record
 * slots) and replayed n_sweeps times on hip_stream, so the host issues one
 * graph launch per sweep instead of a launch per kernel.  The chains are the
 * same, bit for bit, as those of tnmc_sweep with the same contraction choices:
 * the replays use the autotuner's current choices or the pins and run no
 * trials of their own.  Descriptors, counters and the sweep counter are set up
 * on hip_stream before the replays (no memory set is recorded in the graph).
 * stats (may be NULL) receives the counts; the call then synchronises. */
tnmc_status tnmc_sweep_graph(tnmc_lattice* const* lats, int32_t n_lats, int32_t n_sweeps, uint64_t sweep_offset,
                             int32_t record, tnmc_stats* stats, void* hip_stream);

/* As tnmc_sweep, with the slices taken perpendicular to axis `direction`
 * (0: z, identical to tnmc_sweep; 1: y; 2: x), so that chains can cycle the
 * slice direction between sweeps.  A y-slice is the layer of sites with one
 * y, its held neighbours the y-1 and y+1 layers; the sites of a slice are
 * drawn in the order (z, x) for y-slices and (z, y) for x-slices (row index
 * first); the Philox sweep counter of sweep t is sweep_offset + t +
 * direction * 2^56, and the layer counter is the slice index.  The slice's
 * shape must be supported as a layer (TNMC_ERR_UNSUPPORTED otherwise).  Each
 * sweep reorders the spins into the direction's layout and back (two L^3
 * byte copies), and builds its task list on the host. */
tnmc_status tnmc_sweep_direction(tnmc_lattice* const* lats, int32_t n_lats, int32_t direction, int32_t n_sweeps,
                                 uint64_t sweep_offset, int32_t record, int32_t time_kernels, tnmc_stats* stats,
                                 void* hip_stream);

/* One half-sweep (parity 0: even layers, 1: odd layers) of every chain in
 * lats, as inside tnmc_sweep.  trace (DEVICE pointer or NULL) receives, for
 * task t in the order lattice-major, chain, layer z = parity, parity+2, ...:
 * trace[5t..5t+4] = {log q(new), log q(current), dE, accepted, fault}; for a
 * lattice with several candidates per environment: {log q of the final layer,
 * log q of the initial one, E(final) - E(initial), candidates accepted,
 * candidates rejected for a numeric fault}. */
tnmc_status tnmc_half_sweep(tnmc_lattice* const* lats, int32_t n_lats, int32_t parity,
                            uint64_t sweep, double* trace, tnmc_stats* stats, void* hip_stream);

/* State access (HOST buffers, synchronous). */
tnmc_status tnmc_get_spins(tnmc_lattice* lat, int32_t chain, int8_t* out);     /* [Lz][Ly][Lx] */
tnmc_status tnmc_set_spins(tnmc_lattice* lat, int32_t chain, const int8_t* in);
/* Full-lattice energy of a chain, computed on the device in FP64. */
tnmc_status tnmc_energy(tnmc_lattice* lat, int32_t chain, double* E);
/* Recorded observables: E[n][n_chains], M[n][n_chains], q[n][n_pairs] (HOST,
 * each may be NULL); *n receives the number of recorded sweeps (capped at
 * record_capacity; later sweeps are dropped). */
tnmc_status tnmc_timeseries(tnmc_lattice* lat, double* E, double* M, double* q, int64_t* n);
/* Drop the recorded observables. */
tnmc_status tnmc_timeseries_reset(tnmc_lattice* lat);
/* Couplings as given at init: HOST [n_instances][3][Lz][Ly][Lx] (synchronous). */
tnmc_status tnmc_get_couplings(tnmc_lattice* lat, float* out);

/* Checkpoint / resume (synchronous).  save writes the chains' spins, the
 * recorded observables, the learned-proposal counts and fallback flags, and
 * the caller's next sweep counter to the file at path.  load restores them
 * into a lattice created with the same description (shape, d, chi,
 * precision, chains, instances, betas, pairs, Philox seed and keys, and the
 * same couplings, checked by a hash); *next_sweep (may be NULL) receives the
 * saved counter.  Random numbers are a pure function of (seed, key, sweep,
 * layer, site), so sweeps run after a load with that counter reproduce an
 * uninterrupted run.  Errors: TNMC_ERR_IO (message: tnmc_last_error); the
 * lattice is unchanged unless TNMC_OK. */
tnmc_status tnmc_checkpoint_save(tnmc_lattice* lat, uint64_t next_sweep, const char* path);
tnmc_status tnmc_checkpoint_load(tnmc_lattice* lat, const char* path, uint64_t* next_sweep);

/* Algorithmic FP64 flop count of one slice update of an Lx x Ly layer with
 * bond dimension chi, split into the boundary-MPS contraction (textbook
 * counts of the Householder QR, Golub-Reinsch SVD and GEMM steps at the bond
 * dimensions the method uses) and the two sampling passes.  Used for
 * roofline reporting; either output may be NULL. */
tnmc_status tnmc_flop_model(int32_t Lx, int32_t Ly, int32_t d, int32_t chi, double* contract_flops,
                            double* sample_flops);

/* Diagnostics: copy part of the workspace left by the last single-task call
 * (tnmc_slice_propose / tnmc_slice_logq) to the HOST buffer out (at most
 * bytes): what = 0 environments [Ly][Lx][d][chi_max][chi_max] doubles,
 * 1 bond dimensions [Ly][Lx] ints, 2 R-factor row counts [Lx] + fault flag
 * ints, 3 R factors [Lx][(d chi_max)^2] doubles, 4 log scales [Ly] doubles. */
tnmc_status tnmc_debug_workspace(int32_t what, void* out, int64_t bytes);

/* Test hooks, process-wide.  what = 0: send every slice task of the
 * configurations that use the compact two-per-CU contraction layout through
 * its overflow path (a second launch with the full tile layout in LDS, one
 * task per CU), so that path can be checked against the oracle; value 1 = on,
 * 0 = off (default).  what = 1: the contraction autotuner (value 1 = on, the
 * default; 0 = off, which also drops its choices).  what = 2: two
 * learned-proposal tasks per workgroup in tnmc_nn_sweep launches that allow
 * it (value 1 = on, the default; 0 = off).  Results agree within the parity
 * bar either way (what = 2: bit for bit).  what = 3 (an ablation knob, not a
 * test hook): value k in 1..15 sets the relative cut-off of the rank-revealing
 * factorisations to 10^-k for every storage precision, for plans made after
 * the call; 0 restores the defaults (1e-15 for FP64 environments, 1e-6 for
 * FP32 ones).  A proposal made with another cut-off is another q: MH stays
 * exact, but parity with the oracle holds only at the defaults.  what = 4: a
 * contraction class that runs the full tile layout launches its narrow variant
 * (two wavefronts per task, two tasks per CU; otherwise used only when a
 * launch has more tasks than the device has CUs) at any size, so that path
 * can be checked against the oracle on small cases; value 1 = on, 0 = off
 * (default).  Returns TNMC_ERR_ARG for an unknown what or a value out of
 * range. */
tnmc_status tnmc_debug_set(int32_t what, int32_t value);

/* ------------------------------------------------------------------------
 * Learned proposal.  Any exactly normalised proposal q with an exact log q
 * leaves the Metropolis-Hastings chain of main text Eq. 1 exact; here q is an
 * autoregressive masked-convolution network q_theta(s | cond) over the sites
 * of an Ising layer, in the tensor-network sampler's site order (rows, then
 * sites within a row; SM S1.C), used in place of the boundary-MPS
 * conditionals.  The network is not part of the paper; its shape is fixed:
 *  - input per site: four condition channels, seen through full 3x3 windows:
 *    Jz(z-1) s(z-1), Jz(z) s(z+1), Jx(z), Jy(z) (0 where the neighbour layer
 *    or the bond does not exist), and the layer's spins (+1/-1) seen through a
 *    mask that hides the centre and later sites;
 *  - five 3x3 layers of 32 channels with ReLU (the first reads the input, the
 *    next four read the previous layer masked to earlier sites and the
 *    centre), and a 3x3 output channel masked the same way: the logit l of
 *    P(s = +1), clipped to [-30, 30]; zero padding at the open edges;
 *  - parameters: TNMC_NN_PARAMS numbers, per layer W[c_out][c_in][3][3]
 *    then b[c_out] (c_in, c_out = (5,32), (32,32) x4, (32,1)); masked weights
 *    are stored but unused.  The handle keeps FP32 master values (what the
 *    get / set calls exchange and Adam updates) and evaluates the network with
 *    their BF16 roundings (nearest, ties to even), refreshed whenever the
 *    masters change; gradients are taken at the BF16 parameters.
 * Convolutions run in FP32 arithmetic with FP32 accumulation; probabilities,
 * log q, dE and the MH test in FP64.
 * Site j of a drawn layer takes +1 when its uniform (Philox counter
 * (y*Lx+x, z, sweep, 0), as for the TN sampler) is below P(s_j = +1).
 * Ising lattices (d = 2) only.  The batched calls take layers up to 64 sites
 * wide (TNMC_ERR_ARG beyond); the sampler behind propose / logq / sweeps keeps
 * the masked weights and per-layer activation rings in LDS, which limits rows
 * to 47 sites (TNMC_ERR_UNSUPPORTED beyond).
 * Batched entry points take DEVICE pointers: cond [n][4][Ly][Lx] float,
 * s [n][Ly][Lx] int8; they are stream-ordered on hip_stream. */
enum { TNMC_NN_PARAMS = 38753 };
typedef struct tnmc_nn tnmc_nn;   /* opaque; owns its parameters, Adam state and batch buffers */

/* params (HOST, TNMC_NN_PARAMS floats) or NULL for the default
 * initialisation from seed (W ~ N(0, 2/(9 c_in)), b = 0). */
tnmc_status tnmc_nn_create(const float* params, uint64_t seed, tnmc_nn** out);
tnmc_status tnmc_nn_free(tnmc_nn* nn);
/* Parameters to / from a HOST buffer of TNMC_NN_PARAMS floats (synchronous);
 * set also clears the Adam state. */
tnmc_status tnmc_nn_get_params(tnmc_nn* nn, float* out);
tnmc_status tnmc_nn_set_params(tnmc_nn* nn, const float* in);
/* log q_theta(s_i | cond_i) for a batch (logq: DEVICE, n doubles). */
tnmc_status tnmc_nn_logq(tnmc_nn* nn, const float* cond, const int8_t* s, int32_t n, int32_t Lx, int32_t Ly,
                         double* logq, void* hip_stream);
/* Mean of -log q_theta over the batch (*loss, HOST; synchronises) and its
 * gradient with respect to the parameters (grad: DEVICE, TNMC_NN_PARAMS
 * floats, or NULL); masked weights get 0, the clip passes no gradient where
 * it is active. */
tnmc_status tnmc_nn_loss_grad(tnmc_nn* nn, const float* cond, const int8_t* s, int32_t n, int32_t Lx, int32_t Ly,
                              double* loss, float* grad, void* hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * FP32 masters with the DEVICE gradient grad and learning rate lr; the BF16
 * parameters are refreshed from the result. */
tnmc_status tnmc_nn_adam_step(tnmc_nn* nn, const float* grad, double lr, void* hip_stream);
/* epochs passes of minibatch Adam over the n pairs in their given order
 * (minibatches of `batch` consecutive pairs, the last one possibly shorter);
 * *last_loss (HOST, may be NULL) receives the loss of the last minibatch
 * before its step (the call then synchronises). */
tnmc_status tnmc_nn_train(tnmc_nn* nn, const float* cond, const int8_t* s, int64_t n, int32_t Lx, int32_t Ly,
                          int32_t epochs, int32_t batch, double lr, double* last_loss, void* hip_stream);
/* Training pairs from a lattice's current state: for every chain c and layer
 * z, pair c*Lz + z = (condition channels of layer z, spins of layer z) into
 * DEVICE buffers cond [n_chains*Lz][4][Ly][Lx] and s [n_chains*Lz][Ly][Lx]. */
tnmc_status tnmc_nn_dataset(tnmc_lattice* lat, float* cond, int8_t* s, void* hip_stream);
/* As tnmc_slice_propose / tnmc_slice_logq, with the learned proposal. */
tnmc_status tnmc_nn_slice_propose(tnmc_lattice* lat, tnmc_nn* nn, int32_t chain, int32_t z, uint64_t sweep,
                                  int8_t* s_new, double* logq_new, double* logq_old, double* dE, void* hip_stream);
tnmc_status tnmc_nn_slice_logq(tnmc_lattice* lat, tnmc_nn* nn, int32_t chain, int32_t z, const int8_t* s,
                               double* logq, void* hip_stream);
/* As tnmc_sweep, each layer proposed by the learned proposal unless its
 * fallback flag selects the tensor-network proposal (both are exact MH
 * kernels).  The learned proposals of a lattice are counted per (chain, z). */
tnmc_status tnmc_nn_sweep(tnmc_lattice* const* lats, int32_t n_lats, tnmc_nn* nn, int32_t n_sweeps,
                          uint64_t sweep_offset, int32_t record, int32_t time_kernels, tnmc_stats* stats,
                          void* hip_stream);
/* Per-(chain, z) counts of learned proposals made and accepted since the
 * last reset (HOST arrays [n_chains][Lz], either may be NULL). */
tnmc_status tnmc_nn_counts(tnmc_lattice* lat, int64_t* proposed, int64_t* accepted);
tnmc_status tnmc_nn_counts_reset(tnmc_lattice* lat);
/* Fallback flags [n_chains][Lz] (HOST; 1 = tensor-network proposal); NULL
 * clears them all. */
tnmc_status tnmc_nn_set_fallback(tnmc_lattice* lat, const int8_t* flags);
tnmc_status tnmc_nn_get_fallback(tnmc_lattice* lat, int8_t* flags);
/* Freezes the fallback once, after a calibration window: every layer whose
 * learned proposals were accepted at a rate below threshold switches to the
 * tensor-network proposal (layers not yet proposed keep their flag);
 * *n_fallback (may be NULL) receives the number of flagged layers.  Deciding
 * once and then keeping each layer's kernel fixed keeps every later step an
 * exact MH kernel. */
tnmc_status tnmc_nn_calibrate_fallback(tnmc_lattice* lat, double threshold, int32_t* n_fallback);

/* Autotuner of the contraction (batching).  A launch group of slice tasks is
 * keyed by (d, chi bucket, precision, row length, row count, number of
 * tasks); its candidates are the engine of the products M, AT, C and Y
 * (0: FP64 on the vector ALU; 1: the matrix cores, V_MFMA_F64_16X16X4_F64
 * for FP64 environments, V_MFMA_F32_16X16X4_F32 with FP32 operands and
 * accumulation for FP32 ones) and, where the class has the compact tile layout
 * (two tasks per CU, with a full-layout redo of the tasks whose rank outgrows
 * it), the layout (0: compact, 1: full, one task per CU).  Before a group's
 * second sweep each candidate's contraction of that sweep is timed three
 * times with HIP events and the smallest median is kept for the process.
 * All candidates are correct contractions and agree within the parity bar of
 * the storage precision, not bit for bit: pin them (tnmc_autotune_pin) for
 * runs that must reproduce bit for bit across processes.  Single-task calls
 * (tnmc_slice_propose, tnmc_slice_logq and their learned / static variants)
 * use the pins, else engine 0 and the compact layout.
 *
 * tnmc_layout_choice: *layout receives -1 (no tuned class of this (d, chi,
 * precision), or no layout choice) or the chosen layout; ms_compact / ms_full
 * (may be NULL) the median trial durations of the two layouts with the chosen
 * engine (-1 if not tried).
 * tnmc_autotune_choice: the most recently tuned class of this (d, chi,
 * precision): *layout and *engine (-1 if none); ms (may be NULL, 4 doubles)
 * the median trial durations [engine 0 compact, engine 0 full, engine 1
 * compact, engine 1 full] (-1 where not a candidate).
 * tnmc_autotune_pin: fixes the layout and / or the engine for every later
 * launch (-1 leaves that dimension to the autotuner); drops earlier choices.
 * TNMC_ERR_ARG for values outside -1..1. */
tnmc_status tnmc_layout_choice(int32_t d, int32_t chi, int32_t precision, int32_t* layout, double* ms_compact,
                               double* ms_full);
tnmc_status tnmc_autotune_choice(int32_t d, int32_t chi, int32_t precision, int32_t* layout, int32_t* engine,
                                 double* ms);
tnmc_status tnmc_autotune_pin(int32_t layout, int32_t engine);
/* Runs the trials now, on the current states of the chains of lats (the
 * tasks of one sweep of them, both parities), for every launch group, and
 * replaces earlier choices for those groups; the chains are not changed.  A
 * caller that warms its chains up first can tune on representative states
 * (the automatic trial at a group's second sweep may still see the larger
 * bond ranks of a random start).  Synchronises hip_stream. */
tnmc_status tnmc_autotune_now(tnmc_lattice* const* lats, int32_t n_lats, void* hip_stream);

const char* tnmc_status_string(tnmc_status s);
/* Text of the last failed HIP call (thread-local). */
const char* tnmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TNMC_H */
