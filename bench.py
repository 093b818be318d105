#!/usr/bin/env python3
"""Throughput of the TNMCMC-1 slice proposal on one MI355X.

A step is one sweep: every layer of every chain is resampled once (even layers,
then odd layers), each by boundary-MPS contraction, ancestral sampling with
exact log q, teacher-forced log q of the current layer and a Metropolis-Hastings
decision.  Default workload: 3D Edwards-Anderson +-J, 32^3, open boundaries,
beta = 1.0, chi = 32, 16 disorder instances x 2 replicas = 32 chains, FP64,
synthetic couplings and spins from fixed seeds.

Prints one JSON line with slice updates/s, the roofline of the contraction
kernel (HIP events on the launch stream) and the FP64 oracle timed on the host
cores over a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 2.4 GHz x 128 flop/clk

WORKLOADS = {
    # single-lattice 3D EA +-J: L, chi, beta, instances, replicas
    "ea32": dict(L=32, chi=32, beta=1.0, n_inst=16, n_rep=2),
    "ea16": dict(L=16, chi=32, beta=1.0, n_inst=64, n_rep=2),
    "ea8": dict(L=8, chi=16, beta=0.5, n_inst=1, n_rep=1),
    # small layers where the learned proposal is accepted: 8^3 +-J, beta = 1.0, 32 instances x 2 replicas
    "ea8b": dict(L=8, chi=16, beta=1.0, n_inst=32, n_rep=2),
    # the same at beta = 1.5, the low temperature of the paper's main scaling figure
    "ea8h": dict(L=8, chi=16, beta=1.5, n_inst=32, n_rep=2),
    # a truncating proposal (chi = 2 on 16-wide layers), where MH rejects and several candidates per
    # environment pay: 16^3 +-J, beta = 1.0, 64 instances x 2 replicas
    "ea16t": dict(L=16, chi=2, beta=1.0, n_inst=64, n_rep=2),
    # heterogeneous batch: Gaussian couplings, chain k has L = Ls[k % 3],
    # chi = chis[(k // 3) % 3] and beta drawn uniformly in [0.5, 1.5]
    # 3-state Potts, 64^3, uniform J = 1 at beta = 0.5505 (near the transition), chi = 32: 4 chains
    # started ordered (all state 0) and 4 from uniform random states
    "potts64": dict(potts=True, L=64, chi=32, beta=0.5505, n_ordered=4, n_random=4),
    "c3": dict(mixed=True, n_chains=512, Ls=(16, 24, 32), chis=(16, 32, 64), built_chis=(16, 32, 64),
               beta_range=(0.5, 1.5)),
}
PHILOX_SEED = 20250928
# HBM bytes per contraction launch, measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
# (scaled by a plain copy of known size); valid only for the kernel sources it was
# taken on, identified by their hash
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "contract_kernel_ea32_hbm.md")
KERNEL_SOURCES = ["contract_kernel.h", "contract.hip", "device_common.h", "tnmc_internal.h"]


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and whitespace removed."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_23945_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(workload: str, choice=None, path: str = TRAFFIC_FILE):
    """Bytes per launch from the committed counter summary, or None when it is
    missing, for another workload, taken on different kernel sources, or (with
    choice, the autotuner's [{"engine", "layout"}] for the workload's one
    class) taken on another product engine or tile layout than this run's."""
    try:
        with open(path) as fh:
            kv = dict(line.split(":", 1) for line in fh if line.startswith("- ") and ":" in line)
    except OSError:
        return None
    kv = {k[2:].strip(): v.strip().strip("`") for k, v in kv.items()}
    if kv.get("workload") != workload or kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if choice is not None:
        if len(choice) != 1 or any(kv.get(k) != choice[0].get(k) for k in ("engine", "layout")):
            return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def build_inputs(name: str):
    """Single-lattice workloads: (cfg, J[n_inst], spins[n_chains], instance of each chain, pairs, betas)."""
    cfg = WORKLOADS[name]
    L, n_inst, n_rep = cfg["L"], cfg["n_inst"], cfg["n_rep"]
    J = np.stack([synth.couplings_pm_j(L, L, L, i) for i in range(n_inst)])
    spins = np.stack([synth.spins_random(L, L, L, 1000 * i + j) for i in range(n_inst) for j in range(n_rep)])
    inst = np.array([i for i in range(n_inst) for _ in range(n_rep)], dtype=np.int32)
    pairs = np.array([[n_rep * i, n_rep * i + 1] for i in range(n_inst)], dtype=np.int32) if n_rep == 2 else None
    betas = np.full(n_inst * n_rep, cfg["beta"])
    return cfg, J, spins, inst, pairs, betas


def build_groups(name: str):
    """The workload as a list of lattices: dicts with L, chi, J, spins, inst, pairs, betas."""
    cfg = WORKLOADS[name]
    if cfg.get("potts"):
        L = cfg["L"]
        n = cfg["n_ordered"] + cfg["n_random"]
        spins = np.stack([synth.spins_ordered(L, L, L, 3)] * cfg["n_ordered"] +
                         [synth.spins_random(L, L, L, 1000 + c, 3) for c in range(cfg["n_random"])])
        return [dict(L=L, chi=cfg["chi"], d=3, J=synth.couplings_uniform(L, L, L)[None], spins=spins,
                     inst=np.zeros(n, dtype=np.int32), pairs=None, betas=np.full(n, cfg["beta"]))]
    if not cfg.get("mixed"):
        _, J, spins, inst, pairs, betas = build_inputs(name)
        return [dict(L=cfg["L"], chi=cfg["chi"], J=J, spins=spins, inst=inst, pairs=pairs, betas=betas)]
    all_betas = synth.betas_uniform(cfg["n_chains"], *cfg["beta_range"], seed=PHILOX_SEED)
    by_class = {}
    for k in range(cfg["n_chains"]):
        L, chi = cfg["Ls"][k % 3], cfg["chis"][(k // 3) % 3]
        if chi in cfg["built_chis"]:
            by_class.setdefault((L, chi), []).append(k)
    groups = []
    for (L, chi), ks in sorted(by_class.items()):
        J = np.stack([synth.couplings_gauss(L, L, L, k) for k in ks])
        spins = np.stack([synth.spins_random(L, L, L, 1000 * k + 1) for k in ks])
        groups.append(dict(L=L, chi=chi, J=J, spins=spins, inst=np.arange(len(ks), dtype=np.int32), pairs=None,
                           betas=all_betas[ks]))
    return groups


def make_lattice(name: str, record_capacity: int = 0):
    """Single-lattice workloads: (lattice, cfg, J, spins, inst, betas)."""
    import paper_2509_23945_amd as tn
    cfg, J, spins, inst, pairs, betas = build_inputs(name)
    L = cfg["L"]
    lat = tn.tnmc_lattice_init(Lx=L, Ly=L, Lz=L, d=2, chi=cfg["chi"], J=J, beta=betas, spins=spins,
                               chain_instance=inst, seed=PHILOX_SEED, pairs=pairs,
                               record_capacity=record_capacity)
    return lat, cfg, J, spins, inst, betas


def make_lattices(name: str, record_capacity: int = 0, precision: int = 0, n_candidates: int = 1):
    import paper_2509_23945_amd as tn
    groups = build_groups(name)
    lats = [tn.tnmc_lattice_init(Lx=g["L"], Ly=g["L"], Lz=g["L"], d=g.get("d", 2), chi=g["chi"], J=g["J"],
                                 beta=g["betas"],
                                 spins=g["spins"], chain_instance=g["inst"], seed=PHILOX_SEED, pairs=g["pairs"],
                                 record_capacity=record_capacity, precision=precision,
                                 n_candidates=n_candidates) for g in groups]
    return lats, groups


def time_form(tn, lats, warmup: int, steps: int, stream, graph: bool = False):
    """Warm up, tune the contraction on the warmed-up states (untimed), then
    time `steps` sweeps of every lattice; returns (seconds, stats)."""
    import torch
    if warmup:
        tn.tnmc_sweep(lats, warmup, sweep_offset=0, stream=stream)
    tn.tnmc_autotune_now(lats, stream=stream)
    for lat in lats:
        tn.tnmc_timeseries_reset(lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # long runs go in chunks of 500 sweeps with a progress line after each
    st = None
    done = 0
    while done < steps:
        k = min(500, steps - done)
        if graph:
            # HIP-graph replays: no per-kernel events; the launch counts and flops come back, the durations stay 0
            part = tn.tnmc_sweep_graph(lats, k, sweep_offset=warmup + done, record=True, stream=stream)
        else:
            part = tn.tnmc_sweep(lats, k, sweep_offset=warmup + done, record=True, time_kernels=True, stream=stream)
        st = part if st is None else {key: st[key] + part[key] for key in st}
        done += k
        if steps > 500:
            print(f"[bench] {done}/{steps} sweeps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


_INPUTS = {}


def _worker_inputs(name: str):
    if name not in _INPUTS:
        _INPUTS[name] = build_groups(name)
    return _INPUTS[name]


def _oracle_warm(name: str) -> int:
    """Imports the oracle and builds the inputs in a pool worker (not timed)."""
    from oracle import chain  # noqa: F401
    _worker_inputs(name)
    return os.getpid()


def _oracle_task(args):
    """One slice update of the workload by the FP64 oracle (cpu_baseline leg)."""
    name, gi, chain, z = args
    from threadpoolctl import threadpool_limits
    from oracle import chain as ochain
    g = _worker_inputs(name)[gi]
    with threadpool_limits(1):
        t = time.perf_counter()
        ochain.propose(g["J"][g["inst"][chain]], g["spins"][chain], z, g["betas"][chain], g["chi"], g.get("d", 2),
                       seed=PHILOX_SEED, chain=chain, sweep=0)
        return time.perf_counter() - t


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name: str, per_worker: int = 6):
    """The FP64 oracle on the host cores over a bounded sample of the workload's slice updates
    (spread over its lattices in proportion to their share of slice updates)."""
    import multiprocessing as mp
    groups = build_groups(name)
    cores = max(1, len(os.sched_getaffinity(0)))
    n = cores * per_worker
    weights = np.array([len(g["inst"]) * g["L"] for g in groups], dtype=float)
    counts = np.floor(weights / weights.sum() * n).astype(int)
    counts[np.argmax(weights)] += n - counts.sum()
    tasks = []
    for gi, (g, c) in enumerate(zip(groups, counts)):
        nch = len(g["inst"])
        tasks += [(name, gi, k % nch, (2 * k) % g["L"]) for k in range(c)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_warm, [name] * cores, chunksize=1)
        t0 = time.perf_counter()
        per = pool.map(_oracle_task, tasks, chunksize=per_worker)
        wall = time.perf_counter() - t0
    shapes = ", ".join(f"L={g['L']} chi={g['chi']}: {c}" for g, c in zip(groups, counts) if c)
    return {"value": len(tasks) / wall, "unit": "slice updates/s", "cores": cores, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"{len(tasks)} slice updates of the {name} workload ({shapes}), "
                      f"{per_worker} per worker process, numpy single-threaded; wall {wall:.1f} s, "
                      f"{np.sum(per):.1f} s of CPU work, mean {np.mean(per):.2f} s per update per core"}


def indep_of(lat, sweep_s):
    """(independent samples/s, tau_int of the overlap q) from the lattice's record, or Nones when it is
    shorter than 100 sweeps or has no replica pairs."""
    import paper_2509_23945_amd as tn
    from paper_2509_23945_amd import analysis
    _, _, q = tn.tnmc_timeseries(lat)
    if q.shape[0] < 100 or q.shape[1] == 0:
        return None, None
    indep, tau, _ = analysis.independent_samples_per_second(q, sweep_s)
    return indep, tau


# forward flops per site on the taps the masks keep: the first layer sees the 4
# condition channels through all 9 taps and the spin channel through the 4 taps
# of the type-A mask; the four hidden 32 -> 32 layers and the 32 -> 1 output
# keep 5 taps (type-B mask).  Training = forward + input gradient + weight gradient.
NN_FLOPS_PER_SITE = 2 * (32 * (4 * 9 + 1 * 4) + 4 * 32 * 32 * 5 + 32 * 5)
FP32_PEAK_TFLOPS = 157.3


def learned_form(tn, lat, group, args, stream, fp64_value, sweep0, tau_on, fp64_indep):
    """The learned proposal on the same chains: a training set of (condition,
    layer) pairs taken after each of a number of further FP64 TN sweeps (each
    layer then is a fresh draw of the TN proposal given its neighbours),
    minibatch Adam, a calibration window that freezes the TN fallback of layers
    whose acceptance stays below 5%, then timed sweeps."""
    import torch
    L = group["L"]
    n_chains = len(group["inst"])
    per_sweep = n_chains * L
    K = args.learned_data_sweeps
    n = K * per_sweep
    cond = torch.empty((n, 4, L, L), dtype=torch.float32, device="cuda")
    spins = torch.empty((n, L, L), dtype=torch.int8, device="cuda")
    print(f"[bench] learned proposal: {K} TN sweeps -> {n} training pairs", file=sys.stderr, flush=True)
    for k in range(K):
        tn.tnmc_sweep([lat], 1, sweep_offset=sweep0 + k, stream=stream)
        tn.tnmc_nn_dataset(lat, cond.data_ptr() + k * per_sweep * 4 * L * L * 4,
                           spins.data_ptr() + k * per_sweep * L * L, stream=stream)
    torch.cuda.synchronize()
    # shuffle the pairs once (seeded): minibatches then mix sweeps, chains and layers
    perm = torch.from_numpy(np.random.Generator(np.random.PCG64(5)).permutation(n)).cuda()
    cond, spins = cond[perm].contiguous(), spins[perm].contiguous()
    net = tn.tnmc_nn_create(None, seed=1)
    batch = 256
    loss0 = tn.tnmc_nn_loss_grad(net, cond.data_ptr(), spins.data_ptr(), batch, L, L, stream=stream)
    print(f"[bench] learned proposal: training {args.learned_epochs} epochs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = tn.tnmc_nn_train(net, cond.data_ptr(), spins.data_ptr(), n, L, L, args.learned_epochs, batch,
                            args.learned_lr, stream=stream)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    train_flops = 3.0 * NN_FLOPS_PER_SITE * L * L * n * args.learned_epochs
    del cond, spins
    # every layer on the learned proposal: its own rate and acceptance; these
    # sweeps are also the calibration window of the fallback
    sw = sweep0 + K
    tn.tnmc_nn_set_fallback(lat, None)
    tn.tnmc_nn_counts_reset(lat)
    tn.tnmc_timeseries_reset(lat)
    print(f"[bench] learned proposal: timing {args.steps} sweeps, every layer learned", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_nn = tn.tnmc_nn_sweep([lat], net, args.steps, sweep_offset=sw, record=True, time_kernels=True, stream=stream)
    torch.cuda.synchronize()
    secs_nn = time.perf_counter() - t0
    indep_nn = indep_of(lat, secs_nn / args.steps)
    sw += args.steps
    n_fb = tn.tnmc_nn_calibrate_fallback(lat, 0.05)
    print(f"[bench] learned proposal: timing {args.steps} sweeps ({n_fb} of {per_sweep} layers on the TN fallback)",
          file=sys.stderr, flush=True)
    tn.tnmc_nn_counts_reset(lat)
    tn.tnmc_timeseries_reset(lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = tn.tnmc_nn_sweep([lat], net, args.steps, sweep_offset=sw, record=True, time_kernels=True, stream=stream)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    indep = indep_of(lat, secs / args.steps)
    sw += args.steps
    prop, acc = tn.tnmc_nn_counts(lat)
    nn_prop = int(prop.sum())
    value = args.steps * per_sweep / secs
    # log q gap on the current layers of a few (chain, layer) pairs: log q_TN - log q_theta
    gaps = []
    cur = [tn.tnmc_get_spins(lat, c) for c in range(min(n_chains, 4))]
    for c, sc in enumerate(cur):
        for z in range(0, L, 4):
            gaps.append(tn.tnmc_slice_logq(lat, c, z, sc[z]) - tn.tnmc_nn_slice_logq(lat, net, c, z, sc[z]))
    leg = None
    if tau_on:
        leg = tau_leg(tn, lat, lambda k, off: tn.tnmc_nn_sweep([lat], net, k, sweep_offset=sw + off, record=True,
                                                               stream=stream),
                      "learned", args.tau_seconds, args.tau_sweeps)
        indep = (leg["indep_samples_per_s"], leg["tau_int_q"])
    return {
        "form": "masked-conv autoregressive proposal (6 layers, 32 channels, BF16 weights from FP32 masters, FP32 "
                "arithmetic and accumulation) with exact log q, "
                "MH per main text Eq. 1, TN fallback frozen after a calibration window (the learned-only sweeps; acceptance < 5%)",
        "value": value, "unit": "slice updates/s", "ms_per_step": secs / args.steps * 1e3,
        "vs_fp64": value / fp64_value,
        "acceptance": st["accepted"] / max(1, st["proposed"]),
        "acceptance_learned": float(acc.sum()) / max(1, nn_prop),
        "learned_updates_per_step": nn_prop / args.steps, "fallback_layers": n_fb,
        "tau_int_q": indep[1], "indep_samples_per_s": indep[0], "tau_leg": leg,
        "indep_vs_fp64": (indep[0] / fp64_indep) if (indep[0] and fp64_indep) else None,
        "learned_only": {"value": args.steps * per_sweep / secs_nn, "unit": "slice updates/s",
                         "ms_per_step": secs_nn / args.steps * 1e3,
                         "acceptance": st_nn["accepted"] / max(1, st_nn["proposed"]),
                         "sampler_ms_per_launch": st_nn["sample_ms"] / max(1, st_nn["sample_launches"]),
                         "tau_int_q": indep_nn[1], "indep_samples_per_s": indep_nn[0],
                         "tasks_per_launch": per_sweep // 2},
        "sample_ms_per_step": st["sample_ms"] / args.steps, "contract_ms_per_step": st["contract_ms"] / args.steps,
        "logq_gap_tn_minus_learned": {"mean": float(np.mean(gaps)), "median": float(np.median(gaps)),
                                      "layers": len(gaps)},
        "training": {"pairs": n, "epochs": args.learned_epochs, "batch": batch, "lr": args.learned_lr, "seconds": train_s,
                     "loss_first_batch_nats": loss0, "loss_last_batch_nats": last,
                     "tflops": train_flops / train_s / 1e12,
                     "frac_fp32_peak": train_flops / train_s / 1e12 / FP32_PEAK_TFLOPS},
        "numeric_faults": st["numeric_faults"],
    }


def autotune_report(tn, groups, precision):
    """The contraction autotuner's choice per (d, chi) class of the workload
    (product engine and tile layout) with the median trial durations."""
    rep = []
    for d_, c_ in sorted({(g.get("d", 2), g["chi"]) for g in groups}):
        lay, eng, ms = tn.tnmc_autotune_choice(d_, c_, precision)
        if eng >= 0:
            rep.append({"d": d_, "chi": c_, "engine": "mfma" if eng else "valu", "layout": "full" if lay else "compact",
                        "trial_ms": {"valu_compact": ms[0], "valu_full": ms[1], "mfma_compact": ms[2],
                                     "mfma_full": ms[3]}})
    return rep


def copy_probe() -> None:
    """A plain device-to-device copy of 64 MiB, three times: profiled with
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, it scales those counters to bytes
    (each dispatch reads and writes exactly 64 MiB)."""
    import torch
    n = 64 * 1024 * 1024 // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied", a.numel() * 8, "bytes x 3", flush=True)


def tau_leg(tn, lat, run, label: str, budget_s: float, max_sweeps: int, chunk: int = 100, every: int = 500):
    """Runs the form's own sweeps (run(k, offset) does k recorded sweeps) for
    about budget_s seconds (at most max_sweeps), then estimates tau_int of the
    replica overlap q (SM S3; Sokal window) from the recorded series and the
    independent samples per second n_pairs / (tau * t_s) (main text: t_int =
    tau_int * t_s)."""
    import torch
    from paper_2509_23945_amd import analysis
    tn.tnmc_timeseries_reset(lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < max_sweeps:
        k = min(chunk, max_sweeps - done)
        run(k, done)
        done += k
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if done % every == 0 or el > budget_s:
            print(f"[bench] tau leg ({label}): {done} sweeps, {el:.0f} s", file=sys.stderr, flush=True)
        if el > budget_s:
            break
    secs = time.perf_counter() - t0
    _, _, q = tn.tnmc_timeseries(lat)
    out = {"sweeps": done, "seconds": secs, "ms_per_sweep": secs / max(1, done) * 1e3, "tau_int_q": None,
           "window": None, "sweeps_per_tau": None, "tau_converged": False, "indep_samples_per_s": None}
    if q.shape[0] >= 20 and q.shape[1] > 0:
        tau, W = analysis.tau_int(q.T)
        out.update(tau_int_q=tau, window=W, sweeps_per_tau=q.shape[0] / tau, tau_converged=q.shape[0] >= 50 * tau,
                   indep_samples_per_s=q.shape[1] / (tau * secs / done))
    return out


def superspin_leg(tn, args, stream, chi: int = 8):
    """TNMCMC-2 (SM S2.B: layers z0, z0 + 1 merged into 4-state superspins,
    updated in three phases z0 mod 3) on the single-lattice workload's
    couplings, betas and initial spins at bond dimension chi (the composite
    path's largest), with TNMCMC-1 at the same chi on the same inputs beside it:
    updates/s, acceptance, and the composite contraction's flops per launch
    over its HIP-event duration.  A composite task costs several times a
    TNMCMC-1 task (left ranks near d * chi), so the leg times a few sweeps, one
    call per sweep with a progress line after each; tau_int of the overlap is
    estimated only when asked for (--tnmcmc2-tau-seconds)."""
    import torch
    cfg, J, spins, inst, pairs, betas = build_inputs(args.workload)
    L = cfg["L"]
    n_chains = len(inst)
    steps, warm = args.tnmcmc2_steps, 1
    budget = args.tnmcmc2_tau_seconds
    tau_sweeps = args.tau_sweeps if budget > 0 else 0
    cap = warm + steps + tau_sweeps

    def lattice():
        return tn.tnmc_lattice_init(Lx=L, Ly=L, Lz=L, d=2, chi=chi, J=J, beta=betas, spins=spins,
                                    chain_instance=inst, seed=PHILOX_SEED, pairs=pairs, record_capacity=cap)

    out = {"chi": chi, "workload": f"{args.workload} inputs at chi={chi}"}
    # TNMCMC-2: each composite update proposes two layers at once
    print(f"[bench] TNMCMC-2 (superspins, chi={chi}): {warm} warm-up sweep, timing {steps} sweeps", file=sys.stderr,
          flush=True)
    lat = lattice()
    t0 = time.perf_counter()
    tn.tnmc_sweep_superspin([lat], warm, stream=stream)
    torch.cuda.synchronize()
    print(f"[bench] TNMCMC-2 warm-up sweep: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    tn.tnmc_timeseries_reset(lat)
    st = None
    t0 = time.perf_counter()
    for k in range(steps):
        part = tn.tnmc_sweep_superspin([lat], 1, sweep_offset=warm + k, record=True, time_kernels=True, stream=stream)
        st = part if st is None else {key: st[key] + part[key] for key in st}
        print(f"[bench] TNMCMC-2 sweep {k + 1}/{steps}: {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    per_sweep = n_chains * (L - 1)
    launches = max(1, st["contract_launches"])
    avg_s = st["contract_ms"] / 1e3 / launches
    achieved = st["contract_flops"] / launches / avg_s / 1e12 if avg_s > 0 else None
    out["tnmcmc2"] = {
        "value": steps * per_sweep / secs, "unit": "composite updates/s",
        "layer_updates_per_s": 2 * steps * per_sweep / secs, "steps": steps,
        "composite_updates_per_sweep": per_sweep, "ms_per_sweep": secs / steps * 1e3,
        "acceptance": st["accepted"] / max(1, st["proposed"]), "numeric_faults": st["numeric_faults"],
        "contract_ms_per_sweep": st["contract_ms"] / steps, "sample_ms_per_sweep": st["sample_ms"] / steps,
        "roofline": {"bound": "alu", "kernel": f"contract_kernel<4,{chi}>", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
                     "avg_launch_ms": avg_s * 1e3, "launches": launches,
                     "tasks_per_launch": steps * per_sweep / launches,
                     "flops_per_task": st["contract_flops"] / (steps * per_sweep)}}
    if tau_sweeps:
        base = warm + steps
        out["tnmcmc2"]["tau_leg"] = tau_leg(
            tn, lat, lambda k, off: tn.tnmc_sweep_superspin([lat], k, sweep_offset=base + off, record=True,
                                                            stream=stream),
            "TNMCMC-2", budget, tau_sweeps, chunk=1, every=10)
    tn.tnmc_lattice_free(lat)
    # TNMCMC-1 at the same chi
    print(f"[bench] TNMCMC-1 at chi={chi}: timing {args.steps} sweeps", file=sys.stderr, flush=True)
    lat1 = lattice()
    secs1, st1 = time_form(tn, [lat1], args.warmup, args.steps, stream)
    out["tnmcmc1_same_chi"] = {
        "value": args.steps * n_chains * L / secs1, "unit": "slice updates/s", "ms_per_sweep": secs1 / args.steps * 1e3,
        "acceptance": st1["accepted"] / max(1, st1["proposed"]), "numeric_faults": st1["numeric_faults"],
        "contract_ms_per_sweep": st1["contract_ms"] / args.steps,
        "flops_per_task": st1["contract_flops"] / (args.steps * n_chains * L)}
    out["layer_updates_ratio_tnmcmc2_over_tnmcmc1"] = (out["tnmcmc2"]["layer_updates_per_s"] /
                                                       out["tnmcmc1_same_chi"]["value"])
    if tau_sweeps:
        base = args.warmup + args.steps
        out["tnmcmc1_same_chi"]["tau_leg"] = tau_leg(
            tn, lat1, lambda k, off: tn.tnmc_sweep([lat1], k, sweep_offset=base + off, record=True, stream=stream),
            "TNMCMC-1 same chi", budget, tau_sweeps)
        a = out["tnmcmc2"]["tau_leg"]["indep_samples_per_s"]
        b = out["tnmcmc1_same_chi"]["tau_leg"]["indep_samples_per_s"]
        out["indep_ratio_tnmcmc2_over_tnmcmc1"] = a / b if a and b else None
    tn.tnmc_lattice_free(lat1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ea32", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reduced", action="store_true", help="skip the FP32-environment form")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal form")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the FP64-storage run at the reduced form's rank cut-off")
    ap.add_argument("--learned-data-sweeps", type=int, default=98,
                    help="TN sweeps whose layers form the training set of the learned proposal")
    ap.add_argument("--learned-epochs", type=int, default=5)
    ap.add_argument("--learned-lr", type=float, default=2e-3)
    ap.add_argument("--tau-sweeps", type=int, default=1500,
                    help="sweeps per form of the tau_int leg (the same for every form; 0 skips the leg)")
    ap.add_argument("--tau-seconds", type=float, default=120.0,
                    help="wall-time cap per form of the tau_int leg")
    ap.add_argument("--candidates", type=int, default=1,
                    help="candidates drawn per layer environment and chained by MH (every TN form)")
    ap.add_argument("--graph", action="store_true",
                    help="time the FP64 sweeps as HIP-graph replays (tnmc_sweep_graph) instead of eager launches")
    ap.add_argument("--engine", choices=("auto", "valu", "mfma"), default="auto",
                    help="contraction products: chosen by the autotuner (default) or pinned")
    ap.add_argument("--no-tnmcmc2", action="store_true",
                    help="skip the TNMCMC-2 (superspin) leg and its TNMCMC-1 comparison at the same chi")
    ap.add_argument("--tnmcmc2-steps", type=int, default=3,
                    help="timed sweeps of the TNMCMC-2 leg (one warm-up sweep before them)")
    ap.add_argument("--tnmcmc2-tau-seconds", type=float, default=0.0,
                    help="wall-time cap of each tau_int run of the TNMCMC-2 leg (0, the default, skips them)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 64 MiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "design only: chains are independent, so each GPU would run its own share of them", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2509_23945_amd as tn
    from paper_2509_23945_amd import analysis

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    if args.engine != "auto":
        tn.tnmc_autotune_pin(-1, 1 if args.engine == "mfma" else 0)
    tau_on = args.tau_sweeps > 0
    cap = max(args.steps, args.tau_sweeps if tau_on else 0)
    lats, groups = make_lattices(args.workload, record_capacity=cap, n_candidates=args.candidates)
    tau_on = tau_on and len(lats) == 1 and groups[0]["pairs"] is not None
    cfg = WORKLOADS[args.workload]
    n_chains = sum(len(g["inst"]) for g in groups)
    updates_per_sweep = sum(len(g["inst"]) * g["L"] for g in groups)
    print(f"[bench] workload {args.workload}: {n_chains} chains in {len(lats)} lattices, "
          f"{updates_per_sweep} slice updates per sweep, warmup {args.warmup}", file=sys.stderr, flush=True)
    print(f"[bench] timing {args.steps} sweeps", file=sys.stderr, flush=True)
    secs, st = time_form(tn, lats, args.warmup, args.steps, stream, graph=args.graph)
    value = args.steps * updates_per_sweep / secs

    # algorithmic flops: textbook QR/SVD/GEMM counts at the bond dimensions each task used,
    # accumulated by the kernel; the fixed-chi model is reported beside it
    launches = max(1, st["contract_launches"])
    tasks_per_sweep = sum(len(g["inst"]) * g["L"] for g in groups)
    avg_launch_s = st["contract_ms"] / 1e3 / launches   # 0 for graph replays (no per-kernel events)
    flops_per_launch = st["contract_flops"] / launches
    achieved = flops_per_launch / avg_launch_s / 1e12 if avg_launch_s > 0 else None
    kernels = sorted({(g.get("d", 2), g["chi"] if g["chi"] > 16 else 16) for g in groups})
    flops_model = sum(tn.tnmc_flop_model(g["L"], g["L"], g.get("d", 2), g["chi"])[0] * len(g["inst"]) * g["L"]
                      for g in groups) / tasks_per_sweep
    # the per-launch rate (counted flops of a launch / its HIP-event duration)
    # is the roofline figure; the chip-level rate (all flops / wall time, the
    # sampler included) is reported beside it, and so is the rate a fixed-chi
    # implementation would need for the same launch time (the textbook model
    # at full bond dimension, work the rank-revealing path does not do)
    achieved_chip = st["contract_flops"] / secs / 1e12
    tasks_per_launch = args.steps * tasks_per_sweep / launches
    model_rate = flops_model * tasks_per_launch / avg_launch_s / 1e12 if avg_launch_s > 0 else None
    tune = autotune_report(tn, groups, tn.TNMC_FP64)
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
                "traffic": measured_traffic(args.workload, tune),
                "kernel": " + ".join(f"contract_kernel<{d},{c}>" for d, c in kernels),
                "avg_launch_ms": avg_launch_s * 1e3, "launches": launches,
                "achieved_chip": achieved_chip, "frac_chip": achieved_chip / FP64_PEAK_TFLOPS,
                "flops_per_task": st["contract_flops"] / (args.steps * tasks_per_sweep),
                "flops_per_task_fixed_chi": flops_model,
                "fixed_chi_model_rate": model_rate,
                "fixed_chi_model_frac": model_rate / FP64_PEAK_TFLOPS if model_rate else None,
                "tasks_per_launch": tasks_per_launch}

    next_sweep = args.warmup + args.steps   # sweep counters are never reused on a chain
    tau_fp64 = None
    if tau_on:
        # the FP64 chains go on: tau_int of the overlap and independent samples/s
        base = next_sweep
        tau_fp64 = tau_leg(tn, lats[0], lambda k, off: tn.tnmc_sweep(lats, k, sweep_offset=base + off, record=True,
                                                                      stream=stream),
                           "FP64", args.tau_seconds, args.tau_sweeps)
        next_sweep += tau_fp64["sweeps"]
    indep = tau_fp64["indep_samples_per_s"] if tau_fp64 else None
    tau = tau_fp64["tau_int_q"] if tau_fp64 else None

    if cfg.get("potts"):
        desc = (f"3D 3-state Potts {cfg['L']}^3 open BC, J=1, beta={cfg['beta']}, chi={cfg['chi']}, "
                f"{cfg['n_ordered']} chains started ordered + {cfg['n_random']} from random states")
        data = "synthetic (uniform couplings, ordered and seeded random initial states)"
    elif cfg.get("mixed"):
        desc = (f"heterogeneous batch, Gaussian J (2^-20 grid), open BC: chain k of {cfg['n_chains']} has "
                f"L={list(cfg['Ls'])}[k%3], chi={list(cfg['chis'])}[(k//3)%3], beta uniform in "
                f"{list(cfg['beta_range'])}" + (f"; {cfg['n_chains'] - n_chains} chains left out" if n_chains < cfg['n_chains'] else ""))
        data = "synthetic (seeded Gaussian couplings, seeded betas, random initial spins)"
    else:
        L = cfg["L"]
        desc = (f"3D EA +-J {L}^3 open BC, beta={cfg['beta']}, chi={cfg['chi']}, "
                f"{cfg['n_inst']} instances x {cfg['n_rep']} replicas")
        data = "synthetic (seeded +-J couplings, random initial spins)"
    out = {
        "metric": "slice updates/s (TNMCMC-1 slice proposal, FP64 plain)",
        "value": value,
        "unit": "slice updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": data,
        "config": {"workload": desc, "chains": n_chains, "slice_updates_per_step": updates_per_sweep,
                   "candidates_per_environment": args.candidates, "parallelism": "none (1 GPU)"},
        "acceptance": st["accepted"] / max(1, st["proposed"]),
        "numeric_faults": st["numeric_faults"],
        "contract_retries": st["contract_retries"],
        "contract_ms_per_step": st["contract_ms"] / args.steps,
        "sample_ms_per_step": st["sample_ms"] / args.steps,
        "tau_int_q": tau,
        "indep_samples_per_s": indep,
        "tau_leg": tau_fp64,
        "roofline": roofline,
    }
    out["autotune"] = tune
    if not args.no_reduced:
        # the reduced-precision form on the same inputs: FP32 environments, rank
        # cut-off at FP32 resolution, FP64 factorisations, log q and MH
        print(f"[bench] reduced-precision form: timing {args.steps} sweeps", file=sys.stderr, flush=True)
        lats32, _ = make_lattices(args.workload, record_capacity=cap, precision=tn.TNMC_FP32,
                                  n_candidates=args.candidates)
        secs32, st32 = time_form(tn, lats32, args.warmup, args.steps, stream)
        v32 = args.steps * updates_per_sweep / secs32
        out["reduced_precision"] = {
            "form": "environments stored in FP32, rank cut-off 1e-6 (the cut-off, not the storage, gives the speed-up: see ablation); products M, AT, C, Y on the engine the autotuner "
                    "picks (FP32 MFMA operands and accumulation, or FP64 VALU); factorisations, log q, dE, MH in FP64",
            "autotune": autotune_report(tn, groups, tn.TNMC_FP32),
            "value": v32, "unit": "slice updates/s", "ms_per_step": secs32 / args.steps * 1e3,
            "vs_fp64": v32 / value, "acceptance": st32["accepted"] / max(1, st32["proposed"]),
            "tau_int_q": None, "indep_samples_per_s": None,
            "numeric_faults": st32["numeric_faults"],
            "contract_ms_per_step": st32["contract_ms"] / args.steps,
            "sample_ms_per_step": st32["sample_ms"] / args.steps}
        if tau_on:
            base32 = args.warmup + args.steps
            leg = tau_leg(tn, lats32[0], lambda k, off: tn.tnmc_sweep(lats32, k, sweep_offset=base32 + off,
                                                                       record=True, stream=stream),
                          "reduced", args.tau_seconds, args.tau_sweeps)
            out["reduced_precision"].update(tau_int_q=leg["tau_int_q"], indep_samples_per_s=leg["indep_samples_per_s"],
                                            tau_leg=leg)
            if indep and leg["indep_samples_per_s"]:
                out["reduced_precision"]["indep_vs_fp64"] = leg["indep_samples_per_s"] / indep
        for lat in lats32:
            tn.tnmc_lattice_free(lat)
        if not args.no_ablation:
            # which half of the reduced form buys its speed: the same 1e-6 rank
            # cut-off with FP64-stored environments (another q, MH still exact)
            print(f"[bench] ablation: FP64 storage, rank cut-off 1e-6: timing {args.steps} sweeps", file=sys.stderr,
                  flush=True)
            tn.tnmc_debug_set(3, 6)
            try:
                lats_ab, _ = make_lattices(args.workload, record_capacity=cap, precision=tn.TNMC_FP64,
                                           n_candidates=args.candidates)
                secs_ab, st_ab = time_form(tn, lats_ab, args.warmup, args.steps, stream)
            finally:
                tn.tnmc_debug_set(3, 0)
            v_ab = args.steps * updates_per_sweep / secs_ab
            out["reduced_precision"]["ablation"] = {
                "fp64_storage_cut_1e-6": {"value": v_ab, "ms_per_step": secs_ab / args.steps * 1e3,
                                          "contract_ms_per_step": st_ab["contract_ms"] / args.steps,
                                          "acceptance": st_ab["accepted"] / max(1, st_ab["proposed"]),
                                          "numeric_faults": st_ab["numeric_faults"]},
                "fp32_storage_cut_1e-6": {"value": v32, "ms_per_step": secs32 / args.steps * 1e3},
                "fp64_storage_cut_1e-15": {"value": value, "ms_per_step": secs / args.steps * 1e3},
                "speedup_from_cut": v_ab / value, "speedup_from_fp32_storage": v32 / v_ab}
            for lat in lats_ab:
                tn.tnmc_lattice_free(lat)
    if not args.no_learned and len(lats) == 1 and groups[0].get("d", 2) == 2:
        out["learned_proposal"] = learned_form(tn, lats[0], groups[0], args, stream, value, next_sweep,
                                               tau_on, indep)
    if not args.no_tnmcmc2 and not cfg.get("potts") and not cfg.get("mixed"):
        out["superspin"] = superspin_leg(tn, args, stream)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, per_worker=1 if cfg.get("potts") else 6)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
