"""Shared pieces of the GPU parity tests: building a lattice on the device from
the seeded synthetic inputs and comparing one proposal with the oracle's."""
from __future__ import annotations

import os
import sys

import numpy as np

import paper_2509_23945_amd as tn
import synth
from oracle import chain as ochain

# log q tolerance on the FP64 path: 1e-10 absolute, relaxed to 1e-10 relative
# for |log q| > 1.  On full-size 32x32 layers (|log q| ~ 10^3) two independent
# factorisation codes differ by up to ~2e-10 absolute (~1e-13 relative); the
# largest absolute and relative differences observed over every parity case
# and all 512 tasks of a full-size half-sweep are printed at the end of a GPU
# session.
LOGQ_TOL = 1e-10
# reduced-precision form (FP32 environments): log q within 1e-4 relative of the
# FP64 oracle's log q of the same configuration
LOGQ_TOL_REDUCED = 1e-4
TIE = 1e-9


# Observed discrepancies, printed at the end of a GPU session (conftest):
# (label, case, |d log q|, |d log q| / max(1, |log q|)) and per-site draw
# margins of the reduced form.
OBSERVED_LOGQ = []
OBSERVED_MARGINS = []


def logq_close(a: float, b: float, label: str = "", case=None) -> bool:
    if label:
        OBSERVED_LOGQ.append((label, case, abs(a - b), abs(a - b) / max(1.0, abs(a), abs(b))))
    return abs(a - b) <= LOGQ_TOL * max(1.0, abs(a), abs(b))


def record_margin(label, case, sweep, bad, worst, closest):
    OBSERVED_MARGINS.append((label, case, sweep, bad, worst, closest))


def logq_close_reduced(a: float, b: float) -> bool:
    return abs(a - b) <= LOGQ_TOL_REDUCED * max(1.0, abs(a), abs(b))


def announce(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def make_lattice(Lx, Ly, Lz, d, chi, *, kind="pmj", beta=1.0, seed=0, n_chains=1, init="random",
                 pairs=None, record_capacity=0, philox_seed=12345, precision=tn.TNMC_FP64, n_candidates=1):
    """Couplings (one instance per chain pair) and initial spins from synth; returns
    (lattice handle, J[n_inst], spins[n_chains], betas)."""
    n_inst = max(1, (n_chains + 1) // 2) if pairs is not None else n_chains
    Js = []
    for i in range(n_inst):
        if kind == "pmj":
            Js.append(synth.couplings_pm_j(Lx, Ly, Lz, seed + i))
        elif kind == "gauss":
            Js.append(synth.couplings_gauss(Lx, Ly, Lz, seed + i))
        else:
            Js.append(synth.couplings_uniform(Lx, Ly, Lz))
    J = np.stack(Js)
    spins = []
    for c in range(n_chains):
        if init == "random":
            spins.append(synth.spins_random(Lx, Ly, Lz, 1000 * seed + c + 1, d))
        else:
            spins.append(synth.spins_ordered(Lx, Ly, Lz, d))
    spins = np.stack(spins)
    betas = np.broadcast_to(np.asarray(beta, dtype=np.float64), (n_chains,)).copy()
    inst = np.array([c // 2 if pairs is not None else c for c in range(n_chains)], dtype=np.int32)
    lat = tn.tnmc_lattice_init(Lx=Lx, Ly=Ly, Lz=Lz, d=d, chi=chi, J=J, beta=betas, spins=spins,
                               chain_instance=inst, seed=philox_seed, pairs=pairs,
                               record_capacity=record_capacity, precision=precision, n_candidates=n_candidates)
    return lat, J[inst], spins, betas


def compare_proposal(gpu, ref, margins, case=None):
    """gpu = (s_new, lq_new, lq_old, dE, status); ref = oracle.propose record.
    Returns a dict of discrepancies (empty if identical within the parity bar)
    and whether a near-tie explains a spin mismatch."""
    s_new, lq_new, lq_old, dE, st = gpu
    out = {}
    if dE != ref["dE"] and np.array_equal(s_new, ref["new"]):
        out["dE"] = (dE, ref["dE"])
    if not logq_close(lq_old, ref["logq_old"], "fp64 logq_old", case):
        out["logq_old"] = (lq_old, ref["logq_old"])
    if not np.array_equal(s_new, ref["new"]):
        tie = min(margins) < TIE if margins else False
        out["spins"] = ("near-tie" if tie else "mismatch", int(np.sum(s_new != ref["new"])))
    elif not logq_close(lq_new, ref["logq_new"], "fp64 logq_new", case):
        out["logq_new"] = (lq_new, ref["logq_new"])
    return out


def oracle_propose(J, spins, z, beta, chi, d, *, seed, chain, sweep):
    margins = []
    rec = ochain.propose(J, spins, z, beta, chi, d, seed=seed, chain=chain, sweep=sweep, margins=margins)
    return rec, margins


def have_gpu() -> bool:
    if os.environ.get("TNMC_FORCE_NO_GPU"):
        return False
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


# Reduced-precision draws: a site's drawn state must be the one the FP64
# oracle's conditional (given the GPU's own earlier sites) selects for that
# site's uniform, unless the uniform lies within TIE_REDUCED of a cumulative
# threshold.  The reduced form drops directions below 1e-6 of the largest
# (FP32 resolution), so its site conditionals differ from the FP64 ones by
# about that much; the window is ten times it.
TIE_REDUCED = 1e-5


def sitewise_draw_check(J, spins, z, s_new, beta, chi, d, *, seed, chain, sweep):
    """Per-site check of a drawn layer s_new against the oracle's conditionals
    along the forced walk over s_new.  Returns (log q of s_new under the
    oracle, sites whose state differs from the oracle's pick, the largest
    distance of such a site's uniform to its nearest threshold, the smallest
    distance over all sites)."""
    from oracle import model as omodel
    from oracle import sampler as osampler
    from oracle.philox import PURPOSE_SITE, uniform
    probs = []
    lq = ochain.slice_logq(J, spins, z, s_new, beta, chi, d, site_probs=probs)
    states = omodel.to_states(s_new, d)
    Ly, Lx = states.shape
    bad, worst, closest = 0, 0.0, 1.0
    for y in range(Ly):
        for x in range(Lx):
            p = probs[y * Lx + x]
            U = uniform(seed, chain, sweep, z, PURPOSE_SITE, y * Lx + x)
            margin = float(np.min(np.abs(U - np.cumsum(p)[:-1]))) if p.shape[0] > 1 else 1.0
            closest = min(closest, margin)
            if osampler.draw(p, U) != states[y, x]:
                bad += 1
                worst = max(worst, margin)
    return lq, bad, worst, closest
