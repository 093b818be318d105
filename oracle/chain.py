"""TNMCMC-1 slice update, Metropolis-Hastings decision and sweeps.

Oracle code (test infrastructure only).

* Slice update = SM Alg. 2 (SampleLayer + acceptance): build the layer's network
  from the held layers, draw a new layer s' with q(s'), evaluate q of the
  current layer s, and accept with the Metropolis-Hastings probability.
* Acceptance (main text Eq. 1; SM S1.C; SM S2.A):
      A(s -> s') = min{1, q(s) exp(-beta E(s')) / (q(s') exp(-beta E(s)))}
  with s the current and s' the proposed layer.  (The printed Alg. 2 writes
  the inverse ratio; Eq. 1 and the two SM equations agree with the form above,
  which is the one that leaves the Boltzmann distribution invariant.)
* Schedule (SM S2.A, last paragraph; SM S3.D): all even layers are updated
  with the odd ones held, then all odd layers; one sweep visits every layer once.
* A proposal whose sampling or forced path reported a numeric fault is
  rejected.  Faults are a deterministic function of (held layers, layer
  configuration), so rejecting when either path faults keeps detailed balance.
"""
from __future__ import annotations

import math

import numpy as np

from . import bmps, layer, model, sampler
from .philox import PURPOSE_MH, uniform


def mh_accept(logq_old: float, logq_new: float, beta: float, dE: float, u: float) -> bool:
    """Accept iff u < exp(min(0, log q(old) - log q(new) - beta * (E(new) - E(old))))."""
    lr = logq_old - logq_new - beta * dE
    return bool(u < math.exp(min(0.0, lr)))


def propose(J, spins, z: int, beta: float, chi: int, d: int, *, seed: int = 0,
            chain: int = 0, sweep: int = 0, margins=None):
    """One proposal for layer z without changing the state.

    Returns a dict with the new layer (int8 spins [y, x]), log q(new), log q(old),
    dE = E(new) - E(old), the layer's approximate log Z and the fault flag."""
    F = model.slice_field(J, spins, z, d)
    envs, logscale = bmps.environments(J, F, z, beta, chi, d)
    new, lq_new, f_new = sampler.sample_layer(envs, J, F, z, beta, d, seed=seed,
                                              chain=chain, sweep=sweep, margins=margins)
    old = model.to_states(spins[z], d)
    _, lq_old, f_old = sampler.sample_layer(envs, J, F, z, beta, d, forced=old)
    dE = model.slice_energy(J, F, new, z, d) - model.slice_energy(J, F, old, z, d)
    return {
        "new": model.from_states(new, d),
        "logq_new": lq_new,
        "logq_old": lq_old,
        "dE": dE,
        "fault": bool(f_new or f_old),
        "envs": envs,
        "logscale": logscale,
        "F": F,
    }


def slice_logq(J, spins, z: int, layer_spins, beta: float, chi: int, d: int, site_probs=None) -> float:
    """log q of an arbitrary configuration of layer z given the held layers.
    With ``site_probs`` a list, it receives each site's conditional p(u) along
    the forced walk (rows, then sites within a row)."""
    F = model.slice_field(J, spins, z, d)
    envs, _ = bmps.environments(J, F, z, beta, chi, d)
    _, lq, _ = sampler.sample_layer(envs, J, F, z, beta, d,
                                    forced=model.to_states(layer_spins, d), site_probs=site_probs)
    return lq


def slice_update(J, spins, z: int, beta: float, chi: int, d: int, *, seed: int,
                 chain: int, sweep: int):
    """Propose for layer z and apply the MH decision in place.  Returns the proposal
    record extended with the uniform and the decision."""
    rec = propose(J, spins, z, beta, chi, d, seed=seed, chain=chain, sweep=sweep)
    u = uniform(seed, chain, sweep, z, PURPOSE_MH, 0)
    acc = (not rec["fault"]) and mh_accept(rec["logq_old"], rec["logq_new"], beta, rec["dE"], u)
    if acc:
        spins[z] = rec["new"]
    rec["u_acc"] = u
    rec["accepted"] = acc
    return rec


def slice_update_multi(J, spins, z: int, beta: float, chi: int, d: int, n_candidates: int, *, seed: int,
                       chain: int, sweep: int):
    """Several candidates per environment (main text, "TNMCMC": a batch of
    candidate samples is drawn from the same approximate distribution and one
    is kept).  The environments of layer z are contracted once; then
    n_candidates independence-MH steps with the same q are chained, each
    against the layer's state left by the previous one (main text Eq. 1).
    Candidate k draws its sites with Philox purpose 2k and its MH uniform
    with purpose 2k + 1, so one candidate is slice_update.  Every step is an
    exact MH kernel for the layer's conditional, so their product is too.
    Updates spins in place; returns the number of accepted candidates, the
    log q of the initial and final layer, and E(final) - E(initial)."""
    F = model.slice_field(J, spins, z, d)
    envs, _ = bmps.environments(J, F, z, beta, chi, d)
    cur = model.to_states(spins[z], d)
    _, lq_cur, f_cur = sampler.sample_layer(envs, J, F, z, beta, d, forced=cur)
    e_cur = model.slice_energy(J, F, cur, z, d)
    lq0, e0 = lq_cur, e_cur
    n_acc = 0
    for k in range(n_candidates):
        new, lq_new, f_new = sampler.sample_layer(envs, J, F, z, beta, d, seed=seed, chain=chain, sweep=sweep,
                                                  purpose=2 * k)
        e_new = model.slice_energy(J, F, new, z, d)
        u = uniform(seed, chain, sweep, z, 2 * k + 1, 0)
        if not (f_new or f_cur) and mh_accept(lq_cur, lq_new, beta, e_new - e_cur, u):
            cur, lq_cur, e_cur, f_cur = new, lq_new, e_new, f_new
            n_acc += 1
    spins[z] = model.from_states(cur, d)
    return {"accepted": n_acc, "logq_initial": lq0, "logq_final": lq_cur, "dE": e_cur - e0}


def sweep(J, spins, beta: float, chi: int, d: int, *, seed: int, chain: int, sweep_index: int,
          n_candidates: int = 1):
    """Even layers, then odd layers (in place), n_candidates chained candidates
    per layer (one: slice_update).  Returns the number of accepted updates."""
    Lz = spins.shape[0]
    n_acc = 0
    for parity in (0, 1):
        for z in range(parity, Lz, 2):
            if n_candidates == 1:
                rec = slice_update(J, spins, z, beta, chi, d, seed=seed, chain=chain, sweep=sweep_index)
                n_acc += int(rec["accepted"])
            else:
                rec = slice_update_multi(J, spins, z, beta, chi, d, n_candidates, seed=seed, chain=chain,
                                         sweep=sweep_index)
                n_acc += rec["accepted"]
    return n_acc


def run_chain(J, spins, beta: float, chi: int, d: int, n_sweeps: int, *, seed: int,
              chain: int = 0, sweep_offset: int = 0, n_candidates: int = 1):
    """Run n_sweeps sweeps in place; returns per-sweep energies, magnetisations and
    the acceptance count."""
    E = np.zeros(n_sweeps)
    M = np.zeros(n_sweeps)
    acc = 0
    for t in range(n_sweeps):
        acc += sweep(J, spins, beta, chi, d, seed=seed, chain=chain, sweep_index=sweep_offset + t,
                     n_candidates=n_candidates)
        E[t] = model.energy(J, spins, d)
        M[t] = model.magnetisation(spins, d)
    return E, M, acc


# Direction cycling: slices perpendicular to y or x are z-slices of the lattice
# with its axes permuted.  Direction 0 is z (no change), 1 is y, 2 is x.  Each
# direction draws from its own range of Philox sweep counters.
DIRECTION_STRIDE = 2 ** 56


def to_direction(J, spins, direction: int):
    """(J', spins') of the lattice seen as z-slices perpendicular to axis
    `direction`: direction 1 maps site (z, y, x) to (y, z, x), direction 2 to
    (x, z, y); the coupling components follow their bonds (x-, y-, z-bond of
    the permuted lattice)."""
    J = np.asarray(J)
    s = np.asarray(spins)
    if direction == 0:
        return J.copy(), s.copy()
    if direction == 1:
        perm = (1, 0, 2)
        comps = (0, 2, 1)     # x' = x, y' = z, z' = y
    elif direction == 2:
        perm = (2, 0, 1)
        comps = (1, 2, 0)     # x' = y, y' = z, z' = x
    else:
        raise ValueError("direction is 0, 1 or 2")
    Jp = np.stack([J[c].transpose(perm) for c in comps])
    return np.ascontiguousarray(Jp), np.ascontiguousarray(s.transpose(perm))


def from_direction(spins_p, direction: int):
    """Inverse of the spin permutation of to_direction."""
    s = np.asarray(spins_p)
    if direction == 0:
        return s.copy()
    if direction == 1:
        return np.ascontiguousarray(s.transpose(1, 0, 2))
    return np.ascontiguousarray(s.transpose(1, 2, 0))


def sweep_direction(J, spins, beta: float, chi: int, d: int, direction: int, *, seed: int, chain: int,
                    sweep_index: int):
    """One sweep with slices perpendicular to axis `direction` (in place),
    using sweep counter sweep_index + direction * DIRECTION_STRIDE.  Returns the
    number of accepted updates."""
    Jp, sp = to_direction(J, spins, direction)
    n = sweep(Jp, sp, beta, chi, d, seed=seed, chain=chain, sweep_index=sweep_index + direction * DIRECTION_STRIDE)
    spins[...] = from_direction(sp, direction)
    return n


# TNMCMC-2 (SM S2.B): composite layers (z0, z0 + 1) of superspins with d = 4.
# A composite update draws from the sweep counter sweep + SUPERSPIN_STRIDE, so
# its uniforms never coincide with those of TNMCMC-1 updates or of the other
# slice directions; the layer index of the counter is z0.
SUPERSPIN_STRIDE = 3 * 2 ** 56


def superspin_update(J, spins, z0: int, beta: float, chi: int, *, seed: int, chain: int, sweep: int,
                     margins=None):
    """One TNMCMC-2 update of the composite layer (z0, z0 + 1) of an Ising
    lattice, in place: contraction of its 2D network of superspins with the
    blanket z0 - 1, z0 + 2 held, a drawn composite configuration with its log
    q, log q of the current one, and the MH decision of main text Eq. 1."""
    m = layer.composite_layer(J, spins, z0)
    envs, _ = layer.environments(m, beta, chi)
    sw = sweep + SUPERSPIN_STRIDE
    new, lq_new, f_new = layer.sample_layer(envs, m, beta, seed=seed, chain=chain, sweep=sw, z_key=z0,
                                            margins=margins)
    cur = layer.composite_states(spins, z0)
    _, lq_old, f_old = layer.sample_layer(envs, m, beta, forced=cur)
    dE = layer.layer_energy(m, new) - layer.layer_energy(m, cur)
    u = uniform(seed, chain, sw, z0, PURPOSE_MH, 0)
    acc = (not (f_new or f_old)) and mh_accept(lq_old, lq_new, beta, dE, u)
    if acc:
        spins[z0], spins[z0 + 1] = layer.composite_spins(new)
    return {"new": new, "logq_new": lq_new, "logq_old": lq_old, "dE": dE, "accepted": acc,
            "fault": bool(f_new or f_old)}


def superspin_sweep(J, spins, beta: float, chi: int, *, seed: int, chain: int, sweep_index: int):
    """One TNMCMC-2 sweep (in place): every composite layer z0 = 0 .. Lz - 2,
    in three phases z0 = 0, 3, 6, ..., then 1, 4, ..., then 2, 5, ... (composites
    of one phase share no layer and no blanket layer they update, so their
    updates commute).  Returns the number of accepted updates."""
    Lz = spins.shape[0]
    n_acc = 0
    for phase in range(3):
        for z0 in range(phase, Lz - 1, 3):
            n_acc += int(superspin_update(J, spins, z0, beta, chi, seed=seed, chain=chain, sweep=sweep_index)["accepted"])
    return n_acc
