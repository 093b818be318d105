"""The reduced-precision form of the contraction against the FP64 oracle.

Environments are stored in FP32 and the rank-revealing factorisations cut at
FP32 resolution; log q, dE and the MH test stay FP64.  The proposal q is then
an approximation of the FP64 one, so spins are not expected to match the
oracle's draws.  What is checked, on the GPU's own proposals:

* log q of the current layer and of the drawn layer within 1e-4 relative of
  the FP64 oracle's log q of the same configurations (forced evaluation);
* the draws themselves, site by site: every site of a drawn layer holds the
  state that the FP64 oracle's conditional at that site (given the GPU's own
  earlier sites) selects for the site's Philox uniform, except where the
  uniform lies within a tie window of a cumulative threshold (SM S1.C:
  ancestral sampling defines q, so MH is exact only if s is drawn from the q
  whose log q is reported);
* dE exact (a full-lattice energy difference of the oracle's model);
* the same for the narrow variant of the full tile layout (two tasks per CU,
  taken by launches of more tasks than CUs), forced on the cases it serves;
* the Markov chain stays exact: with a truncated (chi = 1) proposal on a
  2x2x4 lattice, chain averages of E and M^2 over independent GPU chains match
  exact enumeration within statistical error.
"""
import math

import numpy as np
import pytest

import bruteforce as bf
import gpu_helpers as gh
import paper_2509_23945_amd as tn
from oracle import chain as ochain
from oracle import model
from test_gpu_parity import CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[0, 1], ids=["valu", "mfma"])
def engine(request):
    """Products on the vector ALU (FP64 arithmetic on FP32-stored
    environments) or on the matrix cores (FP32 operands and accumulation)."""
    tn.tnmc_autotune_pin(-1, request.param)
    try:
        yield request.param
    finally:
        tn.tnmc_autotune_pin(-1, -1)


def case_id(c):
    return "x".join(map(str, c[:3])) + f"-d{c[3]}-{c[4]}-chi{c[6]}-z{c[7]}"


@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_fp32_logq_of_own_proposals(case, engine):
    check_fp32_proposals(case, engine)


# the cases whose class runs the full tile layout, which has a narrow variant
# (two tasks per CU) for launches of more tasks than CUs
NARROW_CASES = [c for c in CASES if (c[3] == 2 and c[6] <= 16) or (c[3] == 3 and c[6] <= 8)]


@pytest.mark.parametrize("case", NARROW_CASES, ids=case_id)
def test_fp32_logq_of_own_proposals_narrow_layout(case, engine):
    tn.tnmc_debug_set(4, 1)
    try:
        check_fp32_proposals(case, engine)
    finally:
        tn.tnmc_debug_set(4, 0)


def check_fp32_proposals(case, engine):
    Lx, Ly, Lz, d, kind, beta, chi, z = case
    gh.announce(f"fp32 propose case {case}, engine {engine}")
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=3, precision=tn.TNMC_FP32)
    lq_cur = ochain.slice_logq(J[0], spins[0], z, spins[0][z], beta, chi, d)
    for sweep in (0, 7):
        s_new, lq_new, lq_old, dE, st = tn.tnmc_slice_propose(lat, 0, z, sweep)
        assert st == 0
        assert gh.logq_close_reduced(lq_old, lq_cur), (lq_old, lq_cur)
        o_new, bad, worst, closest = gh.sitewise_draw_check(J[0], spins[0], z, s_new, beta, chi, d, seed=12345,
                                                            chain=0, sweep=sweep)
        gh.record_margin(f"fp32 sitewise engine {engine}", case, sweep, bad, worst, closest)
        assert bad == 0 or worst < gh.TIE_REDUCED, (bad, worst)
        assert gh.logq_close_reduced(lq_new, o_new), (lq_new, o_new)
        after = spins[0].copy()
        after[z] = s_new
        assert dE == model.energy(J[0], after, d) - model.energy(J[0], spins[0], d)
        # the forced evaluation entry point sees the same environments
        assert abs(tn.tnmc_slice_logq(lat, 0, z, s_new) - lq_new) <= 1e-12 * max(1.0, abs(lq_new))


def test_fp32_exact_regime_is_near_boltzmann(engine):
    """Untruncated 3x3 layer: FP32 log q(s) = -beta E(s) - log Z within 1e-4 relative."""
    gh.announce(f"fp32 exact regime 3x3, engine {engine}")
    lat, J, spins, _ = gh.make_lattice(3, 3, 3, 2, 4, kind="gauss", beta=1.1, seed=5, precision=tn.TNMC_FP32)
    cfgs, E = bf.layer_energies(J[0], spins[0], 1, 2)
    logz = bf.logsumexp(-1.1 * E)
    for i in range(0, len(cfgs), 7):
        layer = model.from_states(np.array(cfgs[i]), 2)
        g = tn.tnmc_slice_logq(lat, 0, 1, layer)
        assert gh.logq_close_reduced(g, -1.1 * E[i] - logz)


def test_fp32_chain_averages_match_enumeration(engine):
    """64 independent chains, each on its own 2x2x4 +-J instance, chi = 1
    (truncated, so proposals are rejected at times): the deviations of each
    chain's averages of E and M^2 over sweeps 50..399 from its exact
    enumeration average have mean zero within four standard errors."""
    gh.announce(f"fp32 chain averages 2x2x4, engine {engine}")
    Lx, Ly, Lz, beta, n_chains, n_sweeps = 2, 2, 4, 1.0, 64, 400
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, 1, kind="pmj", beta=beta, seed=3, n_chains=n_chains,
                                       record_capacity=n_sweeps, precision=tn.TNMC_FP32)
    st = tn.tnmc_sweep([lat], n_sweeps, record=True)
    assert st["numeric_faults"] == 0 and st["accepted"] < st["proposed"]
    E, M, _ = tn.tnmc_timeseries(lat)
    assert E.shape == (n_sweeps, n_chains)
    devs_E, devs_M2 = [], []
    for c in range(n_chains):
        states, En = bf.lattice_states(J[c], Lx, Ly, Lz, 2)
        w = np.exp(-beta * (En - En.min()))
        w /= w.sum()
        Mn = np.sum(1 - 2 * states, axis=(1, 2, 3)) / 16.0
        devs_E.append(E[50:, c].mean() - float(np.sum(w * En)))
        devs_M2.append((M[50:, c] ** 2).mean() - float(np.sum(w * Mn * Mn)))
    for devs in (np.array(devs_E), np.array(devs_M2)):
        err = devs.std(ddof=1) / math.sqrt(len(devs))
        assert abs(devs.mean()) < 4 * err + 1e-12, (devs.mean(), err)


@pytest.mark.parametrize("L,beta,n_sw", [(8, 1.0, 600), (16, 0.7, 400)], ids=["8cubed-beta1", "16cubed-beta0.7"])
def test_reduced_mfma_form_reproduces_fp64_observables(L, beta, n_sw):
    """Stationarity is unchanged by the reduced-precision proposal (main text
    Eq. 1: MH is exact for any q with exact log q).  32 +-J instances x 2
    replicas at chi = 3 (truncated, so proposals are rejected at times), on
    8^3 at beta = 1 and on 16^3 at beta = 0.7 (above the glass transition, so
    that 16^3 chains equilibrate within the discarded sweeps): the FP64 form
    (vector-ALU products) and the reduced form (FP32 environments, FP32 MFMA
    products) each run n_sw sweeps from the same states; per instance the
    averages of E/N and of q^2 over sweeps 100..n_sw-1 are compared, and the
    mean difference over instances must be within four standard errors of
    zero."""
    gh.announce(f"reduced (FP32 MFMA) vs FP64 observables, {L}^3 beta={beta} chi=3, 64 chains x {n_sw} sweeps")
    chi, n_inst = 3, 32
    pairs = np.array([[2 * i, 2 * i + 1] for i in range(n_inst)], dtype=np.int32)
    res = {}
    try:
        for prec, eng in ((tn.TNMC_FP64, 0), (tn.TNMC_FP32, 1)):
            tn.tnmc_autotune_pin(-1, eng)
            lat, J, spins, _ = gh.make_lattice(L, L, L, 2, chi, kind="pmj", beta=beta, seed=70, n_chains=2 * n_inst,
                                               pairs=pairs, record_capacity=n_sw, precision=prec)
            st = tn.tnmc_sweep([lat], n_sw, record=True)
            assert st["numeric_faults"] == 0 and st["accepted"] < st["proposed"]
            E, _, q = tn.tnmc_timeseries(lat)
            tn.tnmc_lattice_free(lat)
            e_inst = (E[100:] / L ** 3).mean(axis=0).reshape(n_inst, 2).mean(axis=1)
            q2_inst = (q[100:] ** 2).mean(axis=0)
            res[prec] = (e_inst, q2_inst)
    finally:
        tn.tnmc_autotune_pin(-1, -1)
    for k in range(2):
        dlt = res[tn.TNMC_FP32][k] - res[tn.TNMC_FP64][k]
        err = dlt.std(ddof=1) / math.sqrt(len(dlt))
        assert abs(dlt.mean()) < 4 * err + 1e-12, (k, dlt.mean(), err)
