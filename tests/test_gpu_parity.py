"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bar (FP64 path): spins and energy changes bit-exact, log q within 1e-10
(relative above |log q| = 1), MH decisions identical; a spin mismatch is
accepted only when the oracle's uniform lies within 1e-9 of a cumulative
threshold (a near-tie, where both draws are correct)."""
import math

import numpy as np
import pytest

import bruteforce as bf
import gpu_helpers as gh
import paper_2509_23945_amd as tn
import synth
from oracle import chain as ochain
from oracle import model

pytestmark = pytest.mark.gpu

CASES = [
    # Lx, Ly, Lz, d, kind, beta, chi, z
    (3, 3, 3, 2, "pmj", 1.0, 4, 1),        # exact, tiny
    (5, 4, 3, 2, "gauss", 0.8, 8, 1),      # ragged rectangle, Gaussian couplings
    (8, 8, 8, 2, "pmj", 0.5, 16, 0),       # 8^3 layer, chi=16 exact (edge layer)
    (8, 8, 8, 2, "pmj", 0.5, 16, 3),
    (12, 12, 1, 2, "ferro", 0.44, 4, 0),   # field-free critical ferromagnet, truncated
    (9, 7, 1, 2, "pmj", 1.0, 3, 0),        # odd chi, truncated, no field
    (7, 6, 2, 2, "pmj", 1.2, 5, 1),        # one held neighbour
    (1, 6, 3, 2, "gauss", 0.9, 1, 1),      # single column
    (6, 1, 3, 2, "pmj", 1.0, 2, 1),        # single row
    (1, 1, 3, 2, "gauss", 0.9, 2, 1),      # one-site layer
    (1, 1, 3, 3, "ferro", 0.55, 2, 1),     # one-site Potts layer
    (4, 3, 3, 3, "ferro", 0.55, 9, 1),     # Potts, exact
    (6, 5, 3, 3, "ferro", 0.55, 4, 1),     # Potts, truncated
    (16, 16, 16, 2, "pmj", 1.0, 32, 5),    # 16^3 layer at chi=32
    (32, 32, 3, 2, "pmj", 1.0, 32, 1),     # 32x32 layer at chi=32 (largest shape)
    (64, 4, 3, 2, "pmj", 1.0, 32, 1),      # widest rows (64 sites), chi=32
    (4, 64, 2, 2, "gauss", 0.9, 8, 0),     # most rows (64), one held neighbour
    (16, 16, 3, 2, "pmj", 1.0, 20, 1),     # compact layout, truncating (rank > chi)
    (7, 6, 3, 3, "ferro", 0.55, 10, 1),    # Potts, compact layout, truncating
    (8, 6, 3, 3, "ferro", 0.55, 14, 1),    # Potts, compact, truncating after an LQ of more than 32 rows
    (5, 4, 3, 3, "ferro", 0.55, 20, 1),    # Potts, chi_max = 32 (every tile in global memory), exact
    (7, 7, 3, 3, "ferro", 0.55, 24, 1),    # Potts, chi_max = 32, truncating
    (64, 6, 3, 3, "ferro", 0.55, 24, 1),   # Potts, chi_max = 32, 64-site rows: the sampler's single-tile layout
    (64, 5, 2, 3, "ferro", 0.55, 32, 0),   # the same with one held neighbour
    (16, 16, 1, 2, "ferro", 0.44, 48, 0),  # chi_max = 64 (tiles in global memory), critical layer truncating at 48
    (32, 32, 1, 2, "ferro", 0.40, 64, 0),  # chi_max = 64 on the largest layer, truncating at 64
    (16, 16, 3, 2, "pmj", 1.0, 40, 1),     # chi_max = 64, +-J layer with held neighbours
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"-d{c[3]}-{c[4]}-chi{c[6]}-z{c[7]}")
def test_propose_matches_oracle(case):
    Lx, Ly, Lz, d, kind, beta, chi, z = case
    gh.announce(f"propose case {case}")
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=3)
    for sweep in (0, 7):
        gpu = tn.tnmc_slice_propose(lat, 0, z, sweep)
        assert gpu[4] == 0
        ref, margins = gh.oracle_propose(J[0], spins[0], z, beta, chi, d, seed=12345, chain=0, sweep=sweep)
        diff = gh.compare_proposal(gpu, ref, margins, case=case)
        assert not diff or diff.get("spins", ("",))[0] == "near-tie", diff


@pytest.fixture
def mfma_engine():
    """Every contraction of the test runs its products on the matrix cores."""
    tn.tnmc_autotune_pin(-1, 1)
    try:
        yield
    finally:
        tn.tnmc_autotune_pin(-1, -1)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"-d{c[3]}-{c[4]}-chi{c[6]}-z{c[7]}")
def test_propose_matches_oracle_mfma(case, mfma_engine):
    """The same bar with the products M, AT, C, Y on FP64 MFMA."""
    Lx, Ly, Lz, d, kind, beta, chi, z = case
    gh.announce(f"propose case {case}, MFMA products")
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=3)
    for sweep in (0, 7):
        gpu = tn.tnmc_slice_propose(lat, 0, z, sweep)
        assert gpu[4] == 0
        ref, margins = gh.oracle_propose(J[0], spins[0], z, beta, chi, d, seed=12345, chain=0, sweep=sweep)
        diff = gh.compare_proposal(gpu, ref, margins, case=case)
        assert not diff or diff.get("spins", ("",))[0] == "near-tie", diff


# cases whose configuration uses the compact two-per-CU contraction layout
COMPACT_CASES = [c for c in CASES if c[3] == 2 and 16 < c[6] <= 32]


@pytest.mark.parametrize("case", COMPACT_CASES, ids=lambda c: "x".join(map(str, c[:3])) + f"-d{c[3]}-chi{c[6]}")
def test_overflow_path_matches_oracle(case):
    """The compact layout's overflow path (full tile layout in global memory),
    forced for every task through the test hook, agrees with the oracle as the
    LDS paths do; one sweep through it equals one through the normal path."""
    Lx, Ly, Lz, d, kind, beta, chi, z = case
    gh.announce(f"overflow path {case}")
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=3)
    tn.tnmc_debug_set(0, 1)
    try:
        gpu = tn.tnmc_slice_propose(lat, 0, z, 0)
        assert gpu[4] == 0
        ref, margins = gh.oracle_propose(J[0], spins[0], z, beta, chi, d, seed=12345, chain=0, sweep=0)
        diff = gh.compare_proposal(gpu, ref, margins)
        assert not diff or diff.get("spins", ("",))[0] == "near-tie", diff
        st = tn.tnmc_sweep([lat], 1, sweep_offset=0)
        assert st["numeric_faults"] == 0
        forced = tn.tnmc_get_spins(lat, 0)
    finally:
        tn.tnmc_debug_set(0, 0)
    lat2 = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=3)[0]
    tn.tnmc_sweep([lat2], 1, sweep_offset=0)
    assert np.array_equal(forced, tn.tnmc_get_spins(lat2, 0))


@pytest.mark.parametrize("case", [(6, 5, 3, 2, "pmj", 1.0, 3), (5, 5, 1, 2, "ferro", 0.44, 2),
                                  (4, 4, 3, 3, "ferro", 0.6, 3)])
def test_logq_of_arbitrary_layers(case):
    Lx, Ly, Lz, d, kind, beta, chi = case
    gh.announce(f"logq case {case}")
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=8)
    rng = np.random.Generator(np.random.PCG64(1))
    z = Lz // 2
    for _ in range(4):
        layer = synth.spins_random(Lx, Ly, 1, int(rng.integers(1 << 30)), d)[0]
        g = tn.tnmc_slice_logq(lat, 0, z, layer)
        o = ochain.slice_logq(J[0], spins[0], z, layer, beta, chi, d)
        assert gh.logq_close(g, o), (g, o)


def test_exact_regime_is_boltzmann_on_gpu():
    """Untruncated contraction: GPU log q(s) = -beta E(s) - log Z for every s of a 3x3 layer."""
    gh.announce("exact regime 3x3")
    lat, J, spins, _ = gh.make_lattice(3, 3, 3, 2, 4, kind="gauss", beta=1.1, seed=5)
    cfgs, E = bf.layer_energies(J[0], spins[0], 1, 2)
    logz = bf.logsumexp(-1.1 * E)
    for i in range(0, len(cfgs), 7):
        layer = model.from_states(np.array(cfgs[i]), 2)
        g = tn.tnmc_slice_logq(lat, 0, 1, layer)
        assert abs(g - (-1.1 * E[i] - logz)) < 1e-11 * max(1.0, abs(logz))


def test_truncated_q_sums_to_one_on_gpu():
    gh.announce("sum q 3x3 chi=1")
    lat, J, spins, _ = gh.make_lattice(3, 3, 1, 2, 1, kind="ferro", beta=0.6, seed=2, init="ordered")
    cfgs, _ = bf.layer_energies(J[0], spins[0], 0, 2)
    tot = math.fsum(math.exp(tn.tnmc_slice_logq(lat, 0, 0, model.from_states(np.array(a), 2))) for a in cfgs)
    assert abs(tot - 1.0) < 1e-12


def test_energy_kernel_matches_oracle():
    for d, kind in ((2, "pmj"), (2, "gauss"), (3, "ferro")):
        gh.announce(f"energy {d} {kind}")
        lat, J, spins, _ = gh.make_lattice(7, 6, 5, d, 4, kind=kind, seed=9, n_chains=2)
        for c in range(2):
            assert tn.tnmc_energy(lat, c) == model.energy(J[c], spins[c], d)


def test_sweeps_match_oracle_c1():
    """8^3 +-J at beta=0.5, chi=16 (exact): three GPU sweeps reproduce the oracle's
    chain bit for bit, and every proposal is accepted."""
    gh.announce("sweep 8^3 chi=16")
    lat, J, spins, _ = gh.make_lattice(8, 8, 8, 2, 16, kind="pmj", beta=0.5, seed=0)
    ref = spins[0].copy()
    for t in range(3):
        st = tn.tnmc_sweep([lat], 1, sweep_offset=t)
        acc = ochain.sweep(J[0], ref, 0.5, 16, 2, seed=12345, chain=0, sweep_index=t)
        assert np.array_equal(tn.tnmc_get_spins(lat, 0), ref)
        assert st["proposed"] == 8 and st["accepted"] == acc == 8


def test_batched_uneven_lattices_match_oracle():
    """Two lattices of different shape, d and chi in one tnmc_sweep call."""
    gh.announce("batched uneven sweep")
    la, Ja, sa, ba = gh.make_lattice(6, 5, 4, 2, 3, kind="gauss", beta=[0.7, 1.3, 1.0], seed=4, n_chains=3)
    lb, Jb, sb, bb = gh.make_lattice(4, 4, 3, 3, 4, kind="ferro", beta=[0.55, 0.6], seed=6, n_chains=2)
    refs = [(Ja[c], sa[c].copy(), ba[c], 3, 2, c) for c in range(3)] + [(Jb[c], sb[c].copy(), bb[c], 4, 3, c) for c in range(2)]
    for t in range(2):
        tn.tnmc_sweep([la, lb], 1, sweep_offset=t)
        for (J, s, beta, chi, d, c) in refs:
            ochain.sweep(J, s, beta, chi, d, seed=12345, chain=c, sweep_index=t)
    for k, (J, s, beta, chi, d, c) in enumerate(refs):
        lat = la if k < 3 else lb
        assert np.array_equal(tn.tnmc_get_spins(lat, c), s), (k, c)


def test_observables_record():
    gh.announce("observables")
    lat, J, spins, _ = gh.make_lattice(6, 6, 6, 2, 8, kind="pmj", beta=1.0, seed=2, n_chains=4,
                                       pairs=np.array([[0, 1], [2, 3]]), record_capacity=5)
    tn.tnmc_sweep([lat], 3, record=True)
    E, M, q = tn.tnmc_timeseries(lat)
    assert E.shape == (3, 4) and q.shape == (3, 2)
    s = [tn.tnmc_get_spins(lat, c) for c in range(4)]
    for c in range(4):
        assert E[-1, c] == model.energy(J[c], s[c], 2)
        assert M[-1, c] == model.magnetisation(s[c], 2)
    assert q[-1, 0] == model.overlap(s[0], s[1]) and q[-1, 1] == model.overlap(s[2], s[3])
    tn.tnmc_timeseries_reset(lat)
    assert tn.tnmc_timeseries(lat)[0].shape[0] == 0


def test_deterministic_replay():
    gh.announce("determinism")
    a = gh.make_lattice(10, 9, 6, 2, 8, kind="pmj", beta=1.0, seed=11, n_chains=2)[0]
    b = gh.make_lattice(10, 9, 6, 2, 8, kind="pmj", beta=1.0, seed=11, n_chains=2)[0]
    tn.tnmc_sweep([a], 2)
    tn.tnmc_sweep([b], 1)
    tn.tnmc_sweep([b], 1, sweep_offset=1)     # resume from the counter
    for c in range(2):
        assert np.array_equal(tn.tnmc_get_spins(a, c), tn.tnmc_get_spins(b, c))


def test_invalid_calls_are_rejected():
    lat = gh.make_lattice(4, 4, 4, 2, 4, seed=1)[0]
    for bad in ((1, 0), (0, 4), (0, -1)):
        with pytest.raises(tn.TnmcError) as ei:
            tn.tnmc_slice_propose(lat, bad[0], bad[1])
        assert ei.value.status == tn.api.TNMC_ERR_ARG
    with pytest.raises(tn.TnmcError):
        tn.tnmc_slice_logq(lat, 0, 0, np.zeros((4, 4), np.int8))
    # chi above 64 (Ising) and above 32 (Potts) is not built
    for d, chi in ((2, 80), (3, 40)):
        with pytest.raises(tn.TnmcError) as ei:
            gh.make_lattice(8, 2, 2, d, chi, kind="ferro", seed=1)
        assert ei.value.status == tn.api.TNMC_ERR_UNSUPPORTED
    # the largest layers are: 64 x 64 Potts at chi = 32 (single-tile sampler layout) and Ising
    for d in (2, 3):
        gh.make_lattice(64, 64, 2, d, 32, kind="ferro", seed=1)


def test_zero_sweeps_change_nothing():
    """n_sweeps = 0 is a valid call: no launch, zero counts, no record, the
    spins as they were."""
    gh.announce("zero sweeps")
    lat, J, spins, _ = gh.make_lattice(5, 4, 4, 2, 4, seed=2, n_chains=2, record_capacity=4)
    st = tn.tnmc_sweep([lat], 0, record=True)
    assert st["proposed"] == 0 and st["accepted"] == 0 and st["numeric_faults"] == 0
    assert st["contract_launches"] == 0 and st["sample_launches"] == 0
    for c in range(2):
        assert np.array_equal(tn.tnmc_get_spins(lat, c), spins[c])
    E, _, _ = tn.tnmc_timeseries(lat)
    assert E.shape[0] == 0
    tn.tnmc_lattice_free(lat)


def test_potts_chain_averages_match_enumeration():
    """64 independent 3-state Potts chains on one 2x2x3 ferromagnet at beta =
    0.55, chi = 1 (truncated, so proposals are rejected at times): each
    chain's averages of E and of the recorded magnetisation
    M = (3 max_k n_k / N - 1) / 2 over sweeps 30..299 deviate from the exact
    Boltzmann averages (all 3^12 states enumerated) by amounts whose mean is
    zero within four standard errors."""
    gh.announce("potts chain averages 2x2x3")
    Lx, Ly, Lz, beta, n_chains, n_sweeps = 2, 2, 3, 0.55, 64, 300
    lat, J, _, _ = gh.make_lattice(Lx, Ly, Lz, 3, 1, kind="ferro", beta=beta, seed=5, n_chains=n_chains,
                                   record_capacity=n_sweeps)
    st = tn.tnmc_sweep([lat], n_sweeps, record=True)
    assert st["numeric_faults"] == 0 and st["accepted"] < st["proposed"]
    E, M, _ = tn.tnmc_timeseries(lat)
    tn.tnmc_lattice_free(lat)
    states, En = bf.lattice_states(J[0], Lx, Ly, Lz, 3)
    counts = np.stack([(states == k).sum(axis=(1, 2, 3)) for k in range(3)])
    Mn = (3.0 * counts.max(axis=0) / (Lx * Ly * Lz) - 1.0) / 2.0
    w = np.exp(-beta * (En - En.min()))
    w /= w.sum()
    for series, exact in ((E, float(np.sum(w * En))), (M, float(np.sum(w * Mn)))):
        devs = series[30:].mean(axis=0) - exact
        err = devs.std(ddof=1) / math.sqrt(len(devs))
        assert abs(devs.mean()) < 4 * err + 1e-12, (devs.mean(), err)


def test_heterogeneous_batch_like_c3():
    """The mixed batch of the c3 workload at small sizes: three lattice sizes x two
    bond dimensions (one truncating), Gaussian couplings and a spread of beta, all in
    one tnmc_sweep call (launches grouped by layer class and bond dimension,
    longest task first).
    Every chain's layers after two sweeps equal the oracle's."""
    gh.announce("c3-like heterogeneous batch")
    rng_b = synth.betas_uniform(12, 0.5, 1.5, seed=7)
    lats, refs = [], []
    k = 0
    for L in (6, 8, 10):
        for chi in (4, 8):
            betas = rng_b[k:k + 2]
            lat, J, spins, b = gh.make_lattice(L, L, L, 2, chi, kind="gauss", beta=betas, seed=50 + k, n_chains=2)
            lats.append(lat)
            refs.append([(J[c], spins[c].copy(), b[c], chi, c) for c in range(2)])
            k += 2
    for t in range(2):
        tn.tnmc_sweep(lats, 1, sweep_offset=t)
        for chains in refs:
            for (J, s, beta, chi, c) in chains:
                ochain.sweep(J, s, beta, chi, 2, seed=12345, chain=c, sweep_index=t)
    for lat, chains in zip(lats, refs):
        for (J, s, beta, chi, c) in chains:
            assert np.array_equal(tn.tnmc_get_spins(lat, c), s), (lat.Lx, chi, c)
