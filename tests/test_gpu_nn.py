"""The learned proposal's HIP kernels against the FP64 oracle (oracle.nn).

The network is evaluated with BF16 parameters (the FP32 masters rounded to
nearest even, on the GPU and in the oracle alike), in FP32 arithmetic on the
GPU and in FP64 in the oracle, so values are compared within tolerances
derived from FP32 rounding (log q and logits 1e-4 relative, the gradient 1e-4
of its largest entry); decisions taken by floating
point (a site's spin) are checked for consistency with the oracle's
probability at that site, except within 1e-5 of a tie.  dE is exact."""
import math

import numpy as np
import pytest

import bruteforce as bf
import gpu_helpers as gh
import paper_2509_23945_amd as tn
import synth
from oracle import model
from oracle import nn as onn
from oracle import philox

pytestmark = pytest.mark.gpu

SHAPES = onn.layer_shapes()
TIE = 1e-5


def torch_dev():
    import torch
    return torch


def to_dev(a):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_pairs(Lx, Ly, Lz, n, seed):
    """n (cond, s) pairs from random +-J lattices (layer z = i % Lz of lattice i // Lz)."""
    conds, spins = [], []
    for i in range(n):
        J = synth.couplings_pm_j(Lx, Ly, Lz, seed + i)
        s = synth.spins_random(Lx, Ly, Lz, 100 * seed + i, 2)
        z = i % Lz
        conds.append(onn.cond_channels(J, s, z))
        spins.append(s[z])
    return np.stack(conds).astype(np.float32), np.stack(spins).astype(np.int8)


def params(seed, scale=1.0):
    return synth.nn_params(seed, SHAPES, scale)


def close(a, b, rel=1e-4):
    return abs(a - b) <= rel * max(1.0, abs(a), abs(b))


@pytest.mark.parametrize("Lx,Ly,n,scale", [(7, 5, 3, 1.0), (8, 8, 2, 2.0), (33, 3, 2, 1.0), (32, 32, 2, 1.0)])
def test_nn_logq_batch(Lx, Ly, n, scale):
    torch = torch_dev()
    gh.announce(f"nn logq batch {Lx}x{Ly} n={n}")
    th = params(1, scale)
    cond, s = make_pairs(Lx, Ly, 4, n, 7)
    net = tn.tnmc_nn_create(th)
    dc, ds = to_dev(cond), to_dev(s)
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    tn.tnmc_nn_logq(net, dc.data_ptr(), ds.data_ptr(), n, Lx, Ly, out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i in range(n):
        ref = onn.logq(onn.weights_bf16(th), cond[i], s[i])
        assert close(got[i], ref), (i, got[i], ref)
    # the kernels use the BF16 parameters: where the FP32 masters' own log q is
    # clearly different (BF16 rounding moves log q by 1e-5 to 1e-3 relative
    # here), the GPU's value is much nearer the BF16 network's
    for i in range(n):
        ref = onn.logq(onn.weights_bf16(th), cond[i], s[i])
        alt = onn.logq(th.astype(np.float64), cond[i], s[i])
        if abs(ref - alt) > 2e-5 * max(1.0, abs(ref)):
            assert abs(got[i] - ref) < 0.5 * abs(ref - alt), (i, got[i], ref, alt)


@pytest.mark.parametrize("Lx,Ly,Lz,z,scale", [(6, 5, 4, 1, 1.0), (9, 7, 3, 0, 2.0), (5, 6, 3, 2, 1.0),
                                               (16, 12, 4, 2, 1.0), (32, 32, 4, 1, 1.0), (47, 4, 3, 1, 1.0),
                                               (1, 5, 3, 1, 1.0), (7, 1, 2, 0, 2.0)])
def test_nn_slice_propose(Lx, Ly, Lz, z, scale):
    gh.announce(f"nn propose {Lx}x{Ly}x{Lz} z={z}")
    th = params(2, scale)
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, 4, kind="pmj", beta=1.0, seed=4)
    net = tn.tnmc_nn_create(th)
    th64 = onn.weights_bf16(th)   # the BF16 parameters the GPU evaluates with
    cond = onn.cond_channels(J[0], spins[0], z)
    for sweep in (0, 5):
        s_new, lq_new, lq_old, dE, st = tn.tnmc_nn_slice_propose(lat, net, 0, z, sweep)
        assert st == 0
        # every site's choice is the one the oracle's probability gives, up to ties
        logits = onn.forward(th64, cond, s_new)
        U = onn.site_uniforms(12345, 0, sweep, z, Ly, Lx)
        p_plus = 1.0 / (1.0 + np.exp(-logits))
        want_plus = U < p_plus
        mismatch = (s_new > 0) != want_plus
        assert np.all(np.abs(U - p_plus)[mismatch] < TIE), np.argwhere(mismatch)
        assert close(lq_new, onn.logq(th64, cond, s_new))
        assert close(lq_old, onn.logq(th64, cond, spins[0][z]))
        after = spins[0].copy()
        after[z] = s_new
        assert dE == model.energy(J[0], after, 2) - model.energy(J[0], spins[0], 2)
        # the forced evaluation runs the same arithmetic as the drawing walk
        assert tn.tnmc_nn_slice_logq(lat, net, 0, z, s_new) == lq_new


def test_nn_slice_propose_matches_oracle_draws():
    """Small layer: the GPU's drawn layer equals the oracle sampler's (no tie
    within 1e-5 on these seeds)."""
    gh.announce("nn propose vs oracle sampler 5x4x3")
    th = params(3, 2.0)
    lat, J, spins, _ = gh.make_lattice(5, 4, 3, 2, 4, kind="gauss", beta=0.7, seed=6)
    net = tn.tnmc_nn_create(th)
    th64 = onn.weights_bf16(th)   # the BF16 parameters the GPU evaluates with
    for z in range(3):
        rec = onn.propose(th64, J[0], spins[0], z, seed=12345, chain_key=0, sweep=3)
        s_new, lq_new, lq_old, dE, st = tn.tnmc_nn_slice_propose(lat, net, 0, z, 3)
        assert st == 0
        U = onn.site_uniforms(12345, 0, 3, z, 4, 5)
        if np.min(np.abs(U - rec["p_plus"])) > TIE:
            assert np.array_equal(s_new, rec["s_new"])
        assert close(lq_new, rec["logq_new"]) and close(lq_old, rec["logq_old"])
        assert dE == rec["dE"]


def test_nn_dataset_matches_oracle():
    torch = torch_dev()
    gh.announce("nn dataset 6x5x4")
    lat, J, spins, _ = gh.make_lattice(6, 5, 4, 2, 4, kind="gauss", seed=2, n_chains=3)
    n = 3 * 4
    cond = torch.zeros((n, 4, 5, 6), dtype=torch.float32, device="cuda")
    s = torch.zeros((n, 5, 6), dtype=torch.int8, device="cuda")
    tn.tnmc_nn_dataset(lat, cond.data_ptr(), s.data_ptr())
    torch.cuda.synchronize()
    cond, s = cond.cpu().numpy(), s.cpu().numpy()
    for c in range(3):
        for z in range(4):
            assert np.array_equal(cond[c * 4 + z], onn.cond_channels(J[c], spins[c], z).astype(np.float32))
            assert np.array_equal(s[c * 4 + z], spins[c][z])


@pytest.mark.parametrize("Lx,Ly,n", [(6, 5, 3), (33, 4, 2)])
def test_nn_gradient(Lx, Ly, n):
    torch = torch_dev()
    gh.announce(f"nn gradient {Lx}x{Ly} n={n}")
    th = params(4, 1.5)
    cond, s = make_pairs(Lx, Ly, 3, n, 11)
    net = tn.tnmc_nn_create(th)
    dc, ds = to_dev(cond), to_dev(s)
    g = torch.zeros(tn.TNMC_NN_PARAMS, dtype=torch.float32, device="cuda")
    loss = tn.tnmc_nn_loss_grad(net, dc.data_ptr(), ds.data_ptr(), n, Lx, Ly, g.data_ptr())
    torch.cuda.synchronize()
    ref_loss, ref_g = onn.loss_and_grad(onn.weights_bf16(th), cond, s)
    assert close(loss, ref_loss, 1e-5), (loss, ref_loss)
    got = g.cpu().numpy().astype(np.float64)
    scale = np.abs(ref_g).max()
    assert np.all(np.abs(got - ref_g) <= 1e-4 * scale + 1e-7), np.abs(got - ref_g).max() / scale
    assert np.array_equal(got == 0, ref_g == 0) or np.all(got[ref_g == 0] == 0)


def test_nn_adam_and_train():
    torch = torch_dev()
    gh.announce("nn adam / train 6x5")
    Lx, Ly = 6, 5
    th = params(5, 1.0)
    cond, s = make_pairs(Lx, Ly, 3, 4, 13)
    th64 = th.astype(np.float64)   # FP32 masters: Adam and train() step them (gradients at their BF16 rounding)
    dc, ds = to_dev(cond), to_dev(s)
    # one explicit step: Adam on the GPU's gradient against the oracle's Adam on the same gradient
    net = tn.tnmc_nn_create(th)
    g = torch.zeros(tn.TNMC_NN_PARAMS, dtype=torch.float32, device="cuda")
    tn.tnmc_nn_loss_grad(net, dc.data_ptr(), ds.data_ptr(), 4, Lx, Ly, g.data_ptr())
    tn.tnmc_nn_adam_step(net, g.data_ptr(), 1e-3)
    torch.cuda.synchronize()
    g64 = g.cpu().numpy().astype(np.float64)
    ref, _, _ = onn.adam_step(th64, np.zeros_like(th64), np.zeros_like(th64), g64, 1, 1e-3)
    got = tn.tnmc_nn_get_params(net).astype(np.float64)
    assert np.abs(got - ref).max() < 2e-6
    # two minibatch steps of train() against the oracle's train()
    net2 = tn.tnmc_nn_create(th)
    last = tn.tnmc_nn_train(net2, dc.data_ptr(), ds.data_ptr(), 4, Lx, Ly, 1, 2, 1e-2)
    ref_th, ref_loss = onn.train(th64, cond, s, 1, 2, 1e-2)
    got2 = tn.tnmc_nn_get_params(net2).astype(np.float64)
    # Adam's step is lr g / |g| to first order: FP32 rounding of the gradient only
    # shows where |g| is near zero, so nearly every parameter agrees closely
    diff = np.abs(got2 - ref_th)
    assert np.mean(diff < 1e-5) > 0.99 and diff.max() <= 2 * 2 * 1e-2 + 1e-6
    assert close(last, ref_loss, 1e-5)


def test_nn_training_lowers_the_loss():
    torch = torch_dev()
    gh.announce("nn training 8x8")
    lat, J, spins, _ = gh.make_lattice(8, 8, 8, 2, 4, kind="pmj", beta=1.0, seed=1, n_chains=8)
    n = 8 * 8
    cond = torch.zeros((n, 4, 8, 8), dtype=torch.float32, device="cuda")
    s = torch.zeros((n, 8, 8), dtype=torch.int8, device="cuda")
    tn.tnmc_nn_dataset(lat, cond.data_ptr(), s.data_ptr())
    net = tn.tnmc_nn_create(None, seed=3)
    l0 = tn.tnmc_nn_loss_grad(net, cond.data_ptr(), s.data_ptr(), n, 8, 8)
    l1 = tn.tnmc_nn_train(net, cond.data_ptr(), s.data_ptr(), n, 8, 8, 30, 16, 3e-3)
    l2 = tn.tnmc_nn_loss_grad(net, cond.data_ptr(), s.data_ptr(), n, 8, 8)
    assert math.isfinite(l1) and l2 < 0.8 * l0, (l0, l2)


def test_nn_chain_averages_match_enumeration():
    """64 independent chains on 2x2x4 +-J instances with an untrained (random)
    learned proposal (acceptance well below 1): each chain's averages of E and
    M^2 over sweeps 50..399 against exact enumeration, deviations with mean
    zero within four standard errors."""
    gh.announce("nn chain averages 2x2x4")
    Lx, Ly, Lz, beta, n_chains, n_sweeps = 2, 2, 4, 1.0, 64, 400
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, 1, kind="pmj", beta=beta, seed=3, n_chains=n_chains,
                                       record_capacity=n_sweeps)
    net = tn.tnmc_nn_create(params(6, 1.0))
    st = tn.tnmc_nn_sweep([lat], net, n_sweeps, record=True)
    assert st["numeric_faults"] == 0 and 0 < st["accepted"] < st["proposed"]
    assert st["proposed"] == n_chains * Lz * n_sweeps
    E, M, _ = tn.tnmc_timeseries(lat)
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


def test_nn_sweep_step_matches_oracle_update():
    """One learned-proposal half-sweep step of a layer equals the oracle's slice
    update (the MH uniform of purpose 1): same decision, same new state."""
    gh.announce("nn sweep step vs oracle 5x4x2")
    th = params(7, 1.0)
    lat, J, spins, _ = gh.make_lattice(5, 4, 2, 2, 4, kind="pmj", beta=0.5, seed=9, n_chains=2)
    net = tn.tnmc_nn_create(th)
    th64 = onn.weights_bf16(th)   # the BF16 parameters the GPU evaluates with
    tn.tnmc_nn_sweep([lat], net, 1, sweep_offset=4)
    for c in range(2):
        ref = spins[c].copy()
        for z in (0, 1):   # even layers, then odd layers
            onn.slice_update(th64, J[c], ref, z, 0.5, seed=12345, chain_key=c, sweep=4)
        assert np.array_equal(tn.tnmc_get_spins(lat, c), ref)


def test_nn_fallback_routing():
    gh.announce("nn fallback 4x4x4")
    lat, J, spins, _ = gh.make_lattice(4, 4, 4, 2, 4, kind="pmj", beta=1.0, seed=5, n_chains=2)
    net = tn.tnmc_nn_create(params(8, 1.0))
    flags = np.zeros((2, 4), dtype=np.int8)
    flags[0, 1] = flags[1, 2] = 1
    tn.tnmc_nn_set_fallback(lat, flags)
    assert np.array_equal(tn.tnmc_nn_get_fallback(lat), flags)
    st = tn.tnmc_nn_sweep([lat], net, 3)
    prop, acc = tn.tnmc_nn_counts(lat)
    assert np.array_equal(prop, np.where(flags == 1, 0, 3))
    assert st["proposed"] == 2 * 4 * 3 and st["contract_launches"] > 0
    # calibration: threshold 0 flags nothing new; threshold 1 flags every proposed
    # layer with a rejection; layers never proposed keep their flag
    assert tn.tnmc_nn_calibrate_fallback(lat, 0.0) == 2
    n = tn.tnmc_nn_calibrate_fallback(lat, 1.0)
    want = np.where(prop > 0, (acc < prop).astype(np.int8), flags)
    assert n == int(want.sum()) and np.array_equal(tn.tnmc_nn_get_fallback(lat), want)
    tn.tnmc_nn_counts_reset(lat)
    st = tn.tnmc_nn_sweep([lat], net, 2)
    assert np.array_equal(tn.tnmc_nn_counts(lat)[0], np.where(want == 1, 0, 2)) and st["proposed"] == 2 * 4 * 2
    with pytest.raises(tn.TnmcError):
        tn.tnmc_nn_calibrate_fallback(lat, 1.5)
    tn.tnmc_nn_set_fallback(lat, None)
    assert np.all(tn.tnmc_nn_get_fallback(lat) == 0)


def test_nn_invalid_calls():
    gh.announce("nn invalid calls")
    net = tn.tnmc_nn_create(None, seed=1)
    potts, _, _, _ = gh.make_lattice(4, 4, 3, 3, 4, kind="ferro", beta=0.5, seed=1)
    with pytest.raises(tn.TnmcError) as e:
        tn.tnmc_nn_slice_propose(potts, net, 0, 1)
    assert e.value.status == tn.api.TNMC_ERR_UNSUPPORTED
    wide, _, _, _ = gh.make_lattice(64, 8, 3, 2, 4, kind="pmj", seed=1)
    with pytest.raises(tn.TnmcError) as e:
        tn.tnmc_nn_sweep([wide], net, 1)
    assert e.value.status == tn.api.TNMC_ERR_UNSUPPORTED
    bad = np.full(tn.TNMC_NN_PARAMS, np.nan, dtype=np.float32)
    with pytest.raises(tn.TnmcError):
        tn.tnmc_nn_set_params(net, bad)


def test_training_gains_acceptance():
    """What training buys: on 8x8 layers of 8^3 +-J lattices at beta = 1 (64 chains,
    chi = 16), the untrained network's proposals are essentially never accepted;
    after 10 epochs of Adam on 20 480 (condition, layer) pairs taken from TN sweeps
    of the same chains, more than 15% are."""
    torch = torch_dev()
    gh.announce("nn training gain 8^3")
    L, n_chains, K = 8, 64, 40
    lat, _, _, _ = gh.make_lattice(L, L, L, 2, 16, kind="pmj", beta=1.0, seed=21, n_chains=n_chains)
    tn.tnmc_sweep([lat], 10)
    per = n_chains * L
    cond = torch.empty((K * per, 4, L, L), dtype=torch.float32, device="cuda")
    s = torch.empty((K * per, L, L), dtype=torch.int8, device="cuda")
    for k in range(K):
        tn.tnmc_sweep([lat], 1, sweep_offset=10 + k)
        tn.tnmc_nn_dataset(lat, cond.data_ptr() + k * per * 4 * L * L * 4, s.data_ptr() + k * per * L * L)
    torch.cuda.synchronize()
    perm = torch.from_numpy(np.random.Generator(np.random.PCG64(5)).permutation(K * per)).cuda()
    cond, s = cond[perm].contiguous(), s[perm].contiguous()
    net = tn.tnmc_nn_create(None, seed=1)
    st0 = tn.tnmc_nn_sweep([lat], net, 2, sweep_offset=100)
    tn.tnmc_nn_train(net, cond.data_ptr(), s.data_ptr(), K * per, L, L, 10, 256, 2e-3)
    st1 = tn.tnmc_nn_sweep([lat], net, 5, sweep_offset=102)
    a0 = st0["accepted"] / st0["proposed"]
    a1 = st1["accepted"] / st1["proposed"]
    print(f"acceptance untrained {a0:.4f}, trained {a1:.4f}")
    assert a0 < 0.01 and a1 > 0.15 and st1["numeric_faults"] == 0


def test_trained_learned_chain_reproduces_tn_observables():
    """Stationarity with the learned proposal at a size where it is accepted
    (main text Eq. 1: MH is exact for any q whose log q is exact).  32 +-J
    instances x 2 replicas on 8^3 at beta = 0.7 (above the glass transition,
    so chains decorrelate within a few sweeps): the FP64 TN chain (chi = 16)
    and a learned-only chain (network trained for 10 epochs on 20 480 TN
    (condition, layer) pairs of the same instances, no TN fallback) each run
    600 recorded sweeps; per instance the averages of E/N and of q^2 over
    sweeps 100..599 are compared, and the mean difference over instances must
    be within four standard errors of zero."""
    torch = torch_dev()
    gh.announce("learned vs TN observables 8^3 beta=0.7, 64 chains x 600 sweeps")
    L, beta, chi, n_inst, n_sw, K = 8, 0.7, 16, 32, 600, 40
    n_chains = 2 * n_inst
    pairs = np.array([[2 * i, 2 * i + 1] for i in range(n_inst)], dtype=np.int32)

    def lattice():
        return gh.make_lattice(L, L, L, 2, chi, kind="pmj", beta=beta, seed=80, n_chains=n_chains, pairs=pairs,
                               record_capacity=n_sw)[0]

    ref = lattice()
    st = tn.tnmc_sweep([ref], n_sw, record=True)
    assert st["numeric_faults"] == 0
    E_ref, _, q_ref = tn.tnmc_timeseries(ref)
    tn.tnmc_lattice_free(ref)

    lat = lattice()
    per = n_chains * L
    cond = torch.empty((K * per, 4, L, L), dtype=torch.float32, device="cuda")
    s_data = torch.empty((K * per, L, L), dtype=torch.int8, device="cuda")
    for k in range(K):
        # Philox counters of their own, so the data sweeps do not replay the reference chain
        tn.tnmc_sweep([lat], 1, sweep_offset=50_000 + k)
        tn.tnmc_nn_dataset(lat, cond.data_ptr() + k * per * 4 * L * L * 4, s_data.data_ptr() + k * per * L * L)
    torch.cuda.synchronize()
    perm = torch.from_numpy(np.random.Generator(np.random.PCG64(7)).permutation(K * per)).cuda()
    cond, s_data = cond[perm].contiguous(), s_data[perm].contiguous()
    net = tn.tnmc_nn_create(None, seed=3)
    tn.tnmc_nn_train(net, cond.data_ptr(), s_data.data_ptr(), K * per, L, L, 10, 256, 2e-3)
    del cond, s_data
    tn.tnmc_timeseries_reset(lat)
    st = tn.tnmc_nn_sweep([lat], net, n_sw, sweep_offset=100_000, record=True)
    acc = st["accepted"] / st["proposed"]
    print(f"learned-only acceptance at 8^3 beta={beta}: {acc:.3f}")
    assert st["numeric_faults"] == 0 and st["nn_fallbacks"] == 0 and acc > 0.15
    E_nn, _, q_nn = tn.tnmc_timeseries(lat)
    tn.tnmc_lattice_free(lat)
    assert E_nn.shape == (n_sw, n_chains) and E_ref.shape == (n_sw, n_chains)

    def per_instance(E, q):
        return ((E[100:] / L ** 3).mean(axis=0).reshape(n_inst, 2).mean(axis=1), (q[100:] ** 2).mean(axis=0))

    for name, a, b in zip(("E/N", "q^2"), per_instance(E_nn, q_nn), per_instance(E_ref, q_ref)):
        dlt = a - b
        err = dlt.std(ddof=1) / math.sqrt(len(dlt))
        print(f"learned minus TN, {name}: {dlt.mean():.3e} +- {err:.3e}")
        assert abs(dlt.mean()) < 4 * err + 1e-12, (name, dlt.mean(), err)


def test_nn_sweep_over_lattices_of_different_shapes():
    """One learned-proposal sweep over two lattices of different (Lx, Ly, Lz) in
    one call (each parity is one launch sized for the widest and tallest
    layer) equals the oracle's slice updates of each lattice."""
    gh.announce("nn sweep two lattices")
    th = params(9, 1.5)
    th64 = onn.weights_bf16(th)   # the BF16 parameters the GPU evaluates with
    net = tn.tnmc_nn_create(th)
    a, Ja, sa, _ = gh.make_lattice(6, 5, 4, 2, 4, kind="gauss", beta=0.7, seed=12, n_chains=2)
    b, Jb, sb, _ = gh.make_lattice(3, 8, 3, 2, 4, kind="pmj", beta=1.2, seed=13, n_chains=1)
    tn.tnmc_nn_sweep([a, b], net, 1, sweep_offset=2)
    for lat, J, s0, beta, nch in ((a, Ja, sa, 0.7, 2), (b, Jb, sb, 1.2, 1)):
        Lz = s0.shape[1]
        for c in range(nch):
            ref = s0[c].copy()
            for z in list(range(0, Lz, 2)) + list(range(1, Lz, 2)):
                onn.slice_update(th64, J[c], ref, z, beta, seed=12345, chain_key=c, sweep=2)
            assert np.array_equal(tn.tnmc_get_spins(lat, c), ref)


def test_paired_sampler_launch_equals_single_task_workgroups():
    """More than 256 learned-proposal tasks of one shape run two per workgroup
    (sharing the weights in LDS); the chain equals the one-task-per-workgroup
    launch bit for bit."""
    gh.announce("nn paired launch 8x8x10, 64 chains")
    th = params(10, 1.5)
    runs = []
    try:
        for pairing in (1, 0):
            tn.tnmc_debug_set(2, pairing)
            lat, _, _, _ = gh.make_lattice(8, 8, 10, 2, 4, kind="pmj", beta=1.0, seed=51, n_chains=64)
            net = tn.tnmc_nn_create(th)
            st = tn.tnmc_nn_sweep([lat], net, 2, sweep_offset=1)
            assert st["proposed"] == 64 * 10 * 2 and st["numeric_faults"] == 0
            runs.append((st["accepted"], [tn.tnmc_get_spins(lat, c) for c in range(64)]))
    finally:
        tn.tnmc_debug_set(2, 1)
    assert runs[0][0] == runs[1][0] > 0
    for a, b in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(a, b)


def test_nn_sweep_with_every_layer_on_the_fallback_is_the_tn_sweep():
    """All layers flagged for the TN proposal (here on a reduced-precision
    lattice): a learned-proposal sweep is then the plain TN sweep, spin for spin."""
    gh.announce("nn sweep all fallback, fp32 lattice")
    net = tn.tnmc_nn_create(params(11, 1.0))
    lats = [gh.make_lattice(6, 5, 4, 2, 4, kind="gauss", beta=0.9, seed=61, n_chains=2, precision=tn.TNMC_FP32)[0]
            for _ in range(2)]
    tn.tnmc_nn_set_fallback(lats[0], np.ones((2, 4), dtype=np.int8))
    st = tn.tnmc_nn_sweep([lats[0]], net, 2, sweep_offset=5)
    tn.tnmc_sweep([lats[1]], 2, sweep_offset=5)
    assert st["proposed"] == 2 * 4 * 2 and np.all(tn.tnmc_nn_counts(lats[0])[0] == 0)
    for c in range(2):
        assert np.array_equal(tn.tnmc_get_spins(lats[0], c), tn.tnmc_get_spins(lats[1], c))
