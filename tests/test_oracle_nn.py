"""Pins of the learned-proposal oracle (oracle.nn), each against something other
than the oracle itself:

* the masked convolution equals scipy's 2D correlation with the masked kernel;
* autoregressive structure: the logit of site j is unchanged by any change of
  the spins at sites >= j, and does depend on earlier ones;
* q is normalised: the sum of q over all 2^(Lx Ly) layers is 1 (enumeration);
* the sampler's draws follow q (frequencies over many uniforms on a 2x2 layer);
* the condition channels hold the held layers' field (the model's slice field,
  itself pinned by brute force) and the in-layer couplings;
* the gradient of the loss matches central finite differences;
* Adam: the first step, and every step under a constant gradient, moves each
  parameter by lr g / (|g| + eps) (closed form);
* BF16 parameters: the rounding equals torch's float32 -> bfloat16 cast (round
  to nearest even) across magnitudes, keeps BF16 values, breaks ties to the
  even neighbour, stays within half a BF16 ulp (2^-8 relative), and train()
  steps the masters by Adam on the gradient taken at their rounding;
* the Metropolis-Hastings kernel with the learned proposal leaves the exact
  conditional Boltzmann distribution of a layer invariant (exact stationarity
  on a 2x2x3 lattice)."""
import itertools
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

import synth
from oracle import chain, model
from oracle import nn

SHAPES = nn.layer_shapes()


def params(seed, scale=1.0):
    return synth.nn_params(seed, SHAPES, scale).astype(np.float64)


def rand_cond(rng, Ly, Lx):
    c = rng.integers(-2, 3, size=(4, Ly, Lx)).astype(np.float64)
    c[2:] = rng.choice([-1.0, 1.0], size=(2, Ly, Lx))
    return c


def test_param_count():
    assert nn.n_params() == 38753
    th = params(0)
    assert th.size == 38753
    assert np.allclose(nn.pack(nn.unpack(th)), th)


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(1)
    for layer in (0, 1, 5):
        ci, co = SHAPES[layer]
        W = rng.standard_normal((co, ci, 3, 3))
        b = rng.standard_normal(co)
        x = rng.standard_normal((ci, 5, 7))
        M = nn.mask(layer)
        out = nn.conv(x, W, b, M)
        for o in range(co):
            ref = b[o] + sum(correlate2d(x[c], W[o, c] * M[c], mode="same", boundary="fill") for c in range(ci))
            assert np.allclose(out[o], ref, atol=1e-12)


def test_masks():
    M0 = nn.mask(0)
    assert M0[:4].sum() == 4 * 9                      # condition channels unmasked
    assert M0[4].sum() == 4 and M0[4, 1, 1] == 0      # type A: centre and later sites hidden
    for l in range(1, 6):
        M = nn.mask(l)
        assert np.all(M.sum(axis=(1, 2)) == 5) and np.all(M[:, 1, 1] == 1)
        assert np.all(M[:, 1, 2] == 0) and np.all(M[:, 2, :] == 0)


def test_autoregressive_property():
    rng = np.random.default_rng(2)
    th = params(3)
    Ly, Lx = 4, 5
    cond = rand_cond(rng, Ly, Lx)
    s = rng.choice([-1, 1], size=(Ly, Lx))
    l0 = nn.forward(th, cond, s)
    for j in range(Ly * Lx):
        y, x = divmod(j, Lx)
        # flip every site >= j: logits of sites <= j are unchanged
        t = s.copy().ravel()
        t[j:] *= -1
        l1 = nn.forward(th, cond, t.reshape(Ly, Lx))
        assert np.array_equal(l1.ravel()[:j + 1], l0.ravel()[:j + 1])
        if j > 0:
            # flipping the left neighbour (first column: the site above) changes the logit of j
            u = s.copy()
            if x > 0:
                u[y, x - 1] *= -1
            else:
                u[y - 1, x] *= -1
            assert nn.forward(th, cond, u)[y, x] != l0[y, x]


@pytest.mark.parametrize("Ly,Lx", [(2, 2), (2, 3), (3, 2)])
def test_q_is_normalised(Ly, Lx):
    rng = np.random.default_rng(Ly * 10 + Lx)
    th = params(4, scale=2.0)
    cond = rand_cond(rng, Ly, Lx)
    lq = [nn.logq(th, cond, np.array(c).reshape(Ly, Lx))
          for c in itertools.product([1, -1], repeat=Ly * Lx)]
    assert abs(math.fsum(math.exp(v) for v in lq) - 1.0) < 1e-12
    assert max(lq) - min(lq) > 1.0    # not uniform


def test_sampler_follows_q():
    rng = np.random.default_rng(5)
    th = params(6, scale=2.0)
    cond = rand_cond(rng, 2, 2)
    cfgs = [np.array(c).reshape(2, 2) for c in itertools.product([1, -1], repeat=4)]
    q = np.array([math.exp(nn.logq(th, cond, c)) for c in cfgs])
    n = 4000
    counts = np.zeros(len(cfgs))
    for _ in range(n):
        s, lq, _ = nn.sample(th, cond, rng.random((2, 2)))
        k = next(i for i, c in enumerate(cfgs) if np.array_equal(c, s))
        counts[k] += 1
        assert abs(lq - math.log(q[k])) < 1e-12
    # each frequency within 5 binomial standard deviations
    sd = np.sqrt(n * q * (1 - q))
    assert np.all(np.abs(counts - n * q) <= 5 * sd + 1)


def test_cond_channels_hold_the_field():
    J = synth.couplings_pm_j(4, 3, 5, 7)
    s = synth.spins_random(4, 3, 5, 8, 2)
    for z in range(5):
        c = nn.cond_channels(J, s, z)
        F = model.slice_field(J, s, z, 2)
        assert np.array_equal(c[0] + c[1], F[:, :, 0])     # state 0 is spin +1
        assert np.array_equal(c[2], J[0, z]) and np.array_equal(c[3], J[1, z])
    assert np.all(nn.cond_channels(J, s, 0)[0] == 0) and np.all(nn.cond_channels(J, s, 4)[1] == 0)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(9)
    th = params(10)
    Ly, Lx, B = 3, 4, 3
    conds = np.stack([rand_cond(rng, Ly, Lx) for _ in range(B)])
    spins = rng.choice([-1, 1], size=(B, Ly, Lx))
    loss, g = nn.loss_and_grad(th, conds, spins)
    ref = np.mean([-nn.logq(th, c, s) for c, s in zip(conds, spins)])
    assert abs(loss - ref) < 1e-12
    # every masked weight has zero gradient
    o = 0
    for i, (ci, co) in enumerate(SHAPES):
        M = np.broadcast_to(nn.mask(i)[None], (co, ci, 3, 3)).ravel()
        assert np.all(g[o:o + co * ci * 9][M == 0] == 0)
        o += co * ci * 9 + co
    idx = rng.choice(th.size, 60, replace=False)
    idx = np.concatenate([idx, [th.size - 1, 0, 1472 - 1]])   # output bias, first weight, layer-0 bias
    h = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fp = nn.loss_and_grad(tp, conds, spins)[0]
        fm = nn.loss_and_grad(tm, conds, spins)[0]
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_closed_forms():
    rng = np.random.default_rng(11)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 1, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    t1, m, v = nn.adam_step(th, m, v, g, 1, lr)
    assert np.allclose(t1, th - lr * g / (np.abs(g) + nn.ADAM_EPS), rtol=0, atol=1e-15)
    cur = t1
    for t in range(2, 6):   # constant gradient: every bias-corrected moment is exact
        nxt, m, v = nn.adam_step(cur, m, v, g, t, lr)
        assert np.allclose(nxt, cur - lr * g / (np.abs(g) + nn.ADAM_EPS), rtol=0, atol=1e-14)
        cur = nxt


def test_bf16_rounding_matches_torch_and_the_format():
    import torch
    rng = np.random.default_rng(12)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-100, 100, 20000))).astype(np.float32)
    r = nn.weights_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).double().numpy()
    assert np.array_equal(r, ref)
    assert np.array_equal(nn.weights_bf16(r), r)                      # BF16 values are kept
    assert np.all(np.abs(r - x) <= np.abs(x.astype(np.float64)) * 2.0 ** -8)   # unit roundoff, 8-bit significand
    # ties go to the even neighbour (spacing 2^-7 on [1, 2))
    for v, want in [(1 + 2.0 ** -8, 1.0), (1 + 3 * 2.0 ** -8, 1 + 2.0 ** -6), (1 + 2.0 ** -8 + 2.0 ** -20, 1 + 2.0 ** -7),
                    (-(1 + 3 * 2.0 ** -8), -(1 + 2.0 ** -6)), (2.0 ** -130, 2.0 ** -130), (0.0, 0.0)]:
        assert nn.weights_bf16([v])[0] == want, (v, want)


def test_train_steps_masters_at_bf16_weights():
    rng = np.random.default_rng(13)
    th = params(9, 1.0) + rng.standard_normal(nn.n_params()) * 1e-4   # masters off the BF16 grid
    conds = np.stack([rand_cond(rng, 3, 4) for _ in range(2)])
    spins = rng.choice([-1, 1], size=(2, 3, 4)).astype(np.int8)
    got, loss = nn.train(th, conds, spins, 1, 2, 1e-3)
    ref_loss, g = nn.loss_and_grad(nn.weights_bf16(th), conds, spins)
    want, _, _ = nn.adam_step(th, np.zeros_like(th), np.zeros_like(th), g, 1, 1e-3)
    assert loss == ref_loss and np.array_equal(got, want)
    assert not np.array_equal(nn.weights_bf16(th), th)


def test_mh_with_learned_proposal_is_exactly_stationary():
    """2x2x3 lattice, layer 1: the one-layer transition kernel (propose from q,
    accept by main text Eq. 1) built from the oracle's q and energies leaves
    the conditional Boltzmann law of the layer invariant."""
    J = synth.couplings_gauss(2, 2, 3, 3)
    s = synth.spins_random(2, 2, 3, 4, 2)
    beta, z = 0.8, 1
    th = params(12, scale=1.5)
    cond = nn.cond_channels(J, s, z)
    cfgs = [np.array(c, dtype=np.int8).reshape(2, 2) for c in itertools.product([1, -1], repeat=4)]
    E = []
    for c in cfgs:
        t = s.copy()
        t[z] = c
        E.append(model.energy(J, t, 2))
    E = np.array(E)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    q = np.array([math.exp(nn.logq(th, cond, c)) for c in cfgs])
    n = len(cfgs)
    P = np.zeros((n, n))
    for a in range(n):
        for b in range(n):
            if a != b:
                lr = math.log(q[a]) - math.log(q[b]) - beta * (E[b] - E[a])
                P[a, b] = q[b] * min(1.0, math.exp(lr))
        P[a, a] = 1.0 - P[a].sum()
    assert np.abs(pi @ P - pi).max() < 1e-14
    # the oracle's own update agrees with that kernel's acceptance rule
    rec = nn.slice_update(th, J, s.copy(), z, beta, seed=1, chain_key=0, sweep=0)
    a = next(i for i, c in enumerate(cfgs) if np.array_equal(c, s[z]))
    b = next(i for i, c in enumerate(cfgs) if np.array_equal(c, rec["s_new"]))
    assert abs(rec["logq_new"] - math.log(q[b])) < 1e-12 and abs(rec["logq_old"] - math.log(q[a])) < 1e-12
    assert abs(rec["dE"] - (E[b] - E[a])) < 1e-12
