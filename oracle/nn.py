"""Learned autoregressive slice proposal q_theta(s | cond), plain FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper proposes a new layer from an exactly normalised distribution q with a
tractable log q and corrects it by Metropolis-Hastings (main text Eq. 1); any
such q leaves the chain exact.  Here q is a masked-convolution autoregressive
network over the layer's sites in the sampling order the tensor-network sampler
uses (rows top to bottom, sites left to right within a row; SM S1.C), in place
of the boundary-MPS conditionals.  The network is not in the paper; its shape
is the one the build fixes:

* input: four condition channels per site, seen through full 3x3 windows
  (field of the held layer below, Jz(z-1) s(z-1); field of the held layer
  above, Jz(z) s(z+1); the in-layer couplings Jx and Jy; 0 where a neighbour
  or bond does not exist), and the layer's own spins (+1 / -1) seen through a
  mask that hides the centre and every later site ("type A");
* five hidden 3x3 layers of 32 channels with ReLU; the first reads the input
  above, the next four read the previous layer through a mask that hides later
  sites but keeps the centre ("type B");
* an output 3x3 type-B layer with one channel: the logit l of P(s = +1), clipped
  to [-LOGIT_CLIP, LOGIT_CLIP];
* zero padding at the layer's open edges.

Parameters are one flat vector: for each layer W[c_out][c_in][3][3] then
b[c_out] (38 753 numbers).  Masked weights are stored but multiply nothing.
The network is evaluated with BF16 parameters: training keeps FP32 master
values, and weights_bf16 rounds them to the BF16 numbers the network uses.
forward, logq, sample, loss_and_grad, propose and slice_update take the
parameters they evaluate with (already rounded); train takes and returns the
masters, takes each gradient at their rounding and applies Adam to the
masters (a straight-through step).

Sampling draws the sites in order; site j takes spin +1 when its uniform is
below P(s_j = +1 | s_<j, cond) (state 0 first, as in the tensor-network
sampler), and log q is the sum of the logs of the probabilities taken.

Training minimises the mean of -log q_theta over (cond, s) pairs with Adam.
"""
from __future__ import annotations

import numpy as np

from . import chain, model, philox

N_LAYERS = 6
CHANNELS = 32
N_COND = 4
LOGIT_CLIP = 30.0
ADAM_B1 = 0.9
ADAM_B2 = 0.999
ADAM_EPS = 1e-8


def layer_shapes():
    """(c_in, c_out) of every layer."""
    shapes = [(N_COND + 1, CHANNELS)]
    shapes += [(CHANNELS, CHANNELS)] * (N_LAYERS - 2)
    shapes += [(CHANNELS, 1)]
    return shapes


def n_params() -> int:
    return sum(ci * co * 9 + co for ci, co in layer_shapes())


def unpack(theta):
    """Flat parameters -> list of (W[c_out, c_in, 3, 3], b[c_out]) in FP64."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for ci, co in layer_shapes():
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def mask(layer: int) -> np.ndarray:
    """M[c_in, ky, kx] in {0, 1}; tap (ky, kx) reads the site at offset (ky - 1, kx - 1)."""
    ci, _ = layer_shapes()[layer]
    earlier = np.zeros((3, 3))
    earlier[0, :] = 1.0          # the row above
    earlier[1, 0] = 1.0          # the site to the left
    M = np.ones((ci, 3, 3))
    if layer == 0:
        M[N_COND] = earlier      # type A on the spin channel; condition channels unmasked
    else:
        M[:] = earlier
        M[:, 1, 1] = 1.0         # type B: the centre is kept
    return M


def cond_channels(J, spins, z: int) -> np.ndarray:
    """The four condition channels [4, Ly, Lx] of layer z of an Ising lattice
    (J[3, Lz, Ly, Lx], spins [Lz, Ly, Lx] of +-1)."""
    J = np.asarray(J, dtype=np.float64)
    s = np.asarray(spins, dtype=np.float64)
    Lz = s.shape[0]
    c = np.zeros((N_COND,) + s.shape[1:])
    if z > 0:
        c[0] = J[2, z - 1] * s[z - 1]
    if z + 1 < Lz:
        c[1] = J[2, z] * s[z + 1]
    c[2] = J[0, z]
    c[3] = J[1, z]
    return c


def conv(x, W, b, M):
    """Masked 3x3 convolution with zero padding: x [c_in, Ly, Lx] -> [c_out, Ly, Lx]."""
    Ly, Lx = x.shape[1:]
    Wm = W * M[None]
    xp = np.zeros((x.shape[0], Ly + 2, Lx + 2))
    xp[:, 1:-1, 1:-1] = x
    out = np.broadcast_to(b[:, None, None], (W.shape[0], Ly, Lx)).copy()
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,cyx->oyx", Wm[:, :, ky, kx], xp[:, ky:ky + Ly, kx:kx + Lx])
    return out


def forward(theta, cond, s, keep=False):
    """Clipped logits l[Ly, Lx] of P(s = +1) for every site, given the whole
    layer s (each logit only sees earlier sites).  keep=True also returns the
    pre-activations and inputs of every layer (for the gradient)."""
    layers = unpack(theta)
    x = np.concatenate([np.asarray(cond, dtype=np.float64), np.asarray(s, dtype=np.float64)[None]])
    xs, pres = [], []
    for i, (W, b) in enumerate(layers):
        xs.append(x)
        pre = conv(x, W, b, mask(i))
        pres.append(pre)
        x = np.maximum(pre, 0.0) if i + 1 < N_LAYERS else pre
    logit = x[0]
    clipped = np.clip(logit, -LOGIT_CLIP, LOGIT_CLIP)
    if keep:
        return clipped, logit, xs, pres
    return clipped


def log_sigmoid(t):
    """log(1 / (1 + exp(-t))), without overflow."""
    t = np.asarray(t, dtype=np.float64)
    return -(np.maximum(-t, 0.0) + np.log1p(np.exp(-np.abs(t))))


def logq(theta, cond, s) -> float:
    """log q_theta(s | cond) = sum over sites of log P(s_j | s_<j, cond)."""
    s = np.asarray(s, dtype=np.float64)
    return float(np.sum(log_sigmoid(s * forward(theta, cond, s))))


def sample(theta, cond, uniforms):
    """Ancestral sampling with the given uniforms [Ly, Lx] (site order: rows,
    then columns).  Returns (spins [Ly, Lx] int8, log q, P(+1) per site)."""
    Ly, Lx = np.asarray(uniforms).shape
    s = np.ones((Ly, Lx))
    p_plus = np.zeros((Ly, Lx))
    lq = 0.0
    for y in range(Ly):
        for x in range(Lx):
            l = forward(theta, cond, s)[y, x]     # later sites are hidden by the masks
            p = 1.0 / (1.0 + np.exp(-l))
            p_plus[y, x] = p
            if uniforms[y][x] < p:
                s[y, x] = 1.0
                lq += float(log_sigmoid(l))
            else:
                s[y, x] = -1.0
                lq += float(log_sigmoid(-l))
    return s.astype(np.int8), lq, p_plus


def loss_and_grad(theta, conds, spins):
    """Mean of -log q_theta over a batch (conds [B, 4, Ly, Lx], spins [B, Ly, Lx])
    and its gradient with respect to the flat parameters, by the chain rule
    through the layers (masked weights get zero gradient; the clip passes no
    gradient where it is active)."""
    layers = unpack(theta)
    B = len(spins)
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in layers]
    total = 0.0
    for cond, s in zip(conds, spins):
        s = np.asarray(s, dtype=np.float64)
        clipped, logit, xs, pres = forward(theta, cond, s, keep=True)
        total -= float(np.sum(log_sigmoid(s * clipped)))
        # d(-log sigma(s l)) / dl = -s sigma(-s l)
        g = -s / (1.0 + np.exp(s * clipped)) / B
        g = np.where(np.abs(logit) < LOGIT_CLIP, g, 0.0)[None]
        for i in range(N_LAYERS - 1, -1, -1):
            W, _ = layers[i]
            Wm = W * mask(i)[None]
            x = xs[i]
            Ly, Lx = x.shape[1:]
            xp = np.zeros((x.shape[0], Ly + 2, Lx + 2))
            xp[:, 1:-1, 1:-1] = x
            gW, gb = grads[i]
            gb += g.sum(axis=(1, 2))
            gxp = np.zeros_like(xp)
            for ky in range(3):
                for kx in range(3):
                    gW[:, :, ky, kx] += np.einsum("oyx,cyx->oc", g, xp[:, ky:ky + Ly, kx:kx + Lx])
                    gxp[:, ky:ky + Ly, kx:kx + Lx] += np.einsum("oc,oyx->cyx", Wm[:, :, ky, kx], g)
            if i > 0:
                g = gxp[:, 1:-1, 1:-1] * (pres[i - 1] > 0.0)
    grads = [(gW * mask(i)[None], gb) for i, (gW, gb) in enumerate(grads)]
    return total / B, pack(grads)


def weights_bf16(theta) -> np.ndarray:
    """The BF16 parameters of FP32 master values: BF16 keeps the upper 16 bits
    of an IEEE binary32 (sign, 8 exponent bits, 7 mantissa bits); a binary32
    rounds to it to nearest, ties to even.  Masters given in float64 are taken
    to FP32 first (they are FP32 values).  Finite inputs; returns float64."""
    x = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).astype(np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF                      # the 16 bits dropped
    keep = u >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((keep & 1) == 1))
    r = (keep + up.astype(np.uint64)) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def adam_step(theta, m, v, grad, t: int, lr: float):
    """One Adam step (Kingma and Ba; t counts from 1).  Returns new (theta, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * grad * grad
    mh = m / (1.0 - ADAM_B1 ** t)
    vh = v / (1.0 - ADAM_B2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


def train(theta, conds, spins, epochs: int, batch: int, lr: float):
    """Plain minibatch Adam over the pairs in their given order (minibatches of
    `batch` consecutive pairs, the last one possibly shorter), on the master
    parameters theta, each gradient taken at their BF16 rounding.  Returns the
    masters and the loss of the last minibatch before its step."""
    theta = np.asarray(theta, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t = 0
    loss = float("nan")
    n = len(spins)
    for _ in range(epochs):
        for i in range(0, n, batch):
            loss, g = loss_and_grad(weights_bf16(theta), conds[i:i + batch], spins[i:i + batch])
            t += 1
            theta, m, v = adam_step(theta, m, v, g, t, lr)
    return theta, loss


def site_uniforms(seed: int, chain_key: int, sweep: int, z: int, Ly: int, Lx: int) -> np.ndarray:
    """The site uniforms of layer z in sweep `sweep` (purpose 0, draw y Lx + x),
    the same stream the tensor-network sampler draws from."""
    return np.array([[philox.uniform(seed, chain_key, sweep, z, 0, y * Lx + x) for x in range(Lx)]
                     for y in range(Ly)])


def propose(theta, J, spins, z: int, *, seed: int, chain_key: int, sweep: int):
    """One learned-proposal slice update of layer z, without changing spins:
    the drawn layer, log q of it and of the current layer, dE and the MH
    decision of main text Eq. 1 (uniform of purpose 1)."""
    Ly, Lx = spins.shape[1:]
    cond = cond_channels(J, spins, z)
    s_new, lq_new, p_plus = sample(theta, cond, site_uniforms(seed, chain_key, sweep, z, Ly, Lx))
    lq_old = logq(theta, cond, spins[z])
    after = spins.copy()
    after[z] = s_new
    dE = model.energy(J, after, 2) - model.energy(J, spins, 2)
    return {"s_new": s_new, "logq_new": lq_new, "logq_old": lq_old, "dE": dE, "p_plus": p_plus}


def slice_update(theta, J, spins, z: int, beta: float, *, seed: int, chain_key: int, sweep: int):
    """propose() followed by the Metropolis-Hastings decision; updates spins in place."""
    rec = propose(theta, J, spins, z, seed=seed, chain_key=chain_key, sweep=sweep)
    u = philox.uniform(seed, chain_key, sweep, z, 1, 0)
    rec["accepted"] = chain.mh_accept(rec["logq_old"], rec["logq_new"], beta, rec["dE"], u)
    if rec["accepted"]:
        spins[z] = rec["s_new"]
    return rec
