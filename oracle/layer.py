"""A layer update in general form, and the TNMCMC-2 composite layer.

Oracle code (test infrastructure only).

TNMCMC-2 (SM S2.B, "coarse-graining with superspins"): two adjacent layers
z0 and z0 + 1 are merged into one composite layer of superspins with d = 2 x 2
= 4 states; the intra-layer couplings of both layers and the inter-layer
couplings between them go into the local tensors of the composite layer's 2D
network, whose Markov blanket is layers z0 - 1 and z0 + 2.  Sampling and the
Metropolis-Hastings step are those of TNMCMC-1 (SM Alg. 2, main text Eq. 1).

To serve both, a layer is described in general form (LayerModel): Ly x Lx
sites with d states and Boltzmann weight

    exp(beta * ( sum_sites F[y, x, u]
                 + sum_{x-bonds} sum_k Jx[k, y, x] sig[k, u, v]
                 + sum_{y-bonds} sum_k Jy[k, y, x] sig[k, u, v] ))

where Jx[k, y, x] couples (x, y)-(x+1, y) and Jy[k, y, x] couples
(x, y)-(x, y+1).

* A TNMCMC-1 layer z: K = 1, sig = s_u s_v (Ising) or delta (Potts),
  Jx = J_x(z), Jy = J_y(z), F = the held-layer field (model.slice_field).
* A composite layer z0 (Ising): u = ua + 2 ub with ua, ub the state indices of
  layers z0 and z0 + 1 (0 is s = +1).  K = 2: component 0 couples the z0
  spins (sig[0, u, v] = s(ua) s(va), couplings of layer z0), component 1 the
  z0 + 1 spins (sig[1, u, v] = s(ub) s(vb), couplings of layer z0 + 1).  The
  on-site term holds the bond between the two layers and the blanket:
  F[y, x, u] = Jz(z0) s(ua) s(ub) + Jz(z0 - 1) s(z0 - 1) s(ua) + Jz(z0 + 1) s(z0 + 2) s(ub)
  (terms with layers outside the lattice are absent).

The contraction (bottom-up boundary MPS with the left-to-right QR sweep and the
right-to-left truncating SVD sweep), the sampling order and the probability
rules are those of oracle/bmps.py and oracle/sampler.py, with the weights above;
on a TNMCMC-1 layer the results are the same.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bmps
from .model import ISING_VALUE, sig_table, to_states
from .philox import PURPOSE_SITE, uniform
from .sampler import draw, site_probabilities


@dataclass
class LayerModel:
    Jx: np.ndarray    # (K, Ly, Lx): x-bond couplings, column Lx-1 unused
    Jy: np.ndarray    # (K, Ly, Lx): y-bond couplings, row Ly-1 unused
    sig: np.ndarray   # (K, d, d)
    F: np.ndarray     # (Ly, Lx, d)

    @property
    def d(self) -> int:
        return self.F.shape[2]


def plain_layer(J, spins, z: int, d: int, F) -> LayerModel:
    """TNMCMC-1 layer z with the held-layer field F (model.slice_field)."""
    Jd = np.asarray(J, dtype=np.float64)
    return LayerModel(Jx=Jd[0, z][None].copy(), Jy=Jd[1, z][None].copy(), sig=sig_table(d)[None], F=np.asarray(F))


def superspin_sig() -> np.ndarray:
    s = ISING_VALUE.astype(np.float64)
    u = np.arange(4)
    ua, ub = u % 2, u // 2
    return np.stack([np.outer(s[ua], s[ua]), np.outer(s[ub], s[ub])])


def composite_layer(J, spins, z0: int) -> LayerModel:
    """Composite layer (z0, z0 + 1) of an Ising lattice, blanket z0 - 1 and z0 + 2."""
    Jd = np.asarray(J, dtype=np.float64)
    Lz, Ly, Lx = spins.shape
    s = ISING_VALUE.astype(np.float64)
    u = np.arange(4)
    sa, sb = s[u % 2], s[u // 2]                           # spin value of each sublayer per state
    F = Jd[2, z0][:, :, None] * (sa * sb)[None, None, :]
    if z0 > 0:
        F = F + (Jd[2, z0 - 1] * spins[z0 - 1])[:, :, None] * sa[None, None, :]
    if z0 + 2 < Lz:
        F = F + (Jd[2, z0 + 1] * spins[z0 + 2])[:, :, None] * sb[None, None, :]
    return LayerModel(Jx=np.stack([Jd[0, z0], Jd[0, z0 + 1]]), Jy=np.stack([Jd[1, z0], Jd[1, z0 + 1]]),
                      sig=superspin_sig(), F=F)


def composite_states(spins, z0: int) -> np.ndarray:
    return to_states(spins[z0], 2) + 2 * to_states(spins[z0 + 1], 2)


def composite_spins(states: np.ndarray):
    """(spins of layer z0, spins of layer z0 + 1) of composite states."""
    s = ISING_VALUE.astype(np.int8)
    return s[states % 2], s[states // 2]


def bond_exponent(m: LayerModel, comp: np.ndarray) -> np.ndarray:
    """sum_k J[k] sig[k] for the couplings comp (K,) of one bond: a (d, d) matrix."""
    return np.tensordot(comp, m.sig, axes=(0, 0))


def row_weights(m: LayerModel, y: int, x: int, beta: float, with_upper: bool):
    """Local MPO weight W[a, r, b] of site (x, y) (as bmps.row_weights)."""
    d = m.d
    na = d if x > 0 else 1
    nr = d if with_upper else 1
    hx = bond_exponent(m, m.Jx[:, y, x - 1]) if x > 0 else np.zeros((d, d))
    vy = bond_exponent(m, m.Jy[:, y - 1, x]) if (with_upper and y > 0) else np.zeros((d, d))
    W = np.empty((na, nr, d))
    for a in range(na):
        for r in range(nr):
            for b in range(d):
                e = m.F[y, x, b]
                if x > 0:
                    e += hx[a, b]
                if with_upper:
                    e += vy[r, b]
                W[a, r, b] = np.exp(beta * e)
    return W


def apply_row_mpo(env, m: LayerModel, y: int, beta: float):
    d = m.d
    Lx = len(env)
    out = []
    for x in range(Lx):
        A = env[x]
        W = row_weights(m, y, x, beta, with_upper=True)
        cl, _, cr = A.shape
        na = W.shape[0]
        if x < Lx - 1:
            B = np.einsum("arb,kbm->karmb", W, A)
            out.append(B.reshape(cl * na, d, cr * d))
        else:
            B = np.einsum("arb,kbm->karm", W, A)
            out.append(B.reshape(cl * na, d, cr))
    return out


def environments(m: LayerModel, beta: float, chi: int):
    """All row environments of the layer (bmps.environments with general weights)."""
    Ly, Lx, d = m.F.shape
    envs = [None] * Ly
    logscale = np.zeros(Ly)
    envs[Ly - 1] = bmps.trivial_env(Lx, d)
    for y in range(Ly - 1, 0, -1):
        B = apply_row_mpo(envs[y], m, y, beta)
        envs[y - 1], lc = bmps.compress(B, chi)
        logscale[y - 1] = logscale[y] + lc
    return envs, logscale


def log_partition(envs, logscale, m: LayerModel, beta: float) -> float:
    Lx = len(envs[0])
    L = np.ones((1, 1))
    lg = 0.0
    for x in range(Lx):
        W = row_weights(m, 0, x, beta, with_upper=False)[:, 0, :]
        L = np.einsum("ka,ab,kbm->mb", L, W, envs[0][x])
        s = np.max(np.abs(L))
        L = L / s
        lg += np.log(s)
    return float(np.log(np.sum(L)) + lg + logscale[0])


def sample_layer(envs, m: LayerModel, beta: float, *, forced=None, seed: int = 0, chain: int = 0, sweep: int = 0,
                 z_key: int = 0, purpose: int = PURPOSE_SITE, margins=None):
    """Draw (or, with forced, evaluate) a layer configuration with its log q:
    sampler.sample_layer with general weights; the site uniforms use the
    Philox counter (y*Lx + x, z_key, sweep, purpose).  Returns (states, logq, fault)."""
    Ly, Lx, d = m.F.shape
    a = np.zeros((Ly, Lx), dtype=np.int64)
    logq = 0.0
    fault = False
    for y in range(Ly):
        Ft = m.F[y].copy()
        if y > 0:
            for x in range(Lx):
                Ft[x] += bond_exponent(m, m.Jy[:, y - 1, x])[a[y - 1, x], :]
        hx = [bond_exponent(m, m.Jx[:, y, x - 1]) if x > 0 else np.zeros((d, d)) for x in range(Lx)]
        env = envs[y]
        R = [None] * (Lx + 1)
        R[Lx] = np.ones((1, d))
        for x in range(Lx - 1, -1, -1):
            v = np.einsum("aub,bu->au", env[x], R[x + 1])
            g = np.exp(beta * (Ft[x][None, :] + hx[x]))      # g[t, u]
            Rx = v @ g.T
            mx = np.max(np.abs(Rx))
            R[x] = Rx / mx if mx > 0 else Rx
        lvec = np.ones(1)
        prev = 0
        for x in range(Lx):
            mvec = np.einsum("a,aub->ub", lvec, env[x])
            loc = beta * Ft[x] + (beta * hx[x][prev] if x > 0 else 0.0)
            w = np.exp(loc) * np.einsum("ub,bu->u", mvec, R[x + 1])
            p, f = site_probabilities(w)
            fault |= f
            if forced is not None:
                u = int(forced[y, x])
            else:
                U = uniform(seed, chain, sweep, z_key, purpose, y * Lx + x)
                u = draw(p, U)
                if margins is not None:
                    margins.append(float(np.min(np.abs(U - np.cumsum(p)[:-1]))))
            logq += float(np.log(p[u]))
            a[y, x] = u
            lvec = mvec[u]
            mx = np.max(np.abs(lvec))
            if mx > 0 and np.isfinite(mx):
                lvec = lvec / mx
            else:
                fault = True
            prev = u
    return a, logq, fault


def layer_energy(m: LayerModel, a: np.ndarray) -> float:
    """Energy of the layer terms in configuration a (minus the exponent above)."""
    E = -float(np.sum(m.F[np.arange(a.shape[0])[:, None], np.arange(a.shape[1])[None, :], a]))
    for k in range(m.sig.shape[0]):
        E -= float(np.sum(m.Jx[k, :, :-1] * m.sig[k][a[:, :-1], a[:, 1:]]))
        E -= float(np.sum(m.Jy[k, :-1, :] * m.sig[k][a[:-1, :], a[1:, :]]))
    return E
