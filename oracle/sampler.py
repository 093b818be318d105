"""Ancestral sampling of one layer from its boundary-MPS environments, with the
exact log-probability of the drawn configuration.

Oracle code (test infrastructure only).

Follows the main text ("TNMCMC"): the conditional of the layer factorises as
P(s | sigma) = prod_i P(s_i | s_<i, sigma), each factor being a ratio of
partition functions with the earlier spins fixed; SM S1.C: fixed spins are
projected on basis vectors and the proposal is q(s) = prod_i q(s_i | s_<i);
SM Alg. 2 (SampleLayer): sample spin by spin, then evaluate q for the new and
for the current configuration of the layer.

Readings:

* Sites are visited row by row from the top (y = 0) and, within a row, from
  x = 0 to Lx-1.  Row y is conditioned on the sampled row y-1 through the
  vertical bonds, and on the rows below through E_y.
* Within a row, right environments R_x(alpha; t) sum the sites x..Lx-1 given
  the state t of site x-1; the weight of state u at site x is
      w(u) = exp(beta*(Ft(x,u) + Jx(x-1) sig(s_{x-1}, u))) * (l A_x[u]) . R_{x+1}(. ; u)
  with l the product of the already-fixed tensors of the row.
* A truncated contraction can make w(u) <= 0.  The weights are clamped at 0,
  normalised, floored at EPS = 1e-12 and normalised again, so every state
  keeps a positive probability.  log q uses these final probabilities.
* Draw rule: the state is the first u with U < p(0) + ... + p(u) (for Ising:
  s = +1 iff U < q(s=+1), as in SM Alg. 1).
* A non-positive or non-finite total weight is a numeric fault; the draw
  then falls back to a uniform choice and the fault is reported.
"""
from __future__ import annotations

import numpy as np

from .model import sig_table
from .philox import PURPOSE_SITE, uniform

EPS = 1e-12


def site_probabilities(w: np.ndarray):
    """Clamp, normalise, floor at EPS, normalise (returns (p, fault))."""
    wp = np.maximum(w, 0.0)
    S = float(np.sum(wp))
    if not (S > 0.0 and np.isfinite(S)):
        return np.full(w.shape[0], 1.0 / w.shape[0]), True
    p = np.maximum(wp / S, EPS)
    return p / np.sum(p), False


def draw(p: np.ndarray, U: float) -> int:
    c = 0.0
    for u in range(p.shape[0] - 1):
        c += p[u]
        if U < c:
            return u
    return p.shape[0] - 1


def sample_layer(envs, J, F, z: int, beta: float, d: int, *, forced=None,
                 seed: int = 0, chain: int = 0, sweep: int = 0, margins=None, site_probs=None,
                 purpose: int = PURPOSE_SITE):
    """Draw a layer configuration (state indices [y, x]) and its log q.

    With ``forced`` given, the draws are replaced by the given states
    (teacher forcing) and the result is log q(forced).  If ``margins`` is a
    list, the distance of every draw's uniform to the nearest cumulative
    threshold is appended to it (to recognise near-ties).  If ``site_probs``
    is a list, every site's final probabilities p(u) are appended to it in
    visiting order (drawn or forced), so a caller can check which state each
    site's uniform selects under these conditionals.  ``purpose`` selects the
    Philox stream of the site uniforms (another candidate drawn from the same
    environments uses another purpose).
    Returns (states, logq, fault)."""
    Ly, Lx, _ = F.shape
    sig = sig_table(d)
    Jd = np.asarray(J, dtype=np.float64)
    a = np.zeros((Ly, Lx), dtype=np.int64)
    logq = 0.0
    fault = False
    for y in range(Ly):
        Ft = F[y].copy()                                   # (Lx, d)
        if y > 0:
            for x in range(Lx):
                Ft[x] += Jd[1, z, y - 1, x] * sig[:, a[y - 1, x]]
        jx = np.zeros(Lx)
        jx[1:] = Jd[0, z, y, :-1]
        env = envs[y]
        # right environments
        R = [None] * (Lx + 1)
        R[Lx] = np.ones((1, d))
        for x in range(Lx - 1, -1, -1):
            A = env[x]
            v = np.einsum("aub,bu->au", A, R[x + 1])      # (chi_l, d)
            g = np.exp(beta * (Ft[x][None, :] + jx[x] * sig))   # g[t, u]
            Rx = v @ g.T                                   # (chi_l, t)
            m = np.max(np.abs(Rx))
            R[x] = Rx / m if m > 0 else Rx
        # left-to-right draws
        lvec = np.ones(1)
        prev = 0
        for x in range(Lx):
            A = env[x]
            mvec = np.einsum("a,aub->ub", lvec, A)         # (d, chi_r)
            loc = beta * Ft[x] + (beta * jx[x] * sig[prev] if x > 0 else 0.0)
            w = np.exp(loc) * np.einsum("ub,bu->u", mvec, R[x + 1])
            p, f = site_probabilities(w)
            fault |= f
            if site_probs is not None:
                site_probs.append(p.copy())
            if forced is not None:
                u = int(forced[y, x])
            else:
                U = uniform(seed, chain, sweep, z, purpose, y * Lx + x)
                u = draw(p, U)
                if margins is not None:
                    margins.append(float(np.min(np.abs(U - np.cumsum(p)[:-1]))))
            logq += float(np.log(p[u]))
            a[y, x] = u
            lvec = mvec[u]
            m = np.max(np.abs(lvec))
            if m > 0 and np.isfinite(m):
                lvec = lvec / m
            else:
                fault = True
            prev = u
    return a, logq, fault
