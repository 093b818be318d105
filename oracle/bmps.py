"""Boundary-MPS environments of one slice, in FP64.

Oracle code (test infrastructure only).

Follows SM S1.B (boundary MPS: a row MPO is applied to the boundary MPS, which
is then truncated back to bond dimension chi by SVD, keeping the largest
singular values) and SM S1.C (the cached intermediate tensors are reused by the
sampler), applied to the 2D network of one layer whose held neighbours enter as
an external field (SM S2.A).

Readings (the paper leaves the boundary-MPS details to its 2D reference):

* Environments are built bottom-up.  E_y(r) is the Boltzmann weight of rows
  y+1..Ly-1 summed over their states, including the vertical bonds from row y
  (state r) to row y+1.  E_{Ly-1} = 1.
* One row step applies the MPO of row y to E_y:
      B_x[r]_{(al,a),(be,b)} = exp(beta*(Jy(x,y-1) sig(r,b) + F(y,x,b) + Jx(x-1,y) sig(a,b))) * A_x[b]_{al,be}
  where b is the state of site (x, y), carried to the right in the bond so that
  the horizontal bond to the next site can be formed; a (the state of x-1) is
  absent at x = 0 and b is summed at x = Lx-1.
* Truncation: the R factors of a left-to-right QR sweep provide the metric of
  the left part; a right-to-left sweep then takes, at each bond, the SVD of the
  centre matrix C = R_{x-1} (B_x T_{x+1}) and keeps exactly min(chi, rows, cols)
  right singular vectors (no relative cut-off).  This is the textbook SVD
  compression of an MPS in mixed-canonical form, and the truncated state it
  produces is independent of the gauge.
* Scales are removed at every step and accumulated in log form, so the result
  is exp(logscale[y]) times an MPS whose first tensor has unit Frobenius norm.
"""
from __future__ import annotations

import numpy as np

from .model import sig_table


def row_weights(J, F, z: int, y: int, x: int, beta: float, d: int, with_upper: bool):
    """Local MPO weight W[a, r, b] of site (x, y); a-dimension 1 at x = 0 and
    r-dimension 1 for the top row (no row above)."""
    sig = sig_table(d)
    jx = float(J[0, z, y, x - 1]) if x > 0 else 0.0
    jy = float(J[1, z, y - 1, x]) if (with_upper and y > 0) else 0.0
    na = d if x > 0 else 1
    nr = d if with_upper else 1
    W = np.empty((na, nr, d))
    for a in range(na):
        for r in range(nr):
            for b in range(d):
                e = F[y, x, b]
                if x > 0:
                    e += jx * sig[a, b]
                if with_upper:
                    e += jy * sig[r, b]
                W[a, r, b] = np.exp(beta * e)
    return W


def apply_row_mpo(env, J, F, z: int, y: int, beta: float, d: int):
    """MPO of row y (vertical bonds to row y-1 as the open index r) applied to E_y."""
    Lx = len(env)
    out = []
    for x in range(Lx):
        A = env[x]                       # (chi_l, d, chi_r)
        W = row_weights(J, F, z, y, x, beta, d, with_upper=True)
        cl, _, cr = A.shape
        na = W.shape[0]
        if x < Lx - 1:
            B = np.einsum("arb,kbm->karmb", W, A)          # (cl, na, d, cr, d)
            out.append(B.reshape(cl * na, d, cr * d))
        else:
            B = np.einsum("arb,kbm->karm", W, A)           # b summed at the right edge
            out.append(B.reshape(cl * na, d, cr))
    return out


def compress(B, chi: int):
    """SVD truncation of an MPS to bond dimension chi (see module docstring).

    Returns (tensors, logscale) with tensors[0] of unit Frobenius norm."""
    Lx = len(B)
    # Left-to-right QR sweep; only the triangular factors are kept.
    Rs = []
    Rprev = np.ones((1, 1))
    for x in range(Lx - 1):
        M = np.tensordot(Rprev, B[x], axes=(1, 0))       # (r, d, Dr)
        r, dd, Dr = M.shape
        R = np.linalg.qr(M.reshape(r * dd, Dr), mode="r")
        s = np.max(np.abs(R))
        if s > 0:
            R = R / s
        Rs.append(R)
        Rprev = R
    # Right-to-left SVD sweep.
    logscale = 0.0
    new = [None] * Lx
    T = np.ones((B[Lx - 1].shape[2], 1))
    for x in range(Lx - 1, 0, -1):
        P = np.tensordot(B[x], T, axes=(2, 0))            # (Dl, d, k)
        Dl, dd, k = P.shape
        C = np.tensordot(Rs[x - 1], P, axes=(1, 0))       # (r, d, k)
        r = C.shape[0]
        _, S, Vt = np.linalg.svd(C.reshape(r, dd * k), full_matrices=False)
        kx = min(chi, S.shape[0])
        V = Vt[:kx]
        new[x] = V.reshape(kx, dd, k)
        T = P.reshape(Dl, dd * k) @ V.T                   # (Dl, kx)
        tn = np.linalg.norm(T)
        if tn > 0:
            T = T / tn
            logscale += np.log(tn)
    P0 = np.tensordot(B[0], T, axes=(2, 0))               # (1, d, k)
    c = np.linalg.norm(P0)
    if c > 0:
        P0 = P0 / c
        logscale += np.log(c)
    new[0] = P0
    return new, logscale


def trivial_env(Lx: int, d: int):
    return [np.ones((1, d, 1)) for _ in range(Lx)]


def environments(J, F, z: int, beta: float, chi: int, d: int):
    """All row environments E_0..E_{Ly-1} of layer z (cached for the sampler, SM S1.C).

    Returns (envs, logscale) where the true E_y equals exp(logscale[y]) times the MPS envs[y]."""
    Ly, Lx, _ = F.shape
    envs = [None] * Ly
    logscale = np.zeros(Ly)
    envs[Ly - 1] = trivial_env(Lx, d)
    for y in range(Ly - 1, 0, -1):
        B = apply_row_mpo(envs[y], J, F, z, y, beta, d)
        envs[y - 1], lc = compress(B, chi)
        logscale[y - 1] = logscale[y] + lc
    return envs, logscale


def log_partition(envs, logscale, J, F, z: int, beta: float, d: int) -> float:
    """log Z of the layer given its field: row 0's weights contracted with E_0.
    Exact when no truncation happened."""
    Lx = len(envs[0])
    L = np.ones((1, 1))                                   # (chi_l, a)
    lg = 0.0
    for x in range(Lx):
        W = row_weights(J, F, z, 0, x, beta, d, with_upper=False)[:, 0, :]   # (na, d)
        A = envs[0][x]
        L = np.einsum("ka,ab,kbm->mb", L, W, A)           # (chi_r, d)
        s = np.max(np.abs(L))
        L = L / s
        lg += np.log(s)
    return float(np.log(np.sum(L)) + lg + logscale[0])
