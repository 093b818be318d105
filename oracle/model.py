"""Lattice model: states, energies, the Markov-blanket field of a slice.

Oracle code (test infrastructure only).

* Ising / Edwards-Anderson energy E(s) = -sum_<ij> J_ij s_i s_j with s in {+1,-1}
  on a cubic lattice with free boundaries (main text, "Sampling 3D spin glasses";
  SM S1.A).
* 3-state Potts energy E = -J sum_<ij> delta(s_i, s_j) (main text, "Sampling the
  3-state 3D Potts model").
* TNMCMC-1 (SM S2.A): with the layers z-1 and z+1 held fixed (the Markov blanket
  of layer z), layer z sees a site-dependent external field.

States are handled as indices u in {0..d-1}.  For Ising, u=0 is s=+1 and u=1 is
s=-1 (SM S1.C projects s=+1 on (1,0)^T and s=-1 on (0,1)^T).  The bond factor
between states u and v is  exp(beta * J * sig(u, v))  with sig = s_u s_v (Ising)
or delta(u, v) (Potts); for Ising this is the matrix W of SM S1.A.
"""
from __future__ import annotations

import numpy as np

ISING_VALUE = np.array([1, -1], dtype=np.int64)


def to_states(spins: np.ndarray, d: int) -> np.ndarray:
    """int8 spins (+-1 for Ising, 0..2 for Potts) -> state indices."""
    spins = np.asarray(spins)
    if d == 2:
        return np.where(spins > 0, 0, 1).astype(np.int64)
    return spins.astype(np.int64)


def from_states(u: np.ndarray, d: int) -> np.ndarray:
    u = np.asarray(u, dtype=np.int64)
    if d == 2:
        return np.where(u == 0, 1, -1).astype(np.int8)
    return u.astype(np.int8)


def sig_table(d: int) -> np.ndarray:
    """sig[u, v]: s_u s_v for Ising, delta(u, v) for Potts."""
    if d == 2:
        return np.outer(ISING_VALUE, ISING_VALUE).astype(np.float64)
    return np.eye(d, dtype=np.float64)


def energy(J: np.ndarray, spins: np.ndarray, d: int) -> float:
    """Full-lattice energy E = -sum over bonds J * sig (spins indexed [z, y, x])."""
    u = to_states(spins, d)
    sig = sig_table(d)
    J = np.asarray(J, dtype=np.float64)
    E = 0.0
    E -= float(np.sum(J[0, :, :, :-1] * sig[u[:, :, :-1], u[:, :, 1:]]))
    E -= float(np.sum(J[1, :, :-1, :] * sig[u[:, :-1, :], u[:, 1:, :]]))
    E -= float(np.sum(J[2, :-1, :, :] * sig[u[:-1, :, :], u[1:, :, :]]))
    return E


def slice_field(J: np.ndarray, spins: np.ndarray, z: int, d: int) -> np.ndarray:
    """F[y, x, u] = sum over held neighbours (z-1, z+1) of J_z * sig(u, s_neighbour).

    This is the external field the Markov blanket exerts on layer z (SM S2.A); the
    Boltzmann factor of state u at (x, y) is exp(beta * F[y, x, u]).
    """
    Lz, Ly, Lx = spins.shape
    u = to_states(spins, d)
    sig = sig_table(d)
    J = np.asarray(J, dtype=np.float64)
    F = np.zeros((Ly, Lx, d))
    for v in range(d):
        if z > 0:
            F[:, :, v] += J[2, z - 1] * sig[v, u[z - 1]]
        if z < Lz - 1:
            F[:, :, v] += J[2, z] * sig[v, u[z + 1]]
    return F


def slice_energy(J: np.ndarray, F: np.ndarray, a: np.ndarray, z: int, d: int) -> float:
    """Energy terms of layer z in configuration a (state indices [y, x]):
    in-layer bonds plus the field of the held layers."""
    sig = sig_table(d)
    J = np.asarray(J, dtype=np.float64)
    Ly, Lx = a.shape
    E = 0.0
    E -= float(np.sum(J[0, z, :, :-1] * sig[a[:, :-1], a[:, 1:]]))
    E -= float(np.sum(J[1, z, :-1, :] * sig[a[:-1, :], a[1:, :]]))
    yy, xx = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    E -= float(np.sum(F[yy, xx, a]))
    return E


def magnetisation(spins: np.ndarray, d: int) -> float:
    """Ising: M = sum s / N.  Potts: M = (d * max_k n_k / N - 1) / (d - 1)."""
    N = spins.size
    if d == 2:
        return float(np.sum(spins.astype(np.int64))) / N
    counts = np.bincount(spins.reshape(-1).astype(np.int64), minlength=d)
    return (d * counts.max() / N - 1.0) / (d - 1)


def overlap(s1: np.ndarray, s2: np.ndarray) -> float:
    """Spin-glass overlap q = (1/N) sum_i s_i^(1) s_i^(2) (main text)."""
    return float(np.sum(s1.astype(np.int64) * s2.astype(np.int64))) / s1.size
