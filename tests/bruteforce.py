"""Independent exact references used to pin the oracle (test helpers).

Everything here is written from the plain definitions (Boltzmann weights of
the model, the conditional of a layer given its neighbours), with explicit
loops over bonds, and shares no code with ``oracle/``:

* ``layer_energies``  - slice energy of every configuration by enumeration
* ``layer_logz_tm``   - exact log Z of a layer by a d^Lx row transfer matrix
* ``lattice_states``  - every configuration of a tiny 3D lattice with its energy
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def sig(u: int, v: int, d: int) -> float:
    if d == 2:
        return float((1 - 2 * u) * (1 - 2 * v))
    return 1.0 if u == v else 0.0


def state_of(spin: int, d: int) -> int:
    if d == 2:
        return 0 if spin > 0 else 1
    return int(spin)


def layer_field(J, spins, z: int, d: int):
    """F[y][x][u] from the held layers z-1 and z+1 (explicit loops)."""
    Lz, Ly, Lx = spins.shape
    F = [[[0.0] * d for _ in range(Lx)] for _ in range(Ly)]
    for y in range(Ly):
        for x in range(Lx):
            for u in range(d):
                f = 0.0
                if z > 0:
                    f += float(J[2, z - 1, y, x]) * sig(u, state_of(spins[z - 1, y, x], d), d)
                if z < Lz - 1:
                    f += float(J[2, z, y, x]) * sig(u, state_of(spins[z + 1, y, x], d), d)
                F[y][x][u] = f
    return F


def config_energy(J, F, z: int, a, d: int) -> float:
    """Energy of layer configuration a[y][x] (state indices): bonds plus field."""
    Ly, Lx = len(a), len(a[0])
    E = 0.0
    for y in range(Ly):
        for x in range(Lx):
            u = a[y][x]
            E -= F[y][x][u]
            if x + 1 < Lx:
                E -= float(J[0, z, y, x]) * sig(u, a[y][x + 1], d)
            if y + 1 < Ly:
                E -= float(J[1, z, y, x]) * sig(u, a[y + 1][x], d)
    return E


def all_layer_configs(Ly: int, Lx: int, d: int):
    for flat in itertools.product(range(d), repeat=Lx * Ly):
        yield [list(flat[y * Lx:(y + 1) * Lx]) for y in range(Ly)]


def layer_energies(J, spins, z: int, d: int):
    """(configs, energies) of every configuration of layer z."""
    Lz, Ly, Lx = spins.shape
    F = layer_field(J, spins, z, d)
    cfgs = list(all_layer_configs(Ly, Lx, d))
    E = np.array([config_energy(J, F, z, a, d) for a in cfgs])
    return cfgs, E


def logsumexp(v) -> float:
    v = np.asarray(v, dtype=np.float64)
    m = float(np.max(v))
    return m + math.log(float(np.sum(np.exp(v - m))))


def layer_logz_tm(J, spins, z: int, beta: float, d: int) -> float:
    """Exact log Z of layer z by a row transfer matrix over all d^Lx row states."""
    Lz, Ly, Lx = spins.shape
    F = layer_field(J, spins, z, d)
    rows = list(itertools.product(range(d), repeat=Lx))
    nr = len(rows)
    S = np.array(rows)                                   # (nr, Lx)
    sig_mat = np.array([[sig(u, v, d) for v in range(d)] for u in range(d)])

    def phi(y):                                          # in-row log weight of each row state
        out = np.zeros(nr)
        for x in range(Lx):
            out += beta * np.array([F[y][x][u] for u in range(d)])[S[:, x]]
            if x + 1 < Lx:
                out += beta * float(J[0, z, y, x]) * sig_mat[S[:, x], S[:, x + 1]]
        return out

    def vert(y):                                         # bond weights between rows y and y+1
        out = np.zeros((nr, nr))
        for x in range(Lx):
            out += beta * float(J[1, z, y, x]) * sig_mat[S[:, x][:, None], S[:, x][None, :]]
        return out

    logv = phi(0)
    for y in range(1, Ly):
        m = float(np.max(logv))
        v = np.exp(logv - m)
        V = np.exp(vert(y - 1))
        nxt = v @ V
        logv = np.log(nxt) + m + phi(y)
    return logsumexp(logv)


def lattice_states(J, Lx: int, Ly: int, Lz: int, d: int):
    """All d^(Lx Ly Lz) configurations of a tiny lattice as state indices
    (n, Lz, Ly, Lx) with their energies."""
    n = Lx * Ly * Lz
    idx = np.arange(d ** n)
    digits = np.zeros((d ** n, n), dtype=np.int64)
    for i in range(n):
        digits[:, i] = (idx // d ** i) % d
    st = digits.reshape(-1, Lz, Ly, Lx)
    sm = np.array([[sig(u, v, d) for v in range(d)] for u in range(d)])
    E = np.zeros(d ** n)
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                if x + 1 < Lx:
                    E -= float(J[0, z, y, x]) * sm[st[:, z, y, x], st[:, z, y, x + 1]]
                if y + 1 < Ly:
                    E -= float(J[1, z, y, x]) * sm[st[:, z, y, x], st[:, z, y + 1, x]]
                if z + 1 < Lz:
                    E -= float(J[2, z, y, x]) * sm[st[:, z, y, x], st[:, z + 1, y, x]]
    return st, E
