"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only *generates inputs*: couplings, initial spins and inverse
temperatures, drawn from numpy's PCG64 from an explicit seed.  It contains none
of the method's arithmetic (no energies, no contractions, no sampling rule), so
both the product path and the oracle may import it without sharing any of the
computation they are compared on.

Conventions (the paper's model, main text "Sampling 3D spin glasses" and SM S1.A):

* Lattice of Lx x Ly x Lz sites with free (open) boundaries.
* Couplings are stored as ``J[3, Lz, Ly, Lx]`` float32: component 0 is the bond
  from (x, y, z) to (x+1, y, z), component 1 to (x, y+1, z), component 2 to
  (x, y, z+1).  Bonds that would leave the lattice are 0.
* Ising spins are int8 in {+1, -1}; Potts states are int8 in {0, 1, 2}.
"""
from __future__ import annotations

import numpy as np

GAUSS_QUANTUM = 2.0 ** -20   # Gaussian couplings are rounded to this grid
GAUSS_CLAMP = 8.0 - 2.0 ** -20


def _open_mask(Lx: int, Ly: int, Lz: int) -> np.ndarray:
    m = np.ones((3, Lz, Ly, Lx), dtype=bool)
    m[0, :, :, Lx - 1] = False
    m[1, :, Ly - 1, :] = False
    m[2, Lz - 1, :, :] = False
    return m


def couplings_pm_j(Lx: int, Ly: int, Lz: int, seed: int, p: float = 0.5) -> np.ndarray:
    """Edwards-Anderson +-J couplings: +1 with probability p, else -1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    J = np.where(rng.random((3, Lz, Ly, Lx)) < p, 1.0, -1.0).astype(np.float32)
    J[~_open_mask(Lx, Ly, Lz)] = 0.0
    return J


def couplings_gauss(Lx: int, Ly: int, Lz: int, seed: int) -> np.ndarray:
    """Gaussian couplings N(0,1), rounded to multiples of 2^-20 and clamped to |J| < 8.

    The rounding makes every coupling exactly representable in float32 and
    every energy an exact dyadic number, so energy differences can be compared
    bit for bit.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    J = rng.standard_normal((3, Lz, Ly, Lx))
    J = np.clip(np.round(J / GAUSS_QUANTUM) * GAUSS_QUANTUM, -GAUSS_CLAMP, GAUSS_CLAMP)
    J = J.astype(np.float32)
    J[~_open_mask(Lx, Ly, Lz)] = 0.0
    return J


def couplings_uniform(Lx: int, Ly: int, Lz: int, J0: float = 1.0) -> np.ndarray:
    """Uniform coupling J0 on every bond (ferromagnetic Ising, or Potts with J=J0)."""
    J = np.full((3, Lz, Ly, Lx), J0, dtype=np.float32)
    J[~_open_mask(Lx, Ly, Lz)] = 0.0
    return J


def spins_random(Lx: int, Ly: int, Lz: int, seed: int, d: int = 2) -> np.ndarray:
    """Uniformly random initial configuration: +-1 for d=2, states 0..d-1 otherwise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if d == 2:
        return np.where(rng.random((Lz, Ly, Lx)) < 0.5, 1, -1).astype(np.int8)
    return rng.integers(0, d, size=(Lz, Ly, Lx)).astype(np.int8)


def spins_ordered(Lx: int, Ly: int, Lz: int, d: int = 2) -> np.ndarray:
    """All spins up (+1) for d=2, all in state 0 for Potts."""
    return np.full((Lz, Ly, Lx), 1 if d == 2 else 0, dtype=np.int8)


def betas_uniform(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """n inverse temperatures uniform on [lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return lo + (hi - lo) * rng.random(n)


def slice_problem(Lx: int, Ly: int, seed: int, d: int = 2, kind: str = "pmj"):
    """A random single-slice problem: a 3-layer lattice (Lz=3) whose middle layer is
    the active slice and whose outer layers provide the fields.

    Returns (J, spins) with J[3,3,Ly,Lx] and spins[3,Ly,Lx].
    """
    if kind == "pmj":
        J = couplings_pm_j(Lx, Ly, 3, seed)
    elif kind == "gauss":
        J = couplings_gauss(Lx, Ly, 3, seed)
    elif kind == "ferro":
        J = couplings_uniform(Lx, Ly, 3)
    else:
        raise ValueError(kind)
    s = spins_random(Lx, Ly, 3, seed + 7919, d)
    return J, s


def nn_params(seed: int, shapes, scale: float = 1.0) -> np.ndarray:
    """Flat float32 parameters of a stack of 3x3 convolutions, shapes = [(c_in,
    c_out), ...]: per layer W[c_out][c_in][3][3] ~ N(0, scale^2 2 / (9 c_in))
    then b[c_out] ~ N(0, (0.1 scale)^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for ci, co in shapes:
        parts.append(rng.standard_normal(co * ci * 9) * scale * np.sqrt(2.0 / (9 * ci)))
        parts.append(rng.standard_normal(co) * 0.1 * scale)
    return np.concatenate(parts).astype(np.float32)
