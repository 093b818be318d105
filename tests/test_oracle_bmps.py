"""Pins of the oracle's boundary-MPS contraction.

Untruncated contraction must reproduce the exact partition function of a layer
(brute-force enumeration for small layers, a row transfer matrix for wider
ones), and the closed forms of the degenerate cases must come out."""
import math

import numpy as np
import pytest

import bruteforce as bf
import synth
from oracle import bmps, model


def _layer(Lx, Ly, d, kind, seed, Lz=3):
    if kind == "pmj":
        J = synth.couplings_pm_j(Lx, Ly, Lz, seed)
    elif kind == "gauss":
        J = synth.couplings_gauss(Lx, Ly, Lz, seed)
    else:
        J = synth.couplings_uniform(Lx, Ly, Lz)
    s = synth.spins_random(Lx, Ly, Lz, seed + 31, d)
    return J, s, Lz // 2


def _logz(J, s, z, beta, chi, d):
    F = model.slice_field(J, s, z, d)
    envs, ls = bmps.environments(J, F, z, beta, chi, d)
    return bmps.log_partition(envs, ls, J, F, z, beta, d)


SMALL = [(1, 1, 2), (4, 1, 2), (1, 4, 2), (2, 3, 2), (3, 3, 2), (4, 3, 2), (4, 4, 2),
         (3, 2, 3), (2, 3, 3), (3, 3, 3)]


@pytest.mark.parametrize("Lx,Ly,d", SMALL)
@pytest.mark.parametrize("beta", [0.3, 1.0, 2.0])
def test_exact_logz_matches_enumeration(Lx, Ly, d, beta):
    kinds = ["pmj", "gauss"] if d == 2 else ["ferro"]
    for kind in kinds:
        J, s, z = _layer(Lx, Ly, d, kind, 17 + Lx * 7 + Ly)
        chi = d ** ((Lx + 1) // 2)          # >= every exact bond dimension
        _, E = bf.layer_energies(J, s, z, d)
        assert abs(_logz(J, s, z, beta, chi, d) - bf.logsumexp(-beta * E)) < 1e-12 * max(1, abs(beta * E).max())


@pytest.mark.parametrize("Lx,Ly,chi", [(6, 5, 8), (8, 6, 16), (8, 8, 16), (9, 4, 16)])
def test_exact_logz_matches_transfer_matrix(Lx, Ly, chi):
    J, s, z = _layer(Lx, Ly, 2, "pmj", 3)
    for beta in (0.5, 1.0):
        ref = bf.layer_logz_tm(J, s, z, beta, 2)
        assert abs(_logz(J, s, z, beta, chi, 2) - ref) < 1e-11 * abs(ref)


def test_exact_logz_potts_transfer_matrix():
    J, s, z = _layer(5, 4, 3, "ferro", 8)
    ref = bf.layer_logz_tm(J, s, z, 0.55, 3)
    assert abs(_logz(J, s, z, 0.55, 9, 3) - ref) < 1e-11 * abs(ref)


def test_beta_zero_is_uniform():
    for d in (2, 3):
        J, s, z = _layer(5, 4, d, "pmj" if d == 2 else "ferro", 2)
        assert abs(_logz(J, s, z, 0.0, 1, d) - 20 * math.log(d)) < 1e-12


def test_no_in_layer_bonds_closed_form():
    """With the in-layer couplings set to zero the layer is a product of independent
    sites in their fields: log Z = sum log sum_u exp(beta F), exact at chi = 1."""
    Lx, Ly = 6, 5
    J = synth.couplings_pm_j(Lx, Ly, 3, 12)
    J[0] = 0.0
    J[1] = 0.0
    s = synth.spins_random(Lx, Ly, 3, 4)
    F = model.slice_field(J, s, 1, 2)
    ref = float(np.sum(np.log(np.sum(np.exp(1.1 * F), axis=2))))
    assert abs(_logz(J, s, 1, 1.1, 1, 2) - ref) < 1e-12 * abs(ref)


def test_single_column_chain_exact_at_chi_one():
    """Lx = 1: each row is one site, the boundary MPS has bond dimension 1 and the
    layer is a 1D chain along y with 2x2 transfer matrices."""
    J, s, z = _layer(1, 7, 2, "gauss", 21)
    beta = 0.8
    F = model.slice_field(J, s, z, 2)
    sv = np.array([1.0, -1.0])
    v = np.exp(beta * F[0, 0])
    for y in range(1, 7):
        T = np.exp(beta * float(J[1, z, y - 1, 0]) * np.outer(sv, sv))
        v = (v @ T) * np.exp(beta * F[y, 0])
    assert abs(_logz(J, s, z, beta, 1, 2) - math.log(v.sum())) < 1e-12


def test_truncation_error_shrinks_with_chi():
    """Truncated regime (field-free critical ferromagnet): |log Z_chi - log Z| decreases
    with chi and vanishes at the exact bond dimension."""
    Lx, Ly = 6, 6
    J = synth.couplings_uniform(Lx, Ly, 1)
    s = synth.spins_ordered(Lx, Ly, 1)
    beta = 0.44
    ref = bf.layer_logz_tm(J, s, 0, beta, 2)
    errs = [abs(_logz(J, s, 0, beta, chi, 2) - ref) for chi in (1, 2, 4, 8)]
    assert errs[0] > errs[1] > errs[2] > 1e-9
    assert errs[3] < 1e-12 * abs(ref)


def test_environments_unit_norm_and_bond_caps():
    J, s, z = _layer(8, 6, 2, "pmj", 5)
    F = model.slice_field(J, s, z, 2)
    envs, _ = bmps.environments(J, F, z, 1.0, 4, 2)
    for env in envs[:-1]:
        assert abs(np.linalg.norm(env[0]) - 1.0) < 1e-12
        for x, A in enumerate(env):
            assert A.shape[0] <= 4 and A.shape[2] <= 4
            if x > 0:   # right-orthonormal tensors from the SVD sweep
                M = A.reshape(A.shape[0], -1)
                assert np.allclose(M @ M.T, np.eye(A.shape[0]), atol=1e-12)
