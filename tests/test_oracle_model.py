"""Pins of the oracle's energies and layer field: integer energies, local energy
changes equal to full-lattice recomputation, and brute-force energies."""
import numpy as np
import pytest

import bruteforce as bf
import synth
from oracle import model


@pytest.mark.parametrize("d,kind", [(2, "pmj"), (2, "gauss"), (3, "ferro")])
def test_energy_matches_enumeration(d, kind):
    Lx, Ly, Lz = 2, 2, 3 if d == 2 else 2
    if kind == "pmj":
        J = synth.couplings_pm_j(Lx, Ly, Lz, 4)
    elif kind == "gauss":
        J = synth.couplings_gauss(Lx, Ly, Lz, 4)
    else:
        J = synth.couplings_uniform(Lx, Ly, Lz)
    st, E = bf.lattice_states(J, Lx, Ly, Lz, d)
    for i in range(0, st.shape[0], max(1, st.shape[0] // 97)):
        spins = model.from_states(st[i], d)
        assert model.energy(J, spins, d) == E[i]


def test_pm_j_and_potts_energies_are_integers():
    for seed in range(5):
        J = synth.couplings_pm_j(6, 5, 4, seed)
        s = synth.spins_random(6, 5, 4, seed + 100)
        E = model.energy(J, s, 2)
        assert E == int(E)
        Jp = synth.couplings_uniform(5, 4, 3)
        sp = synth.spins_random(5, 4, 3, seed, d=3)
        Ep = model.energy(Jp, sp, 3)
        assert Ep == int(Ep)


@pytest.mark.parametrize("d,kind", [(2, "pmj"), (2, "gauss"), (3, "ferro")])
def test_layer_energy_change_equals_full_recompute(d, kind):
    Lx, Ly, Lz = 5, 4, 4
    J = {"pmj": synth.couplings_pm_j, "gauss": synth.couplings_gauss}.get(
        kind, lambda a, b, c, s: synth.couplings_uniform(a, b, c))(Lx, Ly, Lz, 9)
    rng = np.random.Generator(np.random.PCG64(5))
    for z in range(Lz):
        s = synth.spins_random(Lx, Ly, Lz, 11 + z, d)
        F = model.slice_field(J, s, z, d)
        old = model.to_states(s[z], d)
        new = rng.integers(0, d, size=(Ly, Lx))
        s2 = s.copy()
        s2[z] = model.from_states(new, d)
        dE_local = model.slice_energy(J, F, new, z, d) - model.slice_energy(J, F, old, z, d)
        dE_full = model.energy(J, s2, d) - model.energy(J, s, d)
        assert dE_local == dE_full
        Fb = bf.layer_field(J, s, z, d)
        assert np.array_equal(F, np.array(Fb))
        assert model.slice_energy(J, F, new, z, d) == bf.config_energy(J, Fb, z, new.tolist(), d)


def test_overlap_and_magnetisation():
    a = np.array([[[1, -1], [1, 1]]], dtype=np.int8)
    b = np.array([[[1, 1], [-1, 1]]], dtype=np.int8)
    assert model.overlap(a, b) == 0.0
    assert model.overlap(a, a) == 1.0
    assert model.magnetisation(a, 2) == 0.5
    p = np.array([[[0, 0], [0, 0]]], dtype=np.int8)
    assert model.magnetisation(p, 3) == 1.0
