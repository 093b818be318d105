"""Direction cycling through the C ABI: sweeps with slices perpendicular to y
and to x equal the oracle's sweeps of the lattice with permuted axes
(oracle.chain.sweep_direction), spin for spin, on non-cubic lattices (an axis
or coupling mix-up changes the result), and the observables recorded after
cycled sweeps are the energies of the resulting configurations."""
import numpy as np
import pytest

import gpu_helpers as gh
import paper_2509_23945_amd as tn
from oracle import chain as ochain
from oracle import model

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("direction,d,kind", [(1, 2, "gauss"), (2, 2, "gauss"), (1, 3, "ferro"), (2, 2, "pmj")])
def test_direction_sweep_matches_oracle(direction, d, kind):
    gh.announce(f"direction sweep dir={direction} d={d} {kind}")
    Lx, Ly, Lz, chi, beta = 5, 4, 6, 4, (0.55 if d == 3 else 0.8)
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, d, chi, kind=kind, beta=beta, seed=31, n_chains=2)
    tn.tnmc_sweep_direction([lat], direction, 1, sweep_offset=3)
    for c in range(2):
        ref = spins[c].copy()
        ochain.sweep_direction(J[c], ref, beta, chi, d, direction, seed=12345, chain=c, sweep_index=3)
        assert np.array_equal(tn.tnmc_get_spins(lat, c), ref)


def test_cycled_sweeps_and_record():
    gh.announce("cycled sweeps 4x5x3")
    Lx, Ly, Lz, chi, beta = 4, 5, 3, 4, 0.9
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, chi, kind="gauss", beta=beta, seed=32, n_chains=2,
                                       record_capacity=6)
    ref = [spins[c].copy() for c in range(2)]
    for t in range(6):
        direction = t % 3
        tn.tnmc_sweep_direction([lat], direction, 1, sweep_offset=t, record=True)
        for c in range(2):
            ochain.sweep_direction(J[c], ref[c], beta, chi, 2, direction, seed=12345, chain=c, sweep_index=t)
    E, _, _ = tn.tnmc_timeseries(lat)
    assert E.shape == (6, 2)
    for c in range(2):
        assert np.array_equal(tn.tnmc_get_spins(lat, c), ref[c])
        assert E[-1, c] == model.energy(J[c], ref[c], 2)


def test_direction_argument_checked():
    lat, _, _, _ = gh.make_lattice(4, 4, 4, 2, 4, seed=1)
    for bad in (-1, 3):
        with pytest.raises(tn.TnmcError) as e:
            tn.tnmc_sweep_direction([lat], bad, 1)
        assert e.value.status == tn.api.TNMC_ERR_ARG


@pytest.mark.parametrize("direction", [1, 2])
def test_direction_sweep_is_the_z_sweep_of_the_permuted_lattice(direction):
    """On a reduced-precision lattice (no bit-exact oracle there): a sweep along
    `direction` equals a plain z-slice sweep of a second lattice built from the
    permuted couplings and spins, with the direction's sweep counter."""
    gh.announce(f"direction vs permuted lattice dir={direction}")
    Lx, Ly, Lz, chi, beta = 5, 4, 6, 4, 0.8
    lat, J, spins, _ = gh.make_lattice(Lx, Ly, Lz, 2, chi, kind="gauss", beta=beta, seed=33, n_chains=2,
                                       precision=tn.TNMC_FP32)
    perm = [ochain.to_direction(J[c], spins[c], direction) for c in range(2)]
    nz, ny, nx = perm[0][1].shape
    view = tn.tnmc_lattice_init(Lx=nx, Ly=ny, Lz=nz, d=2, chi=chi, J=np.stack([p[0] for p in perm]),
                                beta=np.full(2, beta), spins=np.stack([p[1] for p in perm]),
                                chain_instance=np.arange(2, dtype=np.int32), seed=12345, precision=tn.TNMC_FP32)
    tn.tnmc_sweep_direction([lat], direction, 1, sweep_offset=2)
    tn.tnmc_sweep([view], 1, sweep_offset=2 + direction * ochain.DIRECTION_STRIDE)
    for c in range(2):
        assert np.array_equal(tn.tnmc_get_spins(lat, c), ochain.from_direction(tn.tnmc_get_spins(view, c), direction))
