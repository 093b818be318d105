"""Checkpoint / resume through the C ABI: a run interrupted by save + load
into a fresh lattice reproduces the uninterrupted run bit for bit (spins and
recorded observables), since every random number is a function of (seed,
chain key, sweep, layer, site); checkpoints of another lattice are refused."""
import numpy as np
import pytest

import gpu_helpers as gh
import paper_2509_23945_amd as tn

pytestmark = pytest.mark.gpu


def _lat(seed=4, record=10):
    return gh.make_lattice(6, 5, 4, 2, 4, kind="gauss", beta=0.8, seed=seed, n_chains=2, pairs=[(0, 1)],
                           record_capacity=record)


def test_resume_reproduces_the_uninterrupted_run(tmp_path):
    gh.announce("checkpoint resume 6x5x4")
    a, J, _, _ = _lat()
    assert np.array_equal(tn.tnmc_get_couplings(a), np.stack([J[0]]))
    tn.tnmc_sweep([a], 3, sweep_offset=0, record=True)
    flags = np.zeros((2, 4), dtype=np.int8)
    flags[1, 2] = 1
    tn.tnmc_nn_set_fallback(a, flags)
    path = str(tmp_path / "run.ckpt")
    tn.tnmc_checkpoint_save(a, 3, path)
    tn.tnmc_sweep([a], 2, sweep_offset=3, record=True)

    b, _, _, _ = _lat()
    nxt = tn.tnmc_checkpoint_load(b, path)
    assert nxt == 3
    assert np.array_equal(tn.tnmc_nn_get_fallback(b), flags)
    tn.tnmc_sweep([b], 2, sweep_offset=nxt, record=True)
    for c in range(2):
        assert np.array_equal(tn.tnmc_get_spins(a, c), tn.tnmc_get_spins(b, c))
    for xa, xb in zip(tn.tnmc_timeseries(a), tn.tnmc_timeseries(b)):
        assert xa.shape[0] == 5 and np.array_equal(xa, xb)


def test_checkpoint_of_another_lattice_is_refused(tmp_path):
    gh.announce("checkpoint mismatch")
    a, _, _, _ = _lat(seed=4)
    path = str(tmp_path / "a.ckpt")
    tn.tnmc_checkpoint_save(a, 0, path)
    other, _, _, _ = _lat(seed=5)           # other couplings
    small, _, _, _ = _lat(seed=4, record=0)  # no record capacity: fine, the checkpoint recorded nothing
    with pytest.raises(tn.TnmcError) as e:
        tn.tnmc_checkpoint_load(other, path)
    assert e.value.status == tn.api.TNMC_ERR_IO
    assert tn.tnmc_checkpoint_load(small, path) == 0
    junk = tmp_path / "junk.ckpt"
    junk.write_bytes(b"not a checkpoint at all")
    with pytest.raises(tn.TnmcError) as e:
        tn.tnmc_checkpoint_load(a, str(junk))
    assert e.value.status == tn.api.TNMC_ERR_IO
    with pytest.raises(tn.TnmcError) as e:
        tn.tnmc_checkpoint_load(a, str(tmp_path / "missing.ckpt"))
    assert e.value.status == tn.api.TNMC_ERR_IO
