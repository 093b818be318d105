"""The allocation-free proposal entry point (static device scratch) against
the allocating one, through the C ABI: two calls in a row, the second on a
smaller layer, each equal to tnmc_slice_propose's result on the same lattice
(spins and dE bit-exact, log q within the FP64 bar); a layer whose workspace
exceeds the static scratch is refused."""
import numpy as np
import pytest

import gpu_helpers as gh
import paper_2509_23945_amd as tn

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a[4] == b[4] == 0
    assert np.array_equal(a[0], b[0])
    assert a[3] == b[3]
    assert gh.logq_close(a[1], b[1]) and gh.logq_close(a[2], b[2]), (a[1:3], b[1:3])


@pytest.mark.parametrize("precision", [tn.TNMC_FP64, tn.TNMC_FP32])
def test_static_propose_equals_allocating_propose(precision):
    gh.announce(f"static scratch propose, precision {precision}: 32x32 chi=32, then 8x8 chi=16")
    big = gh.make_lattice(32, 32, 4, 2, 32, kind="pmj", beta=1.0, seed=3, precision=precision)[0]
    small = gh.make_lattice(8, 8, 8, 2, 16, kind="pmj", beta=0.5, seed=4, precision=precision)[0]
    for lat, z, sweep in ((big, 1, 3), (small, 5, 9)):
        want = tn.tnmc_slice_propose(lat, 0, z, sweep)
        got = tn.tnmc_slice_propose_static(lat, 0, z, sweep)
        _same(got, want)
    # once more on the big layer after the small one used the scratch
    _same(tn.tnmc_slice_propose_static(big, 0, 2, 4), tn.tnmc_slice_propose(big, 0, 2, 4))


def test_static_propose_potts_and_refusal():
    gh.announce("static scratch propose: Potts chi=20 (global tiles), then a 64x64 chi=32 layer refused")
    potts = gh.make_lattice(7, 6, 3, 3, 20, kind="ferro", beta=0.55, seed=3)[0]
    _same(tn.tnmc_slice_propose_static(potts, 0, 1, 2), tn.tnmc_slice_propose(potts, 0, 1, 2))
    huge = gh.make_lattice(64, 64, 2, 2, 32, kind="pmj", beta=1.0, seed=1)[0]
    with pytest.raises(tn.TnmcError) as e:
        tn.tnmc_slice_propose_static(huge, 0, 0, 0)
    assert e.value.status == -1 and "static scratch" in str(e.value)
