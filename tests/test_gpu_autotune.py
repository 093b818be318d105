"""The layout autotuner: on the first sweep of a class with a compact layout it
times both layouts and keeps the faster one; the chain it then runs is the
same, bit for bit, as with the default layout (autotuner off)."""
import numpy as np
import pytest

import gpu_helpers as gh
import paper_2509_23945_amd as tn

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,chi,kind,beta", [(2, 20, "gauss", 1.0), (3, 12, "ferro", 0.55)])
def test_autotuned_layout_gives_the_same_chain(d, chi, kind, beta):
    gh.announce(f"autotune d={d} chi={chi}")
    try:
        tn.tnmc_debug_set(1, 0)
        a, _, _, _ = gh.make_lattice(9, 8, 4, d, chi, kind=kind, beta=beta, seed=41, n_chains=2)
        tn.tnmc_sweep([a], 3)
        assert tn.tnmc_layout_choice(d, chi)[0] == -1
        tn.tnmc_debug_set(1, 1)
        b, _, _, _ = gh.make_lattice(9, 8, 4, d, chi, kind=kind, beta=beta, seed=41, n_chains=2)
        tn.tnmc_sweep([b], 3)
        layout, ms_c, ms_f = tn.tnmc_layout_choice(d, chi)
        assert layout in (0, 1) and ms_c > 0 and ms_f > 0
        assert layout == (1 if ms_f < ms_c else 0)
        for c in range(2):
            assert np.array_equal(tn.tnmc_get_spins(a, c), tn.tnmc_get_spins(b, c))
    finally:
        tn.tnmc_debug_set(1, 1)
