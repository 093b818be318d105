"""Sweeps replayed from a captured HIP graph against eager sweeps: two
lattices of different shapes (one in the compact two-per-CU layout with its
retry launch), three rounds of graph replays on one copy and eager sweeps on
the other, with eager work and synchronisation between the rounds; after
every round the chains' spins and the recorded observables are identical."""
import numpy as np
import pytest

import gpu_helpers as gh
import paper_2509_23945_amd as tn

pytestmark = pytest.mark.gpu


def _pair():
    a = gh.make_lattice(9, 8, 6, 2, 20, kind="gauss", beta=1.0, seed=51, n_chains=4, pairs=np.array([[0, 1], [2, 3]],
                        dtype=np.int32), record_capacity=40)[0]
    b = gh.make_lattice(6, 5, 5, 3, 6, kind="ferro", beta=0.55, seed=52, n_chains=2, record_capacity=40)[0]
    return [a, b]


def test_graph_sweeps_equal_eager_sweeps():
    gh.announce("graph replays vs eager sweeps")
    eager, graph = _pair(), _pair()
    sw = 0
    for rnd, k in enumerate((1, 3, 5)):
        tn.tnmc_sweep(eager, k, sweep_offset=sw, record=True)
        st = tn.tnmc_sweep_graph(graph, k, sweep_offset=sw, record=True)
        assert st["numeric_faults"] == 0
        sw += k
        for le, lg in zip(eager, graph):
            n_ch = 4 if le is eager[0] else 2
            for c in range(n_ch):
                assert np.array_equal(tn.tnmc_get_spins(le, c), tn.tnmc_get_spins(lg, c)), (rnd, c)
            for xe, xg in zip(tn.tnmc_timeseries(le), tn.tnmc_timeseries(lg)):
                assert np.array_equal(xe, xg), rnd
        # eager work between the replays
        tn.tnmc_energy(graph[0], 0)


def test_graph_record_capacity_is_respected():
    gh.announce("graph replays past the record capacity")
    lat = gh.make_lattice(5, 4, 4, 2, 4, kind="pmj", beta=0.7, seed=53, n_chains=2, record_capacity=3)[0]
    tn.tnmc_sweep_graph([lat], 5, record=True)
    E, M, q = tn.tnmc_timeseries(lat)
    assert E.shape[0] == 3
