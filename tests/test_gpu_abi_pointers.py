"""Entry-point details that the parity tests do not reach.

* tnmc_slice_propose and tnmc_slice_logq take the layer buffers as host or
  device pointers alike: a drawn layer written to device memory equals the one
  written to host memory, and log q of a device-resident layer equals log q of
  the same layer on the host.
* Statistics: every sweep entry point reports its wall time (seconds > 0),
  and tnmc_nn_sweep counts the layer updates it left to the tensor-network
  fallback (flags per (chain, z), times the sweeps)."""
import ctypes

import numpy as np
import pytest

import gpu_helpers as gh
import paper_2509_23945_amd as tn

pytestmark = pytest.mark.gpu


def test_propose_and_logq_accept_device_buffers():
    import torch
    gh.announce("device s_new / s buffers 6x5x4")
    lat, J, spins, _ = gh.make_lattice(6, 5, 4, 2, 4, kind="gauss", beta=0.8, seed=3, n_chains=1)
    lib = tn.load()
    s_host, lq_new, lq_old, dE, st = tn.tnmc_slice_propose(lat, 0, 2, 7)
    dev = torch.zeros((5, 6), dtype=torch.int8, device="cuda")
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    r = lib.tnmc_slice_propose(lat.handle, 0, 2, ctypes.c_uint64(7),
                               ctypes.cast(ctypes.c_void_p(dev.data_ptr()), ctypes.POINTER(ctypes.c_int8)),
                               ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), None)
    assert r == st
    assert np.array_equal(dev.cpu().numpy(), s_host)
    assert (a.value, b.value, c.value) == (lq_new, lq_old, dE)
    lq_host = tn.tnmc_slice_logq(lat, 0, 2, s_host)
    lq = ctypes.c_double()
    assert lib.tnmc_slice_logq(lat.handle, 0, 2,
                               ctypes.cast(ctypes.c_void_p(dev.data_ptr()), ctypes.POINTER(ctypes.c_int8)),
                               ctypes.byref(lq), None) == 0
    assert lq.value == lq_host == lq_new
    tn.tnmc_lattice_free(lat)


def test_stats_report_wall_time_and_fallbacks():
    gh.announce("stats: seconds, nn_fallbacks")
    lat = gh.make_lattice(6, 6, 4, 2, 4, kind="pmj", beta=0.7, seed=5, n_chains=2)[0]
    st = tn.tnmc_sweep([lat], 2)
    assert st["seconds"] > 0.0 and st["nn_fallbacks"] == 0
    assert tn.tnmc_sweep_graph([lat], 2, sweep_offset=2)["seconds"] > 0.0
    assert tn.tnmc_sweep_superspin([lat], 1)["seconds"] > 0.0
    net = tn.tnmc_nn_create(None, seed=1)
    flags = np.zeros((2, 4), dtype=np.int8)
    flags[0, 1] = flags[1, 3] = flags[1, 0] = 1
    tn.tnmc_nn_set_fallback(lat, flags)
    st = tn.tnmc_nn_sweep([lat], net, 3, sweep_offset=5)
    assert st["nn_fallbacks"] == 3 * 3 and st["seconds"] > 0.0
    assert st["proposed"] == 3 * 8
    tn.tnmc_lattice_free(lat)
