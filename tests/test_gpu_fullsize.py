"""Parity at the full benchmark size, in the launch configuration bench.py times:
one even half-sweep of the 3D +-J workload (32^3, chi = 32, 16 instances x 2
replicas, FP64) as a single batched launch.

The oracle (a fraction of a second per slice at this size, run in worker
processes) checks every one of the 512 tasks: log q of the current layer, and
for each task the proposal visible in the result (the written-back layer if
accepted), dE, log q of the proposal and the MH decision on the shared
uniform.  Every task is also checked through properties that hold at any
size: finite log q <= 0, and per chain the energy change of the half-sweep
equals the sum of dE over its accepted proposals (layers of one parity do not
interact)."""
import numpy as np
import pytest

import bench
import gpu_helpers as gh
import oracle_pool
import paper_2509_23945_amd as tn
from oracle import chain as ochain
from oracle import model
from oracle.philox import PURPOSE_MH, uniform

pytestmark = pytest.mark.gpu


def test_half_sweep_full_size():
    import torch

    gh.announce("full-size half-sweep ea32")
    lat, cfg, J, spins, inst, betas = bench.make_lattice("ea32")
    L, chi = cfg["L"], cfg["chi"]
    n_chains = len(inst)
    tasks = [(c, z) for c in range(n_chains) for z in range(0, L, 2)]   # trace order
    trace = torch.zeros(5 * len(tasks), dtype=torch.float64, device="cuda")
    st = tn.tnmc_half_sweep([lat], 0, 0, trace_ptr=trace.data_ptr())
    torch.cuda.synchronize()
    tr = trace.cpu().numpy().reshape(-1, 5)
    assert st["proposed"] == len(tasks) and st["numeric_faults"] == 0
    assert np.all(np.isfinite(tr[:, :3])) and np.all(tr[:, :2] <= 0.0)
    assert np.all((tr[:, 3] == 0.0) | (tr[:, 3] == 1.0)) and np.all(tr[:, 4] == 0.0)
    assert int(tr[:, 3].sum()) == st["accepted"]

    after = [tn.tnmc_get_spins(lat, c) for c in range(n_chains)]
    for c in range(n_chains):
        Jc = J[inst[c]]
        dE = sum(tr[k, 2] for k, (cc, _) in enumerate(tasks) if cc == c and tr[k, 3] == 1.0)
        assert model.energy(Jc, after[c], 2) - model.energy(Jc, spins[c], 2) == dE, c
        for z in range(1, L, 2):
            assert np.array_equal(after[c][z], spins[c][z])

    gh.announce(f"  oracle on all {len(tasks)} tasks")
    refs = oracle_pool.propose_many(J, spins, [(int(inst[c]), c, z, float(betas[c]), chi, 2, bench.PHILOX_SEED, c, 0)
                                               for (c, z) in tasks])
    checked = 0
    for k, (c, z) in enumerate(tasks):
        ref = refs[k]
        lq_new, lq_old, dE, acc, _ = tr[k]
        label = f"fullsize c{c} z{z}"
        assert gh.logq_close(lq_old, ref["logq_old"], "fp64 fullsize logq_old", (c, z)), (c, z, lq_old,
                                                                                          ref["logq_old"])
        tie = ref["min_margin"] < gh.TIE
        if acc == 1.0:
            if not np.array_equal(after[c][z], ref["new"]):
                assert tie, (c, z)   # a uniform on a cumulative threshold: both draws are correct
                continue
        else:
            assert np.array_equal(after[c][z], spins[c][z])
            if tie:
                continue             # the proposal itself is not visible after a rejection
        assert dE == ref["dE"], label
        assert gh.logq_close(lq_new, ref["logq_new"], "fp64 fullsize logq_new", (c, z)), (c, z, lq_new,
                                                                                          ref["logq_new"])
        u = uniform(bench.PHILOX_SEED, c, 0, z, PURPOSE_MH, 0)
        assert bool(acc) == ochain.mh_accept(ref["logq_old"], ref["logq_new"], betas[c], ref["dE"], u)
        checked += 1
    assert checked >= len(tasks) - 4
