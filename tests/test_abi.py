"""CPU checks of the C ABI: the library loads, exports every declared entry point,
validates its arguments without touching a GPU, and its host-only pieces agree
with the oracle."""
import math
import os

import numpy as np
import pytest

import paper_2509_23945_amd as tn
from oracle import chain as ochain


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tn.api.LIB_PATH):
        from paper_2509_23945_amd import build
        build.build()
    return tn.load()


def test_exports_every_declared_symbol(lib):
    names = tn.declared_symbols()
    assert {"tnmc_lattice_init", "tnmc_slice_propose", "tnmc_mh_accept", "tnmc_sweep"} <= set(names)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing


def test_status_strings(lib):
    assert tn.tnmc_status_string(0) == "ok"
    assert tn.tnmc_status_string(-1) == "invalid argument"
    assert tn.tnmc_status_string(-5) == "unsupported configuration"


def test_mh_accept_matches_oracle(lib):
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(2000):
        lo, ln = rng.normal(-50, 20, size=2)
        beta = rng.uniform(0, 2)
        dE = float(rng.integers(-20, 20))
        u = rng.uniform(1e-12, 1 - 1e-12)
        assert tn.tnmc_mh_accept(lo, ln, beta, dE, u) == ochain.mh_accept(lo, ln, beta, dE, u)
    # boundary: u exactly at A is rejected (strict "<")
    A = math.exp(-1.0)
    assert not tn.tnmc_mh_accept(-1.0, 0.0, 1.0, 0.0, A)
    with pytest.raises(tn.TnmcError):
        tn.tnmc_mh_accept(0.0, 0.0, 1.0, 0.0, 0.0)
    with pytest.raises(tn.TnmcError):
        tn.tnmc_mh_accept(0.0, 0.0, 1.0, 0.0, 1.0)


def _desc(**kw):
    base = dict(Lx=4, Ly=4, Lz=4, d=2, chi=4, J=np.zeros((3, 4, 4, 4), np.float32), beta=1.0,
                spins=np.ones((4, 4, 4), np.int8))
    base.update(kw)
    return base


@pytest.mark.parametrize("bad", [dict(d=4), dict(chi=0), dict(Lx=0),
                                 dict(Lx=65, J=np.zeros((3, 4, 4, 65), np.float32), spins=np.ones((4, 4, 65), np.int8)),
                                 dict(beta=-1.0), dict(spins=np.zeros((4, 4, 4), np.int8)),
                                 dict(d=3, spins=np.full((4, 4, 4), 3, np.int8)),
                                 dict(pairs=np.array([[0, 5]]))])
def test_init_rejects_bad_arguments(lib, bad):
    with pytest.raises(tn.TnmcError) as ei:
        tn.tnmc_lattice_init(**_desc(**bad))
    assert ei.value.status == tn.api.TNMC_ERR_ARG


def test_init_rejects_unbuilt_configuration(lib):
    with pytest.raises(tn.TnmcError) as ei:
        tn.tnmc_lattice_init(**_desc(chi=200))
    assert ei.value.status == tn.api.TNMC_ERR_UNSUPPORTED


def test_flop_model(lib):
    c, s = tn.tnmc_flop_model(32, 32, 2, 32)
    assert 2e9 < c < 6e9 and 0 < s < 1e8
    c8, _ = tn.tnmc_flop_model(8, 8, 2, 16)
    assert c8 < c / 100
    # grows with chi
    assert tn.tnmc_flop_model(16, 16, 2, 32)[0] > tn.tnmc_flop_model(16, 16, 2, 16)[0]
    with pytest.raises(tn.TnmcError):
        tn.tnmc_flop_model(0, 4, 2, 4)


def test_learned_proposal_arguments_checked_on_host(lib):
    """The learned-proposal entry points reject bad arguments before any device work."""
    import ctypes
    ARG = tn.api.TNMC_ERR_ARG
    h = ctypes.c_void_p()
    assert lib.tnmc_nn_create(None, 0, None) == ARG
    bad = np.full(tn.TNMC_NN_PARAMS, np.nan, dtype=np.float32)
    assert lib.tnmc_nn_create(bad.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 0, ctypes.byref(h)) == ARG
    assert not h.value
    assert lib.tnmc_nn_free(None) == ARG
    assert lib.tnmc_nn_logq(None, None, None, 1, 4, 4, None, None) == ARG
    loss = ctypes.c_double()
    assert lib.tnmc_nn_loss_grad(None, None, None, 1, 4, 4, ctypes.byref(loss), None, None) == ARG
    assert lib.tnmc_nn_adam_step(None, None, 1e-3, None) == ARG
    assert lib.tnmc_nn_train(None, None, None, 1, 4, 4, 1, 1, 1e-3, None, None) == ARG
    assert lib.tnmc_nn_dataset(None, None, None, None) == ARG
    assert lib.tnmc_nn_sweep(None, 0, None, 1, 0, 0, 0, None, None) == ARG
    assert lib.tnmc_nn_counts(None, None, None) == ARG
    assert lib.tnmc_nn_set_fallback(None, None) == ARG
    assert lib.tnmc_nn_calibrate_fallback(None, 0.05, None) == ARG
    assert lib.tnmc_nn_slice_logq(None, None, 0, 0, None, None, None) == ARG


def test_checkpoint_arguments_checked_on_host(lib):
    assert tn.tnmc_status_string(-6) == "checkpoint file error"
    assert lib.tnmc_checkpoint_save(None, 0, b"/tmp/x") == tn.api.TNMC_ERR_ARG
    assert lib.tnmc_checkpoint_load(None, b"/tmp/x", None) == tn.api.TNMC_ERR_ARG
    assert lib.tnmc_get_couplings(None, None) == tn.api.TNMC_ERR_ARG


def test_direction_and_layout_arguments_checked_on_host(lib):
    import ctypes
    ARG = tn.api.TNMC_ERR_ARG
    lay = ctypes.c_int32()
    assert lib.tnmc_layout_choice(4, 32, 0, ctypes.byref(lay), None, None) == ARG
    assert lib.tnmc_layout_choice(2, 0, 0, ctypes.byref(lay), None, None) == ARG
    assert lib.tnmc_layout_choice(2, 32, 0, None, None, None) == ARG
    # untuned class: -1
    assert lib.tnmc_layout_choice(2, 32, 1, ctypes.byref(lay), None, None) == 0 and lay.value == -1
    eng = ctypes.c_int32()
    assert lib.tnmc_autotune_choice(2, 32, 0, None, ctypes.byref(eng), None) == ARG
    assert lib.tnmc_autotune_choice(5, 32, 0, ctypes.byref(lay), ctypes.byref(eng), None) == ARG
    assert lib.tnmc_autotune_choice(2, 32, 1, ctypes.byref(lay), ctypes.byref(eng), None) == 0
    assert lay.value == -1 and eng.value == -1
    assert lib.tnmc_autotune_pin(2, 0) == ARG and lib.tnmc_autotune_pin(0, -2) == ARG
    assert lib.tnmc_autotune_now(None, 1, None) == ARG
    assert lib.tnmc_sweep_direction(None, 1, 1, 1, 0, 0, 0, None, None) == ARG
    assert lib.tnmc_debug_set(5, 1) == ARG and lib.tnmc_debug_set(1, 2) == ARG
    assert lib.tnmc_debug_set(4, 2) == ARG
    assert lib.tnmc_debug_set(4, 1) == 0 and lib.tnmc_debug_set(4, 0) == 0
    # the rank cut-off knob takes exponents 0..15 (0 restores the defaults)
    assert lib.tnmc_debug_set(3, 16) == ARG and lib.tnmc_debug_set(3, -1) == ARG
    assert lib.tnmc_debug_set(3, 6) == 0 and lib.tnmc_debug_set(3, 0) == 0


def test_sweep_entry_points_reject_empty_lattice_lists(lib):
    """An empty or NULL lattice list and a negative sweep count are argument
    errors, returned before any device work."""
    import ctypes
    ARG = tn.api.TNMC_ERR_ARG
    empty = (ctypes.c_void_p * 1)()
    for lats in (None, empty):
        assert lib.tnmc_sweep(lats, 0, 1, 0, 0, 0, None, None) == ARG
        assert lib.tnmc_half_sweep(lats, 0, 0, 0, None, None, None) == ARG
        assert lib.tnmc_sweep_graph(lats, 0, 1, 0, 0, None, None) == ARG
        assert lib.tnmc_sweep_superspin(lats, 0, 1, 0, 0, 0, None, None, None) == ARG
        assert lib.tnmc_sweep_direction(lats, 0, 2, 1, 0, 0, 0, None, None) == ARG
        assert lib.tnmc_nn_sweep(lats, 0, None, 1, 0, 0, 0, None, None) == ARG
    # a list holding a NULL handle
    assert lib.tnmc_sweep(empty, 1, 1, 0, 0, 0, None, None) == ARG
    assert lib.tnmc_sweep(None, 1, -1, 0, 0, 0, None, None) == ARG


def test_binding_structs_match_the_header():
    """The ctypes mirrors of the header's by-value structs list the same fields,
    in the same order, with the same types (a field added on one side only
    would shift every later one)."""
    import ctypes
    import re
    hdr = open(os.path.join(os.path.dirname(tn.api.__file__), "..", "include", "tnmc.h")).read()
    hdr = re.sub(r"/\*.*?\*/", " ", hdr, flags=re.S)

    def fields_of(name):
        end = hdr.index("} " + name + ";")
        body = hdr[hdr.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
        out = []
        for decl in body.split(";"):
            words = decl.replace(",", " , ").replace("*", " * ").split()
            if not words:
                continue
            i = 0
            while words[i] == "const":
                i += 1
            ctype, rest = words[i], words[i + 1:]
            ptr = "*" in rest
            out += [(n, ctype + ("*" if ptr else "")) for n in rest if n not in (",", "*")]
        return out

    P = ctypes.POINTER
    kind = {"int64_t": ctypes.c_int64, "double": ctypes.c_double, "int32_t": ctypes.c_int32, "uint64_t": ctypes.c_uint64,
            "float*": P(ctypes.c_float), "int32_t*": P(ctypes.c_int32), "double*": P(ctypes.c_double),
            "int8_t*": P(ctypes.c_int8), "uint64_t*": P(ctypes.c_uint64)}
    for name, mirror in (("tnmc_stats", tn.api._Stats), ("tnmc_lattice_desc", tn.api._Desc)):
        fields = fields_of(name)
        assert [n for n, _ in fields] == [n for n, _ in mirror._fields_], name
        for (n, c), (_, t) in zip(fields, mirror._fields_):
            assert kind[c] == t, (name, n, c, t)
