"""ctypes binding of libtnmc (include/tnmc.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Host arrays are
numpy arrays; device buffers (``trace``) and streams are passed as integer
addresses (for instance ``tensor.data_ptr()`` and
``torch.cuda.current_stream().cuda_stream``).  Nothing here computes any part
of the method: when the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtnmc.so")
HEADER_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tnmc.h")

TNMC_OK = 0
TNMC_ERR_ARG = -1
TNMC_ERR_OOM = -2
TNMC_ERR_DEVICE = -3
TNMC_ERR_NUMERIC = -4
TNMC_ERR_UNSUPPORTED = -5
TNMC_ERR_IO = -6
TNMC_FP64 = 0
TNMC_FP32 = 1

__all__ = [
    "TnmcError", "load", "declared_symbols", "tnmc_lattice_init", "tnmc_lattice_free", "tnmc_slice_propose",
    "tnmc_slice_logq", "tnmc_mh_accept", "tnmc_sweep", "tnmc_half_sweep", "tnmc_get_spins", "tnmc_set_spins",
    "tnmc_energy", "tnmc_timeseries", "tnmc_timeseries_reset", "tnmc_flop_model", "tnmc_debug_workspace", "tnmc_debug_set",
    "tnmc_status_string",
    "tnmc_last_error", "Lattice", "TNMC_FP64", "TNMC_FP32", "TNMC_NN_PARAMS", "Nn", "tnmc_nn_create", "tnmc_nn_free",
    "tnmc_nn_get_params", "tnmc_nn_set_params", "tnmc_nn_logq", "tnmc_nn_loss_grad", "tnmc_nn_adam_step",
    "tnmc_nn_train", "tnmc_nn_dataset", "tnmc_nn_slice_propose", "tnmc_nn_slice_logq", "tnmc_nn_sweep",
    "tnmc_nn_counts", "tnmc_nn_counts_reset", "tnmc_nn_set_fallback", "tnmc_nn_get_fallback",
    "tnmc_nn_calibrate_fallback", "tnmc_get_couplings", "tnmc_checkpoint_save", "tnmc_checkpoint_load",
    "tnmc_sweep_direction", "tnmc_layout_choice", "tnmc_slice_propose_static", "tnmc_autotune_choice",
    "tnmc_autotune_pin", "tnmc_autotune_now", "tnmc_sweep_graph", "tnmc_sweep_superspin",
]
TNMC_NN_PARAMS = 38753


class TnmcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = f"{where}: {tnmc_status_string(status)} ({status})"
        detail = tnmc_last_error()
        if detail:
            msg += f" [{detail}]"
        super().__init__(msg)


class _Desc(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("Lz", ctypes.c_int32),
        ("d", ctypes.c_int32), ("chi", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_chains", ctypes.c_int32), ("n_instances", ctypes.c_int32),
        ("J", ctypes.POINTER(ctypes.c_float)),
        ("chain_instance", ctypes.POINTER(ctypes.c_int32)),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("spins", ctypes.POINTER(ctypes.c_int8)),
        ("seed", ctypes.c_uint64),
        ("chain_key", ctypes.POINTER(ctypes.c_uint64)),
        ("n_pairs", ctypes.c_int32),
        ("pairs", ctypes.POINTER(ctypes.c_int32)),
        ("record_capacity", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("proposed", ctypes.c_int64), ("accepted", ctypes.c_int64), ("numeric_faults", ctypes.c_int64),
        ("contract_ms", ctypes.c_double), ("sample_ms", ctypes.c_double), ("contract_flops", ctypes.c_double),
        ("contract_launches", ctypes.c_int64), ("sample_launches", ctypes.c_int64),
        ("contract_retries", ctypes.c_int64), ("seconds", ctypes.c_double), ("nn_fallbacks", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load libtnmc.so (raises if it has not been built).

    The library links the system HIP runtime; torch wheels carry a runtime of
    their own.  A process that uses both must let torch initialise its GPU
    state first (any torch.cuda call), or torch finds no device afterwards;
    device pointers and the null stream work across the two."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.tnmc_lattice_init.argtypes = [P(_Desc), P(vp)]
    lib.tnmc_lattice_free.argtypes = [vp]
    lib.tnmc_slice_propose.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P(ctypes.c_int8),
                                       P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double), vp]
    lib.tnmc_slice_propose_static.argtypes = lib.tnmc_slice_propose.argtypes
    lib.tnmc_slice_logq.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int8), P(ctypes.c_double), vp]
    lib.tnmc_mh_accept.argtypes = [ctypes.c_double] * 5 + [P(ctypes.c_int32)]
    lib.tnmc_sweep.argtypes = [P(vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                               ctypes.c_int32, P(_Stats), vp]
    lib.tnmc_half_sweep.argtypes = [P(vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, vp, P(_Stats), vp]
    lib.tnmc_get_spins.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int8)]
    lib.tnmc_set_spins.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int8)]
    lib.tnmc_energy.argtypes = [vp, ctypes.c_int32, P(ctypes.c_double)]
    lib.tnmc_timeseries.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double),
                                    P(ctypes.c_int64)]
    lib.tnmc_timeseries_reset.argtypes = [vp]
    lib.tnmc_flop_model.argtypes = [ctypes.c_int32] * 4 + [P(ctypes.c_double), P(ctypes.c_double)]
    lib.tnmc_debug_workspace.argtypes = [ctypes.c_int32, vp, ctypes.c_int64]
    lib.tnmc_debug_workspace.restype = ctypes.c_int
    lib.tnmc_debug_set.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.tnmc_debug_set.restype = ctypes.c_int
    lib.tnmc_status_string.argtypes = [ctypes.c_int]
    lib.tnmc_status_string.restype = ctypes.c_char_p
    lib.tnmc_last_error.argtypes = []
    lib.tnmc_last_error.restype = ctypes.c_char_p
    i32, u64, i64, dbl = ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
    nn_sigs = {
        "tnmc_nn_create": [P(ctypes.c_float), u64, P(vp)],
        "tnmc_nn_free": [vp],
        "tnmc_nn_get_params": [vp, P(ctypes.c_float)],
        "tnmc_nn_set_params": [vp, P(ctypes.c_float)],
        "tnmc_nn_logq": [vp, vp, vp, i32, i32, i32, vp, vp],
        "tnmc_nn_loss_grad": [vp, vp, vp, i32, i32, i32, P(dbl), vp, vp],
        "tnmc_nn_adam_step": [vp, vp, dbl, vp],
        "tnmc_nn_train": [vp, vp, vp, i64, i32, i32, i32, i32, dbl, P(dbl), vp],
        "tnmc_nn_dataset": [vp, vp, vp, vp],
        "tnmc_nn_slice_propose": [vp, vp, i32, i32, u64, P(ctypes.c_int8), P(dbl), P(dbl), P(dbl), vp],
        "tnmc_nn_slice_logq": [vp, vp, i32, i32, P(ctypes.c_int8), P(dbl), vp],
        "tnmc_nn_sweep": [P(vp), i32, vp, i32, u64, i32, i32, P(_Stats), vp],
        "tnmc_nn_counts": [vp, P(i64), P(i64)],
        "tnmc_nn_counts_reset": [vp],
        "tnmc_nn_set_fallback": [vp, P(ctypes.c_int8)],
        "tnmc_nn_get_fallback": [vp, P(ctypes.c_int8)],
        "tnmc_nn_calibrate_fallback": [vp, dbl, P(i32)],
        "tnmc_get_couplings": [vp, P(ctypes.c_float)],
        "tnmc_checkpoint_save": [vp, u64, ctypes.c_char_p],
        "tnmc_checkpoint_load": [vp, ctypes.c_char_p, P(u64)],
        "tnmc_sweep_direction": [P(vp), i32, i32, i32, u64, i32, i32, P(_Stats), vp],
        "tnmc_layout_choice": [i32, i32, i32, P(i32), P(dbl), P(dbl)],
        "tnmc_autotune_choice": [i32, i32, i32, P(i32), P(i32), P(dbl)],
        "tnmc_autotune_pin": [i32, i32],
        "tnmc_autotune_now": [P(vp), i32, vp],
        "tnmc_sweep_graph": [P(vp), i32, i32, u64, i32, P(_Stats), vp],
        "tnmc_sweep_superspin": [P(vp), i32, i32, u64, i32, i32, vp, P(_Stats), vp],
    }
    for name, sig in nn_sigs.items():
        getattr(lib, name).argtypes = sig
        getattr(lib, name).restype = ctypes.c_int
    for name in ("tnmc_lattice_init", "tnmc_lattice_free", "tnmc_slice_propose", "tnmc_slice_logq",
                 "tnmc_mh_accept", "tnmc_sweep", "tnmc_half_sweep", "tnmc_get_spins", "tnmc_set_spins",
                 "tnmc_energy", "tnmc_timeseries", "tnmc_timeseries_reset", "tnmc_flop_model"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def declared_symbols(header: str = HEADER_PATH):
    """Names of the functions declared in include/tnmc.h."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tnmc_[a-z_0-9]+)\s*\(", text)))


def _check(status: int, where: str, allow=()):
    if status != TNMC_OK and status not in allow:
        raise TnmcError(status, where)
    return status


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def tnmc_status_string(status: int) -> str:
    return load().tnmc_status_string(status).decode()


def tnmc_last_error() -> str:
    return load().tnmc_last_error().decode()


class Lattice:
    """Handle of a tnmc_lattice plus its shape (host-side bookkeeping only)."""

    def __init__(self, handle, Lx, Ly, Lz, d, chi, n_chains, n_pairs, record_capacity):
        self.handle = handle
        self.Lx, self.Ly, self.Lz, self.d, self.chi = Lx, Ly, Lz, d, chi
        self.n_chains, self.n_pairs, self.record_capacity = n_chains, n_pairs, record_capacity

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tnmc_lattice_free(self.handle)
            self.handle = None


def tnmc_lattice_init(*, Lx, Ly, Lz, d, chi, J, beta, spins, chain_instance=None, seed=0, chain_key=None,
                      pairs=None, record_capacity=0, precision=TNMC_FP64, n_candidates=1) -> Lattice:
    lib = load()
    J = np.ascontiguousarray(J, dtype=np.float32)
    spins = np.ascontiguousarray(spins, dtype=np.int8)
    n_chains = spins.shape[0] if spins.ndim == 4 else 1
    sites = Lx * Ly * Lz
    if sites > 0:   # shapes are checked here; values and limits by the library
        if spins.size != n_chains * sites or J.size % (3 * sites) != 0:
            raise ValueError("spins / J do not match (Lx, Ly, Lz)")
    n_inst = J.size // (3 * sites) if sites > 0 else 1
    beta = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, dtype=np.float64), (n_chains,)))
    ci = None if chain_instance is None else np.ascontiguousarray(chain_instance, dtype=np.int32)
    ck = None if chain_key is None else np.ascontiguousarray(chain_key, dtype=np.uint64)
    pr = np.zeros((0, 2), dtype=np.int32) if pairs is None else np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    if (ci is not None and ci.size != n_chains) or (ck is not None and ck.size != n_chains):
        raise ValueError("chain_instance / chain_key need one entry per chain")
    desc = _Desc(Lx, Ly, Lz, d, chi, precision, n_chains, n_inst, _ptr(J, ctypes.c_float),
                 _ptr(ci, ctypes.c_int32), _ptr(beta, ctypes.c_double), _ptr(spins, ctypes.c_int8),
                 ctypes.c_uint64(seed), _ptr(ck, ctypes.c_uint64), pr.shape[0],
                 _ptr(pr, ctypes.c_int32) if pr.shape[0] else None, record_capacity, n_candidates)
    h = ctypes.c_void_p()
    _check(lib.tnmc_lattice_init(ctypes.byref(desc), ctypes.byref(h)), "tnmc_lattice_init")
    lat = Lattice(h, Lx, Ly, Lz, d, chi, n_chains, pr.shape[0], record_capacity)
    lat.n_instances = n_inst
    return lat


def tnmc_lattice_free(lat: Lattice):
    if lat.handle:
        _check(load().tnmc_lattice_free(lat.handle), "tnmc_lattice_free")
        lat.handle = None


def tnmc_slice_propose(lat: Lattice, chain: int, z: int, sweep: int = 0, stream=None):
    """Returns (s_new [Ly, Lx] int8, logq_new, logq_old, dE, status)."""
    lib = load()
    s_new = np.zeros((lat.Ly, lat.Lx), dtype=np.int8)
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib.tnmc_slice_propose(lat.handle, chain, z, ctypes.c_uint64(sweep), _ptr(s_new, ctypes.c_int8),
                                ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), stream)
    _check(st, "tnmc_slice_propose", allow=(TNMC_ERR_NUMERIC,))
    return s_new, a.value, b.value, c.value, st


def tnmc_slice_propose_static(lat: Lattice, chain: int, z: int, sweep: int = 0, stream=None):
    """As tnmc_slice_propose, through the allocation-free entry point (static device scratch)."""
    lib = load()
    s_new = np.zeros((lat.Ly, lat.Lx), dtype=np.int8)
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib.tnmc_slice_propose_static(lat.handle, chain, z, ctypes.c_uint64(sweep), _ptr(s_new, ctypes.c_int8),
                                       ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), stream)
    _check(st, "tnmc_slice_propose_static", allow=(TNMC_ERR_NUMERIC,))
    return s_new, a.value, b.value, c.value, st


def tnmc_slice_logq(lat: Lattice, chain: int, z: int, s, stream=None) -> float:
    s = np.ascontiguousarray(s, dtype=np.int8).reshape(lat.Ly, lat.Lx)
    out = ctypes.c_double()
    _check(load().tnmc_slice_logq(lat.handle, chain, z, _ptr(s, ctypes.c_int8), ctypes.byref(out), stream),
           "tnmc_slice_logq")
    return out.value


def tnmc_mh_accept(logq_old: float, logq_new: float, beta: float, dE: float, u: float) -> bool:
    acc = ctypes.c_int32()
    _check(load().tnmc_mh_accept(logq_old, logq_new, beta, dE, u, ctypes.byref(acc)), "tnmc_mh_accept")
    return bool(acc.value)


def _handles(lats):
    lats = list(lats) if isinstance(lats, (list, tuple)) else [lats]
    arr = (ctypes.c_void_p * len(lats))(*[l.handle for l in lats])
    return arr, len(lats)


def tnmc_sweep(lats, n_sweeps: int, sweep_offset: int = 0, record: bool = False, time_kernels: bool = False,
               stream=None) -> dict:
    arr, n = _handles(lats)
    st = _Stats()
    _check(load().tnmc_sweep(arr, n, n_sweeps, ctypes.c_uint64(sweep_offset), int(record), int(time_kernels),
                             ctypes.byref(st), stream), "tnmc_sweep")
    return st.as_dict()


def tnmc_sweep_direction(lats, direction: int, n_sweeps: int, sweep_offset: int = 0, record: bool = False,
                         time_kernels: bool = False, stream=None) -> dict:
    arr, n = _handles(lats)
    st = _Stats()
    _check(load().tnmc_sweep_direction(arr, n, direction, n_sweeps, ctypes.c_uint64(sweep_offset), int(record),
                                       int(time_kernels), ctypes.byref(st), stream), "tnmc_sweep_direction")
    return st.as_dict()


def tnmc_half_sweep(lats, parity: int, sweep: int, trace_ptr=None, stream=None) -> dict:
    arr, n = _handles(lats)
    st = _Stats()
    _check(load().tnmc_half_sweep(arr, n, parity, ctypes.c_uint64(sweep), trace_ptr, ctypes.byref(st), stream),
           "tnmc_half_sweep")
    return st.as_dict()


def tnmc_get_spins(lat: Lattice, chain: int) -> np.ndarray:
    out = np.zeros((lat.Lz, lat.Ly, lat.Lx), dtype=np.int8)
    _check(load().tnmc_get_spins(lat.handle, chain, _ptr(out, ctypes.c_int8)), "tnmc_get_spins")
    return out


def tnmc_set_spins(lat: Lattice, chain: int, spins) -> None:
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(lat.Lz, lat.Ly, lat.Lx)
    _check(load().tnmc_set_spins(lat.handle, chain, _ptr(s, ctypes.c_int8)), "tnmc_set_spins")


def tnmc_energy(lat: Lattice, chain: int) -> float:
    e = ctypes.c_double()
    _check(load().tnmc_energy(lat.handle, chain, ctypes.byref(e)), "tnmc_energy")
    return e.value


def tnmc_timeseries(lat: Lattice):
    """Returns (E [n, n_chains], M [n, n_chains], q [n, n_pairs])."""
    cap = max(lat.record_capacity, 1)
    E = np.zeros((cap, lat.n_chains))
    M = np.zeros((cap, lat.n_chains))
    q = np.zeros((cap, max(lat.n_pairs, 1)))
    n = ctypes.c_int64()
    _check(load().tnmc_timeseries(lat.handle, _ptr(E, ctypes.c_double), _ptr(M, ctypes.c_double),
                                  _ptr(q, ctypes.c_double), ctypes.byref(n)), "tnmc_timeseries")
    k = n.value
    return E[:k], M[:k], q[:k, : lat.n_pairs]


def tnmc_timeseries_reset(lat: Lattice) -> None:
    _check(load().tnmc_timeseries_reset(lat.handle), "tnmc_timeseries_reset")


def tnmc_debug_workspace(what: int, nbytes: int) -> bytes:
    """Raw copy of part of the last single-task workspace (diagnostics)."""
    buf = ctypes.create_string_buffer(nbytes)
    _check(load().tnmc_debug_workspace(what, buf, nbytes), "tnmc_debug_workspace")
    return buf.raw


def tnmc_debug_set(what: int, value: int) -> None:
    """Test hooks and knobs (see include/tnmc.h): what = 0 forces the compact layout's overflow path,
    1 the autotuner, 2 learned-task pairing, 3 the rank cut-off 10^-value (0 = defaults), 4 forces the
    narrow (two tasks per CU) variant of full-layout launches."""
    _check(load().tnmc_debug_set(what, value), "tnmc_debug_set")


def tnmc_flop_model(Lx: int, Ly: int, d: int, chi: int):
    """Returns (contraction flops, sampling flops) of one slice update."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().tnmc_flop_model(Lx, Ly, d, chi, ctypes.byref(a), ctypes.byref(b)), "tnmc_flop_model")
    return a.value, b.value


# ------------------------------------------------------------ learned proposal
# Batched calls take device buffers as integer addresses (tensor.data_ptr()):
# cond [n][4][Ly][Lx] float32, s [n][Ly][Lx] int8, logq [n] float64,
# grad [TNMC_NN_PARAMS] float32.


class Nn:
    """Handle of a tnmc_nn."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tnmc_nn_free(self.handle)
            self.handle = None


def tnmc_nn_create(params=None, seed: int = 0) -> Nn:
    p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
    if p is not None and p.size != TNMC_NN_PARAMS:
        raise ValueError(f"params need {TNMC_NN_PARAMS} entries")
    h = ctypes.c_void_p()
    _check(load().tnmc_nn_create(_ptr(p, ctypes.c_float), ctypes.c_uint64(seed), ctypes.byref(h)), "tnmc_nn_create")
    return Nn(h)


def tnmc_nn_free(nn: Nn) -> None:
    if nn.handle:
        _check(load().tnmc_nn_free(nn.handle), "tnmc_nn_free")
        nn.handle = None


def tnmc_nn_get_params(nn: Nn) -> np.ndarray:
    out = np.zeros(TNMC_NN_PARAMS, dtype=np.float32)
    _check(load().tnmc_nn_get_params(nn.handle, _ptr(out, ctypes.c_float)), "tnmc_nn_get_params")
    return out


def tnmc_nn_set_params(nn: Nn, params) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != TNMC_NN_PARAMS:
        raise ValueError(f"params need {TNMC_NN_PARAMS} entries")
    _check(load().tnmc_nn_set_params(nn.handle, _ptr(p, ctypes.c_float)), "tnmc_nn_set_params")


def tnmc_nn_logq(nn: Nn, cond_ptr: int, s_ptr: int, n: int, Lx: int, Ly: int, logq_ptr: int, stream=None) -> None:
    _check(load().tnmc_nn_logq(nn.handle, cond_ptr, s_ptr, n, Lx, Ly, logq_ptr, stream), "tnmc_nn_logq")


def tnmc_nn_loss_grad(nn: Nn, cond_ptr: int, s_ptr: int, n: int, Lx: int, Ly: int, grad_ptr=None, stream=None) -> float:
    loss = ctypes.c_double()
    _check(load().tnmc_nn_loss_grad(nn.handle, cond_ptr, s_ptr, n, Lx, Ly, ctypes.byref(loss), grad_ptr, stream),
           "tnmc_nn_loss_grad")
    return loss.value


def tnmc_nn_adam_step(nn: Nn, grad_ptr: int, lr: float, stream=None) -> None:
    _check(load().tnmc_nn_adam_step(nn.handle, grad_ptr, lr, stream), "tnmc_nn_adam_step")


def tnmc_nn_train(nn: Nn, cond_ptr: int, s_ptr: int, n: int, Lx: int, Ly: int, epochs: int, batch: int, lr: float,
                  stream=None) -> float:
    loss = ctypes.c_double()
    _check(load().tnmc_nn_train(nn.handle, cond_ptr, s_ptr, n, Lx, Ly, epochs, batch, lr, ctypes.byref(loss), stream),
           "tnmc_nn_train")
    return loss.value


def tnmc_nn_dataset(lat: Lattice, cond_ptr: int, s_ptr: int, stream=None) -> None:
    _check(load().tnmc_nn_dataset(lat.handle, cond_ptr, s_ptr, stream), "tnmc_nn_dataset")


def tnmc_nn_slice_propose(lat: Lattice, nn: Nn, chain: int, z: int, sweep: int = 0, stream=None):
    """Returns (s_new [Ly, Lx] int8, logq_new, logq_old, dE, status)."""
    s_new = np.zeros((lat.Ly, lat.Lx), dtype=np.int8)
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = load().tnmc_nn_slice_propose(lat.handle, nn.handle, chain, z, ctypes.c_uint64(sweep),
                                      _ptr(s_new, ctypes.c_int8), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                      stream)
    _check(st, "tnmc_nn_slice_propose", allow=(TNMC_ERR_NUMERIC,))
    return s_new, a.value, b.value, c.value, st


def tnmc_nn_slice_logq(lat: Lattice, nn: Nn, chain: int, z: int, s, stream=None) -> float:
    s = np.ascontiguousarray(s, dtype=np.int8).reshape(lat.Ly, lat.Lx)
    out = ctypes.c_double()
    _check(load().tnmc_nn_slice_logq(lat.handle, nn.handle, chain, z, _ptr(s, ctypes.c_int8), ctypes.byref(out),
                                     stream), "tnmc_nn_slice_logq")
    return out.value


def tnmc_nn_sweep(lats, nn: Nn, n_sweeps: int, sweep_offset: int = 0, record: bool = False,
                  time_kernels: bool = False, stream=None) -> dict:
    arr, n = _handles(lats)
    st = _Stats()
    _check(load().tnmc_nn_sweep(arr, n, nn.handle, n_sweeps, ctypes.c_uint64(sweep_offset), int(record),
                                int(time_kernels), ctypes.byref(st), stream), "tnmc_nn_sweep")
    return st.as_dict()


def tnmc_nn_counts(lat: Lattice):
    """Returns (proposed, accepted), each [n_chains, Lz] int64."""
    p = np.zeros((lat.n_chains, lat.Lz), dtype=np.int64)
    a = np.zeros((lat.n_chains, lat.Lz), dtype=np.int64)
    _check(load().tnmc_nn_counts(lat.handle, _ptr(p, ctypes.c_int64), _ptr(a, ctypes.c_int64)), "tnmc_nn_counts")
    return p, a


def tnmc_nn_counts_reset(lat: Lattice) -> None:
    _check(load().tnmc_nn_counts_reset(lat.handle), "tnmc_nn_counts_reset")


def tnmc_nn_set_fallback(lat: Lattice, flags=None) -> None:
    f = None if flags is None else np.ascontiguousarray(flags, dtype=np.int8).reshape(lat.n_chains, lat.Lz)
    _check(load().tnmc_nn_set_fallback(lat.handle, _ptr(f, ctypes.c_int8)), "tnmc_nn_set_fallback")


def tnmc_nn_get_fallback(lat: Lattice) -> np.ndarray:
    f = np.zeros((lat.n_chains, lat.Lz), dtype=np.int8)
    _check(load().tnmc_nn_get_fallback(lat.handle, _ptr(f, ctypes.c_int8)), "tnmc_nn_get_fallback")
    return f


def tnmc_nn_calibrate_fallback(lat: Lattice, threshold: float) -> int:
    n = ctypes.c_int32()
    _check(load().tnmc_nn_calibrate_fallback(lat.handle, threshold, ctypes.byref(n)), "tnmc_nn_calibrate_fallback")
    return n.value


def tnmc_get_couplings(lat: Lattice) -> np.ndarray:
    """Returns J [n_instances, 3, Lz, Ly, Lx]."""
    out = np.zeros((lat.n_instances, 3, lat.Lz, lat.Ly, lat.Lx), dtype=np.float32)
    _check(load().tnmc_get_couplings(lat.handle, _ptr(out, ctypes.c_float)), "tnmc_get_couplings")
    return out


def tnmc_checkpoint_save(lat: Lattice, next_sweep: int, path: str) -> None:
    _check(load().tnmc_checkpoint_save(lat.handle, ctypes.c_uint64(next_sweep), os.fsencode(path)),
           "tnmc_checkpoint_save")


def tnmc_checkpoint_load(lat: Lattice, path: str) -> int:
    """Returns the saved next sweep counter."""
    nxt = ctypes.c_uint64()
    _check(load().tnmc_checkpoint_load(lat.handle, os.fsencode(path), ctypes.byref(nxt)), "tnmc_checkpoint_load")
    return nxt.value


def tnmc_layout_choice(d: int, chi: int, precision: int = TNMC_FP64):
    """Returns (layout, ms_compact, ms_full): layout -1 (not tuned / no choice), 0 compact, 1 full."""
    lay = ctypes.c_int32()
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(load().tnmc_layout_choice(d, chi, precision, ctypes.byref(lay), ctypes.byref(a), ctypes.byref(b)),
           "tnmc_layout_choice")
    return lay.value, a.value, b.value


def tnmc_autotune_choice(d: int, chi: int, precision: int = TNMC_FP64):
    """Returns (layout, engine, ms[4]) of the most recently tuned class of (d, chi, precision):
    -1 where not tuned; ms = median trial ms [VALU compact, VALU full, MFMA compact, MFMA full], -1 if not tried."""
    lay, eng = ctypes.c_int32(), ctypes.c_int32()
    ms = (ctypes.c_double * 4)()
    _check(load().tnmc_autotune_choice(d, chi, precision, ctypes.byref(lay), ctypes.byref(eng), ms),
           "tnmc_autotune_choice")
    return lay.value, eng.value, list(ms)


def tnmc_autotune_pin(layout: int = -1, engine: int = -1) -> None:
    """Fix the contraction layout (0 compact, 1 full) and / or product engine (0 VALU, 1 MFMA); -1 = tuned."""
    _check(load().tnmc_autotune_pin(layout, engine), "tnmc_autotune_pin")


def tnmc_autotune_now(lats, stream=None) -> None:
    """Time the contraction candidates now on the chains' current states (replaces earlier choices)."""
    arr, n = _handles(lats)
    _check(load().tnmc_autotune_now(arr, n, stream), "tnmc_autotune_now")


def tnmc_sweep_graph(lats, n_sweeps: int, sweep_offset: int = 0, record: bool = False, stream=None) -> dict:
    """As tnmc_sweep, with one sweep captured into a HIP graph and replayed n_sweeps times."""
    arr, n = _handles(lats)
    st = _Stats()
    _check(load().tnmc_sweep_graph(arr, n, n_sweeps, ctypes.c_uint64(sweep_offset), int(record), ctypes.byref(st),
                                   stream), "tnmc_sweep_graph")
    return st.as_dict()


def tnmc_sweep_superspin(lats, n_sweeps: int, sweep_offset: int = 0, record: bool = False, time_kernels: bool = False,
                         trace_ptr=None, stream=None) -> dict:
    """TNMCMC-2 composite-layer (superspin) sweeps of Ising lattices, chi_max <= 8; TnmcError otherwise."""
    arr, n = _handles(lats)
    st = _Stats()
    _check(load().tnmc_sweep_superspin(arr, n, n_sweeps, ctypes.c_uint64(sweep_offset), int(record),
                                       int(time_kernels), trace_ptr, ctypes.byref(st), stream), "tnmc_sweep_superspin")
    return st.as_dict()
