"""ctypes binding of libtanq (the C ABI in include/tanq.h).

Functions named ``tanq_*`` are the C entry points with argument marshalling only; the
classes :class:`DM`, :class:`Circuit` and :class:`Fused` wrap the handles.  Every compute
step runs in the library's HIP kernels.  There is no fallback: if ``libtanq.so`` is not
built, loading raises :class:`TanqError`.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtanq.so")

TANQ_OK = 0
TANQ_E_ARG = -1
TANQ_E_OOM = -2
TANQ_E_HIP = -3
TANQ_E_STATE = -4
TANQ_E_UNSUPPORTED = -5
TANQ_E_AGAIN = -6
TANQ_E_CANCELED = -7
TANQ_E_TIMEOUT = -8

TANQ_F64 = 0
TANQ_F32 = 1

TANQ_FUSE_AUTO = 0
TANQ_FUSE_NONE = -1
TANQ_FUSE_PAPER = -2

# every symbol include/tanq.h declares
EXPORTED = [
    "tanq_last_error", "tanq_version",
    "tanq_dm_init", "tanq_dm_wrap", "tanq_dm_free", "tanq_dm_reset", "tanq_dm_query",
    "tanq_dm_read", "tanq_dm_write", "tanq_dm_fill_random", "tanq_dm_gather", "tanq_sync", "tanq_dm_scale",
    "tanq_mfma_rate",
    "tanq_circuit_create", "tanq_circuit_free", "tanq_circuit_add_gate", "tanq_circuit_add_kraus",
    "tanq_circuit_add_ops", "tanq_circuit_size",
    "tanq_fuse", "tanq_fuse_plan", "tanq_fused_info", "tanq_fused_free", "tanq_fused_get",
    "tanq_apply_superop", "tanq_apply_fused", "tanq_apply_fused_range",
    "tanq_variant_count", "tanq_variant_get", "tanq_variant_select", "tanq_variant_selected", "tanq_autotune",
    "tanq_variant_for", "tanq_tuning_export", "tanq_tuning_import", "tanq_autotune_dense",
    "tanq_set_pass_limit", "tanq_get_pass_limit", "tanq_pass_layout_info", "tanq_fused_passes",
    "tanq_fused_launches", "tanq_fuse_plan_ordered",
    "tanq_probs", "tanq_probs_readout", "tanq_sample", "tanq_sample_noalloc", "tanq_dm_set_basis", "tanq_reduced_dm",
    "tanq_process_chi_1q",
    "tanq_expect_pauli", "tanq_expect_pauli_c", "tanq_expect_pauli_batch",
    "tanq_dm_compare",
    "tanq_server_create", "tanq_server_submit", "tanq_server_poll", "tanq_server_wait", "tanq_server_release", "tanq_server_cancel",
    "tanq_server_stats_get", "tanq_server_destroy",
]


class TanqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("tanq error %d: %s" % (code, msg))
        self.code = code


class Variant(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("prec", ctypes.c_int), ("tile_bits", ctypes.c_int), ("threads", ctypes.c_int),
                ("staging", ctypes.c_int)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int), ("prec", ctypes.c_int),
                ("width", ctypes.c_int), ("steps_per_launch", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("cohort_bytes", ctypes.c_size_t), ("request_timeout_s", ctypes.c_double)]


class Outputs(ctypes.Structure):
    _fields_ = [("probs", ctypes.c_int), ("npauli", ctypes.c_int), ("paulis", ctypes.POINTER(ctypes.c_char_p))]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n", ctypes.c_int), ("trace", ctypes.c_double),
                ("probs", ctypes.POINTER(ctypes.c_double)), ("pauli", ctypes.POINTER(ctypes.c_double)),
                ("npauli", ctypes.c_int), ("fused_applies", ctypes.c_int),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("launches", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("budget_bytes", ctypes.c_size_t),
                ("active", ctypes.c_int), ("pending", ctypes.c_int), ("clock", ctypes.c_double),
                ("tiles", ctypes.c_uint64), ("chunks", ctypes.c_uint64), ("dropped", ctypes.c_uint64)]


class FusedInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("count_k", ctypes.c_int * 4), ("source_ops", ctypes.c_int),
                ("max_width", ctypes.c_int), ("prec", ctypes.c_int), ("n", ctypes.c_int)]


_lib = None

_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "tanq_last_error": ([], ctypes.c_char_p),
    "tanq_version": ([], ctypes.c_int),
    "tanq_dm_init": ([ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tanq_dm_wrap": ([ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tanq_dm_free": ([_vp], ctypes.c_int),
    "tanq_dm_reset": ([_vp], ctypes.c_int),
    "tanq_dm_query": ([_vp, _ip, _ip, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_vp)], ctypes.c_int),
    "tanq_dm_read": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int),
    "tanq_dm_write": ([_vp, _vp, ctypes.c_size_t], ctypes.c_int),
    "tanq_dm_fill_random": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "tanq_dm_gather": ([_vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64), _vp], ctypes.c_int),
    "tanq_sync": ([_vp], ctypes.c_int),
    "tanq_circuit_create": ([ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
    "tanq_circuit_free": ([_vp], ctypes.c_int),
    "tanq_circuit_add_gate": ([_vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
    "tanq_circuit_add_kraus": ([_vp, ctypes.c_int, _ip, ctypes.c_int, _dp], ctypes.c_int),
    "tanq_circuit_add_ops": ([_vp, ctypes.c_int, _ip, _ip, _ip, ctypes.POINTER(ctypes.c_int64), _dp,
                              ctypes.c_size_t], ctypes.c_int),
    "tanq_circuit_size": ([_vp, _ip], ctypes.c_int),
    "tanq_fuse": ([_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_vp)], ctypes.c_int),
    "tanq_fuse_plan": ([_vp, ctypes.c_int, _ip, _ip], ctypes.c_int),
    "tanq_fused_info": ([_vp, ctypes.POINTER(FusedInfo)], ctypes.c_int),
    "tanq_fused_free": ([_vp], ctypes.c_int),
    "tanq_fused_get": ([_vp, ctypes.c_int, _ip, _ip, _dp], ctypes.c_int),
    "tanq_apply_superop": ([_vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
    "tanq_apply_fused": ([_vp, _vp], ctypes.c_int),
    "tanq_apply_fused_range": ([_vp, _vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "tanq_variant_count": ([ctypes.c_int, ctypes.c_int, _ip], ctypes.c_int),
    "tanq_variant_get": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Variant)], ctypes.c_int),
    "tanq_variant_select": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "tanq_variant_selected": ([ctypes.c_int, ctypes.c_int, _ip], ctypes.c_int),
    "tanq_autotune": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "tanq_probs": ([_vp, _dp, ctypes.c_int, _dp], ctypes.c_int),
    "tanq_probs_readout": ([_vp, _dp, _dp, _dp], ctypes.c_int),
    "tanq_dm_set_basis": ([_vp, ctypes.c_uint64, ctypes.c_uint64], ctypes.c_int),
    "tanq_variant_for": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip], ctypes.c_int),
    "tanq_autotune_dense": ([_vp, ctypes.c_int, _dp], ctypes.c_int),
    "tanq_set_pass_limit": ([ctypes.c_int], ctypes.c_int),
    "tanq_get_pass_limit": ([_ip], ctypes.c_int),
    "tanq_pass_layout_info": ([ctypes.c_int, ctypes.c_int, _ip, ctypes.c_int, _ip, _ip], ctypes.c_int),
    "tanq_fused_passes": ([_vp, _ip, _ip], ctypes.c_int),
    "tanq_fused_launches": ([_vp, _ip, ctypes.c_int, _ip], ctypes.c_int),
    "tanq_fuse_plan_ordered": ([_vp, ctypes.c_int, ctypes.c_int, _ip, _ip], ctypes.c_int),
    "tanq_tuning_export": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tanq_tuning_import": ([ctypes.c_char_p], ctypes.c_int),
    "tanq_reduced_dm": ([_vp, ctypes.c_int, _ip, _dp], ctypes.c_int),
    "tanq_process_chi_1q": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp], ctypes.c_int),
    "tanq_sample": ([_vp, ctypes.c_uint64, ctypes.c_uint64, _dp, _dp, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "tanq_sample_noalloc": ([_vp, ctypes.c_uint64, ctypes.c_uint64, _dp, _dp, ctypes.POINTER(ctypes.c_uint64)],
                            ctypes.c_int),
    "tanq_expect_pauli": ([_vp, ctypes.c_char_p, _dp], ctypes.c_int),
    "tanq_expect_pauli_c": ([_vp, ctypes.c_char_p, _dp, _dp], ctypes.c_int),
    "tanq_expect_pauli_batch": ([_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), _dp, _dp], ctypes.c_int),
    "tanq_dm_compare": ([_vp, _vp, _dp], ctypes.c_int),
    "tanq_dm_scale": ([_vp, ctypes.c_double], ctypes.c_int),
    "tanq_mfma_rate": ([ctypes.c_int, _dp], ctypes.c_int),
    "tanq_server_create": ([ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)], ctypes.c_int),
    "tanq_server_submit": ([_vp, _vp, ctypes.POINTER(Outputs), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "tanq_server_poll": ([_vp, ctypes.c_uint64, ctypes.POINTER(Result)], ctypes.c_int),
    "tanq_server_wait": ([_vp, ctypes.c_uint64, ctypes.POINTER(Result)], ctypes.c_int),
    "tanq_server_release": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "tanq_server_cancel": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "tanq_server_stats_get": ([_vp, ctypes.POINTER(ServerStats)], ctypes.c_int),
    "tanq_server_destroy": ([_vp], ctypes.c_int),
}


def load(path: str = LIB_PATH):
    """Load libtanq.so (raises TanqError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise TanqError(TANQ_E_STATE, "libtanq.so not built at %s (run __graft_entry__.build())" % path)
        lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != TANQ_OK:
        raise TanqError(rc, load().tanq_last_error().decode())


def _ints(seq: Sequence[int]):
    return (ctypes.c_int * len(seq))(*[int(x) for x in seq])


def _cdoubles(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(_dp)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # a torch.cuda.Stream


# ---------------------------------------------------------------------------------------
# C entry points, same names
# ---------------------------------------------------------------------------------------

def tanq_last_error() -> str:
    return load().tanq_last_error().decode()


def tanq_version() -> int:
    return int(load().tanq_version())


def tanq_dm_init(n: int, prec: int, stream=None) -> int:
    h = _vp()
    _check(load().tanq_dm_init(n, prec, _stream_ptr(stream), ctypes.byref(h)))
    return h.value


def tanq_dm_wrap(n: int, prec: int, dev_ptr: int, stream=None) -> int:
    h = _vp()
    _check(load().tanq_dm_wrap(n, prec, dev_ptr, _stream_ptr(stream), ctypes.byref(h)))
    return h.value


def tanq_dm_free(h: int):
    _check(load().tanq_dm_free(h))


def tanq_dm_reset(h: int):
    _check(load().tanq_dm_reset(h))


def tanq_dm_scale(h: int, factor: float):
    _check(load().tanq_dm_scale(h, float(factor)))


def tanq_mfma_rate(prec) -> float:
    """Sustained matrix-unit rate (TFLOP/s) of the pass kernels' multiplication loop shape."""
    v = ctypes.c_double()
    _check(load().tanq_mfma_rate(_prec(prec), ctypes.byref(v)))
    return v.value


def tanq_dm_query(h: int):
    n, p, e, ptr = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64(), _vp()
    _check(load().tanq_dm_query(h, ctypes.byref(n), ctypes.byref(p), ctypes.byref(e), ctypes.byref(ptr)))
    return n.value, p.value, e.value, ptr.value


def tanq_dm_read(h: int, out: np.ndarray):
    _check(load().tanq_dm_read(h, out.ctypes.data, out.nbytes))


def tanq_dm_write(h: int, data: np.ndarray):
    data = np.ascontiguousarray(data)
    _check(load().tanq_dm_write(h, data.ctypes.data, data.nbytes))


def tanq_dm_fill_random(h: int, seed: int):
    _check(load().tanq_dm_fill_random(h, seed))


def tanq_dm_gather(h: int, idx: np.ndarray, dtype) -> np.ndarray:
    idx = np.ascontiguousarray(idx, dtype=np.uint64).reshape(-1)
    out = np.empty(idx.size, dtype=dtype)
    _check(load().tanq_dm_gather(h, idx.size, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), out.ctypes.data))
    return out


def tanq_sync(h: int):
    _check(load().tanq_sync(h))


def tanq_circuit_create(n: int) -> int:
    h = _vp()
    _check(load().tanq_circuit_create(n, ctypes.byref(h)))
    return h.value


def tanq_circuit_free(h: int):
    _check(load().tanq_circuit_free(h))


def tanq_circuit_add_gate(h: int, qubits: Sequence[int], U: np.ndarray):
    U, p = _cdoubles(U)
    _check(load().tanq_circuit_add_gate(h, len(qubits), _ints(qubits), p))


def tanq_circuit_add_kraus(h: int, qubits: Sequence[int], K: np.ndarray):
    K, p = _cdoubles(K)
    _check(load().tanq_circuit_add_kraus(h, len(qubits), _ints(qubits), K.shape[0], p))


def tanq_circuit_add_ops(h: int, j: np.ndarray, q: np.ndarray, m: np.ndarray, koff: np.ndarray, pool: np.ndarray):
    j = np.ascontiguousarray(j, dtype=np.int32)
    q = np.ascontiguousarray(q, dtype=np.int32).reshape(-1)
    m = np.ascontiguousarray(m, dtype=np.int32)
    koff = np.ascontiguousarray(koff, dtype=np.int64)
    pool = np.ascontiguousarray(pool, dtype=np.float64)
    _check(load().tanq_circuit_add_ops(h, int(j.size), j.ctypes.data_as(_ip), q.ctypes.data_as(_ip),
                                       m.ctypes.data_as(_ip), koff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       pool.ctypes.data_as(_dp), pool.size))


def tanq_circuit_size(h: int) -> int:
    c = ctypes.c_int()
    _check(load().tanq_circuit_size(h, ctypes.byref(c)))
    return c.value


def tanq_fuse(circuit: int, max_width: int, prec: int, stream=None) -> int:
    h = _vp()
    _check(load().tanq_fuse(circuit, max_width, prec, _stream_ptr(stream), ctypes.byref(h)))
    return h.value


def tanq_fuse_plan(circuit: int, max_width: int, nops: int):
    ob = (ctypes.c_int * max(nops, 1))()
    nb = ctypes.c_int()
    _check(load().tanq_fuse_plan(circuit, max_width, ob, ctypes.byref(nb)))
    return list(ob[:nops]), nb.value


def tanq_fuse_plan_ordered(circuit: int, max_width: int, prec, nops: int):
    ob = (ctypes.c_int * max(nops, 1))()
    nb = ctypes.c_int()
    _check(load().tanq_fuse_plan_ordered(circuit, max_width, _prec(prec), ob, ctypes.byref(nb)))
    return list(ob[:nops]), nb.value


def tanq_fused_info(h: int) -> dict:
    info = FusedInfo()
    _check(load().tanq_fused_info(h, ctypes.byref(info)))
    return {"count": info.count, "count_k": list(info.count_k), "source_ops": info.source_ops,
            "max_width": info.max_width, "prec": info.prec, "n": info.n}


def tanq_fused_free(h: int):
    _check(load().tanq_fused_free(h))


def tanq_fused_get(h: int, idx: int):
    k = ctypes.c_int()
    q = (ctypes.c_int * 3)()
    _check(load().tanq_fused_get(h, idx, ctypes.byref(k), q, None))
    S = np.empty((4 ** k.value, 4 ** k.value), dtype=np.complex128)
    _check(load().tanq_fused_get(h, idx, None, None, S.ctypes.data_as(_dp)))
    return k.value, tuple(q[:k.value]), S


def tanq_fused_block(h: int, idx: int):
    """(k, qubits) of fused block idx without copying its superoperator."""
    k = ctypes.c_int()
    q = (ctypes.c_int * 3)()
    _check(load().tanq_fused_get(h, idx, ctypes.byref(k), q, None))
    return k.value, tuple(q[:k.value])


def tanq_apply_superop(h: int, qubits: Sequence[int], S: np.ndarray):
    S, p = _cdoubles(S)
    _check(load().tanq_apply_superop(h, len(qubits), _ints(qubits), p))


def tanq_apply_fused(h: int, fused: int):
    _check(load().tanq_apply_fused(h, fused))


def tanq_apply_fused_range(h: int, fused: int, begin: int, end: int):
    _check(load().tanq_apply_fused_range(h, fused, begin, end))


def tanq_variant_count(k: int, prec: int) -> int:
    c = ctypes.c_int()
    _check(load().tanq_variant_count(k, prec, ctypes.byref(c)))
    return c.value


def tanq_variant_get(k: int, prec: int, index: int) -> dict:
    v = Variant()
    _check(load().tanq_variant_get(k, prec, index, ctypes.byref(v)))
    return {"k": v.k, "prec": v.prec, "tile_bits": v.tile_bits, "threads": v.threads, "staging": v.staging}


def tanq_variant_select(k: int, prec: int, index: int):
    _check(load().tanq_variant_select(k, prec, index))


def tanq_variant_selected(k: int, prec: int) -> int:
    c = ctypes.c_int()
    _check(load().tanq_variant_selected(k, prec, ctypes.byref(c)))
    return c.value


def tanq_autotune(h: int, reps: int = 3) -> list:
    ms = (ctypes.c_double * 4)()
    _check(load().tanq_autotune(h, reps, ms))
    return list(ms)


def tanq_autotune_dense(h: int, reps: int = 3) -> list:
    ms = (ctypes.c_double * 4)()
    _check(load().tanq_autotune_dense(h, reps, ms))
    return list(ms)


def tanq_probs(h: int, dim: int, renormalize: bool = True):
    out = np.empty(dim, dtype=np.float64)
    tr = ctypes.c_double()
    _check(load().tanq_probs(h, out.ctypes.data_as(_dp), int(bool(renormalize)), ctypes.byref(tr)))
    return out, tr.value


def tanq_probs_readout(h: int, n: int, p01, p10) -> np.ndarray:
    a = np.ascontiguousarray(p01, dtype=np.float64)
    b = np.ascontiguousarray(p10, dtype=np.float64)
    out = np.empty(1 << n, dtype=np.float64)
    _check(load().tanq_probs_readout(h, a.ctypes.data_as(_dp), b.ctypes.data_as(_dp), out.ctypes.data_as(_dp)))
    return out


def tanq_variant_for(n: int, k: int, prec) -> int:
    v = ctypes.c_int()
    _check(load().tanq_variant_for(n, k, _prec(prec), ctypes.byref(v)))
    return v.value


def tanq_set_pass_limit(max_superops: int):
    _check(load().tanq_set_pass_limit(int(max_superops)))


def tanq_get_pass_limit() -> int:
    v = ctypes.c_int()
    _check(load().tanq_get_pass_limit(ctypes.byref(v)))
    return v.value


def tanq_fused_passes(h: int):
    """(passes, blocks applied inside passes) of a fused list under the current pass limit."""
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(load().tanq_fused_passes(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def tanq_fused_launches(h: int) -> List[int]:
    """Blocks per launch of tanq_apply_fused for a fused list (1 = single apply, >= 2 = pass)."""
    cnt = ctypes.c_int()
    _check(load().tanq_fused_launches(h, None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_int * max(cnt.value, 1))()
    _check(load().tanq_fused_launches(h, buf, cnt.value, ctypes.byref(cnt)))
    return list(buf[:cnt.value])


def tanq_pass_layout_info(n: int, pairs: Sequence[Sequence[int]], prec):
    """(conflict-free LDS access patterns, their achievable maximum) of one pass layout; two
    patterns per superoperator."""
    flat = [int(q) for pr in pairs for q in pr]
    v, b = ctypes.c_int(), ctypes.c_int()
    _check(load().tanq_pass_layout_info(n, len(pairs), _ints(flat), _prec(prec), ctypes.byref(v), ctypes.byref(b)))
    return v.value, b.value


def tanq_tuning_export() -> str:
    need = ctypes.c_size_t()
    _check(load().tanq_tuning_export(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(load().tanq_tuning_export(buf, need.value, ctypes.byref(need)))
    return buf.value.decode()


def tanq_tuning_import(text: str):
    _check(load().tanq_tuning_import(text.encode()))


def tanq_dm_set_basis(h: int, r: int, c: int):
    _check(load().tanq_dm_set_basis(h, r, c))


def tanq_reduced_dm(h: int, keep: Sequence[int]) -> np.ndarray:
    k = len(keep)
    out = np.empty((1 << k, 1 << k), dtype=np.complex128)
    _check(load().tanq_reduced_dm(h, k, _ints(keep), out.ctypes.data_as(_dp)))
    return out


def tanq_process_chi_1q(circuit: int, max_width: int, prec, in_qubit: int, out_qubit: int):
    """(chi, S): the process matrix in the Pauli basis and the 4x4 superoperator."""
    prec = _prec(prec)
    chi = np.empty((4, 4), dtype=np.complex128)
    S = np.empty((4, 4), dtype=np.complex128)
    _check(load().tanq_process_chi_1q(circuit, max_width, prec, in_qubit, out_qubit, chi.ctypes.data_as(_dp),
                                      S.ctypes.data_as(_dp)))
    return chi, S


def _sample_call(fn, h: int, shots: int, seed: int, p01=None, p10=None) -> np.ndarray:
    out = np.empty(shots, dtype=np.uint64)
    a = b = None
    if p01 is not None:
        a = np.ascontiguousarray(p01, dtype=np.float64)
        b = np.ascontiguousarray(p10, dtype=np.float64)
    _check(fn(h, shots, seed, a.ctypes.data_as(_dp) if a is not None else None,
              b.ctypes.data_as(_dp) if b is not None else None,
              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return out


def tanq_sample(h: int, shots: int, seed: int, p01=None, p10=None) -> np.ndarray:
    return _sample_call(load().tanq_sample, h, shots, seed, p01, p10)


def tanq_sample_noalloc(h: int, shots: int, seed: int, p01=None, p10=None) -> np.ndarray:
    return _sample_call(load().tanq_sample_noalloc, h, shots, seed, p01, p10)


def tanq_expect_pauli(h: int, pauli: str) -> float:
    v = ctypes.c_double()
    _check(load().tanq_expect_pauli(h, pauli.encode(), ctypes.byref(v)))
    return v.value


def tanq_expect_pauli_c(h: int, pauli: str) -> complex:
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(load().tanq_expect_pauli_c(h, pauli.encode(), ctypes.byref(re), ctypes.byref(im)))
    return complex(re.value, im.value)


def tanq_expect_pauli_batch(h: int, paulis: Sequence[str]) -> np.ndarray:
    cnt = len(paulis)
    arr = (ctypes.c_char_p * max(cnt, 1))(*[p.encode() for p in paulis])
    re = np.empty(cnt, dtype=np.float64)
    im = np.empty(cnt, dtype=np.float64)
    _check(load().tanq_expect_pauli_batch(h, cnt, arr, re.ctypes.data_as(_dp), im.ctypes.data_as(_dp)))
    return re + 1j * im


def tanq_dm_compare(a: int, b: int):
    """(||a-b||_F, max|a-b|, ||a||_F) computed on the GPU in FP64."""
    out = (ctypes.c_double * 3)()
    _check(load().tanq_dm_compare(a, b, out))
    return tuple(out)


def tanq_server_create(hbm_budget: int, max_slots: int, prec: int, width: int = 2,
                       steps_per_launch: int = 8, use_graphs: bool = True, cohort_bytes: int = 0,
                       request_timeout_s: float = 0.0) -> int:
    cfg = ServerConfig(hbm_budget, max_slots, prec, width, steps_per_launch, int(bool(use_graphs)),
                       int(cohort_bytes), float(request_timeout_s))
    h = _vp()
    _check(load().tanq_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def tanq_server_submit(h: int, circuit: int, probs: bool = True, paulis: Sequence[str] = ()) -> int:
    arr = (ctypes.c_char_p * max(len(paulis), 1))(*[p.encode() for p in paulis])
    outs = Outputs(int(bool(probs)), len(paulis), arr)
    t = ctypes.c_uint64()
    _check(load().tanq_server_submit(h, circuit, ctypes.byref(outs), ctypes.byref(t)))
    return t.value


def _result_dict(r: Result) -> dict:
    out = {"status": r.status, "n": r.n, "trace": r.trace, "fused_applies": r.fused_applies,
           "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
           "probs": None, "pauli": None}
    if r.probs:
        out["probs"] = np.ctypeslib.as_array(r.probs, shape=(1 << r.n,)).copy()
    if r.pauli and r.npauli:
        out["pauli"] = np.ctypeslib.as_array(r.pauli, shape=(r.npauli,)).copy()
    return out


def tanq_server_poll(h: int, ticket: int):
    """Result dict, or None while the request is not finished."""
    r = Result()
    rc = load().tanq_server_poll(h, ticket, ctypes.byref(r))
    if rc == TANQ_E_AGAIN:
        return None
    _check(rc)
    return _result_dict(r)


def tanq_server_wait(h: int, ticket: int) -> dict:
    r = Result()
    _check(load().tanq_server_wait(h, ticket, ctypes.byref(r)))
    return _result_dict(r)


def tanq_server_release(h: int, ticket: int):
    _check(load().tanq_server_release(h, ticket))


def tanq_server_cancel(h: int, ticket: int):
    _check(load().tanq_server_cancel(h, ticket))


def tanq_server_stats_get(h: int) -> dict:
    st = ServerStats()
    _check(load().tanq_server_stats_get(h, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in ServerStats._fields_}


def tanq_server_destroy(h: int):
    _check(load().tanq_server_destroy(h))


# ---------------------------------------------------------------------------------------
# handle wrappers
# ---------------------------------------------------------------------------------------

def _prec(p) -> int:
    if p in (TANQ_F64, "f64", "fp64", np.complex128):
        return TANQ_F64
    if p in (TANQ_F32, "f32", "fp32", np.complex64):
        return TANQ_F32
    raise ValueError("precision %r" % (p,))


class DM:
    """A device-resident vec(rho) (owned, or wrapping caller memory via ``dev_ptr``)."""

    def __init__(self, n: int, prec="f64", stream=None, dev_ptr: Optional[int] = None):
        self.n = n
        self.prec = _prec(prec)
        self.h = tanq_dm_init(n, self.prec, stream) if dev_ptr is None else tanq_dm_wrap(n, self.prec, dev_ptr, stream)

    @property
    def dtype(self):
        return np.complex128 if self.prec == TANQ_F64 else np.complex64

    def free(self):
        if self.h:
            tanq_dm_free(self.h)
            self.h = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def reset(self):
        tanq_dm_reset(self.h)

    def scale(self, factor: float):
        tanq_dm_scale(self.h, factor)

    def read(self) -> np.ndarray:
        out = np.empty(4 ** self.n, dtype=self.dtype)
        tanq_dm_read(self.h, out)
        return out

    def write(self, v: np.ndarray):
        tanq_dm_write(self.h, np.ascontiguousarray(v, dtype=self.dtype))

    def fill_random(self, seed: int):
        tanq_dm_fill_random(self.h, seed)

    def sync(self):
        tanq_sync(self.h)

    def gather(self, idx) -> np.ndarray:
        return tanq_dm_gather(self.h, np.asarray(idx), self.dtype)

    def apply_superop(self, qubits: Sequence[int], S: np.ndarray):
        tanq_apply_superop(self.h, qubits, S)

    def apply_fused(self, fused: "Fused", begin: Optional[int] = None, end: Optional[int] = None):
        if begin is None and end is None:
            tanq_apply_fused(self.h, fused.h)
        else:
            tanq_apply_fused_range(self.h, fused.h, begin or 0, fused.count if end is None else end)

    def probs(self, renormalize: bool = True):
        return tanq_probs(self.h, 1 << self.n, renormalize)

    def compare(self, other: "DM"):
        return tanq_dm_compare(self.h, other.h)

    def autotune(self, reps: int = 3, dense: bool = False) -> list:
        """Tune the apply variants on this state; dense=True overwrites it with pseudo-random
        values and times a dense superoperator (the costs real circuits see)."""
        return tanq_autotune_dense(self.h, reps) if dense else tanq_autotune(self.h, reps)

    def probs_readout(self, p01, p10) -> np.ndarray:
        return tanq_probs_readout(self.h, self.n, p01, p10)

    def set_basis(self, r: int, c: int):
        tanq_dm_set_basis(self.h, r, c)

    def reduced(self, keep: Sequence[int]) -> np.ndarray:
        return tanq_reduced_dm(self.h, keep)

    def sample(self, shots: int, seed: int, p01=None, p10=None) -> np.ndarray:
        return tanq_sample(self.h, shots, seed, p01, p10)

    def expect_pauli(self, pauli: str) -> complex:
        return tanq_expect_pauli_c(self.h, pauli)

    def expect_paulis(self, paulis: Sequence[str]) -> np.ndarray:
        return tanq_expect_pauli_batch(self.h, paulis)


class Circuit:
    def __init__(self, n: int, ops: Iterable = (), arrays=None):
        self.n = n
        self.h = tanq_circuit_create(n)
        if arrays is not None:
            self.add_arrays(arrays)
        for op in ops:
            self.add(op)

    def process_chi_1q(self, in_qubit: int, out_qubit: int, max_width: int = TANQ_FUSE_AUTO, prec="f64"):
        """(chi, S) of the one-qubit channel in_qubit -> out_qubit defined by this circuit."""
        return tanq_process_chi_1q(self.h, max_width, prec, in_qubit, out_qubit)

    def add_arrays(self, ca):
        """Append a pooled circuit (workloads.CircuitArrays) in one call."""
        tanq_circuit_add_ops(self.h, ca.j, ca.q, ca.m, ca.koff, ca.pool)

    def add(self, op):
        if op.mats.shape[0] == 1 and op.kind == "gate":
            tanq_circuit_add_gate(self.h, op.qubits, op.mats[0])
        else:
            tanq_circuit_add_kraus(self.h, op.qubits, op.mats)

    def __len__(self):
        return tanq_circuit_size(self.h)

    def free(self):
        if self.h:
            tanq_circuit_free(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def plan(self, max_width: int):
        return tanq_fuse_plan(self.h, max_width, len(self))

    def plan_ordered(self, max_width: int, prec="f64"):
        """The block assignment fuse() makes: the plan ordered for multi-superoperator passes."""
        return tanq_fuse_plan_ordered(self.h, max_width, prec, len(self))

    def fuse(self, max_width: int = TANQ_FUSE_AUTO, prec="f64", stream=None) -> "Fused":
        return Fused(tanq_fuse(self.h, max_width, _prec(prec), stream))


class Fused:
    def __init__(self, h: int):
        self.h = h
        self.info = tanq_fused_info(h)
        self.count = self.info["count"]

    def get(self, idx: int):
        return tanq_fused_get(self.h, idx)

    def passes(self):
        """(passes, blocks inside passes) that apply_fused uses under the current pass limit."""
        return tanq_fused_passes(self.h)

    def launches(self) -> List[int]:
        """Blocks per launch of apply_fused, in order (1 = single apply, >= 2 = pass)."""
        return tanq_fused_launches(self.h)

    def get_k(self, idx: int) -> int:
        if getattr(self, "_ks", None) is None:
            self._ks = [tanq_fused_block(self.h, i)[0] for i in range(self.count)]
        return self._ks[idx]

    def free(self):
        if self.h:
            tanq_fused_free(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def simulate(n: int, ops: Iterable, max_width: int = TANQ_FUSE_AUTO, prec="f64", stream=None) -> DM:
    """Fuse ``ops`` and apply them to |0..0><0..0|; returns the DM handle."""
    c = Circuit(n, ops)
    f = c.fuse(max_width, prec, stream)
    d = DM(n, prec, stream)
    d.apply_fused(f)
    f.free()
    c.free()
    return d


class Server:
    """Continuous-batching server (see tanq_server_* in include/tanq.h)."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, prec="f32", width: int = 2,
                 steps_per_launch: int = 8, use_graphs: bool = True, cohort_bytes: int = 0,
                 request_timeout_s: float = 0.0):
        self.h = tanq_server_create(hbm_budget, max_slots, _prec(prec), width, steps_per_launch, use_graphs,
                                    cohort_bytes, request_timeout_s)

    def submit(self, n: int, ops: Iterable = (), probs: bool = True, paulis: Sequence[str] = (), arrays=None) -> int:
        c = Circuit(n, ops, arrays=arrays)
        try:
            return tanq_server_submit(self.h, c.h, probs, paulis)
        finally:
            c.free()

    def poll(self, ticket: int):
        return tanq_server_poll(self.h, ticket)

    def wait(self, ticket: int) -> dict:
        return tanq_server_wait(self.h, ticket)

    def release(self, ticket: int):
        tanq_server_release(self.h, ticket)

    def cancel(self, ticket: int):
        tanq_server_cancel(self.h, ticket)

    def stats(self) -> dict:
        return tanq_server_stats_get(self.h)

    def close(self):
        if self.h:
            tanq_server_destroy(self.h)
            self.h = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
