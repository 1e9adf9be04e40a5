"""Python driver for the CPU FP64 reference (``oracle.c``).  TEST INFRASTRUCTURE ONLY.

Functions:

* :func:`run` -- rho_out = E_m(...E_1(rho_in)...), each E(rho) = sum_i K_i rho K_i^dag
  applied operation by operation, unfused, FP64 (Sec. 2.1, Eq. eq:dmsim; the Kraus form of
  each noisy transformation, Sec. 3.1).  rho is a row-major 2^n x 2^n complex128 matrix.
* :func:`diag`, :func:`expect_pauli` -- measurement statistics of rho (Sec. 2.1: rho holds
  the probabilities of every measurement outcome).
* :func:`statevector` -- a plain state-vector simulator for circuits made only of unitary
  gates; for those circuits rho_out = |psi><psi| (the pure-state case of Sec. 2.1).
* :func:`readout_probs`, :func:`sample` -- measurement through readout errors and sampled
  outcomes (Sec. 3.5).
* :func:`reduced_dm`, :func:`process_chi_1q` -- partial trace and single-qubit process
  tomography of a circuit (Sec. 5, teleportation case study: the chi matrix).
* :func:`trace_distance`, :func:`vec_to_matrix`, :func:`matrix_to_vec` -- comparison
  helpers; vec() is column stacking (Sec. 3.1): rho[r, c] sits at index r + c 2^n.

The library is built from ``oracle.c`` with gcc/OpenMP by :func:`build`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class OracleError(RuntimeError):
    pass


def library_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_apply_kraus.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ip, ctypes.c_int, dp]
        lib.oracle_apply_kraus.restype = ctypes.c_int
        lib.oracle_init_zero.argtypes = [ctypes.c_int, dp]
        lib.oracle_init_zero.restype = ctypes.c_int
        lib.oracle_diagonal.argtypes = [ctypes.c_int, dp, dp, dp]
        lib.oracle_diagonal.restype = ctypes.c_int
        lib.oracle_expect_pauli.argtypes = [ctypes.c_int, dp, ctypes.c_char_p, dp, dp]
        lib.oracle_expect_pauli.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def run_on(rho: np.ndarray, ops: Iterable) -> np.ndarray:
    """Apply ``ops`` in order to the row-major matrix ``rho`` (modified in place, returned).

    ``rho`` need not be Hermitian or of unit trace: each step is the linear map
    X -> sum_i K_i X K_i^dag.
    """
    lib = _load()
    assert rho.dtype == np.complex128 and rho.flags.c_contiguous
    dim = rho.shape[0]
    n = dim.bit_length() - 1
    assert rho.shape == (dim, dim) and (1 << n) == dim
    T = np.empty_like(rho)
    acc = None
    for op in ops:
        K = np.ascontiguousarray(op.mats, dtype=np.complex128)
        m = K.shape[0]
        if m > 1 and acc is None:
            acc = np.empty_like(rho)
        q = (ctypes.c_int * len(op.qubits))(*op.qubits)
        rc = lib.oracle_apply_kraus(n, _dptr(rho), _dptr(T), _dptr(acc) if acc is not None else None,
                                    len(op.qubits), q, m, _dptr(K))
        if rc != 0:
            raise OracleError("oracle_apply_kraus rejected op %r on n=%d" % (op.qubits, n))
    return rho


def run(n: int, ops: Iterable, rho_in: Optional[np.ndarray] = None) -> np.ndarray:
    """rho_out for ``ops`` applied to rho_in (default |0..0><0..0|); row-major complex128."""
    if rho_in is None:
        rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        rho[0, 0] = 1.0
    else:
        rho = np.array(rho_in, dtype=np.complex128, order="C", copy=True)
    return run_on(rho, ops)


def diag(rho: np.ndarray):
    """(p, trace): p[x] = Re rho[x, x] (not renormalised) and the trace."""
    lib = _load()
    dim = rho.shape[0]
    n = dim.bit_length() - 1
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    out = np.empty(dim, dtype=np.float64)
    tr = ctypes.c_double()
    if lib.oracle_diagonal(n, _dptr(rho), _dptr(out), ctypes.byref(tr)) != 0:
        raise OracleError("oracle_diagonal")
    return out, tr.value


def expect_pauli(rho: np.ndarray, pauli: str) -> complex:
    """Tr(P rho) for the Pauli string ``pauli`` (character t acts on qubit t)."""
    lib = _load()
    dim = rho.shape[0]
    n = dim.bit_length() - 1
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    re, im = ctypes.c_double(), ctypes.c_double()
    if lib.oracle_expect_pauli(n, _dptr(rho), pauli.encode(), ctypes.byref(re), ctypes.byref(im)) != 0:
        raise OracleError("oracle_expect_pauli(%r)" % pauli)
    return complex(re.value, im.value)


def statevector(n: int, ops: Iterable, psi_in: Optional[np.ndarray] = None) -> np.ndarray:
    """|psi_out> for unitary-only ``ops`` (each op must hold exactly one matrix)."""
    psi = np.zeros(1 << n, dtype=np.complex128)
    if psi_in is None:
        psi[0] = 1.0
    else:
        psi[:] = psi_in
    for op in ops:
        if op.mats.shape[0] != 1:
            raise OracleError("statevector: op %r is a channel" % (op.label,))
        U = op.mats[0]
        q = list(op.qubits)
        j = len(q)
        offs = np.zeros(1 << j, dtype=np.int64)
        for a in range(1 << j):
            offs[a] = sum(((a >> t) & 1) << q[t] for t in range(j))
        tmask = sum(1 << x for x in q)
        idx = np.arange(1 << n, dtype=np.int64)
        bases = idx[(idx & tmask) == 0]
        gidx = bases[:, None] + offs[None, :]
        psi[gidx] = psi[gidx] @ U.T
    return psi


def trace_distance(a: np.ndarray, b: np.ndarray) -> float:
    """(1/2) sum |eig(a - b)| for Hermitian a, b (LAPACK eigvalsh of the difference)."""
    d = np.asarray(a, dtype=np.complex128) - np.asarray(b, dtype=np.complex128)
    d = 0.5 * (d + d.conj().T)
    return 0.5 * float(np.abs(np.linalg.eigvalsh(d)).sum())


def vec_to_matrix(v: np.ndarray, n: int) -> np.ndarray:
    """Column-stacked vec(rho) (index r + c 2^n) -> row-major matrix rho[r, c]."""
    dim = 1 << n
    return np.ascontiguousarray(np.asarray(v).reshape(dim, dim).T)


def matrix_to_vec(rho: np.ndarray) -> np.ndarray:
    """Row-major rho[r, c] -> column-stacked vec(rho)."""
    return np.ascontiguousarray(np.asarray(rho).T).reshape(-1)


def sample_block(vec_in_values, n: int, ops: Sequence, row_free: int, col_free: int):
    """One group of outputs computed directly from the definition.

    For operations that all act inside the qubit set Q = union of their targets (|Q| = k),
    the entries rho[r, c] whose row and column bits outside Q are fixed to ``row_free`` and
    ``col_free`` form a 2^k x 2^k block M[a, b] that evolves on its own: M -> sum K M K^dag
    with K acting on the local qubits.  ``vec_in_values(indices)`` returns vec(rho_in) at the
    given column-stacked indices.  Returns (Q, M_in, M_out).
    """
    Q = sorted({q for op in ops for q in op.qubits})
    k = len(Q)
    loc = {q: i for i, q in enumerate(Q)}
    dep = np.array([sum(((a >> t) & 1) << Q[t] for t in range(k)) for a in range(1 << k)], dtype=np.int64)
    rows = row_free + dep
    cols = col_free + dep
    idx = rows[:, None] + (cols[None, :] << n)
    M_in = np.asarray(vec_in_values(idx.reshape(-1)), dtype=np.complex128).reshape(1 << k, 1 << k)

    class _L:  # the op relabelled onto local qubits 0..k-1
        def __init__(self, op):
            self.qubits = tuple(loc[q] for q in op.qubits)
            self.mats = op.mats
            self.label = getattr(op, "label", "")

    M_out = run(k, [_L(op) for op in ops], rho_in=M_in)
    return Q, M_in, M_out


# --------------------------------------------------------------------------------------
# measurement with readout error, and sampling (Sec. 3.5, measurement error)
# --------------------------------------------------------------------------------------

def splitmix64(x):
    """SplitMix64 output for counter value(s) x (Steele, Lea & Flood, OOPSLA 2014): the state
    advanced once by the golden gamma 0x9E3779B97F4A7C15, then the variant-13 finaliser."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def readout_probs(p: np.ndarray, p01, p10) -> np.ndarray:
    """Probabilities seen through independent per-qubit readout errors: qubit t is read as 0
    when it is 1 with probability p01[t] and as 1 when it is 0 with p10[t].  Definition: the
    confusion matrix (x)_t A_t, A_t = [[1 - p10, p01], [p10, 1 - p01]] (qubit t = bit t, the
    right-most Kronecker factor first), applied to p."""
    n = len(p01)
    M = np.array([[1.0]])
    for t in range(n):
        A = np.array([[1.0 - p10[t], p01[t]], [p10[t], 1.0 - p01[t]]])
        M = np.kron(A, M)
    return M @ np.asarray(p, dtype=np.float64)


def sample(p: np.ndarray, shots: int, seed: int) -> np.ndarray:
    """All-qubit measurement outcomes: outcome i is the smallest x with cdf(x) > u_i cdf(end),
    u_i = top 53 bits of SplitMix64((seed << 40) + i) / 2^53, cdf the prefix sums of p."""
    cdf = np.cumsum(np.asarray(p, dtype=np.float64))
    u = (splitmix64((np.uint64(seed) << np.uint64(40)) + np.arange(shots, dtype=np.uint64)) >> np.uint64(11))
    u = u.astype(np.float64) * (2.0 ** -53) * cdf[-1]
    return np.searchsorted(cdf, u, side="right").astype(np.uint64), u, cdf


# --------------------------------------------------------------------------------------
# partial trace and process tomography (Sec. 5, case study 1)
# --------------------------------------------------------------------------------------

_PAULI = (np.eye(2, dtype=np.complex128),
          np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128))


def reduced_dm(rho: np.ndarray, keep: Sequence[int]) -> np.ndarray:
    """Partial trace over every qubit not in ``keep``: out[a, b] = sum_f rho[a|f, b|f], where
    bit t of a and b is qubit keep[t] and f runs over the values of the other qubits."""
    dim = rho.shape[0]
    n = dim.bit_length() - 1
    keep = list(keep)
    others = [q for q in range(n) if q not in keep]
    k = len(keep)
    out = np.zeros((1 << k, 1 << k), dtype=np.complex128)
    dep_k = np.array([sum(((a >> t) & 1) << keep[t] for t in range(k)) for a in range(1 << k)], dtype=np.int64)
    dep_f = np.array([sum(((f >> t) & 1) << others[t] for t in range(len(others)))
                      for f in range(1 << len(others))], dtype=np.int64)
    for a in range(1 << k):
        for b in range(1 << k):
            out[a, b] = rho[dep_k[a] + dep_f, dep_k[b] + dep_f].sum()
    return out


def process_chi_1q(n: int, ops: Iterable, src: int, dst: int) -> np.ndarray:
    """chi of the channel that carries qubit ``src`` to qubit ``dst`` (every other qubit
    starting in |0>), in the Pauli basis I, X, Y, Z: E(rho) = sum_ij chi_ij sigma_i rho sigma_j.

    Standard process tomography: E is linear, so the outputs E(|a><b|) for the four basis
    operators fix it; chi is the solution of the 16 linear equations
    E(|a><b|)[r, c] = sum_ij chi_ij (sigma_i |a><b| sigma_j)[r, c]."""
    ops = list(ops)
    rows, rhs = [], []
    for a in range(2):
        for b in range(2):
            E_ab = np.zeros((2, 2), dtype=np.complex128)
            E_ab[a, b] = 1.0
            rho_in = np.zeros((1 << n, 1 << n), dtype=np.complex128)
            rho_in[a << src, b << src] = 1.0
            out = reduced_dm(run(n, ops, rho_in), [dst])
            for r in range(2):
                for c in range(2):
                    rows.append([(_PAULI[i] @ E_ab @ _PAULI[j])[r, c] for i in range(4) for j in range(4)])
                    rhs.append(out[r, c])
    return np.linalg.solve(np.array(rows), np.array(rhs)).reshape(4, 4)
