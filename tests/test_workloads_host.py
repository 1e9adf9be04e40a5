"""Host-side checks of the workload generators and the pooled circuit ABI (no GPU)."""
import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W


@pytest.fixture(scope="module")
def lib():
    if not __import__("os").path.exists(T.LIB_PATH):
        from paper_2404_13184_amd import build_lib

        build_lib.build()
    return T.load()


def test_config_shapes():
    n, ops = W.config1()
    assert n == 8 and len(ops) == 20 * (8 * 3 + 4 * 2)
    n, ops = W.config4(layers=3)
    assert n == 16 and len(ops) == 3 * (16 * 2 + 8 * 2)
    n, ops = W.config3(steps=2, n=5)
    assert len(ops) == 2 * (4 * 3 + 5 * 2)
    n, ops = W.config2(layers=2, n=6)
    assert len(ops) == 6 * 3 + 3 * 4 + 6 * 3 + 2 * 4
    reqs = W.config5(num_requests=300)
    arr = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(arr) > 0)
    rate = len(reqs) / arr[-1]
    assert 150 < rate < 260  # Poisson at 200/s
    assert {r.kind for r in reqs} == {"u3cx", "ising", "teleport"}
    assert min(r.n for r in reqs) == 4 and max(r.n for r in reqs) == 12


def test_channels_trace_preserving():
    for K in (W.depolarizing(0.3, 1), W.depolarizing(0.05, 2), W.amplitude_damping(0.2), W.phase_damping(0.4),
              W.thermal_relaxation(1.0, 0.5, 0.2), W.dephase()):
        S = sum(k.conj().T @ k for k in K)
        assert np.abs(S - np.eye(S.shape[0])).max() < 1e-14


@pytest.mark.parametrize("kind", ["u3cx", "ising", "teleport"])
def test_request_arrays_roundtrip(kind):
    req = W.Request(7, 0.0, 6, kind, 5, 3e-3, [])
    ca = W.request_arrays(req)
    ops = W.arrays_to_ops(ca)
    assert len(ops) == ca.count
    back = W.ops_to_arrays(6, ops)
    for i, op in enumerate(ops):
        j, m = int(back.j[i]), int(back.m[i])
        d = 1 << j
        mats = back.pool[back.koff[i]:back.koff[i] + m * d * d * 2].view(np.complex128).reshape(m, d, d)
        assert np.array_equal(mats, op.mats)
    # every operation's Kraus set is a channel (or a unitary)
    for op in ops:
        S = sum(k.conj().T @ k for k in op.mats)
        assert np.abs(S - np.eye(S.shape[0])).max() < 1e-12


def test_request_is_a_physical_circuit(oracle_mod):
    req = W.Request(3, 0.0, 5, "teleport", 2, 5e-3, [])
    rho = oracle_mod.run(5, W.request_ops(req))
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.linalg.eigvalsh(rho).min() > -1e-12


def test_add_ops_equals_single_adds(lib):
    req = W.Request(11, 0.0, 7, "u3cx", 4, 2e-3, [])
    ca = W.request_arrays(req)
    ops = W.arrays_to_ops(ca)
    c1 = T.Circuit(7, ops)
    c2 = T.Circuit(7, arrays=ca)
    assert len(c1) == len(c2) == ca.count
    for mode in (T.TANQ_FUSE_NONE, T.TANQ_FUSE_PAPER, 2, 3):
        assert c1.plan(mode) == c2.plan(mode)
    c1.free()
    c2.free()


def test_add_ops_validation_is_all_or_nothing(lib):
    ca = W.ops_to_arrays(3, [W.gate(W.hadamard(), (0,)), W.gate(W.cx(), (0, 1))])
    c = T.Circuit(3)
    bad_q = ca.q.copy()
    bad_q[1, 1] = 5
    with pytest.raises(T.TanqError):
        T.tanq_circuit_add_ops(c.h, ca.j, bad_q, ca.m, ca.koff, ca.pool)
    bad_off = ca.koff.copy()
    bad_off[1] = ca.pool.size  # reads past the pool
    with pytest.raises(T.TanqError):
        T.tanq_circuit_add_ops(c.h, ca.j, ca.q, ca.m, bad_off, ca.pool)
    assert len(c) == 0
    c.add_arrays(ca)
    assert len(c) == 2
    c.free()
