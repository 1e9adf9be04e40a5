"""Multi-superoperator passes: runs of 2-qubit blocks applied in one pass over vec(rho).

A pass multiplies each superoperator in 3M form (three real products) where a single apply
uses the real-block form, so the state after tanq_apply_fused with passes must match the state
of the same fused list applied with passes switched off (limit 1) to rounding (relative 1e-12
in FP64, 1e-5 in FP32); FP64 must also match the CPU oracle within 1e-10.  Sizes: the smallest
states that use passes (n = 10 in FP64, n = 11 in FP32: at least 256 pass tiles) and a
12-qubit state, compared on every element.  Circuits: the random U3/CX circuit (random pairs, so passes mix
low and high qubits) and the nearest-neighbour brickwork (passes on neighbouring qubits, low
qubits inside the bank window)."""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def run_fused(n, ops, prec, limit, rho_in=None, fuse_limit=8, width=2):
    """Fuse at the given width under pass limit fuse_limit (which orders the blocks for
    passes), then apply under pass limit `limit` (1 = every block on its own)."""
    old = T.tanq_get_pass_limit()
    try:
        T.tanq_set_pass_limit(fuse_limit)
        c = T.Circuit(n, ops)
        f = c.fuse(width, prec)
        T.tanq_set_pass_limit(limit)
        passes = f.passes()
        d = T.DM(n, prec)
        if rho_in is not None:
            d.write(rho_in)
        d.apply_fused(f)
        out = d.read()
        d.free()
        f.free()
        c.free()
        return out, passes
    finally:
        T.tanq_set_pass_limit(old)


def circuits(n):
    return [("u3cx", W.random_u3_cx(n, 6, 11 + n, 1e-3, 1e-2, gamma=5e-4)),
            ("brick", W.brickwork_cz(n, 6, 7 + n, 1e-3, 1e-2, 1e-3))]


TOL = {"f64": 1e-12, "f32": 1e-5}


def close(got, want, prec):
    return np.abs(got - want).max() <= TOL[prec] * np.abs(want).max()


@pytest.mark.parametrize("prec,n", [("f64", 10), ("f64", 11), ("f32", 11)])
def test_passes_match_single_applies(prec, n):
    for name, ops in circuits(n):
        say("passes %s n=%d %s" % (prec, n, name))
        want, p0 = run_fused(n, ops, prec, 1)
        got, p1 = run_fused(n, ops, prec, 8)
        assert p0 == (0, 0)
        assert p1[0] > 0 and p1[1] >= 2 * p1[0]  # passes were used
        assert close(got, want, prec)


@pytest.mark.parametrize("prec,n", [("f64", 10), ("f32", 11)])
@pytest.mark.parametrize("limit", [2, 3, 5])
def test_pass_limits(prec, n, limit):
    ops = W.random_u3_cx(n, 5, 3, 1e-3, 1e-2)
    say("pass limit %d %s n=%d" % (limit, prec, n))
    want, _ = run_fused(n, ops, prec, 1)
    got, (np_, nin) = run_fused(n, ops, prec, limit)
    assert np_ > 0 and nin <= limit * np_
    assert close(got, want, prec)


@pytest.mark.parametrize("prec,n", [("f64", 11), ("f32", 12)])
def test_passes_in_width_3_plans(prec, n):
    """A width-3 plan mixes 3-qubit blocks (single applies) with runs of 2-qubit blocks that
    form passes; the two kinds must interleave in circuit order."""
    ops = W.random_u3_cx(n, 6, 17 + n, 1e-3, 1e-2, gamma=5e-4)
    say("passes in a width-3 plan %s n=%d" % (prec, n))
    want, _ = run_fused(n, ops, prec, 1, width=3)
    got, (np_, _) = run_fused(n, ops, prec, 8, width=3)
    assert np_ > 0
    assert close(got, want, prec)


def test_passes_match_oracle_f64(oracle_mod):
    n = 10
    for name, ops in circuits(n):
        say("passes vs oracle n=%d %s" % (n, name))
        got, (np_, _) = run_fused(n, ops, "f64", 8)
        assert np_ > 0
        want = oracle_mod.matrix_to_vec(oracle_mod.run(n, ops))
        assert np.abs(got - want).max() <= 1e-10


def test_passes_on_a_dense_input_f32(oracle_mod):
    """FP32 against the FP64 oracle from a dense random state (every element nonzero)."""
    n = 11
    rng = np.random.default_rng(5)
    A = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    rho = A @ A.conj().T
    rho /= np.trace(rho)
    vec = oracle_mod.matrix_to_vec(rho)
    ops = W.random_u3_cx(n, 2, 21, 1e-3, 1e-2)
    say("passes f32 dense n=%d" % n)
    got, (np_, _) = run_fused(n, ops, "f32", 8, rho_in=vec.astype(np.complex64))
    assert np_ > 0
    want = oracle_mod.matrix_to_vec(oracle_mod.run(n, ops, rho))
    g = oracle_mod.vec_to_matrix(got.astype(np.complex128), n)
    w = oracle_mod.vec_to_matrix(want, n)
    assert oracle_mod.trace_distance(g, w) <= 1e-4


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_passes_12_qubits(prec):
    n = 12
    ops = W.random_u3_cx(n, 3, 12, 1e-3, 1e-2, gamma=5e-4)
    say("passes %s n=%d full compare" % (prec, n))
    want, _ = run_fused(n, ops, prec, 1)
    got, (np_, _) = run_fused(n, ops, prec, 8)
    assert np_ > 0
    assert close(got, want, prec)


def test_launch_ranges_reproduce_apply_fused():
    """tanq_fused_launches lists the launches of tanq_apply_fused; replaying them range by range
    gives the same bits (the benchmark times launches this way)."""
    n = 11
    ops = W.random_u3_cx(n, 5, 31, 1e-3, 1e-2)
    c = T.Circuit(n, ops)
    for prec in ("f64", "f32"):
        say("launch ranges %s" % prec)
        f = c.fuse(2, prec)
        runs = f.launches()
        np_, nin = f.passes()
        assert sum(runs) == f.count and np_ > 0
        assert max(runs) >= 3  # blocks reordered by qubit set make passes of three
        assert sum(1 for r in runs if r >= 2) == np_ and sum(r for r in runs if r >= 2) == nin
        d1, d2 = T.DM(n, prec), T.DM(n, prec)
        d1.apply_fused(f)
        pos = 0
        for r in runs:
            d2.apply_fused(f, pos, pos + r)
            pos += r
        assert np.array_equal(d1.read().view(np.uint8), d2.read().view(np.uint8))
        d1.free()
        d2.free()
        f.free()
    c.free()


def test_autotune_times_passes():
    for prec, mmax in (("f64", 4), ("f32", 6)):
        say("autotune passes %s" % prec)
        d = T.DM(11, prec)
        d.autotune(reps=1)
        out = T.tanq_tuning_export()
        for m in range(2, mmax + 1):
            assert "pass 11 %s %d " % (prec, m) in out
        assert "pass 11 %s %d " % (prec, mmax + 1) not in out
        d.free()
