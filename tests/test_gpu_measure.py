"""Readout-error probabilities and all-qubit sampling on the GPU vs the oracle."""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def state(oracle_mod):
    n = 7
    ops = W.random_u3_cx(n, 3, seed=17, p1=2e-3, p2=2e-2, gamma=1e-3)
    rho = oracle_mod.run(n, ops)
    p, tr = oracle_mod.diag(rho)
    return n, ops, p / tr


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_readout_probs(oracle_mod, state, prec):
    n, ops, p = state
    rng = np.random.default_rng(2)
    p01, p10 = rng.uniform(0, 0.05, n), rng.uniform(0, 0.03, n)
    say("readout %s" % prec)
    d = T.simulate(n, ops, 2, prec)
    q = d.probs_readout(p01, p10)
    d.free()
    want = oracle_mod.readout_probs(p, p01, p10)
    tol = 1e-13 if prec == "f64" else 1e-6
    assert np.abs(q - want).max() <= tol
    assert abs(q.sum() - 1) <= tol


@pytest.mark.parametrize("readout", [False, True])
def test_sampling_matches_oracle_draws(oracle_mod, state, readout):
    n, ops, p = state
    shots, seed = 50000, 21
    p01 = np.full(n, 0.02) if readout else None
    p10 = np.full(n, 0.01) if readout else None
    say("sample readout=%s" % readout)
    d = T.simulate(n, ops, 3, "f64")
    x = d.sample(shots, seed, p01, p10)
    d.free()
    q = oracle_mod.readout_probs(p, p01, p10) if readout else p
    want, u, cdf = oracle_mod.sample(q, shots, seed)
    # the same draws decide the same outcome except where u is within rounding of a cdf edge
    xi = x.astype(np.int64)
    assert xi.min() >= 0 and xi.max() < (1 << n)
    lower = np.where(xi > 0, cdf[np.maximum(xi - 1, 0)], 0.0)
    eps = 1e-12
    assert np.all(lower <= u + eps) and np.all(u < cdf[xi] + eps)
    differ = np.nonzero(x != want)[0]
    assert differ.size <= 2


def test_sampling_edge_cases():
    with T.DM(3, "f64") as d:  # |000><000|: every shot is 0
        assert np.all(d.sample(1000, 1) == 0)
        assert d.sample(0, 1).size == 0
        with pytest.raises(T.TanqError):
            d.sample(10, 1 << 30)
        with pytest.raises(T.TanqError):
            d.probs_readout(np.full(3, 1.5), np.zeros(3))


# ---------------------------------------------------------------------------------------
# reset to |0> (Kraus set {|0><0|, |0><1|}) inside fused circuits
# ---------------------------------------------------------------------------------------

def _check(oracle_mod, d, want, prec, ctx):
    got = oracle_mod.vec_to_matrix(d.read().astype(np.complex128), d.n)
    p, tr = d.probs(renormalize=True)
    pw, trw = oracle_mod.diag(want)
    if prec == "f64":
        err = np.abs(got - want).max()
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert err <= 1e-10 and rel <= 1e-12, "%s: max abs %.3e rel %.3e" % (ctx, err, rel)
    else:
        td = oracle_mod.trace_distance(got, want)
        assert td <= 1e-4, "%s: trace distance %.3e" % (ctx, td)
    assert np.abs(p - pw / trw).max() <= (1e-12 if prec == "f64" else 1e-5), ctx
    assert abs(tr - 1.0) <= (1e-12 if prec == "f64" else 1e-5), ctx


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("width", [T.TANQ_FUSE_NONE, 2, 3])
def test_reset_in_fused_circuits(oracle_mod, prec, width):
    n = 7
    ops = W.random_u3_cx_reset(n, 5, seed=23, p1=2e-3, p2=2e-2, resets_per_layer=2)
    want = oracle_mod.run(n, ops)
    say("reset n=%d %s width=%d" % (n, prec, width))
    d = T.simulate(n, ops, width, prec)
    _check(oracle_mod, d, want, prec, "reset n=%d %s w=%d" % (n, prec, width))
    d.free()


@pytest.mark.parametrize("prec,n", [("f64", 10), ("f32", 11)])
def test_reset_in_passes(oracle_mod, prec, n):
    """States large enough for the multi-superoperator pass kernels (width 2)."""
    ops = W.random_u3_cx_reset(n, 2, seed=29, p1=1e-3, p2=1e-2, resets_per_layer=3)
    want = oracle_mod.run(n, ops)
    say("reset passes n=%d %s" % (n, prec))
    c = T.Circuit(n, ops)
    f = c.fuse(2, prec)
    npass = f.passes()[0]
    d = T.DM(n, prec)
    d.apply_fused(f)
    f.free()
    c.free()
    assert npass > 0
    _check(oracle_mod, d, want, prec, "reset passes n=%d %s" % (n, prec))
    d.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_reset_every_qubit_gives_ground_state(prec):
    """Resetting every qubit of a noisy entangled state leaves |0..0><0..0| (exact in FP64 up
    to rounding)."""
    n = 6
    ops = W.random_u3_cx(n, 3, seed=31, p1=1e-2, p2=5e-2) + [W.channel(W.reset(), (q,)) for q in range(n)]
    say("reset all n=%d %s" % (n, prec))
    for width in (2, 3):
        d = T.simulate(n, ops, width, prec)
        v = d.read().astype(np.complex128)
        d.free()
        want = np.zeros_like(v)
        want[0] = 1.0
        assert np.abs(v - want).max() <= (1e-13 if prec == "f64" else 1e-6), width
