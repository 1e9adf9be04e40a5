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
