"""Pins for the oracle's readout-error model and all-qubit sampling (no GPU)."""
import itertools
import os

import numpy as np
import pytest


def test_splitmix64_published_outputs(oracle_mod):
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    xs = np.array([int(a, 16) for a, _ in rows], dtype=np.uint64)
    want = [int(b, 16) for _, b in rows]
    assert [int(v) for v in oracle_mod.splitmix64(xs)] == want


def test_readout_definition_by_outcome_sum(oracle_mod):
    """q[m] = sum_x prod_t P(m_t | x_t) p[x], evaluated outcome by outcome."""
    rng = np.random.default_rng(3)
    n = 4
    p = rng.random(1 << n)
    p /= p.sum()
    p01, p10 = rng.uniform(0, 0.2, n), rng.uniform(0, 0.2, n)
    q = oracle_mod.readout_probs(p, p01, p10)
    for m in range(1 << n):
        s = 0.0
        for x in range(1 << n):
            w = 1.0
            for t in range(n):
                mt, xt = (m >> t) & 1, (x >> t) & 1
                if xt == 0:
                    w *= p10[t] if mt == 1 else 1 - p10[t]
                else:
                    w *= p01[t] if mt == 0 else 1 - p01[t]
            s += w * p[x]
        assert abs(q[m] - s) < 1e-15


def test_readout_limits(oracle_mod):
    rng = np.random.default_rng(4)
    p = rng.random(8)
    p /= p.sum()
    z = np.zeros(3)
    assert np.array_equal(oracle_mod.readout_probs(p, z, z), p)
    q = oracle_mod.readout_probs(p, [0.1, 0.0, 0.3], [0.05, 0.2, 0.0])
    assert abs(q.sum() - 1) < 1e-15 and q.min() >= 0
    # full flip on qubit 0: outcomes swap pairwise
    q = oracle_mod.readout_probs(p, [1.0, 0, 0], [1.0, 0, 0])
    assert np.allclose(q, p.reshape(4, 2)[:, ::-1].reshape(-1), atol=0, rtol=0)
    # one qubit in |1>: P(read 0) = p01 (the paper's P(0|1))
    q = oracle_mod.readout_probs(np.array([0.0, 1.0]), [0.07], [0.02])
    assert np.allclose(q, [0.07, 0.93], rtol=0, atol=2e-16)


def test_sampling(oracle_mod):
    p = np.zeros(16)
    p[5] = 1.0
    x, _, _ = oracle_mod.sample(p, 100, seed=3)
    assert np.all(x == 5)
    rng = np.random.default_rng(1)
    p = rng.random(16)
    p /= p.sum()
    shots = 200000
    x, u, cdf = oracle_mod.sample(p, shots, seed=9)
    freq = np.bincount(x.astype(np.int64), minlength=16) / shots
    assert np.abs(freq - p).max() < 5 * np.sqrt(p.max() / shots)
    # each outcome satisfies its defining inequality
    xi = x.astype(np.int64)
    lower = np.where(xi > 0, cdf[np.maximum(xi - 1, 0)], 0.0)
    assert np.all(lower <= u) and np.all(u < cdf[xi])
