"""tanq_sample_noalloc (sampling without device allocations) against tanq_sample."""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_sampling_matches_allocating_entry_point(oracle_mod):
    T.load()
    # two calls in a row on the shared array, the second with a smaller state and fewer shots
    cases = [(10, 120000, 11, True, "f64"), (6, 777, 12, False, "f32")]
    for n, shots, seed, readout, prec in cases:
        ops = W.random_u3_cx(n, 3, seed=40 + n, p1=2e-3, p2=2e-2, gamma=1e-3)
        say("noalloc sample n=%d shots=%d readout=%s %s" % (n, shots, readout, prec))
        rng = np.random.default_rng(n)
        p01 = rng.uniform(0, 0.05, n) if readout else None
        p10 = rng.uniform(0, 0.03, n) if readout else None
        d = T.simulate(n, ops, 2, prec)
        want = T.tanq_sample(d.h, shots, seed, p01, p10)
        got = T.tanq_sample_noalloc(d.h, shots, seed, p01, p10)
        assert np.array_equal(got, want), (n, shots)  # integer outcomes: bit-exact
        # the outcomes are also the oracle's draws up to CDF-edge rounding
        rho = oracle_mod.run(n, ops)
        p, tr = oracle_mod.diag(rho)
        q = oracle_mod.readout_probs(p / tr, p01, p10) if readout else p / tr
        ref, u, cdf = oracle_mod.sample(q, shots, seed)
        assert np.count_nonzero(got.astype(np.int64) != ref) <= (2 if prec == "f64" else shots // 100)
        # limits: more shots than the array holds; zero shots
        with pytest.raises(T.TanqError):
            T.tanq_sample_noalloc(d.h, (1 << 17) + 1, seed)
        assert T.tanq_sample_noalloc(d.h, 0, seed).size == 0
        d.free()
