"""Every apply-kernel variant (tile shape x workgroup size) against the CPU FP64 oracle: the
autotuner may select any of them, so each is held to the same bar as the default.

Sizes: n = 8 gives full tiles for every variant (2n >= tile bits), n = 5 and n = 6 give
partial tiles (the whole state is one tile smaller than the variant's)."""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def superop_of(op):
    """sum_i conj(K_i) (x) K_i with local index row + 2^j col (test-side construction)."""
    return sum(np.kron(K.conj(), K) for K in op.mats)


def random_density(rng, n):
    dim = 1 << n
    A = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    rho = A @ A.conj().T
    return rho / np.trace(rho)


def cases():
    out = []
    try:
        T.load()
    except (T.TanqError, OSError):  # library missing or not loadable: nothing to parametrize
        return out
    for k in (2, 3):
        for prec in ("f64", "f32"):
            for v in range(T.tanq_variant_count(k, T._prec(prec))):
                out.append((k, prec, v))
    return out


@pytest.mark.parametrize("k,prec,v", cases())
def test_variant_matches_oracle(oracle_mod, k, prec, v):
    P = T._prec(prec)
    desc = T.tanq_variant_get(k, P, v)
    rng = np.random.default_rng(100 * k + 10 * v + (prec == "f32"))
    try:
        T.tanq_variant_select(k, P, v)
        for n in (5, 6, 8):
            qsets = [tuple(range(k)), tuple(range(n - k, n)), tuple(int(x) for x in rng.choice(n, k, replace=False))]
            for qs in qsets:
                say("variant k=%d %s tile_bits=%d threads=%d n=%d qubits=%s"
                    % (k, prec, desc["tile_bits"], desc["threads"], n, qs))
                rho = random_density(rng, n)
                d4 = 1 << k
                mats = [rng.standard_normal((d4, d4)) + 1j * rng.standard_normal((d4, d4)) for _ in range(2)]
                op = W.channel([m * 0.4 for m in mats], qs)
                want = oracle_mod.run(n, [op], rho)
                with T.DM(n, prec) as d:
                    d.write(oracle_mod.matrix_to_vec(rho))
                    d.apply_superop(qs, superop_of(op))
                    got = oracle_mod.vec_to_matrix(d.read().astype(np.complex128), n)
                err = np.abs(got - want).max()
                rel = np.linalg.norm(got - want) / np.linalg.norm(want)
                if prec == "f64":
                    assert err <= 1e-10 and rel <= 1e-12, (err, rel)
                else:
                    assert rel <= 2e-6, (err, rel)
    finally:
        T.tanq_variant_select(k, P, 0)


@pytest.mark.parametrize("k,prec,v", cases())
def test_variant_full_size_sampled(oracle_mod, k, prec, v):
    """At 16 qubits (64 GiB FP64 / 32 GiB FP32, the benchmark's launch shapes): one apply on a
    seeded pseudo-random vec(rho), sampled output groups recomputed by the oracle on the
    2^k x 2^k block each forms."""
    n = 16
    P = T._prec(prec)
    desc = T.tanq_variant_get(k, P, v)
    rng = np.random.default_rng(7 + 100 * k + 10 * v)
    qsets = [tuple(int(x) for x in rng.choice(n, k, replace=False)), tuple(range(n - k, n))]
    try:
        T.tanq_variant_select(k, P, v)
        with T.DM(n, prec) as d:
            for qs in qsets:
                say("n=16 variant k=%d %s tile_bits=%d threads=%d staging=%d qubits=%s"
                    % (k, prec, desc["tile_bits"], desc["threads"], desc["staging"], qs))
                mats = [rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
                        for _ in range(2)]
                op = W.channel([m * 0.4 for m in mats], qs)
                seed = 11 + v
                d.fill_random(seed)
                d.apply_superop(qs, superop_of(op))
                frees = [q for q in range(n) if q not in qs]
                for _ in range(8):
                    rf = sum(int(rng.integers(0, 2)) << q for q in frees)
                    cf = sum(int(rng.integers(0, 2)) << q for q in frees)
                    vals = (lambda idx: W.hash_fill_values(seed, idx)) if prec == "f64" else \
                        (lambda idx: W.hash_fill_values(seed, idx).astype(np.complex64).astype(np.complex128))
                    Q, _, M_out = oracle_mod.sample_block(vals, n, [op], rf, cf)
                    dep = np.array([sum(((a >> t) & 1) << Q[t] for t in range(k)) for a in range(1 << k)],
                                   dtype=np.uint64)
                    idx = (np.uint64(rf) + dep)[:, None] + ((np.uint64(cf) + dep)[None, :] << np.uint64(n))
                    got = d.gather(idx.reshape(-1)).astype(np.complex128).reshape(1 << k, 1 << k)
                    tol = 1e-12 if prec == "f64" else 2e-5
                    assert np.abs(got - M_out).max() <= tol * max(1.0, np.abs(M_out).max()), (qs, rf, cf)
    finally:
        T.tanq_variant_select(k, P, 0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dense_autotune_records_costs(prec):
    """Dense autotuning: every width gets a cost and a tuned variant for this n; the state it
    leaves stays finite (a unitary applied to bounded data) and reset restores |0><0|."""
    n = 8
    P = T._prec(prec)
    say("dense autotune %s n=%d" % (prec, n))
    with T.DM(n, prec) as d:
        ms = d.autotune(reps=1, dense=True)
        assert all(m > 0 for m in ms[1:4])
        for k in (2, 3):
            assert 0 <= T.tanq_variant_for(n, k, prec) < T.tanq_variant_count(k, P)
        v = d.read()
        assert np.all(np.isfinite(v.view(np.float64 if prec == "f64" else np.float32)))
        d.reset()
        v = d.read()
        assert v[0] == 1 and np.count_nonzero(v) == 1
    for k in (2, 3):
        T.tanq_variant_select(k, P, 0)  # clear the tuned entries for later tests
