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
