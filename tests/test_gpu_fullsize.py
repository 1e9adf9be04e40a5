"""Full-size (16-qubit, 64 GiB FP64 / 32 GiB FP32) parity on sampled outputs.

The oracle cannot hold a 16-qubit rho next to its scratch in host memory for a whole
circuit, so these checks use cases it can compute one output at a time:

* one superoperator applied to a seeded pseudo-random vec(rho): every group of outputs
  depends only on its own 4^k inputs, so sampled groups are recomputed by the oracle on the
  2^k x 2^k block they form (sum K M K^dag);
* a noiseless circuit: rho = |psi><psi| with psi from the oracle's state-vector simulator;
* a noisy circuit confined to four interleaved 4-qubit groups: rho is the tensor product of
  the four 4-qubit oracle results.

All run through the same apply launches (tile shapes, persistent grids) as the benchmark; at
fusion width 2 that includes the multi-superoperator pass kernels.
"""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 16


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def random_channel(rng, qubits):
    d = 1 << len(qubits)
    mats = [rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)) for _ in range(2)]
    return W.channel([m * 0.5 for m in mats], qubits)


def superop_of(op):
    return sum(np.kron(K.conj(), K) for K in op.mats)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("qubits", [(0, 15), (7, 3), (14, 15), (0, 1, 2), (15, 8, 0), (13, 14, 15), (5,), (0,)])
def test_single_apply_sampled_groups(oracle_mod, prec, qubits):
    rng = np.random.default_rng(sum(qubits) + 7 * len(qubits))
    op = random_channel(rng, qubits)
    seed = 5 + len(qubits)
    say("n=16 apply %s qubits=%s" % (prec, qubits))
    with T.DM(N, prec) as d:
        d.fill_random(seed)
        d.apply_superop(qubits, superop_of(op))
        tmask = sum(1 << q for q in qubits)
        frees = [q for q in range(N) if q not in qubits]
        checked = 0
        for _ in range(24):
            rf = sum(int(rng.integers(0, 2)) << q for q in frees)
            cf = sum(int(rng.integers(0, 2)) << q for q in frees)
            vals = (lambda idx: W.hash_fill_values(seed, idx)) if prec == "f64" else \
                (lambda idx: W.hash_fill_values(seed, idx).astype(np.complex64).astype(np.complex128))
            Q, M_in, M_out = oracle_mod.sample_block(vals, N, [op], rf, cf)
            k = len(Q)
            dep = np.array([sum(((a >> t) & 1) << Q[t] for t in range(k)) for a in range(1 << k)], dtype=np.uint64)
            idx = (np.uint64(rf) + dep)[:, None] + ((np.uint64(cf) + dep)[None, :] << np.uint64(N))
            got = d.gather(idx.reshape(-1)).astype(np.complex128).reshape(1 << k, 1 << k)
            tol = 1e-12 if prec == "f64" else 2e-5
            assert np.abs(got - M_out).max() <= tol * max(1.0, np.abs(M_out).max()), (rf, cf)
            assert (rf & tmask) == 0 and (cf & tmask) == 0
            checked += 1
        assert checked == 24


@pytest.mark.parametrize("mode,prec", [(2, "f64"), (2, "f32"), (3, "f64"), (3, "f32")])
def test_noiseless_circuit_vs_statevector(oracle_mod, mode, prec):
    ops = W.random_u3_cx(N, 6, seed=44, p1=0.0, p2=0.0)
    psi = oracle_mod.statevector(N, ops)
    say("n=16 noiseless mode=%d %s" % (mode, prec))
    c = T.Circuit(N, ops)
    f = c.fuse(mode, prec)
    if mode == 2:
        assert f.passes()[0] > 0  # width 2 runs as multi-superoperator passes, as in the benchmark
    rng = np.random.default_rng(3)
    with T.DM(N, prec) as d:
        d.apply_fused(f)
        r = rng.integers(0, 1 << N, size=4000, dtype=np.int64)
        cc = rng.integers(0, 1 << N, size=4000, dtype=np.int64)
        r[:1000] = cc[:1000]  # include diagonal entries
        idx = (r.astype(np.uint64) + (cc.astype(np.uint64) << np.uint64(N)))
        got = d.gather(idx).astype(np.complex128)
        p, tr = d.probs(renormalize=False)
    f.free()
    c.free()
    want = psi[r] * psi[cc].conj()
    scale = np.abs(psi).max() ** 2
    if prec == "f64":
        assert np.abs(got - want).max() <= 1e-10
        assert np.abs(got - want).max() <= 1e-9 * scale
        assert np.abs(p - np.abs(psi) ** 2).max() <= 1e-12
        assert abs(tr - 1) <= 1e-12
    else:
        assert np.abs(got - want).max() <= 1e-5 * scale
        assert np.abs(p - np.abs(psi) ** 2).max() <= 1e-5


@pytest.mark.parametrize("mode,prec", [(2, "f64"), (3, "f64"), (2, "f32")])
def test_block_separable_noisy_circuit(oracle_mod, mode, prec):
    """Noisy U3/CX layers confined to the groups {0,4,8,12}, {1,5,9,13}, ...: rho is the
    tensor product of four 4-qubit oracle results."""
    groups = [[g + 4 * i for i in range(4)] for g in range(4)]
    ops, parts = [], []
    for gi, grp in enumerate(groups):
        local = W.random_u3_cx(4, 8, seed=90 + gi, p1=2e-3, p2=2e-2, gamma=1e-3)
        parts.append(oracle_mod.run(4, local))
        for op in local:
            ops.append(W.Op(op.kind, tuple(grp[q] for q in op.qubits), op.mats, op.label))
    # interleave the groups' operations round-robin (they commute)
    rng = np.random.default_rng(1)
    per_group = {}
    for i, op in enumerate(ops):
        per_group.setdefault(op.qubits[0] % 4, []).append(op)
    merged = []
    while any(per_group.values()):
        for gk in sorted(per_group):
            if per_group[gk]:
                merged.append(per_group[gk].pop(0))
    say("n=16 block-separable mode=%d %s" % (mode, prec))
    c = T.Circuit(N, merged)
    f = c.fuse(mode, prec)
    with T.DM(N, prec) as d:
        d.apply_fused(f)
        r = rng.integers(0, 1 << N, size=3000, dtype=np.int64)
        cc = rng.integers(0, 1 << N, size=3000, dtype=np.int64)
        r[:500] = cc[:500]
        got = d.gather(r.astype(np.uint64) + (cc.astype(np.uint64) << np.uint64(N))).astype(np.complex128)
        zz = d.expect_paulis(W.zz_paulis(N)[:3])
    f.free()
    c.free()

    def local_index(x, grp):
        return sum(((x >> q) & 1) << t for t, q in enumerate(grp))

    want = np.ones(r.size, dtype=np.complex128)
    for grp, rb in zip(groups, parts):
        ri = np.array([local_index(int(x), grp) for x in r])
        ci = np.array([local_index(int(x), grp) for x in cc])
        want *= rb[ri, ci]
    z0 = oracle_mod.expect_pauli(parts[0], "ZIII")
    z1 = oracle_mod.expect_pauli(parts[1], "ZIII")
    if prec == "f64":
        assert np.abs(got - want).max() <= 1e-10
        assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()
        # <Z_0 Z_1>: qubits 0 and 1 are in different groups, so it factorises
        assert abs(zz[0] - z0 * z1) <= 1e-12
    else:
        assert np.abs(got - want).max() <= 1e-5 * np.abs(want).max()
        assert abs(zz[0] - z0 * z1) <= 1e-5


@pytest.mark.parametrize("qubits", [(16, 3), (0, 16, 9)])
def test_largest_register_fp32(oracle_mod, qubits):
    """n = 17, the largest register the library accepts: 4^17 complex64 = 128 GiB, element
    indices beyond 2^32.  One apply on a seeded fill, sampled groups against the oracle."""
    n = 17
    rng = np.random.default_rng(17 + len(qubits))
    op = random_channel(rng, qubits)
    seed = 3
    say("n=17 f32 apply qubits=%s" % (qubits,))
    with T.DM(n, "f32") as d:
        d.fill_random(seed)
        d.apply_superop(qubits, superop_of(op))
        frees = [q for q in range(n) if q not in qubits]
        for _ in range(12):
            rf = sum(int(rng.integers(0, 2)) << q for q in frees)
            cf = sum(int(rng.integers(0, 2)) << q for q in frees)
            vals = lambda idx: W.hash_fill_values(seed, idx).astype(np.complex64).astype(np.complex128)
            Q, _, M_out = oracle_mod.sample_block(vals, n, [op], rf, cf)
            k = len(Q)
            dep = np.array([sum(((a >> t) & 1) << Q[t] for t in range(k)) for a in range(1 << k)], dtype=np.uint64)
            idx = (np.uint64(rf) + dep)[:, None] + ((np.uint64(cf) + dep)[None, :] << np.uint64(n))
            got = d.gather(idx.reshape(-1)).astype(np.complex128).reshape(1 << k, 1 << k)
            assert np.abs(got - M_out).max() <= 2e-5 * max(1.0, np.abs(M_out).max()), (rf, cf)


def test_largest_register_fp32_pass(oracle_mod):
    """n = 17 FP32 through the multi-superoperator pass kernel: five 2-qubit channels on qubits
    {0, 13, 14, 15, 16} (one pass; tile offsets and element indices beyond 2^32), sampled
    32 x 32 blocks against the oracle applying the same channels in order."""
    n = 17
    rng = np.random.default_rng(1717)
    ops = [random_channel(rng, q) for q in ((16, 15), (14, 13), (0, 16), (16, 13), (15, 14))]
    seed = 4
    say("n=17 f32 pass")
    c = T.Circuit(n, ops)
    f = c.fuse(2, "f32")
    assert f.passes() == (1, 5)
    with T.DM(n, "f32") as d:
        d.fill_random(seed)
        d.apply_fused(f)
        Q = [0, 13, 14, 15, 16]
        frees = [q for q in range(n) if q not in Q]
        vals = lambda idx: W.hash_fill_values(seed, idx).astype(np.complex64).astype(np.complex128)
        for _ in range(8):
            rf = sum(int(rng.integers(0, 2)) << q for q in frees)
            cf = sum(int(rng.integers(0, 2)) << q for q in frees)
            Qs, _, M_out = oracle_mod.sample_block(vals, n, ops, rf, cf)
            assert Qs == Q
            dep = np.array([sum(((a >> t) & 1) << Q[t] for t in range(5)) for a in range(32)], dtype=np.uint64)
            idx = (np.uint64(rf) + dep)[:, None] + ((np.uint64(cf) + dep)[None, :] << np.uint64(n))
            got = d.gather(idx.reshape(-1)).astype(np.complex128).reshape(32, 32)
            assert np.abs(got - M_out).max() <= 5e-5 * max(1.0, np.abs(M_out).max()), (rf, cf)
    f.free()
    c.free()
