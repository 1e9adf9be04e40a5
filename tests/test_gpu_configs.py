"""The 14-qubit brickwork and 15-qubit Ising workloads at their full sizes (4 GiB and 16 GiB
FP64 states), checked where the oracle cannot hold the whole run:

* properties that hold at any size: unit trace, Hermiticity of sampled element pairs,
  probabilities in [0, 1] summing to 1, Pauli expectations in [-1, 1];
* the FP32 form against the FP64 result at the same size (trace-distance bound, |dp|);
* the noiseless brickwork against the oracle's state vector on sampled elements;
* Ising limits: with h = 0, |0..0> is a ZZ eigenstate and the relaxation fixed point, so
  <Z_i> = 1 exactly; with J = 0 the qubits evolve independently, so <Z_i> and sampled
  elements follow from single-qubit oracle runs;
* FP64 results under different fusion widths agree (consistency of the fused path).
"""
import os
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def sampled_pairs(rng, n, count):
    r = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    c = rng.integers(0, 1 << n, size=count, dtype=np.uint64)
    return r, c


def check_properties(d, n, rng, tol):
    p, tr = d.probs(renormalize=False)
    assert abs(tr - 1.0) <= tol
    assert p.min() >= -tol and abs(p.sum() - 1.0) <= tol
    r, c = sampled_pairs(rng, n, 256)
    a = d.gather(r + (c << np.uint64(n))).astype(np.complex128)
    b = d.gather(c + (r << np.uint64(n))).astype(np.complex128)
    assert np.abs(a - np.conj(b)).max() <= tol
    return p


def test_brickwork_14q_full_size():
    n, ops = W.config2()
    rng = np.random.default_rng(1)
    say("brickwork n=14 full depth: FP64 width 2, FP32 width 2, FP64 width 3")
    c = T.Circuit(n, ops)
    f64 = T.DM(n, "f64")
    f64.apply_fused(c.fuse(2, "f64"))
    p64 = check_properties(f64, n, rng, 1e-12)
    zz = np.real(f64.expect_paulis(W.zz_paulis(n)))
    assert np.all(np.abs(zz) <= 1.0 + 1e-12)
    d32 = T.DM(n, "f32")
    d32.apply_fused(c.fuse(2, "f32"))
    p32 = check_properties(d32, n, rng, 1e-5)
    fro, mx, _ = d32.compare(f64)
    assert 0.5 * 2 ** (n / 2) * fro <= 1e-4  # trace-distance bound
    assert np.abs(p32 / p32.sum() - p64).max() <= 1e-5
    d32.free()
    w3 = T.DM(n, "f64")
    w3.apply_fused(c.fuse(3, "f64"))
    fro, mx, nrm = w3.compare(f64)
    assert mx <= 1e-12 and fro <= 1e-12 * nrm
    w3.free()
    f64.free()
    c.free()


def test_brickwork_14q_noiseless_vs_statevector(oracle_mod):
    n = 14
    ops = W.brickwork_cz(n, 40, seed=2, p1=0.0, p2=0.0, lam=0.0)
    ops = [op for op in ops if op.mats.shape[0] == 1]  # the unitary gates only
    psi = oracle_mod.statevector(n, ops)
    rng = np.random.default_rng(4)
    for prec, tol in (("f64", 1e-12), ("f32", 2e-6)):
        say("noiseless brickwork n=14 %s" % prec)
        d = T.simulate(n, ops, 2, prec)
        r, c = sampled_pairs(rng, n, 512)
        got = d.gather(r + (c << np.uint64(n))).astype(np.complex128)
        want = psi[r.astype(np.int64)] * np.conj(psi[c.astype(np.int64)])
        assert np.abs(got - want).max() <= tol * max(1.0, np.abs(want).max())
        d.free()


def ising_variant(n, steps, h_zero=False, j_zero=False):
    ops, h = W.ising_trotter(n, steps, seed=3)
    out, skip = [], 0
    for op in ops:
        if h_zero and op.label == "rx":
            out.append(W.gate(W.rx(0.0), op.qubits, "rx"))
            continue
        if j_zero and op.label == "rzz":
            skip = 2  # the relaxation of its two qubits goes with it
            continue
        if skip and op.label == "tr":
            skip -= 1
            continue
        out.append(op)
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ising_15q_limits(oracle_mod, prec):
    n, steps = 15, 50
    tol = 1e-12 if prec == "f64" else 1e-5
    say("ising n=15 h=0 %s" % prec)
    d = T.simulate(n, ising_variant(n, steps, h_zero=True), 3, prec)
    z = np.real(d.expect_paulis(W.z_paulis(n)))
    assert np.abs(z - 1.0).max() <= tol
    d.free()
    say("ising n=15 J=0 %s" % prec)
    ops = ising_variant(n, steps, j_zero=True)
    d = T.simulate(n, ops, 3, prec)
    z = np.real(d.expect_paulis(W.z_paulis(n)))
    singles = []
    for q in range(n):
        local = [W.Op(op.kind, (0,), op.mats, op.label) for op in ops if op.qubits == (q,)]
        singles.append(oracle_mod.run(1, local))
    want_z = np.array([(s[0, 0] - s[1, 1]).real for s in singles])
    assert np.abs(z - want_z).max() <= tol
    # sampled elements of the product state
    rng = np.random.default_rng(8)
    r, c = sampled_pairs(rng, n, 256)
    got = d.gather(r + (c << np.uint64(n))).astype(np.complex128)
    want = np.ones(r.size, dtype=np.complex128)
    for q in range(n):
        rb = ((r >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
        cb = ((c >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
        want *= singles[q][rb, cb]
    assert np.abs(got - want).max() <= tol * max(1.0, np.abs(want).max())
    d.free()


def test_ising_15q_full_size_widths_agree():
    n, ops = W.config3()
    rng = np.random.default_rng(5)
    say("ising n=15 full: FP64 width 3 vs width 2")
    c = T.Circuit(n, ops)
    a = T.DM(n, "f64")
    a.apply_fused(c.fuse(3, "f64"))
    check_properties(a, n, rng, 1e-12)
    b = T.DM(n, "f64")
    b.apply_fused(c.fuse(2, "f64"))
    fro, mx, nrm = a.compare(b)
    assert mx <= 1e-12 and fro <= 1e-12 * nrm
    za = np.real(a.expect_paulis(W.z_paulis(n)))
    zb = np.real(b.expect_paulis(W.z_paulis(n)))
    assert np.abs(za - zb).max() <= 1e-12
    a.free()
    b.free()
    c.free()


GOLDEN_BRICK = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "brickwork14_2layers.npz")


@pytest.mark.parametrize("prec,width", [("f64", 2), ("f64", 3), ("f32", 2)])
def test_brickwork_14q_prefix_against_oracle(prec, width):
    """The first two layers of the noisy 14-qubit brickwork (every bond entangled once, all
    noise channels present) against the oracle's result, written by tests/golden/make_golden.py:
    all 2^14 probabilities, 4096 sampled elements of vec(rho) and <Z_i Z_i+1>.  FP64 runs as
    passes at width 2 and as 3-qubit applies at width 3."""
    if not os.path.exists(GOLDEN_BRICK):
        pytest.skip("oracle values not generated (tests/golden/make_golden.py brickwork)")
    g = np.load(GOLDEN_BRICK)
    n, ops = W.config2(layers=2)
    say("brickwork n=14 2-layer prefix vs oracle: %s width %d" % (prec, width))
    c = T.Circuit(n, ops)
    f = c.fuse(width, prec)
    if prec == "f64" and width == 2:
        assert f.passes()[0] > 0
    d = T.DM(n, prec)
    d.apply_fused(f)
    p, tr = d.probs(renormalize=True)
    vals = d.gather(g["idx"]).astype(np.complex128)
    zz = np.real(d.expect_paulis(W.zz_paulis(n)))
    d.free()
    f.free()
    c.free()
    if prec == "f64":
        assert np.abs(vals - g["val"]).max() <= 1e-10
        assert np.linalg.norm(vals - g["val"]) <= 1e-12 * np.linalg.norm(g["val"])
        assert np.abs(p - g["probs"]).max() <= 1e-12
        assert abs(tr - float(g["trace"])) <= 1e-12
        assert np.abs(zz - g["zz"]).max() <= 1e-12
    else:
        assert np.abs(p - g["probs"]).max() <= 1e-5
        assert np.abs(vals - g["val"]).max() <= 1e-6
        assert abs(tr - float(g["trace"])) <= 1e-5
        assert np.abs(zz - g["zz"]).max() <= 1e-5
