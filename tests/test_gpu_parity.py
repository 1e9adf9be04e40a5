"""HIP path vs the CPU FP64 oracle (needs an MI355X).

FP64 bar: max |rho_gpu - rho_oracle| <= 1e-10 element-wise, plus a relative Frobenius
bound of 1e-12 (entries are ~2^-n, so the absolute bar alone is loose).
FP32 bar: trace distance <= 1e-4 and |p_gpu - p_oracle| <= 1e-5 per probability.
"""
import itertools
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu

ABS64 = 1e-10
REL64 = 1e-12


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def device():
    T.load()
    d = T.DM(1, "f64")  # raises if no device is usable
    d.free()


def superop_of(op):
    """sum_i conj(K_i) (x) K_i with local index row + 2^j col (test-side construction)."""
    return sum(np.kron(K.conj(), K) for K in op.mats)


def random_density(rng, n):
    dim = 1 << n
    A = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    rho = A @ A.conj().T
    return rho / np.trace(rho)


def random_channel(rng, qubits):
    j = len(qubits)
    d = 1 << j
    mats = [rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)) for _ in range(int(rng.integers(1, 4)))]
    return W.channel([m * 0.5 for m in mats], qubits)


def check64(got_mat, want, ctx=""):
    err = np.abs(got_mat - want).max()
    rel = np.linalg.norm(got_mat - want) / np.linalg.norm(want)
    assert err <= ABS64 and rel <= REL64, "%s: max abs %.3e rel %.3e" % (ctx, err, rel)


def gpu_rho(d, oracle_mod):
    return oracle_mod.vec_to_matrix(d.read().astype(np.complex128), d.n)


# ---------------------------------------------------------------------------------------
# single applies, every width and placement class
# ---------------------------------------------------------------------------------------

def placements(n, k):
    """Low, high, straddling, reversed and random qubit tuples (first = LSB of S)."""
    cands = [tuple(range(k)), tuple(range(n - k, n)), tuple(reversed(range(k)))]
    if n > k:
        cands.append(tuple([0] + list(range(n - k + 1, n))))
        cands.append(tuple(reversed([0] + list(range(n - k + 1, n)))))
    rng = np.random.default_rng(n * 10 + k)
    for _ in range(2):
        cands.append(tuple(int(x) for x in rng.choice(n, size=k, replace=False)))
    out = []
    for c in cands:
        if c not in out:
            out.append(c)
    return out


@pytest.mark.parametrize("k,n", [(1, 1), (1, 2), (1, 5), (1, 9), (2, 2), (2, 3), (2, 5), (2, 6), (2, 9),
                                 (3, 3), (3, 4), (3, 5), (3, 6), (3, 7), (3, 9)])
def test_apply_superop_f64(oracle_mod, k, n):
    rng = np.random.default_rng(1000 + 17 * k + n)
    for qs in placements(n, k):
        say("apply_superop f64 k=%d n=%d qubits=%s" % (k, n, qs))
        op = random_channel(rng, qs)
        rho = random_density(rng, n)
        with T.DM(n, "f64") as d:
            d.write(oracle_mod.matrix_to_vec(rho))
            d.apply_superop(qs, superop_of(op))
            got = gpu_rho(d, oracle_mod)
        check64(got, oracle_mod.run(n, [op], rho), "k=%d n=%d q=%s" % (k, n, qs))


@pytest.mark.parametrize("k,n", [(1, 6), (2, 6), (2, 8), (3, 6), (3, 8)])
def test_apply_superop_f32(oracle_mod, k, n):
    rng = np.random.default_rng(2000 + 17 * k + n)
    for qs in placements(n, k)[:4]:
        say("apply_superop f32 k=%d n=%d qubits=%s" % (k, n, qs))
        op = W.channel([W.random_unitary(rng, 1 << k)], qs)
        rho = random_density(rng, n)
        with T.DM(n, "f32") as d:
            d.write(oracle_mod.matrix_to_vec(rho))
            d.apply_superop(qs, superop_of(op))
            got = gpu_rho(d, oracle_mod)
        want = oracle_mod.run(n, [op], rho)
        assert np.abs(got - want).max() <= 1e-6


def test_repeated_applies_no_upload_race(oracle_mod):
    """Many consecutive uploads through the pinned ring (more than its slot count)."""
    n = 6
    rng = np.random.default_rng(5)
    ops = [random_channel(rng, tuple(int(x) for x in rng.choice(n, size=int(rng.integers(1, 4)), replace=False)))
           for _ in range(30)]
    rho = random_density(rng, n)
    say("30 queued applies n=6")
    with T.DM(n, "f64") as d:
        d.write(oracle_mod.matrix_to_vec(rho))
        for op in ops:
            d.apply_superop(op.qubits, superop_of(op))
        got = gpu_rho(d, oracle_mod)
    want = oracle_mod.run(n, ops, rho)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-11


# ---------------------------------------------------------------------------------------
# fused circuits (Sec. 3.3) vs the unfused oracle
# ---------------------------------------------------------------------------------------

MODES = [T.TANQ_FUSE_NONE, T.TANQ_FUSE_PAPER, 1, 2, 3, T.TANQ_FUSE_AUTO]


@pytest.mark.parametrize("mode", MODES)
def test_config1_fused_f64(oracle_mod, mode):
    """8 qubits, depth 20, U3 + dep + AD, CX + dep2 (the plain-method configuration)."""
    n, ops = W.config1()
    say("config1 f64 mode=%d" % mode)
    want = oracle_mod.run(n, ops)
    d = T.simulate(n, ops, mode, "f64")
    got = gpu_rho(d, oracle_mod)
    p, tr = d.probs(renormalize=False)
    d.free()
    check64(got, want, "config1 mode %d" % mode)
    pw, trw = oracle_mod.diag(want)
    assert abs(tr - trw) <= 1e-12 and np.abs(p - pw).max() <= 1e-12


@pytest.mark.parametrize("layers", [1, 3])
@pytest.mark.parametrize("mode", [2, 3])
def test_shallow_random_circuits_f64(oracle_mod, layers, mode):
    """Shallow circuits keep rho far from I/2^n, so a wrong kernel cannot hide."""
    n = 9
    ops = W.random_u3_cx(n, layers, seed=70 + layers, p1=1e-3, p2=1e-2, gamma=5e-4)
    say("shallow n=9 layers=%d mode=%d" % (layers, mode))
    want = oracle_mod.run(n, ops)
    d = T.simulate(n, ops, mode, "f64")
    got = gpu_rho(d, oracle_mod)
    d.free()
    check64(got, want, "shallow")
    assert np.trace(want @ want).real > 0.5


def test_config2_small_f64(oracle_mod):
    n, ops = W.config2(layers=8, n=8)
    say("config2 small n=8")
    want = oracle_mod.run(n, ops)
    d = T.simulate(n, ops, 2, "f64")
    got = gpu_rho(d, oracle_mod)
    zz = d.expect_paulis(W.zz_paulis(n))
    d.free()
    check64(got, want, "config2")
    for s, v in zip(W.zz_paulis(n), zz):
        assert abs(v - oracle_mod.expect_pauli(want, s)) <= 1e-12


def test_config3_small_f64(oracle_mod):
    n, ops = W.config3(steps=6, n=7)
    say("config3 small n=7 k=3")
    want = oracle_mod.run(n, ops)
    d = T.simulate(n, ops, 3, "f64")
    got = gpu_rho(d, oracle_mod)
    z = d.expect_paulis(W.z_paulis(n))
    d.free()
    check64(got, want, "config3")
    for s, v in zip(W.z_paulis(n), z):
        assert abs(v - oracle_mod.expect_pauli(want, s)) <= 1e-12


def test_teleport_layers_f64(oracle_mod):
    n = 7
    ops = W.teleport_layers(n, 3, seed=9, p1=2e-3, p2=2e-2)
    say("teleport n=7")
    want = oracle_mod.run(n, ops)
    for mode in (2, 3):
        d = T.simulate(n, ops, mode, "f64")
        check64(gpu_rho(d, oracle_mod), want, "teleport mode %d" % mode)
        d.free()


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_registers(oracle_mod, n):
    rng = np.random.default_rng(n)
    ops = []
    for _ in range(12):
        j = int(rng.integers(1, n + 1))
        qs = tuple(int(x) for x in rng.choice(n, size=j, replace=False))
        ops.append(random_channel(rng, qs))
    say("tiny n=%d" % n)
    rho = random_density(rng, n)
    want = oracle_mod.run(n, ops, rho)
    for mode in (T.TANQ_FUSE_NONE, 1, 2, 3):
        c = T.Circuit(n, ops)
        f = c.fuse(mode, "f64")
        with T.DM(n, "f64") as d:
            d.write(oracle_mod.matrix_to_vec(rho))
            d.apply_fused(f)
            got = gpu_rho(d, oracle_mod)
        f.free()
        c.free()
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 1e-12, (n, mode, err)


def test_fused_composition_matches_oracle(oracle_mod):
    """Each fused FP64 superoperator equals the oracle's action of its member operations on
    the basis operators |r><c| of the block's qubits."""
    n, ops = W.config3(steps=2, n=6)
    c = T.Circuit(n, ops)
    blocks, nb = c.plan(3)
    f = c.fuse(3, "f64")
    assert f.count == nb
    say("composition readback, %d blocks" % nb)
    for b in range(nb):
        k, Q, S = f.get(b)
        members = [ops[i] for i in range(len(ops)) if blocks[i] == b]
        loc = {q: i for i, q in enumerate(Q)}
        local = [W.Op(op.kind, tuple(loc[q] for q in op.qubits), op.mats, op.label) for op in members]
        D = 1 << k
        want = np.zeros((D * D, D * D), dtype=np.complex128)
        for col in range(D * D):
            E = np.zeros((D, D), dtype=np.complex128)
            E[col % D, col // D] = 1.0
            want[:, col] = oracle_mod.matrix_to_vec(oracle_mod.run(k, local, E))
        assert np.abs(S - want).max() <= 1e-13, b
    f.free()
    c.free()


# ---------------------------------------------------------------------------------------
# FP32 form
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [T.TANQ_FUSE_NONE, 2, 3])
def test_config1_f32_error_bounds(oracle_mod, mode):
    n, ops = W.config1()
    say("config1 f32 mode=%d" % mode)
    want = oracle_mod.run(n, ops)
    d = T.simulate(n, ops, mode, "f32")
    got = gpu_rho(d, oracle_mod)
    p, tr = d.probs(renormalize=True)
    d.free()
    td = oracle_mod.trace_distance(got, want)
    pw, _ = oracle_mod.diag(want)
    assert td <= 1e-4, td
    assert np.abs(p - pw).max() <= 1e-5
    assert abs(tr - 1.0) <= 1e-5


def test_shallow_f32_relative(oracle_mod):
    n = 8
    ops = W.random_u3_cx(n, 2, seed=3, p1=1e-3, p2=1e-2)
    say("shallow f32")
    want = oracle_mod.run(n, ops)
    d = T.simulate(n, ops, 3, "f32")
    got = gpu_rho(d, oracle_mod)
    d.free()
    assert oracle_mod.trace_distance(got, want) <= 1e-5


# ---------------------------------------------------------------------------------------
# reductions
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_probs_and_paulis_random_state(oracle_mod, prec):
    rng = np.random.default_rng(77)
    n = 7
    rho = random_density(rng, n)
    strings = ["".join(rng.choice(list("IXYZ"), size=n)) for _ in range(40)] + W.zz_paulis(n) + ["I" * n]
    say("reductions %s" % prec)
    with T.DM(n, prec) as d:
        d.write(oracle_mod.matrix_to_vec(rho))
        p, tr = d.probs(renormalize=False)
        vals = d.expect_paulis(strings)
        single = d.expect_pauli(strings[0])
    pw, trw = oracle_mod.diag(rho)
    tol = 1e-13 if prec == "f64" else 1e-6
    assert abs(tr - trw) <= tol and np.abs(p - pw).max() <= tol
    for s, v in zip(strings, vals):
        assert abs(v - oracle_mod.expect_pauli(rho, s)) <= tol, s
    assert abs(single - vals[0]) == 0


def test_reset_and_initial_state(oracle_mod):
    with T.DM(5, "f64") as d:
        v = d.read()
        assert v[0] == 1 and np.count_nonzero(v) == 1
        d.fill_random(3)
        d.reset()
        v = d.read()
        assert v[0] == 1 and np.count_nonzero(v) == 1


def test_fill_random_matches_definition():
    with T.DM(6, "f64") as d:
        d.fill_random(11)
        v = d.read()
    want = W.hash_fill_values(11, np.arange(4 ** 6))
    assert np.array_equal(v, want)


def test_error_paths_on_device():
    with T.DM(4, "f64") as d:
        with pytest.raises(T.TanqError):
            d.apply_superop((0, 4), np.eye(16))
        with pytest.raises(T.TanqError):
            d.apply_superop((1, 1), np.eye(16))
        with pytest.raises(T.TanqError):
            d.expect_pauli("XXZ")
        with pytest.raises(T.TanqError):
            d.gather([4 ** 4])
        c = T.Circuit(5, [W.gate(W.hadamard(), (0,))])
        f = c.fuse(2, "f64")
        with pytest.raises(T.TanqError) as e:
            d.apply_fused(f)
        assert e.value.code == T.TANQ_E_STATE
        f.free()
        f2 = T.Circuit(4, [W.gate(W.hadamard(), (0,))]).fuse(2, "f32")
        with pytest.raises(T.TanqError):
            d.apply_fused(f2)
        f2.free()


@pytest.mark.parametrize("pa,pb", [("f64", "f64"), ("f32", "f64"), ("f64", "f32")])
def test_dm_compare(oracle_mod, pa, pb):
    rng = np.random.default_rng(123)
    n = 6
    ra, rb = random_density(rng, n), random_density(rng, n)
    say("compare %s %s" % (pa, pb))
    with T.DM(n, pa) as a, T.DM(n, pb) as b:
        a.write(oracle_mod.matrix_to_vec(ra))
        b.write(oracle_mod.matrix_to_vec(rb))
        fro, mx, nrm = a.compare(b)
        va, vb = a.read().astype(np.complex128), b.read().astype(np.complex128)
    assert abs(fro - np.linalg.norm(va - vb)) <= 1e-12 * np.linalg.norm(va - vb)
    assert abs(mx - np.abs(va - vb).max()) <= 1e-15
    assert abs(nrm - np.linalg.norm(va)) <= 1e-12 * np.linalg.norm(va)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_empty_circuit(prec):
    """Fusing a circuit with no operations gives no blocks; applying it leaves |0><0|."""
    say("empty circuit %s" % prec)
    c = T.Circuit(5)
    f = c.fuse(T.TANQ_FUSE_AUTO, prec)
    assert f.count == 0 and f.info["source_ops"] == 0
    with T.DM(5, prec) as d:
        d.apply_fused(f)
        p, tr = d.probs()
        assert tr == 1.0 and p[0] == 1.0 and np.count_nonzero(p) == 1
    f.free()
    c.free()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_three_qubit_operations_fused(oracle_mod, prec):
    """Circuits with 3-qubit gates and 3-qubit Kraus channels between 1- and 2-qubit ones,
    fused at width 3 (the composition's whole-column path) and unfused."""
    rng = np.random.default_rng(33)
    n = 6
    ops = []
    for _ in range(6):
        q3 = tuple(int(x) for x in rng.choice(n, 3, replace=False))
        ops.append(W.gate(W.random_unitary(rng, 8), q3))
        ops.append(random_channel(rng, q3))
        q1 = int(q3[0])
        ops.append(W.gate(W.u3(*rng.uniform(0, 6.28, 3)), (q1,)))
        q2 = (int(q3[1]), int(q3[2]))
        ops.append(W.gate(W.cx(), q2))
        ops.append(W.channel(W.depolarizing(0.02, 2), q2))
    want = oracle_mod.run(n, ops)
    for mode in (3, T.TANQ_FUSE_NONE):
        say("three-qubit ops %s mode=%d" % (prec, mode))
        d = T.simulate(n, ops, mode, prec)
        got = gpu_rho(d, oracle_mod)
        d.free()
        if prec == "f64":
            check64(got, want, "mode %d" % mode)
        else:
            assert oracle_mod.trace_distance(got / np.trace(got), want / np.trace(want)) <= 1e-4


# ---------------------------------------------------------------------------------------
# in-place scaling (the plain streaming pass over the state)
# ---------------------------------------------------------------------------------------


@pytest.mark.parametrize("prec,peak", [("f64", 78.6), ("f32", 157.3)])
def test_mfma_rate_is_plausible(prec, peak):
    """The measured matrix-unit rate of the multiplication loop alone lies below the datasheet
    peak (products of 16 x 16 x 4 at the chip's top clock) and well above a quarter of it."""
    say("mfma rate %s" % prec)
    r = T.tanq_mfma_rate(prec)
    assert 0.25 * peak < r <= 1.02 * peak, r

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 4, 5, 9, 12])
def test_scale_in_place(prec, n):
    """Partial workgroups (n <= 4), one exact workgroup (n = 5 FP64) and grid-stride sweeps
    (n = 12): every element equals the host product in the state's precision."""
    say("scale n=%d %s" % (n, prec))
    with T.DM(n, prec) as d:
        d.fill_random(3 + n)
        x = d.read()
        for f in (0.5, 1.0 / 3.0, -2.0):
            d.scale(f)
            ft = x.real.dtype.type(f)
            x = (x.real * ft + 1j * (x.imag * ft)).astype(x.dtype)
            got = d.read()
            assert np.array_equal(got, x), (n, prec, f)
        with pytest.raises(T.TanqError):
            d.scale(float("inf"))
