"""Pins for the calibration-driven noise builder (no GPU): channel identities, closed forms and
the reported gate error reproduced through an independent oracle simulation."""
import math

import numpy as np
import pytest

from paper_2404_13184_amd import workloads as W


def rand_rho(rng, n):
    A = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    r = A @ A.conj().T
    return r / np.trace(r)


def test_general_relaxation_reduces_to_zero_temperature(oracle_mod):
    rng = np.random.default_rng(1)
    rho = rand_rho(rng, 1)
    a = oracle_mod.run(1, [W.channel(W.thermal_relaxation(80.0, 100.0, 3.0), (0,))], rho)
    b = oracle_mod.run(1, [W.channel(W.thermal_relaxation_general(80.0, 100.0, 3.0, 0.0), (0,))], rho)
    assert np.abs(a - b).max() < 1e-15


def test_general_relaxation_closed_forms(oracle_mod):
    t1, t2, t, pe = 60.0, 90.0, 5.0, 0.03
    rng = np.random.default_rng(2)
    rho = rand_rho(rng, 1)
    out = oracle_mod.run(1, [W.channel(W.thermal_relaxation_general(t1, t2, t, pe), (0,))], rho)
    assert abs(out[1, 1] - (pe + (rho[1, 1] - pe) * math.exp(-t / t1))) < 1e-14
    assert abs(out[0, 1] - rho[0, 1] * math.exp(-t / t2)) < 1e-14
    eq = np.diag([1 - pe, pe]).astype(np.complex128)  # thermal state is the fixed point
    assert np.abs(oracle_mod.run(1, [W.channel(W.thermal_relaxation_general(t1, t2, t, pe), (0,))], eq) - eq).max() < 1e-15


@pytest.mark.parametrize("j", [1, 2])
def test_canonical_kraus_same_channel(oracle_mod, j):
    rng = np.random.default_rng(3 + j)
    K = W.kraus_compose(W.depolarizing(0.07, j), [W.random_unitary(rng, 1 << j) * 0.6, np.eye(1 << j) * 0.8])
    C = W.kraus_canonical(K)
    assert len(C) <= 4 ** j
    rho = rand_rho(rng, 3)
    qs = (2, 0) if j == 2 else (1,)
    a = oracle_mod.run(3, [W.channel(K, qs)], rho)
    b = oracle_mod.run(3, [W.channel(C, qs)], rho)
    assert np.abs(a - b).max() < 1e-14


def process_fidelity_by_simulation(oracle_mod, kraus, j):
    """<Phi|(E (x) I)(|Phi><Phi|)|Phi> with Phi maximally entangled between system qubits
    0..j-1 and ancillas j..2j-1, prepared by H and CX gates and simulated by the oracle."""
    n = 2 * j
    prep = []
    for t in range(j):
        prep.append(W.gate(W.hadamard(), (j + t,)))
        prep.append(W.gate(W.cx(), (j + t, t)))
    ops = prep + [W.channel(kraus, tuple(range(j)))]
    rho = oracle_mod.run(n, ops)
    phi = oracle_mod.statevector(n, prep)
    return (phi.conj() @ rho @ phi).real


@pytest.mark.parametrize("gate_name", ["sx", "cx"])
def test_gate_noise_reproduces_reported_error(oracle_mod, gate_name):
    dev = W.synthetic_device(4, seed=11)
    qs = (1,) if gate_name == "sx" else (1, 2)
    j = len(qs)
    d = 1 << j
    K = W.device_gate_noise(dev, gate_name, qs)
    err = dev.err_1q[1] if gate_name == "sx" else dev.err_cx[(1, 2)]
    f_pro = process_fidelity_by_simulation(oracle_mod, K, j)
    f_avg = (d * f_pro + 1) / (d + 1)
    assert abs((1 - f_avg) - err) < 1e-12
    # relaxation alone stays below the reported error (depolarizing makes up the rest)
    assert W.depolarizing_for_gate_error(err, W.kraus_compose(K, [np.eye(d)])) >= 0


def test_u3_decomposition_into_basis():
    rng = np.random.default_rng(5)
    for _ in range(5):
        th, ph, la = rng.uniform(0, 2 * math.pi, 3)
        U = np.eye(2, dtype=np.complex128)
        for name, _, ang in W.u3_to_basis(0, th, ph, la):
            U = (W.rz(ang) if name == "rz" else W.sx()) @ U
        overlap = abs(np.trace(W.u3(th, ph, la).conj().T @ U))
        assert abs(overlap - 2) < 1e-12


def test_device_circuit_is_physical(oracle_mod):
    dev = W.synthetic_device(4, seed=2)
    ops = W.device_random_circuit(dev, 2, seed=9)
    assert any(op.label == "noise_cx" for op in ops)
    assert all(op.mats.shape[0] <= 4 ** op.width for op in ops)
    rho = oracle_mod.run(4, ops)
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.linalg.eigvalsh(rho).min() > -1e-12
    with pytest.raises(ValueError):
        W.noisy_basis_circuit(dev, [("cx", (0, 3), 0.0)])  # not a coupler on the line
