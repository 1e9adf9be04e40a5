"""Pins for the oracle's partial trace and single-qubit process tomography (Sec. 5, case study
1: the chi matrix of the teleportation channel), against brute force, closed forms and an
independent entanglement-fidelity simulation (no GPU)."""
import dataclasses
import math
import os

import numpy as np
import pytest

from paper_2404_13184_amd import workloads as W

SIG = [W.I2, W.PX, W.PY, W.PZ]


def rand_rho(rng, n):
    A = rng.standard_normal((1 << n, 1 << n)) + 1j * rng.standard_normal((1 << n, 1 << n))
    r = A @ A.conj().T
    return r / np.trace(r)


def brute_reduced(rho, n, keep):
    k = len(keep)
    out = np.zeros((1 << k, 1 << k), dtype=np.complex128)
    for x in range(1 << n):
        for y in range(1 << n):
            same = all(((x >> q) & 1) == ((y >> q) & 1) for q in range(n) if q not in keep)
            if same:
                a = sum(((x >> keep[t]) & 1) << t for t in range(k))
                b = sum(((y >> keep[t]) & 1) << t for t in range(k))
                out[a, b] += rho[x, y]
    return out


@pytest.mark.parametrize("keep", [[2], [3, 0], [1, 2, 3], [0, 1, 2, 3]])
def test_reduced_dm_brute_force(oracle_mod, keep):
    rng = np.random.default_rng(len(keep))
    rho = rand_rho(rng, 4)
    assert np.abs(oracle_mod.reduced_dm(rho, keep) - brute_reduced(rho, 4, keep)).max() < 1e-15


def test_reduced_dm_of_product_state(oracle_mod):
    rng = np.random.default_rng(9)
    lo, hi = rand_rho(rng, 2), rand_rho(rng, 1)  # qubits 0, 1 and qubit 2
    rho = np.kron(hi, lo)
    assert np.abs(oracle_mod.reduced_dm(rho, [0, 1]) - lo).max() < 1e-15
    assert np.abs(oracle_mod.reduced_dm(rho, [2]) - hi).max() < 1e-15
    # keep order swaps the qubits of the result: (1, 0) is lo with its two bits exchanged
    P = W.swap()
    assert np.abs(oracle_mod.reduced_dm(rho, [1, 0]) - P @ lo @ P).max() < 1e-15


def chi_of_kraus(kraus):
    """chi = sum_k c_k c_k^dag with K_k = sum_i c_ki sigma_i (the Pauli expansion)."""
    chi = np.zeros((4, 4), dtype=np.complex128)
    for K in kraus:
        c = np.array([np.trace(s.conj().T @ K) / 2 for s in SIG])
        chi += np.outer(c, c.conj())
    return chi


def test_chi_closed_forms(oracle_mod):
    p = 0.12
    chi = oracle_mod.process_chi_1q(1, [W.channel(W.depolarizing(p, 1), (0,))], 0, 0)
    assert np.abs(chi - np.diag([1 - 3 * p / 4, p / 4, p / 4, p / 4])).max() < 1e-14
    g = 0.3  # amplitude damping: K0 = a I + b Z, K1 = sqrt(g) (X + iY) / 2
    a, b = (1 + math.sqrt(1 - g)) / 2, (1 - math.sqrt(1 - g)) / 2
    c0 = np.array([a, 0, 0, b])
    c1 = np.array([0, math.sqrt(g) / 2, 1j * math.sqrt(g) / 2, 0])
    want = np.outer(c0, c0.conj()) + np.outer(c1, c1.conj())
    chi = oracle_mod.process_chi_1q(1, [W.channel(W.amplitude_damping(g), (0,))], 0, 0)
    assert np.abs(chi - want).max() < 1e-14
    th = 0.7  # RX(th) = cos(th/2) I - i sin(th/2) X
    c = np.array([math.cos(th / 2), -1j * math.sin(th / 2), 0, 0])
    chi = oracle_mod.process_chi_1q(2, [W.gate(W.rx(th), (1,))], 1, 1)
    assert np.abs(chi - np.outer(c, c.conj())).max() < 1e-14
    # a spectator in |0> and a SWAP carry the channel from qubit 0 to qubit 1
    chi = oracle_mod.process_chi_1q(2, [W.channel(W.amplitude_damping(g), (0,)), W.gate(W.swap(), (0, 1))], 0, 1)
    assert np.abs(chi - want).max() < 1e-14
    # and the chi of a random channel equals its Pauli expansion
    rng = np.random.default_rng(4)
    K = W.kraus_compose(W.thermal_relaxation(50.0, 70.0, 4.0), [W.random_unitary(rng, 2)])
    chi = oracle_mod.process_chi_1q(1, [W.channel(K, (0,))], 0, 0)
    assert np.abs(chi - chi_of_kraus(K)).max() < 1e-14


def test_measurement_with_readout_error(oracle_mod):
    rng = np.random.default_rng(3)
    rho = rand_rho(rng, 1)
    out = oracle_mod.run(1, [W.channel(W.measure_with_readout_error(0.04, 0.01), (0,))], rho)
    p0, p1 = rho[0, 0].real, rho[1, 1].real
    assert abs(out[0, 0] - (0.99 * p0 + 0.04 * p1)) < 1e-15
    assert abs(out[1, 1] - (0.01 * p0 + 0.96 * p1)) < 1e-15
    assert abs(out[0, 1]) == 0 and abs(out[1, 0]) == 0


def noiseless(dev):
    """The device with zero gate times and zero gate errors: every injected channel is the
    identity."""
    return dataclasses.replace(W.with_gate_errors(dev, 0.0, 0.0), t_1q=0.0, t_cx={k: 0.0 for k in dev.t_cx})


def test_transpiled_teleport_is_identity_channel(oracle_mod):
    golden = os.path.join(os.path.dirname(__file__), "golden", "teleport_chi_ideal.txt")
    want = np.loadtxt(golden, comments="#").reshape(4, 4)
    dev = noiseless(W.synthetic_device(3, seed=1, line=False))
    ops = W.teleport_device_circuit(dev, 0, 1, 2, readout=False)
    assert np.abs(oracle_mod.process_chi_1q(3, ops, 0, 2) - want).max() < 1e-12


@pytest.mark.parametrize("worse", [False, True])
def test_noisy_teleport_chi(oracle_mod, worse):
    dev = W.synthetic_device(3, seed=1, line=False)
    if worse:
        dev = W.with_gate_errors(dev, 0.1, 0.1)
    ops = W.teleport_device_circuit(dev, 0, 1, 2)
    chi = oracle_mod.process_chi_1q(3, ops, 0, 2)
    # a channel's chi is Hermitian, positive semidefinite and trace preserving:
    # sum_ij chi_ij sigma_j sigma_i = I
    assert np.abs(chi - chi.conj().T).max() < 1e-13
    assert np.linalg.eigvalsh(chi).min() > -1e-13
    tp = sum(chi[i, j] * SIG[j] @ SIG[i] for i in range(4) for j in range(4))
    assert np.abs(tp - np.eye(2)).max() < 1e-13
    # chi_00 is the entanglement fidelity: teleport half of a Bell pair (a, ancilla 3) and
    # measure the overlap of (c, ancilla) with the Bell state
    prep = [W.gate(W.hadamard(), (3,)), W.gate(W.cx(), (3, 0))]
    rho = oracle_mod.run(4, prep + ops)
    pair = oracle_mod.reduced_dm(rho, [2, 3])
    phi = np.array([1, 0, 0, 1], dtype=np.complex128) / math.sqrt(2)
    f_e = (phi.conj() @ pair @ phi).real
    assert abs(chi[0, 0].real - f_e) < 1e-13
    assert (0.3 < f_e < 0.8) if worse else (0.9 < f_e < 1.0)
