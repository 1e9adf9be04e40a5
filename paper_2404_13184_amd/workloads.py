"""Seeded synthetic workloads: gate matrices, Kraus channels and circuit generators.

This module is the single source of inputs for both the CPU reference (``oracle/``)
and the HIP path.  It holds no superoperator arithmetic: it only emits an explicit,
ordered list of operations, each a set of Kraus matrices acting on named qubits.
A unitary gate is the one-element case (the problem statement of Sec. 2.1, Eq.
``eq:dmsim``: the input is rho_in plus a sequence of not-necessarily-unitary
transformations).

Conventions (shared by every consumer):

* A j-qubit matrix acting on ``qubits = (q_0, ..., q_{j-1})`` is indexed by the local
  basis index ``sum_t b_{q_t} 2^t``: the first listed qubit is the least-significant
  bit.  Matrices are ``M[out, in]``.
* Qubit q of an n-qubit register is bit q of the row index of rho (little-endian), as
  in the strided index map of Sec. 3.1, whose 2^q terms address qubit q.

Noise channels follow the Qiskit-Aer conventions the paper adopts (Sec. 3.5):
depolarizing with parameter p on j qubits is (1-p) rho + p Tr_Q(rho) (x) I/2^j,
amplitude damping, phase damping, and thermal relaxation built from the two.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------------------
# Operation record
# --------------------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Op:
    """One circuit operation: Kraus matrices ``mats`` (m, 2^j, 2^j) on ``qubits``.

    ``kind`` is ``"gate"`` for a unitary (m == 1) and ``"kraus"`` for a channel.
    ``label`` is informational only (e.g. ``"u3"``, ``"dep1"``).
    """

    kind: str
    qubits: Tuple[int, ...]
    mats: np.ndarray
    label: str = ""

    @property
    def width(self) -> int:
        return len(self.qubits)


def gate(U: np.ndarray, qubits: Sequence[int], label: str = "") -> Op:
    U = np.asarray(U, dtype=np.complex128)
    j = len(qubits)
    assert U.shape == (2 ** j, 2 ** j)
    return Op("gate", tuple(int(q) for q in qubits), U.reshape(1, 2 ** j, 2 ** j).copy(), label)


def channel(kraus: Sequence[np.ndarray], qubits: Sequence[int], label: str = "") -> Op:
    K = np.asarray(np.stack([np.asarray(k, dtype=np.complex128) for k in kraus]))
    j = len(qubits)
    assert K.shape[1:] == (2 ** j, 2 ** j)
    return Op("kraus", tuple(int(q) for q in qubits), K, label)


# --------------------------------------------------------------------------------------
# Gate matrices
# --------------------------------------------------------------------------------------

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULIS = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """OpenQASM 2 U3(theta, phi, lambda)."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array(
        [[c, -np.exp(1j * lam) * s], [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
        dtype=np.complex128,
    )


def rx(theta: float) -> np.ndarray:
    """exp(-i theta X / 2)."""
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    """exp(-i theta Z / 2)."""
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)


def hadamard() -> np.ndarray:
    return np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)


def rzz(theta: float) -> np.ndarray:
    """exp(-i theta Z(x)Z / 2); diagonal, eigenvalue of ZZ is (-1)^(b0 xor b1)."""
    d = []
    for idx in range(4):
        b0, b1 = idx & 1, (idx >> 1) & 1
        zz = 1 - 2 * (b0 ^ b1)
        d.append(np.exp(-0.5j * theta * zz))
    return np.diag(d).astype(np.complex128)


def controlled(U1: np.ndarray) -> np.ndarray:
    """Two-qubit controlled-U on qubits (control, target): local index b_c + 2 b_t.

    Defined by its action on basis states: if b_c == 1 the target's 2x2 block is U1.
    """
    M = np.zeros((4, 4), dtype=np.complex128)
    for bc in range(2):
        for bt_in in range(2):
            col = bc + 2 * bt_in
            if bc == 0:
                M[col, col] = 1.0
            else:
                for bt_out in range(2):
                    M[bc + 2 * bt_out, col] = U1[bt_out, bt_in]
    return M


def cx() -> np.ndarray:
    return controlled(PX)


def cz() -> np.ndarray:
    return controlled(PZ)


def swap() -> np.ndarray:
    M = np.zeros((4, 4), dtype=np.complex128)
    for b0 in range(2):
        for b1 in range(2):
            M[b1 + 2 * b0, b0 + 2 * b1] = 1.0
    return M


def random_unitary(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Haar-random unitary via QR of a complex Ginibre matrix (Mezzadri's phase fix)."""
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph


# --------------------------------------------------------------------------------------
# Noise channels (Kraus sets), Sec. 3.5
# --------------------------------------------------------------------------------------


def pauli_string_matrix(labels: str) -> np.ndarray:
    """Matrix of a j-qubit Pauli string; ``labels[t]`` acts on local qubit t (bit t)."""
    M = np.array([[1.0 + 0j]])
    for ch in labels:  # local qubit t is bit t: it is the right-most Kronecker factor so far
        M = np.kron(PAULIS[ch], M)
    return M


def depolarizing(p: float, j: int) -> List[np.ndarray]:
    """Kraus set of (1-p) rho + p Tr_Q(rho) (x) I/2^j on j qubits (Qiskit-Aer convention).

    Pauli-mixture form: identity with weight 1 - (4^j - 1) p / 4^j, every other Pauli
    string with weight p / 4^j.
    """
    d4 = 4 ** j
    if not (0.0 <= p <= d4 / (d4 - 1)):
        raise ValueError("depolarizing parameter out of range")
    out = []
    for labels in itertools.product("IXYZ", repeat=j):
        s = "".join(labels)
        w = 1.0 - (d4 - 1) * p / d4 if set(s) == {"I"} else p / d4
        if w > 0.0:
            out.append(math.sqrt(w) * pauli_string_matrix(s))
    return out


def amplitude_damping(gamma: float) -> List[np.ndarray]:
    k0 = np.array([[1, 0], [0, math.sqrt(1 - gamma)]], dtype=np.complex128)
    k1 = np.array([[0, math.sqrt(gamma)], [0, 0]], dtype=np.complex128)
    return [k0, k1]


def phase_damping(lam: float) -> List[np.ndarray]:
    k0 = np.array([[1, 0], [0, math.sqrt(1 - lam)]], dtype=np.complex128)
    k1 = np.array([[0, 0], [0, math.sqrt(lam)]], dtype=np.complex128)
    return [k0, k1]


def thermal_relaxation(t1: float, t2: float, t: float) -> List[np.ndarray]:
    """Thermal relaxation toward |0> (zero excited-state population), requires T2 <= 2 T1.

    Populations relax as exp(-t/T1) and coherences as exp(-t/T2).  Built as amplitude
    damping with gamma = 1 - exp(-t/T1) followed by phase damping with
    lambda = 1 - exp(-2t/T2 + t/T1); the Kraus set is the non-zero products.
    """
    if t2 > 2 * t1:
        raise ValueError("thermal_relaxation needs T2 <= 2 T1")
    gamma = 1.0 - math.exp(-t / t1)
    lam = 1.0 - math.exp(-2.0 * t / t2 + t / t1)
    out = []
    for P in phase_damping(lam):
        for A in amplitude_damping(gamma):
            K = P @ A
            if np.abs(K).max() > 0:
                out.append(K)
    return out


def generalized_amplitude_damping(gamma: float, excited: float) -> List[np.ndarray]:
    """Relaxation with rate gamma toward the thermal state diag(1 - excited, excited)."""
    a, b = math.sqrt(1.0 - excited), math.sqrt(excited)
    g, h = math.sqrt(gamma), math.sqrt(1.0 - gamma)
    return [np.array([[a, 0], [0, a * h]], dtype=np.complex128),
            np.array([[0, a * g], [0, 0]], dtype=np.complex128),
            np.array([[b * h, 0], [0, b]], dtype=np.complex128),
            np.array([[0, 0], [b * g, 0]], dtype=np.complex128)]


def thermal_relaxation_general(t1: float, t2: float, t: float, excited: float = 0.0) -> List[np.ndarray]:
    """Thermal relaxation with equilibrium excited-state population ``excited``: populations
    relax toward diag(1 - excited, excited) as exp(-t/T1), coherences decay as exp(-t/T2)
    (T2 <= 2 T1).  Generalised amplitude damping followed by phase damping; the Kraus set is the
    non-zero products.  excited = 0 gives :func:`thermal_relaxation`."""
    if t2 > 2 * t1:
        raise ValueError("thermal relaxation needs T2 <= 2 T1")
    gamma = 1.0 - math.exp(-t / t1)
    lam = 1.0 - math.exp(-2.0 * t / t2 + t / t1)
    out = []
    for P in phase_damping(lam):
        for A in generalized_amplitude_damping(gamma, excited):
            K = P @ A
            if np.abs(K).max() > 0:
                out.append(K)
    return out


def kraus_compose(first: Sequence[np.ndarray], second: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Kraus set of the channel `second` after `first` (all products, zero products dropped)."""
    out = []
    for B in second:
        for A in first:
            K = B @ A
            if np.abs(K).max() > 0:
                out.append(K)
    return out


def kraus_tensor(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Kraus set of channel a on local qubit 0 and b on local qubit 1 (a is the LSB factor)."""
    return [np.kron(B, A) for B in b for A in a]


def kraus_canonical(kraus: Sequence[np.ndarray], tol: float = 1e-15) -> List[np.ndarray]:
    """An equivalent Kraus set of at most d^2 operators: eigenvectors of the Choi matrix
    J = sum_i vec(K_i) vec(K_i)^dag (column stacking), K'_j = sqrt(l_j) unvec(v_j) for the
    eigenvalues l_j above tol * max(l)."""
    d = kraus[0].shape[0]
    vecs = np.stack([np.asarray(K, dtype=np.complex128).T.reshape(-1) for K in kraus], axis=1)
    J = vecs @ vecs.conj().T
    J = 0.5 * (J + J.conj().T)
    w, v = np.linalg.eigh(J)
    keep = w > tol * max(w.max(), 1e-300)
    return [math.sqrt(float(w[i])) * v[:, i].reshape(d, d).T for i in np.nonzero(keep)[0][::-1]]


def process_fidelity_to_identity(kraus: Sequence[np.ndarray]) -> float:
    """F_pro = sum_i |Tr K_i|^2 / d^2 (overlap of the channel with the identity channel)."""
    d = kraus[0].shape[0]
    return float(sum(abs(np.trace(K)) ** 2 for K in kraus).real) / (d * d)


def depolarizing_for_gate_error(gate_error: float, relax: Sequence[np.ndarray]) -> float:
    """Depolarizing parameter p such that depolarizing(p) after the relaxation channel has
    average gate infidelity `gate_error` (the device-noise rule of Qiskit-Aer, which the paper
    follows: the reported gate error is split into relaxation during the gate plus
    depolarizing).  With F_avg = (d F_pro + 1) / (d + 1) and
    F_pro(dep_p o R) = (1 - p) F_pro(R) + p / d^2.  Clamped to [0, 4^j / (4^j - 1)]."""
    d = relax[0].shape[0]
    f_target = 1.0 - gate_error
    fpro_target = ((d + 1) * f_target - 1.0) / d
    fr = process_fidelity_to_identity(relax)
    if fr - 1.0 / (d * d) <= 0:
        return 0.0
    p = (fr - fpro_target) / (fr - 1.0 / (d * d))
    return min(max(p, 0.0), d * d / (d * d - 1.0))


def dephase() -> List[np.ndarray]:
    """Mid-circuit Z-basis measurement with the outcome discarded: complete dephasing."""
    return [np.diag([1.0, 0.0]).astype(np.complex128), np.diag([0.0, 1.0]).astype(np.complex128)]


def reset() -> List[np.ndarray]:
    """Reset to |0> (Sec. 3, measurement and reset as operations of their own): the Kraus set
    {|0><0|, |0><1|}, i.e. a Z measurement whose outcome is discarded followed by a flip to
    |0> where 1 was read.  On qubit q it maps rho to Tr_q(rho) (x) |0><0|_q; trace preserving."""
    return [np.array([[1, 0], [0, 0]], dtype=np.complex128), np.array([[0, 1], [0, 0]], dtype=np.complex128)]


# --------------------------------------------------------------------------------------
# Device calibration and noise injection into basis circuits (Sec. 3.5, Sec. 4)
# --------------------------------------------------------------------------------------


@dataclasses.dataclass
class Device:
    """Calibration of a synthetic device: per-qubit T1, T2 (us), excited-state population,
    readout errors P(0|1) = p01 and P(1|0) = p10, 1q gate time (us) and error; per-coupler CX
    time and error.  Couplers are directed (control, target) pairs."""

    n: int
    t1: np.ndarray
    t2: np.ndarray
    excited: np.ndarray
    p01: np.ndarray
    p10: np.ndarray
    t_1q: float
    err_1q: np.ndarray
    couplers: List[Tuple[int, int]]
    t_cx: dict
    err_cx: dict


def synthetic_device(n: int, seed: int = 7, line: bool = True) -> Device:
    """Seeded calibration in the ranges of current superconducting devices: T1 ~ U[50, 150],
    T2 ~ U[0.5, 1.5] T1 capped at 2 T1, SX/X time 0.035 us with error ~ U[1e-4, 5e-4], CX
    time ~ U[0.25, 0.5] us with error ~ U[5e-3, 1.5e-2], readout p01 ~ U[1e-2, 4e-2] (relaxation
    during readout makes it the larger) and p10 ~ U[5e-3, 2e-2]; couplers on a line (both
    directions) or all-to-all."""
    rng = np.random.default_rng(seed)
    t1 = rng.uniform(50.0, 150.0, n)
    t2 = np.minimum(rng.uniform(0.5, 1.5, n) * t1, 2.0 * t1)
    excited = rng.uniform(0.0, 0.02, n)
    p01 = rng.uniform(1e-2, 4e-2, n)
    p10 = rng.uniform(5e-3, 2e-2, n)
    err_1q = rng.uniform(1e-4, 5e-4, n)
    if line:
        couplers = [(a, a + 1) for a in range(n - 1)] + [(a + 1, a) for a in range(n - 1)]
    else:
        couplers = [(a, b) for a in range(n) for b in range(n) if a != b]
    t_cx = {c: float(rng.uniform(0.25, 0.5)) for c in couplers}
    err_cx = {c: float(rng.uniform(5e-3, 1.5e-2)) for c in couplers}
    return Device(n, t1, t2, excited, p01, p10, 0.035, err_1q, couplers, t_cx, err_cx)


def sx() -> np.ndarray:
    """sqrt(X) = [[1 + i, 1 - i], [1 - i, 1 + i]] / 2."""
    return np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128) / 2.0


def device_gate_noise(dev: Device, gate: str, qubits: Sequence[int]) -> List[np.ndarray]:
    """Noise channel that follows a basis gate on the device (Qiskit-Aer's device model):
    thermal relaxation of every touched qubit for the gate time, then depolarizing with the
    parameter that makes the total average gate infidelity the reported gate error.  RZ is
    virtual (no noise, empty list)."""
    if gate == "rz":
        return []
    if gate in ("sx", "x", "id"):
        q = qubits[0]
        relax = thermal_relaxation_general(dev.t1[q], dev.t2[q], dev.t_1q, dev.excited[q])
        p = depolarizing_for_gate_error(float(dev.err_1q[q]), relax)
        return kraus_canonical(kraus_compose(relax, depolarizing(p, 1)) if p > 0 else relax)
    if gate == "cx":
        c, t = qubits
        tg = dev.t_cx[(c, t)]
        rc = thermal_relaxation_general(dev.t1[c], dev.t2[c], tg, dev.excited[c])
        rt = thermal_relaxation_general(dev.t1[t], dev.t2[t], tg, dev.excited[t])
        relax = kraus_tensor(rc, rt)
        p = depolarizing_for_gate_error(dev.err_cx[(c, t)], relax)
        return kraus_canonical(kraus_compose(relax, depolarizing(p, 2)) if p > 0 else relax)
    raise ValueError(gate)


def noisy_basis_circuit(dev: Device, gates: Sequence[Tuple[str, Tuple[int, ...], float]]) -> List[Op]:
    """Inject the device's noise after every basis gate.  gates: (name, qubits, angle) with
    name in {"rz", "sx", "x", "id", "cx"} (the angle is used by rz only); CX must be on a
    coupler of the device."""
    ops: List[Op] = []
    for name, qs, ang in gates:
        if name == "rz":
            ops.append(gate(rz(ang), qs, "rz"))
        elif name == "sx":
            ops.append(gate(sx(), qs, "sx"))
        elif name == "x":
            ops.append(gate(PX, qs, "x"))
        elif name == "id":
            ops.append(gate(I2, qs, "id"))
        elif name == "cx":
            if tuple(qs) not in dev.t_cx:
                raise ValueError("CX %r is not a coupler of the device" % (tuple(qs),))
            ops.append(gate(cx(), qs, "cx"))
        else:
            raise ValueError(name)
        noise = device_gate_noise(dev, name, qs)
        if noise:
            ops.append(channel(noise, qs, "noise_" + name))
    return ops


def u3_to_basis(q: int, theta: float, phi: float, lam: float) -> List[Tuple[str, Tuple[int, ...], float]]:
    """U3(theta, phi, lambda) = RZ(phi + pi) SX RZ(theta + pi) SX RZ(lambda) up to global phase."""
    return [("rz", (q,), lam), ("sx", (q,), 0.0), ("rz", (q,), theta + math.pi), ("sx", (q,), 0.0),
            ("rz", (q,), phi + math.pi)]


def measure_with_readout_error(p01: float, p10: float) -> List[np.ndarray]:
    """Z-basis measurement whose outcome is kept in the qubit (deferred-measurement form) and
    misread with P(0|1) = p01, P(1|0) = p10: coherences vanish and the populations pass
    through the confusion matrix [[1 - p10, p01], [p10, 1 - p01]].  Four Kraus operators
    sqrt(P(y|x)) |y><x|."""
    if not (0.0 <= p01 <= 1.0 and 0.0 <= p10 <= 1.0):
        raise ValueError("readout error out of range")
    out = []
    for x in range(2):
        for y in range(2):
            w = (p10 if y else 1.0 - p10) if x == 0 else (1.0 - p01 if y else p01)
            if w > 0.0:
                K = np.zeros((2, 2), dtype=np.complex128)
                K[y, x] = math.sqrt(w)
                out.append(K)
    return out


def with_gate_errors(dev: Device, err_1q: float, err_cx: float) -> Device:
    """The same device with every 1q gate error set to err_1q and every CX error to err_cx
    (the 'turned-up' noise of the teleportation case study, Sec. 5)."""
    return dataclasses.replace(dev, err_1q=np.full(dev.n, float(err_1q)),
                               err_cx={k: float(err_cx) for k in dev.err_cx})


def teleport_device_circuit(dev: Device, a: int, b: int, c: int, u3_in: Tuple[float, float, float] = None,
                            readout: bool = True) -> List[Op]:
    """Teleportation of qubit a onto c through the Bell pair (b, c), transpiled to the device's
    basis {RZ, SX, CX} with the device noise after every basis gate (Sec. 5, case study 1):
    [U3(a)] H(b) CX(b,c) CX(a,b) H(a), measurement of a and b (kept in the qubits, misread
    with the device's readout errors when `readout`), then the corrections CX(b,c) and
    CZ(a,c) = H(c) CX(a,c) H(c).  H = RZ(pi/2) SX RZ(pi/2) up to a global phase.  Needs the
    couplers (b,c), (a,b) and (a,c)."""
    def h(q):
        return [("rz", (q,), math.pi / 2), ("sx", (q,), 0.0), ("rz", (q,), math.pi / 2)]

    ops: List[Op] = []
    pre = [] if u3_in is None else u3_to_basis(a, *u3_in)
    ops += noisy_basis_circuit(dev, pre + h(b) + [("cx", (b, c), 0.0), ("cx", (a, b), 0.0)] + h(a))
    for q in (a, b):
        p01, p10 = (float(dev.p01[q]), float(dev.p10[q])) if readout else (0.0, 0.0)
        ops.append(channel(measure_with_readout_error(p01, p10), (q,), "meas"))
    ops += noisy_basis_circuit(dev, [("cx", (b, c), 0.0)] + h(c) + [("cx", (a, c), 0.0)] + h(c))
    return ops


def device_random_circuit(dev: Device, layers: int, seed: int) -> List[Op]:
    """Random U3 layers (decomposed into RZ/SX) and CX on random disjoint couplers, with the
    device's noise after every basis gate."""
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(dev.n):
            th, ph, la = rng.uniform(0.0, 2 * math.pi, size=3)
            gates += u3_to_basis(q, th, ph, la)
        used = set()
        for idx in rng.permutation(len(dev.couplers)):
            c, t = dev.couplers[int(idx)]
            if c not in used and t not in used:
                gates.append(("cx", (c, t), 0.0))
                used.update((c, t))
    return noisy_basis_circuit(dev, gates)


# --------------------------------------------------------------------------------------
# Circuit generators (seeded, PCG64)
# --------------------------------------------------------------------------------------


def _pairing(rng: np.random.Generator, n: int) -> List[Tuple[int, int]]:
    perm = rng.permutation(n)
    return [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]


def _rand_u3(rng: np.random.Generator) -> np.ndarray:
    th, ph, la = rng.uniform(0.0, 2 * math.pi, size=3)
    return u3(th, ph, la)


def random_u3_cx(n: int, layers: int, seed: int, p1: float, p2: float,
                 gamma: float | None = None) -> List[Op]:
    """Layers of U3 on every qubit (+1q noise) then CX on a random disjoint pairing (+2q dep).

    Each 1q gate is followed by depolarizing(p1) and, if ``gamma`` is given, amplitude
    damping(gamma); each CX (control = first of the pair) by 2q depolarizing(p2).
    """
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    dep1 = depolarizing(p1, 1) if p1 > 0 else None
    dep2 = depolarizing(p2, 2) if p2 > 0 else None
    ad = amplitude_damping(gamma) if gamma else None
    for _ in range(layers):
        for q in range(n):
            ops.append(gate(_rand_u3(rng), (q,), "u3"))
            if dep1 is not None:
                ops.append(channel(dep1, (q,), "dep1"))
            if ad is not None:
                ops.append(channel(ad, (q,), "ad"))
        for c, t in _pairing(rng, n):
            ops.append(gate(cx(), (c, t), "cx"))
            if dep2 is not None:
                ops.append(channel(dep2, (c, t), "dep2"))
    return ops


def random_u3_cx_reset(n: int, layers: int, seed: int, p1: float, p2: float,
                       resets_per_layer: int = 1) -> List[Op]:
    """:func:`random_u3_cx` with mid-circuit resets (ancilla reuse): after each layer's CX
    gates, ``resets_per_layer`` distinct random qubits are reset to |0> (:func:`reset`)."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    rst = reset()
    for layer in range(layers):
        ops.extend(random_u3_cx(n, 1, int(rng.integers(0, 2 ** 31)), p1, p2))
        for q in rng.choice(n, size=min(resets_per_layer, n), replace=False):
            ops.append(channel(rst, (int(q),), "reset"))
    return ops


def config1(layers: int = 20, seed: int = 1, n: int = 8) -> Tuple[int, List[Op]]:
    """8-qubit random U3/CX circuit, depth 20, dep 1e-3 + AD 5e-4 per 1q gate, dep2 1e-2."""
    return n, random_u3_cx(n, layers, seed, 1e-3, 1e-2, gamma=5e-4)


def brickwork_cz(n: int, layers: int, seed: int, p1: float, p2: float, lam: float) -> List[Op]:
    """U3 on every qubit (+dep1 +PD) then CZ on even/odd nearest-neighbour bonds (+dep2 +PD)."""
    rng = np.random.default_rng(seed)
    dep1, dep2, pd = depolarizing(p1, 1), depolarizing(p2, 2), phase_damping(lam)
    ops: List[Op] = []
    for layer in range(layers):
        for q in range(n):
            ops.append(gate(_rand_u3(rng), (q,), "u3"))
            ops.append(channel(dep1, (q,), "dep1"))
            ops.append(channel(pd, (q,), "pd"))
        for a in range(layer % 2, n - 1, 2):
            ops.append(gate(cz(), (a, a + 1), "cz"))
            ops.append(channel(dep2, (a, a + 1), "dep2"))
            ops.append(channel(pd, (a,), "pd"))
            ops.append(channel(pd, (a + 1,), "pd"))
    return ops


def config2(layers: int = 200, seed: int = 2, n: int = 14) -> Tuple[int, List[Op]]:
    return n, brickwork_cz(n, layers, seed, 1e-3, 1e-2, 1e-3)


def ising_trotter(n: int, steps: int, seed: int, J: float = 1.0, dt: float = 0.05,
                  t1: float = 100.0, t2: float = 80.0, tg: float = 0.05,
                  noisy: bool = True) -> Tuple[List[Op], np.ndarray]:
    """Open-chain TFIM H = J sum Z_i Z_{i+1} + sum h_i X_i, first-order Trotter.

    Each step: RZZ(2 J dt) on every bond then RX(2 h_i dt) on every qubit; h_i ~ U[0.5,1.5]
    drawn once.  Thermal relaxation (T1, T2, gate time tg) follows every gate on each
    qubit it touches.  Returns (ops, h).
    """
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.5, 1.5, size=n)
    tr = thermal_relaxation(t1, t2, tg) if noisy else None
    ops: List[Op] = []
    for _ in range(steps):
        for a in range(n - 1):
            ops.append(gate(rzz(2 * J * dt), (a, a + 1), "rzz"))
            if tr is not None:
                ops.append(channel(tr, (a,), "tr"))
                ops.append(channel(tr, (a + 1,), "tr"))
        for q in range(n):
            ops.append(gate(rx(2 * h[q] * dt), (q,), "rx"))
            if tr is not None:
                ops.append(channel(tr, (q,), "tr"))
    return ops, h


def config3(steps: int = 50, seed: int = 3, n: int = 15) -> Tuple[int, List[Op]]:
    ops, _ = ising_trotter(n, steps, seed)
    return n, ops


def config4(layers: int = 100, seed: int = 4, n: int = 16) -> Tuple[int, List[Op]]:
    return n, random_u3_cx(n, layers, seed, 1e-3, 1e-2)


def teleport_block(a: int, b: int, c: int, U_in: np.ndarray, p1: float, p2: float) -> List[Op]:
    """Teleport qubit a's state (prepared by U_in) onto c through the Bell pair (b, c).

    H(b), CX(b,c); CX(a,b), H(a); Z-measurements of a and b modelled as dephasing;
    corrections CX(b,c), CZ(a,c) (deferred-measurement form).  1q gates are followed by
    depolarizing(p1), 2q gates by 2q depolarizing(p2) when the rates are positive.
    """
    d1 = depolarizing(p1, 1) if p1 > 0 else None
    d2 = depolarizing(p2, 2) if p2 > 0 else None
    ops: List[Op] = []

    def g1(U, q, lab):
        ops.append(gate(U, (q,), lab))
        if d1 is not None:
            ops.append(channel(d1, (q,), "dep1"))

    def g2(U, q0, q1, lab):
        ops.append(gate(U, (q0, q1), lab))
        if d2 is not None:
            ops.append(channel(d2, (q0, q1), "dep2"))

    g1(U_in, a, "u3")
    g1(hadamard(), b, "h")
    g2(cx(), b, c, "cx")
    g2(cx(), a, b, "cx")
    g1(hadamard(), a, "h")
    ops.append(channel(dephase(), (a,), "meas"))
    ops.append(channel(dephase(), (b,), "meas"))
    g2(cx(), b, c, "cx")
    g2(cz(), a, c, "cz")
    return ops


def teleport_layers(n: int, layers: int, seed: int, p1: float, p2: float) -> List[Op]:
    """Layers of teleport blocks on a random disjoint set of qubit triples."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for _ in range(layers):
        perm = rng.permutation(n)
        for i in range(n // 3):
            a, b, c = (int(x) for x in perm[3 * i:3 * i + 3])
            ops.extend(teleport_block(a, b, c, _rand_u3(rng), p1, p2))
    return ops


# --------------------------------------------------------------------------------------
# Nested entanglement purification (the distillation case study, Sec. 5; the protocol of
# Deutsch et al. 1996)
# --------------------------------------------------------------------------------------


def agree_projector() -> List[np.ndarray]:
    """Post-selection on equal Z outcomes of a qubit pair: the single Kraus operator
    |00><00| + |11><11|.  It is not trace preserving: after it, the trace of the state is the
    probability that the two measurements agreed."""
    return [np.diag([1.0, 0.0, 0.0, 1.0]).astype(np.complex128)]


def werner_pair(a: int, b: int, fidelity: float) -> List[Op]:
    """The Bell pair |Phi+> on (a, b) degraded to a Werner state of the given fidelity with
    |Phi+>: H(a), CX(a, b), then one-qubit depolarizing p = 4 (1 - F) / 3 on b (which keeps
    |Phi+> with weight 1 - 3p/4 and gives each other Bell state p/4)."""
    if not 0.25 <= fidelity <= 1.0:
        raise ValueError("Werner fidelity must lie in [1/4, 1]")
    ops = [gate(hadamard(), (a,), "h"), gate(cx(), (a, b), "cx")]
    p = 4.0 * (1.0 - fidelity) / 3.0
    if p > 0:
        ops.append(channel(depolarizing(p, 1), (b,), "werner"))
    return ops


def purify_step(control: Tuple[int, int], target: Tuple[int, int], cx_error: float) -> List[Op]:
    """One purification step on two pairs, each given as (Alice's qubit, Bob's qubit):
    Rx(pi/2) on Alice's qubits and Rx(-pi/2) on Bob's, a CX from the control pair to the
    target pair on each side (each followed by two-qubit depolarizing cx_error when it is
    positive), then the target pair is measured in Z and kept only when both outcomes agree
    (agree_projector)."""
    (ac, bc), (at, bt) = control, target
    ops: List[Op] = []
    for q in (ac, at):
        ops.append(gate(rx(math.pi / 2), (q,), "rx"))
    for q in (bc, bt):
        ops.append(gate(rx(-math.pi / 2), (q,), "rx"))
    for c_, t_ in ((ac, at), (bc, bt)):
        ops.append(gate(cx(), (c_, t_), "cx"))
        if cx_error > 0:
            ops.append(channel(depolarizing(cx_error, 2), (c_, t_), "dep2"))
    ops.append(channel(agree_projector(), (at, bt), "agree"))
    return ops


def nested_purification(rounds: int, fidelity: float, cx_error: float) -> Tuple[int, List[Op]]:
    """2^rounds Werner pairs of the given fidelity purified in `rounds` nested rounds down to
    one pair on qubits (0, 1).  Pair i sits on qubits (2i, 2i + 1) (Alice, Bob).  Round r
    (from 1) purifies pair i (control) with pair i + 2^(r-1) (target) for every i that is a
    multiple of 2^r.  The trace of the final state is the probability that every step
    succeeded, and the kept pair's fidelity is <Phi+| rho_01 |Phi+> divided by that trace."""
    if rounds < 1:
        raise ValueError("at least one round")
    npairs = 1 << rounds
    ops: List[Op] = []
    for i in range(npairs):
        ops.extend(werner_pair(2 * i, 2 * i + 1, fidelity))
    for r in range(1, rounds + 1):
        half = 1 << (r - 1)
        for i in range(0, npairs, 1 << r):
            j = i + half
            ops.extend(purify_step((2 * i, 2 * i + 1), (2 * j, 2 * j + 1), cx_error))
    return 2 * npairs, ops


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    kind: str
    depth: int
    p1: float
    ops: List[Op]


def config5(num_requests: int = 5000, rate_hz: float = 200.0, seed: int = 5,
            n_range: Tuple[int, int] = (4, 12), depth_range: Tuple[int, int] = (20, 200)
            ) -> List[Request]:
    """Serving stream: Poisson arrivals; n ~ U{4..12}; depth ~ U{20..200}; mixed types.

    Types: random U3/CX (depth = layers), Ising Trotter (depth = Trotter steps) and
    teleport blocks (depth = layers of triples; n >= 3).  p1 ~ U[1e-4, 1e-2], p2 = 10 p1.
    Circuits are generated lazily by :func:`request_ops` from the per-request seed.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=num_requests)
    t = np.cumsum(gaps)
    out = []
    kinds = ("u3cx", "ising", "teleport")
    for i in range(num_requests):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        kind = kinds[int(rng.integers(0, 3))]
        p1 = float(rng.uniform(1e-4, 1e-2))
        out.append(Request(i, float(t[i]), n, kind, depth, p1, []))
    return out


# --------------------------------------------------------------------------------------
# Pooled array form (for large request streams): one matrix pool per circuit plus, per
# operation, its width j, qubits (padded to 3), Kraus count m and offset into the pool
# (in doubles).  Repeated channels point at one copy.
# --------------------------------------------------------------------------------------


@dataclasses.dataclass
class CircuitArrays:
    n: int
    j: np.ndarray       # int32 [count]
    q: np.ndarray       # int32 [count, 3]
    m: np.ndarray       # int32 [count]
    koff: np.ndarray    # int64 [count]
    pool: np.ndarray    # float64, interleaved complex matrices
    labels: List[str]

    @property
    def count(self) -> int:
        return int(self.j.size)


class _PoolBuilder:
    def __init__(self):
        self.chunks: List[np.ndarray] = []
        self.size = 0

    def add(self, mats: np.ndarray) -> int:
        """Append matrices (complex, any leading shape); returns their offset in doubles."""
        a = np.ascontiguousarray(mats, dtype=np.complex128).view(np.float64).reshape(-1)
        off = self.size
        self.chunks.append(a)
        self.size += a.size
        return off

    def pool(self) -> np.ndarray:
        return np.concatenate(self.chunks) if self.chunks else np.zeros(0)


def u3_batch(theta: np.ndarray, phi: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """U3 for arrays of angles: shape (..., 2, 2)."""
    c, s_ = np.cos(theta / 2), np.sin(theta / 2)
    out = np.empty(theta.shape + (2, 2), dtype=np.complex128)
    out[..., 0, 0] = c
    out[..., 0, 1] = -np.exp(1j * lam) * s_
    out[..., 1, 0] = np.exp(1j * phi) * s_
    out[..., 1, 1] = np.exp(1j * (phi + lam)) * c
    return out


class _OpRecorder:
    def __init__(self, n):
        self.n = n
        self.j, self.q, self.m, self.koff, self.labels = [], [], [], [], []

    def op(self, qubits, m, koff, label):
        self.j.append(len(qubits))
        self.q.append(tuple(qubits) + (0,) * (3 - len(qubits)))
        self.m.append(m)
        self.koff.append(koff)
        self.labels.append(label)

    def finish(self, pb: _PoolBuilder) -> CircuitArrays:
        return CircuitArrays(self.n, np.asarray(self.j, dtype=np.int32),
                             np.asarray(self.q, dtype=np.int32).reshape(-1, 3),
                             np.asarray(self.m, dtype=np.int32), np.asarray(self.koff, dtype=np.int64),
                             pb.pool(), self.labels)


def request_arrays(req: Request, seed_base: int = 1000) -> CircuitArrays:
    """The request's circuit in pooled array form (the definition of its operations).

    Types: "u3cx" (layers of U3 + dep(p1) on every qubit, CX on a random disjoint pairing +
    dep2(p2)), "ising" (Trotter steps as in :func:`ising_trotter`, thermal relaxation with
    T1 = T2 = 0.05 / p1 and gate time 0.05 after every gate), "teleport" (layers of teleport
    blocks on a random disjoint set of triples, as in :func:`teleport_block`).
    """
    rng = np.random.default_rng(seed_base + req.rid)
    n = req.n
    p1, p2 = req.p1, min(10 * req.p1, 0.5)
    pb, rec = _PoolBuilder(), _OpRecorder(n)
    two_pi = 2 * math.pi
    if req.kind == "u3cx":
        d1 = pb.add(np.stack(depolarizing(p1, 1)))
        d2 = pb.add(np.stack(depolarizing(p2, 2)))
        cxo = pb.add(cx())
        for _ in range(req.depth):
            ang = rng.uniform(0.0, two_pi, size=(n, 3))
            uo = pb.add(u3_batch(ang[:, 0], ang[:, 1], ang[:, 2]))
            for qq in range(n):
                rec.op((qq,), 1, uo + 8 * qq, "u3")
                rec.op((qq,), 4, d1, "dep1")
            perm = rng.permutation(n)
            for i in range(n // 2):
                c, t = int(perm[2 * i]), int(perm[2 * i + 1])
                rec.op((c, t), 1, cxo, "cx")
                rec.op((c, t), 16, d2, "dep2")
    elif req.kind == "ising":
        dt, J = 0.05, 1.0
        h = rng.uniform(0.5, 1.5, size=n)
        t1 = 0.05 / p1
        tr = thermal_relaxation(t1, t1, 0.05)
        tro = pb.add(np.stack(tr))
        rzo = pb.add(rzz(2 * J * dt))
        rxo = pb.add(np.stack([rx(2 * h[qq] * dt) for qq in range(n)]))
        for _ in range(req.depth):
            for a in range(n - 1):
                rec.op((a, a + 1), 1, rzo, "rzz")
                rec.op((a,), len(tr), tro, "tr")
                rec.op((a + 1,), len(tr), tro, "tr")
            for qq in range(n):
                rec.op((qq,), 1, rxo + 8 * qq, "rx")
                rec.op((qq,), len(tr), tro, "tr")
    elif req.kind == "teleport":
        d1 = pb.add(np.stack(depolarizing(p1, 1)))
        d2 = pb.add(np.stack(depolarizing(p2, 2)))
        ho, cxo, czo = pb.add(hadamard()), pb.add(cx()), pb.add(cz())
        meo = pb.add(np.stack(dephase()))
        for _ in range(req.depth):
            perm = rng.permutation(n)
            ang = rng.uniform(0.0, two_pi, size=(n // 3, 3))
            uo = pb.add(u3_batch(ang[:, 0], ang[:, 1], ang[:, 2]))
            for i in range(n // 3):
                a, b, c = (int(x) for x in perm[3 * i:3 * i + 3])
                rec.op((a,), 1, uo + 8 * i, "u3")
                rec.op((a,), 4, d1, "dep1")
                rec.op((b,), 1, ho, "h")
                rec.op((b,), 4, d1, "dep1")
                rec.op((b, c), 1, cxo, "cx")
                rec.op((b, c), 16, d2, "dep2")
                rec.op((a, b), 1, cxo, "cx")
                rec.op((a, b), 16, d2, "dep2")
                rec.op((a,), 1, ho, "h")
                rec.op((a,), 4, d1, "dep1")
                rec.op((a,), 2, meo, "meas")
                rec.op((b,), 2, meo, "meas")
                rec.op((b, c), 1, cxo, "cx")
                rec.op((b, c), 16, d2, "dep2")
                rec.op((a, c), 1, czo, "cz")
                rec.op((a, c), 16, d2, "dep2")
    else:
        raise ValueError(req.kind)
    return rec.finish(pb)


def arrays_to_ops(ca: CircuitArrays) -> List[Op]:
    """Expand the pooled form into explicit :class:`Op` records."""
    ops = []
    for i in range(ca.count):
        j, m, off = int(ca.j[i]), int(ca.m[i]), int(ca.koff[i])
        d = 1 << j
        mats = ca.pool[off:off + m * d * d * 2].view(np.complex128).reshape(m, d, d).copy()
        qs = tuple(int(x) for x in ca.q[i, :j])
        ops.append(Op("gate" if m == 1 else "kraus", qs, mats, ca.labels[i]))
    return ops


def ops_to_arrays(n: int, ops: Sequence[Op]) -> CircuitArrays:
    """Pooled form of an explicit operation list (matrices deduplicated by identity)."""
    pb, rec = _PoolBuilder(), _OpRecorder(n)
    seen = {}
    for op in ops:
        key = id(op.mats)
        if key not in seen:
            seen[key] = pb.add(op.mats)
        rec.op(op.qubits, op.mats.shape[0], seen[key], op.label)
    return rec.finish(pb)


def request_ops(req: Request, seed_base: int = 1000) -> List[Op]:
    return arrays_to_ops(request_arrays(req, seed_base))


def zz_paulis(n: int) -> List[str]:
    """Pauli strings <Z_i Z_{i+1}> for i = 0..n-2 (character t acts on qubit t)."""
    out = []
    for i in range(n - 1):
        s = ["I"] * n
        s[i] = s[i + 1] = "Z"
        out.append("".join(s))
    return out


def z_paulis(n: int) -> List[str]:
    out = []
    for i in range(n):
        s = ["I"] * n
        s[i] = "Z"
        out.append("".join(s))
    return out


# --------------------------------------------------------------------------------------
# Counter-based input generator (SplitMix64, Steele, Lea & Flood, OOPSLA 2014)
# --------------------------------------------------------------------------------------

_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied to counters ``x`` (uint64 array): returns uint64."""
    z = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(_M64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def hash_fill_values(seed: int, index: np.ndarray) -> np.ndarray:
    """Pseudo-random complex value at vec index ``index`` for the seeded fill.

    re = u(2*(seed*2^40 + index)), im = u(2*(seed*2^40 + index) + 1), u(c) = the top 53 bits
    of splitmix64(c) as a double in [-0.5, 0.5).  The device fill implements the same
    definition independently.
    """
    with np.errstate(over="ignore"):
        idx = np.asarray(index, dtype=np.uint64)
        base = (np.uint64(seed) << np.uint64(40)) + idx
        c0 = base * np.uint64(2)
        c1 = c0 + np.uint64(1)
        r0 = (splitmix64(c0) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 0.5
        r1 = (splitmix64(c1) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 0.5
    return r0 + 1j * r1
