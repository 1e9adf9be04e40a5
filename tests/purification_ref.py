"""Reference computations for the distillation case study (Sec. 5, case study 2: nested
entanglement purification after Deutsch et al. 1996), shared by its CPU and GPU tests.

Without gate noise the protocol maps Bell-diagonal states to Bell-diagonal states by a closed
recurrence.  With weights (A, B, C, D) on (Phi+, Psi-, Psi+, Phi-) and success probability
N = (A + B)^2 + (C + D)^2, one step gives A' = (A^2 + B^2)/N, B' = 2CD/N, C' = (C^2 + D^2)/N
and D' = 2AB/N.  With noise, the pairs entering a step are independent, so the final pair of
the nested circuit is also the result of running each step on its own (a 4-qubit oracle run
on the product of two copies of the previous round's pair).  The step-by-step form reaches
register sizes the oracle cannot hold whole."""
import numpy as np

from paper_2404_13184_amd import workloads as W

_S = 1.0 / np.sqrt(2.0)
BELL = {
    "phi+": np.array([1, 0, 0, 1], dtype=np.complex128) * _S,
    "psi-": np.array([0, 1, -1, 0], dtype=np.complex128) * _S,
    "psi+": np.array([0, 1, 1, 0], dtype=np.complex128) * _S,
    "phi-": np.array([1, 0, 0, -1], dtype=np.complex128) * _S,
}
ORDER = ("phi+", "psi-", "psi+", "phi-")


def bell_weights(r2: np.ndarray) -> np.ndarray:
    """<B| r2 |B> for the four Bell states, in ORDER (r2: 4x4, qubit 0 = index bit 0)."""
    return np.array([np.real(BELL[k].conj() @ r2 @ BELL[k]) for k in ORDER])


def dejmps(w):
    """One noiseless purification step on Bell weights; returns (new weights, success prob)."""
    A, B, C, D = w
    N = (A + B) ** 2 + (C + D) ** 2
    return np.array([(A * A + B * B) / N, 2 * C * D / N, (C * C + D * D) / N, 2 * A * B / N]), N


def recurrence(rounds: int, F: float):
    """Final Bell weights and overall success probability of `rounds` nested noiseless steps
    on Werner pairs of fidelity F."""
    w = np.array([F, (1 - F) / 3, (1 - F) / 3, (1 - F) / 3])
    p = 1.0
    for _ in range(rounds):
        w, N = dejmps(w)
        p = p * p * N
    return w, p


def final_pair(oracle_mod, rounds: int, F: float, e: float):
    """(normalised state of pair (0, 1), trace) of the whole nested circuit on the oracle."""
    n, ops = W.nested_purification(rounds, F, e)
    rho = oracle_mod.run(n, ops)
    r = oracle_mod.reduced_dm(rho, (0, 1))
    tr = float(np.real(np.trace(r)))
    return r / tr, tr


def stepwise_pair(oracle_mod, rounds: int, F: float, e: float):
    """The same result step by step: each step is a 4-qubit oracle run on two independent
    copies of the previous round's pair (control on qubits 0, 1, target on 2, 3)."""
    r = oracle_mod.run(2, W.werner_pair(0, 1, F))
    p = 1.0
    step = W.purify_step((0, 1), (2, 3), e)
    for _ in range(rounds):
        rho4 = np.kron(r, r)  # target pair on the high qubits, control pair on the low ones
        out = oracle_mod.reduced_dm(oracle_mod.run(4, step, rho4), (0, 1))
        N = float(np.real(np.trace(out)))
        r = out / N
        p = p * p * N
    return r, p


def fidelity_from_reduced(r2: np.ndarray):
    """(<Phi+| r2 |Phi+> / tr r2, tr r2) for an unnormalised pair state."""
    tr = float(np.real(np.trace(r2)))
    return float(np.real(BELL["phi+"].conj() @ r2 @ BELL["phi+"])) / tr, tr
