"""The distillation case study (Sec. 5, case study 2: nested entanglement purification) on the
GPU.  Nested purification circuits are fused and applied by the HIP path, and the kept pair
is read back through the GPU partial trace.  At 4 and 8 qubits (one and two rounds) it is
compared with the oracle on the whole circuit.  At 16 qubits (three rounds, the 64 GiB FP64
state of the benchmark) it is compared with the step-by-step oracle and, without noise, with
the closed recurrence of the protocol.  The projector that post-selects agreeing outcomes is
not trace preserving: the state's trace is the overall success probability, which is
compared as well."""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

import purification_ref as PR

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def gpu_pair(rounds, F, e, prec, width):
    """Unnormalised 4x4 state of pair (0, 1) after the nested circuit on the GPU."""
    n, ops = W.nested_purification(rounds, F, e)
    c = T.Circuit(n, ops)
    f = c.fuse(width, prec)
    with T.DM(n, prec) as d:
        d.apply_fused(f)
        r = d.reduced((0, 1))
    f.free()
    c.free()
    return r


@pytest.mark.parametrize("prec,width", [("f64", 2), ("f64", 3), ("f32", 2)])
@pytest.mark.parametrize("rounds", [1, 2])
@pytest.mark.parametrize("F,e", [(0.7, 0.0), (0.8, 0.02), (0.9, 0.07)])
def test_small_registers_match_oracle(oracle_mod, prec, width, rounds, F, e):
    say("purification rounds=%d F=%.2f e=%.2f %s width %d" % (rounds, F, e, prec, width))
    got = gpu_pair(rounds, F, e, prec, width)
    n, ops = W.nested_purification(rounds, F, e)
    want = oracle_mod.reduced_dm(oracle_mod.run(n, ops), (0, 1))
    fg, tg = PR.fidelity_from_reduced(got)
    fw, tw = PR.fidelity_from_reduced(want)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert np.abs(got - want).max() <= tol
    assert abs(tg - tw) <= tol and abs(fg - fw) <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_three_rounds_at_16_qubits(oracle_mod, prec):
    F, e = 0.8, 0.01
    say("purification rounds=3 n=16 F=%.2f e=%.2f %s" % (F, e, prec))
    got = gpu_pair(3, F, e, prec, 2)
    want, p = PR.stepwise_pair(oracle_mod, 3, F, e)
    fg, tg = PR.fidelity_from_reduced(got)
    tol = 1e-10 if prec == "f64" else 1e-5
    assert abs(tg - p) <= tol
    assert np.abs(got / tg - want).max() <= tol
    assert abs(fg - float(np.real(PR.BELL["phi+"].conj() @ want @ PR.BELL["phi+"]))) <= tol
    assert fg > F  # three rounds at this error rate still purify


def test_three_rounds_noiseless_closed_form():
    F = 0.7
    say("purification rounds=3 n=16 noiseless f64")
    got = gpu_pair(3, F, 0.0, "f64", 2)
    w, p = PR.recurrence(3, F)
    tr = float(np.real(np.trace(got)))
    assert abs(tr - p) <= 1e-12
    assert np.abs(PR.bell_weights(got / tr) - w).max() <= 1e-10
