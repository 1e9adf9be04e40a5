"""Continuous-batching server on the GPU: results against the oracle, identical alone and in a
mix, admission within the device-memory budget, rejection of requests that can never fit."""
import sys

import numpy as np
import pytest

from paper_2404_13184_amd import tanq as T
from paper_2404_13184_amd import workloads as W

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def small_requests(count, seed, n_range=(4, 7), depth_range=(2, 6)):
    reqs = W.config5(num_requests=count, seed=seed, n_range=n_range, depth_range=depth_range)
    return [(r.n, W.request_ops(r), r) for r in reqs]


@pytest.mark.parametrize("prec,width", [("f64", 2), ("f64", 3), ("f32", 2), ("f32", 3)])
def test_server_results_match_oracle(oracle_mod, prec, width):
    reqs = small_requests(12, seed=50 + width)
    say("server parity %s width %d" % (prec, width))
    with T.Server(256 * MiB, max_slots=8, prec=prec, width=width, steps_per_launch=4) as srv:
        tickets = []
        for n, ops, _ in reqs:
            tickets.append(srv.submit(n, ops, probs=True, paulis=W.zz_paulis(n)[:2] + W.z_paulis(n)[:1]))
        for (n, ops, _), t in zip(reqs, tickets):
            res = srv.wait(t)
            assert res["status"] == T.TANQ_OK
            want = oracle_mod.run(n, ops)
            p, tr = oracle_mod.diag(want)
            tol = 1e-12 if prec == "f64" else 1e-5
            assert abs(res["trace"] - tr) <= tol
            assert np.abs(res["probs"] - p / tr).max() <= tol
            strings = W.zz_paulis(n)[:2] + W.z_paulis(n)[:1]
            for s, v in zip(strings, res["pauli"]):
                assert abs(v - oracle_mod.expect_pauli(want, s).real) <= (1e-12 if prec == "f64" else 1e-5)
            srv.release(t)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["bytes_in_use"] == 0


@pytest.mark.parametrize("use_graphs,cohort", [(True, 0), (False, 0), (True, 1 * MiB)])
def test_alone_equals_in_mix(use_graphs, cohort):
    reqs = small_requests(24, seed=77, n_range=(4, 9), depth_range=(3, 12))
    target = reqs[5]
    say("alone vs mix, graphs=%s cohort=%d" % (use_graphs, cohort))
    with T.Server(512 * MiB, max_slots=16, prec="f32", width=2, steps_per_launch=8, use_graphs=use_graphs) as srv:
        t = srv.submit(target[0], target[1], probs=True, paulis=W.z_paulis(target[0]))
        alone = srv.wait(t)
    with T.Server(512 * MiB, max_slots=16, prec="f32", width=2, steps_per_launch=8, use_graphs=use_graphs,
                  cohort_bytes=cohort) as srv:
        tickets = [srv.submit(n, ops, probs=True, paulis=W.z_paulis(n)) for n, ops, _ in reqs]
        mixed = [srv.wait(t) for t in tickets]
    got = mixed[5]
    assert got["status"] == T.TANQ_OK and alone["status"] == T.TANQ_OK
    assert np.array_equal(got["probs"], alone["probs"])  # bitwise
    assert np.array_equal(got["pauli"], alone["pauli"])
    assert got["trace"] == alone["trace"]


def test_graph_and_direct_launches_agree():
    reqs = small_requests(10, seed=31, n_range=(5, 8), depth_range=(4, 8))
    say("graph vs direct")
    outs = []
    for g in (True, False):
        with T.Server(256 * MiB, max_slots=4, prec="f32", width=3, steps_per_launch=3, use_graphs=g) as srv:
            tickets = [srv.submit(n, ops) for n, ops, _ in reqs]
            outs.append([srv.wait(t)["probs"] for t in tickets])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_admission_respects_budget():
    # each 9-qubit FP32 request holds 2 MiB of state plus its operands; a 64 MiB budget admits a few
    reqs = small_requests(40, seed=8, n_range=(9, 9), depth_range=(5, 10))
    say("admission budget")
    with T.Server(64 * MiB, max_slots=64, prec="f32", width=2, steps_per_launch=4) as srv:
        tickets = [srv.submit(n, ops) for n, ops, _ in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(r["status"] == T.TANQ_OK for r in res)
    assert st["peak_bytes"] <= st["budget_bytes"]
    assert st["completed"] == len(reqs)
    assert all(abs(r["trace"] - 1.0) <= 1e-5 for r in res)
    # FIFO admission: admit times do not decrease with submission order
    admits = [r["t_admit"] for r in res]
    assert all(b >= a for a, b in zip(admits, admits[1:]))


def test_rejects_requests_that_never_fit():
    with T.Server(64 * MiB, max_slots=4, prec="f64", width=2) as srv:
        n = 12  # FP64 state alone is 256 MiB
        with pytest.raises(T.TanqError) as e:
            srv.submit(n, W.random_u3_cx(n, 1, seed=1, p1=1e-3, p2=1e-2))
        assert e.value.code == T.TANQ_E_OOM
        with pytest.raises(T.TanqError) as e:
            srv.submit(1, [W.gate(W.hadamard(), (0,))])  # narrower than the fusion width
        assert e.value.code == T.TANQ_E_ARG
        assert srv.stats()["rejected"] == 1


def test_arrivals_while_busy_overlap():
    """Requests submitted while others are resident join the running batch."""
    # a first wave long enough (12 qubits, 100+ layers: hundreds of ms on the GPU) that the
    # second wave's submissions (host-side planning of small circuits) land while it runs
    heavy = small_requests(4, seed=12, n_range=(12, 12), depth_range=(100, 120))
    light = small_requests(8, seed=13, n_range=(8, 10), depth_range=(20, 30))
    say("arrivals while busy")
    with T.Server(2048 * MiB, max_slots=16, prec="f32", width=2, steps_per_launch=4) as srv:
        first = [srv.submit(n, ops) for n, ops, _ in heavy]
        second = [srv.submit(n, ops) for n, ops, _ in light]
        res = [srv.wait(t) for t in first + second]
    assert all(r["status"] == T.TANQ_OK for r in res)
    # some request of the second wave was admitted before the last of the first wave finished
    last_first_done = max(r["t_done"] for r in res[:4])
    assert min(r["t_admit"] for r in res[4:]) < last_first_done


@pytest.mark.parametrize("cohort", [0, 1 * MiB])
def test_empty_circuit_request_completes(cohort):
    """A request with no operations finishes with the outputs of |0..0><0..0|, alone and
    between ordinary requests (it must not wait for a superoperator that never comes)."""
    reqs = small_requests(6, seed=91)
    say("empty-circuit request, cohort=%d" % cohort)
    with T.Server(256 * MiB, max_slots=8, prec="f32", width=3, steps_per_launch=4, cohort_bytes=cohort) as srv:
        t_empty = srv.submit(5, [], probs=True, paulis=["ZIIII", "XIIII"])
        tickets = [srv.submit(n, ops, probs=True) for n, ops, _ in reqs]
        t_empty2 = srv.submit(4, [], probs=True)
        for t in (t_empty, t_empty2):
            res = srv.wait(t)
            assert res["status"] == T.TANQ_OK and res["fused_applies"] == 0
            p = res["probs"]
            assert p[0] == 1.0 and np.count_nonzero(p) == 1 and res["trace"] == 1.0
        assert list(srv.wait(t_empty)["pauli"]) == [1.0, 0.0]
        for t in tickets:
            assert srv.wait(t)["status"] == T.TANQ_OK
        assert srv.stats()["completed"] == len(reqs) + 2


def test_request_size_limits():
    with T.Server(256 * MiB, max_slots=4, prec="f32", width=3) as srv:
        for n in (2, 15):  # below the fusion width, above the serving limit
            with pytest.raises(T.TanqError):
                srv.submit(n, [W.gate(W.hadamard(), (0,))])


def test_cancel_queued_and_resident_requests(oracle_mod):
    """A queued request leaves the queue; a resident one stops and frees its slot and memory;
    the others finish with correct results; a finished request keeps its result."""
    heavy = small_requests(2, seed=21, n_range=(12, 12), depth_range=(150, 180))
    light = small_requests(6, seed=22)
    say("cancel queued and resident")
    with T.Server(1024 * MiB, max_slots=1, prec="f64", width=2, steps_per_launch=4) as srv:
        t_heavy = srv.submit(heavy[0][0], heavy[0][1])  # admitted first (one slot)
        t_light = [srv.submit(n, ops, probs=True) for n, ops, _ in light]
        t_queued = srv.submit(heavy[1][0], heavy[1][1])  # behind the others in the queue
        srv.cancel(t_queued)
        srv.cancel(t_heavy)
        r_heavy = srv.wait(t_heavy)
        r_queued = srv.wait(t_queued)
        assert r_queued["status"] == T.TANQ_E_CANCELED and r_queued["probs"] is None
        assert r_queued["t_admit"] == 0.0  # never admitted
        # the heavy request may have finished before the cancel reached the scheduler; if not,
        # it is cancelled without outputs
        assert r_heavy["status"] in (T.TANQ_OK, T.TANQ_E_CANCELED)
        if r_heavy["status"] == T.TANQ_E_CANCELED:
            assert r_heavy["probs"] is None
        for (n, ops, _), t in zip(light, t_light):
            res = srv.wait(t)
            assert res["status"] == T.TANQ_OK
            want = oracle_mod.run(n, ops)
            p, tr = oracle_mod.diag(want)
            assert np.abs(res["probs"] - p / tr).max() <= 1e-12
        done = srv.wait(t_light[0])
        srv.cancel(t_light[0])  # finished: nothing changes
        assert srv.wait(t_light[0])["status"] == T.TANQ_OK and np.array_equal(srv.wait(t_light[0])["probs"], done["probs"])
        with pytest.raises(T.TanqError):
            srv.cancel(987654321)
        st = srv.stats()
        assert st["completed"] + st["dropped"] == len(light) + 2
        assert st["dropped"] >= 1 and st["bytes_in_use"] == 0 and st["active"] == 0


def test_request_timeout():
    """With a timeout far below a request's run time, requests time out (queued or resident)
    and free their memory; with a generous one, every request finishes."""
    reqs = small_requests(6, seed=31, n_range=(11, 12), depth_range=(100, 150))
    say("request timeout")
    with T.Server(1024 * MiB, max_slots=2, prec="f32", width=3, steps_per_launch=4,
                  request_timeout_s=0.002) as srv:
        tickets = [srv.submit(n, ops) for n, ops, _ in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(r["status"] in (T.TANQ_OK, T.TANQ_E_TIMEOUT) for r in res)
    assert sum(r["status"] == T.TANQ_E_TIMEOUT for r in res) >= len(reqs) - 2
    assert st["bytes_in_use"] == 0 and st["dropped"] == sum(r["status"] == T.TANQ_E_TIMEOUT for r in res)
    with T.Server(1024 * MiB, max_slots=2, prec="f32", width=3, steps_per_launch=4, request_timeout_s=600.0) as srv:
        res = [srv.wait(t) for t in [srv.submit(n, ops) for n, ops, _ in reqs[:3]]]
    assert all(r["status"] == T.TANQ_OK for r in res)
