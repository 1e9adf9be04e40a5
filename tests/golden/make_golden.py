"""Writes the oracle-computed expected values that the large GPU parity tests compare against.

Only the CPU oracle (``oracle/``) and the seeded generators (``workloads``) run here; nothing of
the HIP library is loaded.  Each output is a NumPy ``.npz`` (no pickled objects):

* ``serve_stream_n10_12.npz`` -- requests of the 5000-request serving stream (seed 5) at 10, 11
  and 12 qubits, one per (qubit count, circuit type): the lowest-depth request of each pair.
  For each request ``rid``: ``probs_<rid>`` (the 2^n outcome probabilities, renormalised by the
  trace), ``trace_<rid>`` and ``z_<rid>`` (Tr(Z_q rho) for every qubit q, not renormalised).  ``rids`` lists them.
* ``brickwork14_2layers.npz`` -- the first two layers of the 14-qubit noisy CZ brickwork
  (U3 + depolarizing 1e-3 + phase damping 1e-3 on every qubit, CZ on nearest-neighbour bonds +
  two-qubit depolarizing 1e-2 + phase damping on both qubits; seed 2): ``probs`` (all 2^14),
  ``trace``, ``zz`` (<Z_i Z_{i+1}>), and ``idx``/``val``: 4096 sampled elements of vec(rho)
  (index r + c 2^n, value rho[r, c]).

Usage (CPU, from the repository root; the 14-qubit run needs ~12 GiB of host memory and about
half an hour on 8 cores, the serving requests about an hour):

    python tests/golden/make_golden.py serve brickwork
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2404_13184_amd import workloads as W  # noqa: E402

SERVE_FILE = os.path.join(HERE, "serve_stream_n10_12.npz")
BRICK_FILE = os.path.join(HERE, "brickwork14_2layers.npz")


def serve_selection(reqs):
    """The lowest-depth request (first on ties) of each (n, type) with n in 10..12."""
    best = {}
    for r in reqs:
        if 10 <= r.n <= 12:
            k = (r.n, r.kind)
            if k not in best or r.depth < best[k].depth:
                best[k] = r
    return [best[k] for k in sorted(best)]


def make_serve():
    reqs = W.config5(num_requests=5000, seed=5)
    out = {}
    sel = serve_selection(reqs)
    for r in sel:
        t0 = time.time()
        ops = W.request_ops(r)
        rho = oracle.run(r.n, ops)
        p, tr = oracle.diag(rho)
        out["probs_%d" % r.rid] = p / tr
        out["trace_%d" % r.rid] = np.array(tr)
        out["z_%d" % r.rid] = np.array([oracle.expect_pauli(rho, s).real for s in W.z_paulis(r.n)])
        print("request %d: n=%d %s depth %d, %d ops, %.0f s" % (r.rid, r.n, r.kind, r.depth, len(ops),
                                                              time.time() - t0), flush=True)
        del rho
    out["rids"] = np.array([r.rid for r in sel], dtype=np.int64)
    np.savez_compressed(SERVE_FILE, **out)


def make_brickwork():
    n, ops = W.config2(layers=2)
    t0 = time.time()
    rho = oracle.run(n, ops)
    secs = time.time() - t0
    p, tr = oracle.diag(rho)
    zz = np.array([oracle.expect_pauli(rho, s).real for s in W.zz_paulis(n)])
    rng = np.random.default_rng(1402)
    dim = 1 << n
    r = rng.integers(0, dim, size=4096)
    c = rng.integers(0, dim, size=4096)
    c[:1024] = r[:1024]  # a quarter on the diagonal
    val = rho[r, c]
    print("brickwork n=%d, %d ops, %.0f s" % (n, len(ops), secs), flush=True)
    np.savez_compressed(BRICK_FILE, probs=p / tr, trace=np.array(tr), zz=zz,
                        idx=(r.astype(np.uint64) + c.astype(np.uint64) * np.uint64(dim)), val=val,
                        oracle_seconds=np.array(secs), oracle_threads=np.array(oracle.max_threads()))


if __name__ == "__main__":
    oracle.build(force=False)
    what = sys.argv[1:] or ["serve", "brickwork"]
    if "brickwork" in what:
        make_brickwork()
    if "serve" in what:
        make_serve()
