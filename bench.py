"""Benchmark: 16-qubit density-matrix superoperator applies/s on one MI355X.

Workload: the 16-qubit noisy random circuit (2^32-element vec(rho): 64 GiB in FP64,
32 GiB in FP32), depth 100, each layer U3 on every qubit + 1q depolarizing(1e-3), then CX
on a random disjoint pairing + 2q depolarizing(1e-2); seeded, synthetic.

One step = the whole hot path on that circuit: reset rho to |0..0><0..0|, fuse the
circuit (GPU superoperator construction + FP64 composition + packing), apply every fused
superoperator, and reduce the 2^16 probabilities in FP64.  `value` = fused superoperator
applies per second over the timed FP64 steps; FP32 is reported beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_kernel_traffic_16q.txt")
TRAFFIC_N = 16  # qubits of the state the traffic summary was taken on
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2404_13184_amd", "csrc", f) for f in ("apply.hip", "tile.hpp", "pass.hip")]
# multi-superoperator pass kernels, by precision
PASS_KERNELS = {"f64": "apply_pass_kernel<double, 12, 512>", "f32": "apply_pass_ws_kernel<float, 13, 640, 2>"}


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_name(prec, k, variant) -> str:
    t = "double" if prec == "f64" else "float"
    if variant.get("staging", 0) == 1:
        return "apply_dma_kernel<%s, %d, %d, %d>" % (t, k, variant["tile_bits"], variant["threads"])
    return "apply_tiles_kernel<%s, %d, %d, %d, true>" % (t, k, variant["tile_bits"], variant["threads"])


def measured_traffic(name: str, n: int = TRAFFIC_N):
    """HBM bytes per launch of `name` from the committed rocprofv3 counter summary (FETCH_SIZE
    and WRITE_SIZE, each scaled by what the counter reads for a copy kernel of known size), or
    None when there is no summary for it, the kernel sources changed since it was taken, or
    the state size differs from the summary's (TRAFFIC_N qubits)."""
    if n != TRAFFIC_N or not os.path.exists(TRAFFIC_FILE):
        return None
    src_hash, rows = None, {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if len(f) >= 2 and f[0] == "source_hash":
                src_hash = f[1]
            elif len(f) >= 4 and f[0] == "kernel":
                # kernel <name without spaces> <fetch bytes> <write bytes>
                rows[f[1]] = (float(f[2]), float(f[3]))
    if src_hash != kernel_source_hash():
        return None
    hit = rows.get(name.replace(" ", ""))
    return None if hit is None else hit[0] + hit[1]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--layers", type=int, default=100)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--width", type=int, default=0, help="fusion width: 0 = autotuned, 2, 3, -1 none")
    ap.add_argument("--precs", default="f64,f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=5000, help="0 skips the serving stream")
    ap.add_argument("--serve-width", type=int, default=3)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=8)
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-cohort-mib", type=float, default=0.0,
                    help="states advanced together per scheduler iteration (0 = all resident requests)")
    ap.add_argument("--plain-budget-s", type=float, default=30.0)
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="first run one device copy of this size (reads and writes it once): the "
                         "known-size kernel that scales HBM byte counters")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def run_precision(T, torch, n, ops, prec, width, steps, warmup):
    """Autotune, then time `steps` full passes of the hot path.  Returns (measurements, dm);
    the caller frees the dm."""
    stream = torch.cuda.current_stream()
    circ = T.Circuit(n, ops)
    d = T.DM(n, prec, stream)
    t0 = time.perf_counter()
    tuned_ms = d.autotune(reps=2, dense=True)  # dense data: the matrix units' real clock
    d.reset()
    variants = {k: T.tanq_variant_get(k, T._prec(prec), T.tanq_variant_for(n, k, prec))
                for k in (2, 3) if k <= n}
    log("%s autotune %.1fs: ms/apply by k %s" % (prec, time.perf_counter() - t0, tuned_ms[1:]))

    # the method's own work per fused block: 8 flops per complex multiply-add at the block's
    # true width k (the qubits its operations touch), 8 * 4^k * 4^n per apply; a one-qubit
    # block that a pass widens to two qubits still counts as k = 1
    f0 = circ.fuse(width, prec, stream)
    chosen = f0.info["max_width"]
    op_block, nblocks = circ.plan_ordered(chosen, prec)
    if nblocks != f0.count:
        raise RuntimeError("ordered plan has %d blocks, the fused list %d" % (nblocks, f0.count))
    block_qubits = [set() for _ in range(nblocks)]
    for op, b in zip(ops, op_block):
        block_qubits[b].update(op.qubits)
    block_flops = [8.0 * 4 ** len(q) * 4 ** n for q in block_qubits]
    if any(len(q) > f0.get_k(b) for b, q in enumerate(block_qubits)):
        raise RuntimeError("a fused block is narrower than the qubits of its operations")
    f0.free()

    def one_step(events=None):
        d.reset()
        f = circ.fuse(width, prec, stream)
        if events is None:
            d.apply_fused(f)
        else:
            # the launches apply_fused makes (single applies and multi-superoperator passes),
            # each bracketed by events on the library's stream
            pos = 0
            for r in f.launches():
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(stream)
                d.apply_fused(f, pos, pos + r)
                ev1.record(stream)
                events.append((f.get_k(pos) if r == 1 else "pass", r, ev0, ev1, sum(block_flops[pos:pos + r])))
                pos += r
        p, tr = d.probs(renormalize=True)
        info = f.info
        f.free()
        return info, p, tr

    # the other fusion width, for context: one whole apply_fused timed end to end
    alt_w = 3 if chosen == 2 else 2
    d.reset()
    fa = circ.fuse(alt_w, prec, stream)
    npass, nin = fa.passes()
    d.apply_fused(fa, 0, min(fa.count, 8))  # loads the kernels
    d.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.apply_fused(fa)
    torch.cuda.synchronize()
    T.tanq_sync(d.h)
    dt = time.perf_counter() - t0
    alternative = {"fusion_width": alt_w, "fused_applies": fa.count, "passes": npass, "blocks_in_passes": nin,
                   "s": round(dt, 3), "applies_per_s": round(fa.count / dt, 3),
                   "gates_per_s": round(len(ops) / dt, 1)}
    fa.free()
    log("%s fusion width %d (not chosen): %s" % (prec, alt_w, alternative))

    for w in range(warmup):
        one_step()
        log("%s warmup step %d done" % (prec, w + 1))
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for st in range(steps):
        info, p, tr = one_step(events)
        log("%s step %d done (%.1fs)" % (prec, st + 1, time.perf_counter() - t0))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_k, pass_sizes, alg_flops = {}, [], {}
    for k, r, e0, e1, fl in events:
        per_k.setdefault(k, []).append(e0.elapsed_time(e1) * 1e-3)
        alg_flops.setdefault(k, []).append(fl)
        if r >= 2:
            pass_sizes.append(r)
    circ.free()
    stream_s = time_stream(torch, d, stream)
    log("%s in-place stream over the state: %.3f ms (%.1f GB/s)" % (prec, stream_s * 1e3, d_bytes(d) / stream_s / 1e9))
    mfma_tf = T.tanq_mfma_rate(prec)
    log("%s matrix units, multiplication loop alone: %.1f TFLOP/s" % (prec, mfma_tf))
    applies = info["count"] * steps
    return {"wall_s": wall, "applies": applies, "info": info, "per_k": per_k, "trace": tr, "probs": p,
            "tuned_ms": tuned_ms[1:], "variants": variants, "alternative": alternative,
            "pass_sizes": pass_sizes, "alg_flops": alg_flops, "launches": len(events) // max(steps, 1),
            "stream_s": stream_s, "mfma_tflops": mfma_tf}, d


def d_bytes(d):
    """Algorithmic bytes of one in-place pass over the state: every element read and written."""
    return 2.0 * (4 ** d.n) * (16 if d.prec == 0 else 8)


def time_stream(torch, d, stream, reps=5):
    """Average time of the library's plain in-place streaming kernel (rho <- 1.0 * rho, which
    leaves the state unchanged) on the state buffer, HIP events on the library's stream."""
    d.scale(1.0)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        d.scale(1.0)
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return sum(ts) / len(ts)


def roofline(prec, k, n, secs):
    es = 16 if prec == "f64" else 8
    nbytes = 2.0 * (4 ** n) * es
    flops = 8.0 * (4 ** k) * (4 ** n)
    peak_f = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    t_mem = nbytes / (HBM_PEAK_GBS * 1e9)
    t_cmp = flops / (peak_f * 1e12)
    if t_mem >= t_cmp:
        ach = nbytes / secs / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel_k": k,
                "avg_launch_ms": round(secs * 1e3, 3), "algorithmic_bytes": nbytes}
    ach = flops / secs / 1e12
    # the k = 3 kernel multiplies in 3M form: three real products instead of four
    executed = 6.0 * (4 ** k) * (4 ** n) if k == 3 else flops
    return {"bound": "mfma", "achieved": round(ach, 2), "peak": peak_f, "unit": "TFLOP/s",
            "frac": round(ach / peak_f, 4), "traffic": None, "kernel_k": k,
            "avg_launch_ms": round(secs * 1e3, 3), "algorithmic_flops": flops,
            "mfma_flops_executed": executed, "mfma_frac_executed": round(executed / secs / 1e12 / peak_f, 4),
            "hbm_GBs": round(nbytes / secs / 1e9, 1)}


def roofline_pass(prec, n, secs, m_avg, alg_flops):
    """A pass reads and writes the state once and multiplies it by m_avg superoperators.

    The kernel multiplies every member, one-qubit blocks widened to two qubits included, as a
    16 x 16 complex product in 3M form: three real 16 x 16 products per 16-element group, i.e.
    6 flops per complex multiply-add, 1536 per group.  Those executed flops and the bytes set
    the floor: the bound is the resource whose ideal time at its datasheet peak is the longer,
    and `frac` is that ideal time over the measured one.  `alg_flops` is the method's own work
    per launch (8 flops per complex multiply-add of each member at its true width, 8 * 4^k
    * 4^n); its rate is reported beside as the effective throughput."""
    es = 16 if prec == "f64" else 8
    nbytes = 2.0 * (4 ** n) * es
    executed = m_avg * 6.0 * 16 * (4 ** n)
    peak_f = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    gbs = nbytes / secs / 1e9
    tfs = executed / secs / 1e12
    common = {"traffic": None, "kernel_k": "pass", "superops_per_launch": round(m_avg, 3),
              "avg_launch_ms": round(secs * 1e3, 3), "algorithmic_bytes": nbytes,
              "mfma_flops_executed": executed, "mfma_frac_executed": round(tfs / peak_f, 4),
              "algorithmic_flops": alg_flops,
              "effective_TFLOPs_algorithmic": round(alg_flops / secs / 1e12, 2),
              "effective_frac_algorithmic": round(alg_flops / secs / 1e12 / peak_f, 4),
              "hbm_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    if nbytes / (HBM_PEAK_GBS * 1e9) >= executed / (peak_f * 1e12):
        return dict({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4)}, **common)
    return dict({"bound": "mfma", "achieved": round(tfs, 2), "peak": peak_f, "unit": "TFLOP/s",
                 "frac": round(tfs / peak_f, 4)}, **common)


def host_info():
    """CPU model, hardware threads and memory of the host doing the timing."""
    model, ram_gib = None, None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    ram_gib = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "ram_gib": ram_gib}


# one instance of each operation of the benchmark circuit: (label, Kraus set builder, qubits)
CPU_OP_TYPES = ("u3", "dep1", "cx", "dep2")


def _cpu_op(W, kind):
    if kind == "u3":
        return W.gate(W.u3(0.7, 1.9, 4.1), (0,))
    if kind == "dep1":
        return W.channel(W.depolarizing(1e-3, 1), (0,))
    if kind == "cx":
        return W.gate(W.cx(), (0, 1))
    return W.channel(W.depolarizing(1e-2, 2), (0, 1))


def cpu_baseline(W, n_full, ops_full, gates_per_apply, big_n=14):
    """The oracle (unfused FP64 sum K rho K^dag, all host threads) as the CPU baseline.

    * the 8-qubit workload (20 layers, 640 operations) in full;
    * the time of one operation of each kind of the benchmark circuit (U3, one-qubit
      depolarizing, CX, two-qubit depolarizing) at 8, 10, 12 and `big_n` qubits (the
      two-qubit depolarizing channel, 16 Kraus terms, only up to 12 qubits: about 25 s at 14
      on 16 threads);
    * per kind, the 16-qubit time extrapolated from its largest measured size by 4^(16 - n)
      (the oracle's work per operation is proportional to the 4^n elements; the measured
      ratios between sizes are reported beside it), weighted by the benchmark circuit's mix
      of kinds: the extrapolated gates/s at 16 qubits, and applies/s after dividing by the
      operations one fused apply absorbs;
    * the first operations of the 14-qubit brickwork workload, until ~8 s have passed, and its
      10-layer prefix extrapolated from the per-kind times (phase damping timed once more)."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    out = dict(host_info(), threads=oracle.max_threads())
    n1, ops1 = W.config1()
    t0 = time.perf_counter()
    oracle.run(n1, ops1)
    t1 = time.perf_counter() - t0
    out["config_8q_full"] = {"n": n1, "ops": len(ops1), "s": round(t1, 3), "ops_per_s": round(len(ops1) / t1, 1)}
    log("cpu baseline: 8-qubit workload %d ops in %.2f s" % (len(ops1), t1))
    per = {k: {} for k in CPU_OP_TYPES + ("pd",)}
    for n in (8, 10, 12, big_n):
        rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
        rho[0, 0] = 1.0
        kinds = CPU_OP_TYPES + (("pd",) if n == big_n else ())
        for kind in kinds:
            if kind == "dep2" and n > 12:
                continue
            op = W.channel(W.phase_damping(1e-3), (0,)) if kind == "pd" else _cpu_op(W, kind)
            reps = 4 if n <= 10 else 1
            t0 = time.perf_counter()
            for _ in range(reps):
                oracle.run_on(rho, [op])
            per[kind][n] = (time.perf_counter() - t0) / reps
        log("cpu baseline: per-operation times at n=%d: %s" % (n, {k: round(v[n], 4) for k, v in per.items() if n in v}))
        del rho
    mix = {k: 0 for k in CPU_OP_TYPES}
    for op in ops_full:
        mix[op.label if op.label in mix else ("dep1" if op.width == 1 else "dep2")] += 1
    t16 = {}
    for kind in CPU_OP_TYPES:
        nmax = max(per[kind])
        t16[kind] = per[kind][nmax] * 4.0 ** (n_full - nmax)
    secs16 = sum(mix[k] * t16[k] for k in CPU_OP_TYPES)
    gates16 = len(ops_full) / secs16
    ratios = {k: {"%d->%d" % (a, b): round(per[k][b] / per[k][a], 2)
                  for a, b in ((8, 10), (10, 12), (12, big_n)) if a in per[k] and b in per[k]}
              for k in CPU_OP_TYPES}
    out["per_op_s"] = {k: {str(n): round(v, 5) for n, v in sorted(per[k].items())} for k in per}
    out["ratio_per_2_qubits"] = ratios
    out["extrapolated_16q"] = {"method": "per kind: time at its largest measured n x 4^(16 - n); "
                                         "weighted by the benchmark circuit's mix %s" % mix,
                               "s_per_op": {k: round(v, 3) for k, v in t16.items()},
                               "gates_per_s": gates16, "applies_per_s": gates16 / gates_per_apply,
                               "label": "extrapolated"}
    n2, ops2 = W.config2(layers=10)
    rho = np.zeros((1 << n2, 1 << n2), dtype=np.complex128)
    rho[0, 0] = 1.0
    t0 = time.perf_counter()
    done = 0
    for op in ops2:
        oracle.run_on(rho, [op])
        done += 1
        if time.perf_counter() - t0 > 8.0:
            break
    t2 = time.perf_counter() - t0
    del rho
    tk = {"u3": per["u3"][big_n], "dep1": per["dep1"][big_n], "pd": per["pd"][big_n],
          "cz": per["cx"][big_n], "dep2": per["dep2"][12] * 4.0 ** (big_n - 12)}
    pre = sum(tk[op.label] for op in ops2)
    out["config_14q_prefix"] = {"n": n2, "ops_timed": done, "s": round(t2, 2),
                                "s_per_op": round(t2 / done, 3),
                                "prefix_10_layers_ops": len(ops2),
                                "prefix_10_layers_s_extrapolated": round(pre, 1),
                                "label": "first operations measured; 10-layer time extrapolated from "
                                         "per-kind times (two-qubit depolarizing from 12 qubits by 4^2)"}
    log("cpu baseline: 14-qubit brickwork, %d ops in %.1f s; 10-layer prefix ~%.0f s (extrapolated)"
        % (done, t2, pre))
    return out


def _gen_arrays(args):
    from paper_2404_13184_amd import workloads as W

    return W.request_arrays(args)


def serving_requests(W, num, seed=5):
    """The request stream and each request's circuit (pooled arrays), generated in parallel.

    Called before anything loads the HIP library or touches the GPU: the workers are forks of
    this process, and a fork of a process that has initialised HIP inherits its runtime (and a
    profiler's) state.  The pool is closed and joined, so every worker ends on its own rather
    than by a signal."""
    import multiprocessing as mp

    reqs = W.config5(num_requests=num, seed=seed)
    workers = max(1, min(16, (os.cpu_count() or 2) - 1))
    pool = mp.get_context("fork").Pool(workers)
    try:
        arrays = pool.map(_gen_arrays, reqs, chunksize=32)
    finally:
        pool.close()
        pool.join()
    return reqs, arrays


def _latency_summary(lat, done, first_arrival, last_done):
    import numpy as np

    lat = np.asarray(lat)
    span = max(1e-9, last_done - first_arrival)
    return {"completed": int(done), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2) if lat.size else None,
            "mean_ms": round(float(lat.mean()) * 1e3, 2) if lat.size else None,
            "circuits_per_s": round(done / span, 2)}


def serve_batched(T, W, reqs, arrays, prec, width, budget, slots, steps, cohort_bytes=0):
    """Open-loop replay of the stream through the continuous-batching server."""
    srv = T.Server(budget, slots, prec, width, steps, use_graphs=True, cohort_bytes=cohort_bytes)
    outs = {}
    t0 = time.perf_counter()
    c0 = srv.stats()["clock"]
    tickets = []
    for r, ca in zip(reqs, arrays):
        dt = r.arrival_s - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(r.n, arrays=ca, probs=True, paulis=W.z_paulis(r.n)[:1]))
    lat, last = [], 0.0
    for r, t in zip(reqs, tickets):
        res = srv.wait(t)
        if res["status"] != 0:
            raise RuntimeError("request %d failed: %d" % (r.rid, res["status"]))
        done = res["t_done"] - c0
        lat.append(done - r.arrival_s)
        last = max(last, done)
        outs[r.rid] = res["trace"]
        srv.release(t)
    st = srv.stats()
    srv.close()
    out = _latency_summary(lat, len(lat), reqs[0].arrival_s, last)
    out.update({"peak_device_bytes": int(st["peak_bytes"]), "budget_bytes": int(st["budget_bytes"]),
                "batched_applies": int(st["steps"]), "graph_launches": int(st["launches"]),
                "tile_applies": int(st["tiles"]), "chunks": int(st["chunks"]),
                "avg_chunk_tiles": round(st["tiles"] / max(1, st["chunks"]), 2),
                "wall_s": round(time.perf_counter() - t0, 2)})
    return out


def serve_plain(T, W, reqs, arrays, time_budget_s):
    """The unbatched baseline: one request at a time in arrival order, FP64, one superoperator
    per operation (no fusion).  Stops admitting new work after time_budget_s."""
    lat = []
    t0 = time.perf_counter()
    last = 0.0
    for r, ca in zip(reqs, arrays):
        now = time.perf_counter() - t0
        if now > time_budget_s:
            break
        if r.arrival_s > now:
            time.sleep(r.arrival_s - now)
        c = T.Circuit(r.n, arrays=ca)
        f = c.fuse(T.TANQ_FUSE_NONE, "f64")
        d = T.DM(r.n, "f64")
        d.apply_fused(f)
        d.probs(renormalize=True)
        d.expect_pauli(W.z_paulis(r.n)[0])
        d.free()
        f.free()
        c.free()
        done = time.perf_counter() - t0
        lat.append(done - r.arrival_s)
        last = done
    out = _latency_summary(lat, len(lat), reqs[0].arrival_s, last)
    out["latency_note"] = "p50/p99/mean over the requests served inside the window only"
    out["arrived_in_window"] = int(sum(1 for r in reqs if r.arrival_s <= last))
    # every request that arrived before the window closed but was not served waited at least
    # until then: counted with that lower bound, the percentiles cover every arrival
    import numpy as np

    cens = list(lat) + [last - r.arrival_s for r in reqs[len(lat):] if r.arrival_s <= last]
    if cens:
        out["censored"] = {"requests": len(cens), "p50_ms_at_least": round(float(np.percentile(cens, 50)) * 1e3, 2),
                           "p99_ms_at_least": round(float(np.percentile(cens, 99)) * 1e3, 2),
                           "note": "arrived but unserved requests counted with latency >= window end - arrival"}
    out["wall_s"] = round(time.perf_counter() - t0, 2)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU sharding (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_2404_13184_amd import workloads as W

    stream_reqs = None
    if a.serve_requests > 0:
        # before any HIP or torch GPU call: the generator forks worker processes
        log("serving: generating %d requests ..." % a.serve_requests)
        stream_reqs = serving_requests(W, a.serve_requests)
    import torch

    from paper_2404_13184_amd import tanq as T

    T.load()
    torch.cuda.init()
    if a.copy_calibration_gib > 0:
        nel = int(a.copy_calibration_gib * (1 << 30)) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read and %d bytes written by one copy kernel" % (nel * 8, nel * 8))
        del src, dst
    n, ops = W.config4(layers=a.layers, n=a.n)
    results, dms = {}, {}
    for prec in a.precs.split(","):
        results[prec], dms[prec] = run_precision(T, torch, n, ops, prec, a.width, a.steps, a.warmup)
    accuracy = None
    if "f64" in dms and "f32" in dms:
        fro, mx, nrm = dms["f32"].compare(dms["f64"])
        p32, p64 = results["f32"]["probs"], results["f64"]["probs"]
        dp = float(np.abs(p32 - p64).max())
        pos = p64 > 0
        dp_rel = float((np.abs(p32 - p64)[pos] / p64[pos]).max()) if pos.any() else None
        accuracy = {"fro_diff": fro, "max_abs_diff": mx, "fro_f64": nrm,
                    "trace_distance_bound": 0.5 * (2 ** (n / 2)) * fro, "max_abs_dprob": dp,
                    "max_rel_dprob": dp_rel, "min_prob_f64": float(p64.min())}
        log("f32 vs f64: ||d||_F %.3e, max %.3e, TD <= %.3e, max|dp| %.3e, max|dp|/p %.3e" %
            (fro, mx, accuracy["trace_distance_bound"], dp, dp_rel))
    for d in dms.values():
        d.free()

    main_prec = "f64" if "f64" in results else a.precs.split(",")[0]
    r = results[main_prec]
    # fusion ratio (Sec. 3.3): source operations per fused apply, next to the paper's own rule
    # (consecutive operations on the same ordered qubit tuple) planned on the host
    cc = T.Circuit(n, ops)
    paper_blocks = cc.plan(T.TANQ_FUSE_PAPER)[1]
    cc.free()
    fusion = {"source_ops": len(ops), "fused_applies": r["info"]["count"],
              "ratio": round(len(ops) / r["info"]["count"], 2), "paper_rule_applies": paper_blocks,
              "paper_rule_ratio": round(len(ops) / paper_blocks, 2)}
    value = r["applies"] / r["wall_s"]

    def measured_mfma(rl, rr, secs):
        """The executed products' rate against the measured rate of the same multiplication loop
        with nothing else in it (tanq_mfma_rate), beside the datasheet fraction."""
        if "mfma_flops_executed" in rl and rr.get("mfma_tflops"):
            rl["mfma_measured_TFLOPs"] = round(rr["mfma_tflops"], 2)
            rl["mfma_frac_of_measured"] = round(rl["mfma_flops_executed"] / secs / 1e12 / rr["mfma_tflops"], 4)
        return rl

    def dominant(rr, prec):
        k = max(rr["per_k"], key=lambda kk: sum(rr["per_k"][kk]))
        secs = sum(rr["per_k"][k]) / len(rr["per_k"][k])
        if k == "pass":
            rl = roofline_pass(prec, n, secs, sum(rr["pass_sizes"]) / len(rr["pass_sizes"]),
                               sum(rr["alg_flops"][k]) / len(rr["alg_flops"][k]))
            name = PASS_KERNELS[prec]
            rl["kernel"] = name
            rl["traffic"] = measured_traffic(name, n)
            if rl["traffic"] is not None:
                rl["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
            return measured_mfma(rl, rr, secs)
        rl = measured_mfma(roofline(prec, k, n, secs), rr, secs)
        if k in rr["variants"]:
            name = kernel_name(prec, k, rr["variants"][k])
            rl["kernel"] = name
            rl["traffic"] = measured_traffic(name, n)
            if rl["traffic"] is not None:
                rl["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        return rl

    def hbm_summary(prec, rr):
        """State bandwidth of the plain in-place stream (the measured peak for this access
        pattern), of a single 2-qubit apply (autotuned, dense data) and of a pass, each as a
        fraction of the datasheet peak and of the measured stream."""
        es = 16 if prec == "f64" else 8
        nbytes = 2.0 * (4 ** n) * es
        st = nbytes / rr["stream_s"] / 1e9
        k2 = nbytes / (rr["tuned_ms"][1] * 1e-3) / 1e9
        res = {"stream_GBs": round(st, 1), "stream_frac_datasheet": round(st / HBM_PEAK_GBS, 4),
               "apply_k2_GBs": round(k2, 1), "apply_k2_frac_datasheet": round(k2 / HBM_PEAK_GBS, 4),
               "apply_k2_frac_stream": round(k2 / st, 4)}
        if "pass" in rr["per_k"]:
            ps = nbytes / (sum(rr["per_k"]["pass"]) / len(rr["per_k"]["pass"])) / 1e9
            res.update({"pass_GBs": round(ps, 1), "pass_frac_datasheet": round(ps / HBM_PEAK_GBS, 4),
                        "pass_frac_stream": round(ps / st, 4)})
        return res

    out = {
        "metric": "16-qubit DM superop applies/s",
        "value": round(value, 3),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["wall_s"] / a.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": "16-qubit noisy random U3/CX circuit, depth 100, dep 1e-3/1e-2 "
                               "(2^32-element vec(rho), %s)" % ("64 GiB FP64" if main_prec == "f64" else "32 GiB FP32"),
                   "n_qubits": n, "layers": a.layers, "source_ops": len(ops),
                   "fused_applies_per_step": r["info"]["count"], "fusion_width": r["info"]["max_width"],
                   "count_by_k": r["info"]["count_k"][1:]},
        "gates_per_s": round(len(ops) * a.steps / r["wall_s"], 1),
        "fusion": fusion,
        "roofline": dominant(r, main_prec),
    }
    for prec, rr in results.items():
        out[prec] = {"applies_per_s": round(rr["applies"] / rr["wall_s"], 3),
                     "gates_per_s": round(len(ops) * a.steps / rr["wall_s"], 1),
                     "ms_per_step": round(rr["wall_s"] / a.steps * 1e3, 2),
                     "fused_applies": rr["info"]["count"], "fusion_width": rr["info"]["max_width"],
                     "count_by_k": rr["info"]["count_k"][1:],
                     "avg_launch_ms_by_kind": {str(k): round(sum(v) / len(v) * 1e3, 3) for k, v in rr["per_k"].items()},
                     "roofline": dominant(rr, prec), "trace": rr["trace"],
                     "autotuned_ms_per_apply_by_k": [round(x, 3) for x in rr["tuned_ms"]],
                     "variants": rr["variants"], "launches_per_step": rr["launches"],
                     "passes_per_step": len(rr["pass_sizes"]) // max(a.steps, 1),
                     "other_fusion_width": rr["alternative"],
                     "hbm": hbm_summary(prec, rr)}
    if accuracy is not None:
        out["f32_vs_f64"] = accuracy
    if a.serve_requests > 0:
        reqs, arrays = stream_reqs
        log("serving: FP32 continuous batching ...")
        batched = serve_batched(T, W, reqs, arrays, "f32", a.serve_width, int(a.serve_budget_gb * (1 << 30)),
                                a.serve_slots, a.serve_steps, int(a.serve_cohort_mib * (1 << 20)))
        log("serving batched: %s" % batched)
        log("serving: plain FP64 per request ...")
        plain = serve_plain(T, W, reqs, arrays, a.plain_budget_s)
        log("serving plain: %s" % plain)
        out["serving"] = {"workload": "%d requests, Poisson 200/s, n ~ U{4..12}, depth ~ U{20..200}, "
                                      "U3/CX, Ising Trotter and teleport blocks" % a.serve_requests,
                          "batched_f32": dict(batched, width=a.serve_width, slots=a.serve_slots,
                                              steps_per_launch=a.serve_steps,
                                              cohort_mib=a.serve_cohort_mib),
                          "plain_f64": plain}
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        gates_per_apply = len(ops) / r["info"]["count"]
        cb = cpu_baseline(W, n, ops, gates_per_apply)
        ex = cb["extrapolated_16q"]
        out["cpu_baseline"] = dict({
            "value": ex["applies_per_s"],
            "unit": "applies/s",
            "cores": cb["threads"],
            "kind": "oracle",
            "sample": "oracle (unfused FP64 sum K rho K^dag, %d threads): the 8-qubit workload in full; one "
                      "operation of each kind of the benchmark circuit at 8/10/12/14 qubits, extrapolated to 16 "
                      "qubits by 4^n and weighted by the circuit's mix (%.2f operations per fused apply); the "
                      "first operations of the 14-qubit brickwork workload" % (cb["threads"], gates_per_apply),
            "gates_per_s_16q_extrapolated": ex["gates_per_s"],
        }, **{k: v for k, v in cb.items() if k != "threads"})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
