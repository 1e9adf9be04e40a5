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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2404_13184_amd", "csrc", f) for f in ("apply.hip", "tile.hpp", "pass.hip")]
# multi-superoperator pass kernels, by precision
PASS_KERNELS = {"f64": "apply_pass_ws_kernel<double, 12, 640, 2>", "f32": "apply_pass_ws_kernel<float, 13, 640, 2>"}


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


def measured_traffic(name: str):
    """HBM bytes per launch of `name` from the committed rocprofv3 counter summary (FETCH_SIZE
    and WRITE_SIZE, each scaled by what the counter reads for a copy kernel of known size), or
    None when there is no summary for it or the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
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
    ap.add_argument("--cpu-n", type=int, default=12)
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
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
                events.append((f.get_k(pos) if r == 1 else "pass", r, ev0, ev1))
                pos += r
        p, tr = d.probs(renormalize=True)
        info = f.info
        f.free()
        return info, p, tr

    # the other fusion width, for context: one whole apply_fused timed end to end
    f0 = circ.fuse(width, prec, stream)
    chosen = f0.info["max_width"]
    f0.free()
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
    per_k, pass_sizes = {}, []
    for k, r, e0, e1 in events:
        per_k.setdefault(k, []).append(e0.elapsed_time(e1) * 1e-3)
        if r >= 2:
            pass_sizes.append(r)
    circ.free()
    applies = info["count"] * steps
    return {"wall_s": wall, "applies": applies, "info": info, "per_k": per_k, "trace": tr, "probs": p,
            "tuned_ms": tuned_ms[1:], "variants": variants, "alternative": alternative,
            "pass_sizes": pass_sizes, "launches": len(events) // max(steps, 1)}, d


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


def roofline_pass(prec, n, secs, m_avg):
    """A pass reads and writes the state once and multiplies it by m_avg 2-qubit
    superoperators (8 algorithmic flops per complex MAC; the kernel's 3M form executes 6): the
    bound is the resource whose ideal time at its datasheet peak is the longer, the other one
    beside it."""
    es = 16 if prec == "f64" else 8
    nbytes = 2.0 * (4 ** n) * es
    flops = m_avg * 8.0 * 16 * (4 ** n)
    peak_f = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    gbs = nbytes / secs / 1e9
    tfs = flops / secs / 1e12
    executed = 0.75 * flops
    common = {"traffic": None, "kernel_k": "pass", "superops_per_launch": round(m_avg, 3),
              "avg_launch_ms": round(secs * 1e3, 3), "algorithmic_bytes": nbytes, "algorithmic_flops": flops,
              "mfma_flops_executed": executed, "mfma_frac_executed": round(executed / secs / 1e12 / peak_f, 4)}
    if nbytes / (HBM_PEAK_GBS * 1e9) >= flops / (peak_f * 1e12):
        return dict({"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "mfma_frac": round(tfs / peak_f, 4)}, **common)
    return dict({"bound": "mfma", "achieved": round(tfs, 2), "peak": peak_f, "unit": "TFLOP/s",
                 "frac": round(tfs / peak_f, 4), "hbm_GBs": round(gbs, 1),
                 "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}, **common)


def cpu_baseline(W, n_full, layers_full, cpu_n, budget_s):
    """The oracle (unfused FP64 sum K rho K^dag, all host threads) on a bounded sample of
    the same circuit family at cpu_n qubits, scaled by 4^(n_full - cpu_n) to the 16-qubit
    unit; returns gates/s and the equivalent applies/s."""
    import oracle

    oracle.build(force=False)
    n_c, ops = W.config4(layers=layers_full, n=cpu_n)
    rho = None
    import numpy as np

    rho = np.zeros((1 << cpu_n, 1 << cpu_n), dtype=np.complex128)
    rho[0, 0] = 1.0
    t0 = time.perf_counter()
    done = 0
    for op in ops:
        oracle.run_on(rho, [op])
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    secs = time.perf_counter() - t0
    gates_per_s_small = done / secs
    scale = 4.0 ** (n_full - cpu_n)
    return {"gates_per_s_16q_equiv": gates_per_s_small / scale, "ops_done": done, "secs": secs,
            "cores": oracle.max_threads(), "cpu_n": cpu_n}


def _gen_arrays(args):
    from paper_2404_13184_amd import workloads as W

    return W.request_arrays(args)


def serving_requests(W, num, seed=5):
    """The request stream and each request's circuit (pooled arrays), generated in parallel."""
    import multiprocessing as mp

    reqs = W.config5(num_requests=num, seed=seed)
    workers = max(1, min(16, (os.cpu_count() or 2) - 1))
    with mp.get_context("fork").Pool(workers) as pool:
        arrays = pool.map(_gen_arrays, reqs, chunksize=32)
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
    out["arrived_in_window"] = int(sum(1 for r in reqs if r.arrival_s <= last))
    out["wall_s"] = round(time.perf_counter() - t0, 2)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this path has no multi-GPU sharding (use --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2404_13184_amd import tanq as T
    from paper_2404_13184_amd import workloads as W

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
        dp = float(np.abs(results["f32"]["probs"] - results["f64"]["probs"]).max())
        accuracy = {"fro_diff": fro, "max_abs_diff": mx, "fro_f64": nrm,
                    "trace_distance_bound": 0.5 * (2 ** (n / 2)) * fro, "max_abs_dprob": dp}
        log("f32 vs f64: ||d||_F %.3e, max %.3e, TD <= %.3e, max|dp| %.3e" %
            (fro, mx, accuracy["trace_distance_bound"], dp))
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

    def dominant(rr, prec):
        k = max(rr["per_k"], key=lambda kk: sum(rr["per_k"][kk]))
        secs = sum(rr["per_k"][k]) / len(rr["per_k"][k])
        if k == "pass":
            rl = roofline_pass(prec, n, secs, sum(rr["pass_sizes"]) / len(rr["pass_sizes"]))
            name = PASS_KERNELS[prec]
            rl["kernel"] = name
            rl["traffic"] = measured_traffic(name)
            if rl["traffic"] is not None:
                rl["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
            return rl
        rl = roofline(prec, k, n, secs)
        if k in rr["variants"]:
            name = kernel_name(prec, k, rr["variants"][k])
            rl["kernel"] = name
            rl["traffic"] = measured_traffic(name)
            if rl["traffic"] is not None:
                rl["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        return rl

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
                     "other_fusion_width": rr["alternative"]}
    if accuracy is not None:
        out["f32_vs_f64"] = accuracy
    if a.serve_requests > 0:
        log("serving: generating %d requests ..." % a.serve_requests)
        reqs, arrays = serving_requests(W, a.serve_requests)
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
        cb = cpu_baseline(W, n, a.layers, a.cpu_n, a.cpu_budget_s)
        gates_per_apply = len(ops) / r["info"]["count"]
        out["cpu_baseline"] = {
            "value": cb["gates_per_s_16q_equiv"] / gates_per_apply,
            "unit": "applies/s",
            "cores": cb["cores"],
            "kind": "oracle",
            "sample": "oracle (unfused FP64 sum K rho K^dag) on the first %d operations of the same "
                      "circuit family at %d qubits (%.1f s), scaled by 4^%d to 16 qubits and by %.2f "
                      "operations per fused apply" % (cb["ops_done"], cb["cpu_n"], cb["secs"],
                                                      n - cb["cpu_n"], gates_per_apply),
            "gates_per_s_16q_equiv": cb["gates_per_s_16q_equiv"],
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
