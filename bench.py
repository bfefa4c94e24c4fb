"""Benchmark: TMFG construction on one MI355X.

One step = one whole build on the GPU from series already resident in HBM: Pearson
similarity (standardise + FP32-MFMA GEMM), seed scores, the per-vertex row sort and the
persistent insertion loop (seed selection, initial faces, n-4 insertions). The default
workload is n=20000 series of length L=1024 (50 planted random-walk clusters plus 10%
white-noise series).

value = whole-job insertions per second = steps * (n-4) / (time of the timed steps).
Also printed: per-phase times from HIP events on the build stream, the loop-only
insertion rate, the roofline of the dominant kernel (the insertion loop: its dependent
trips to memory against the measured latency of one trip), the CPU oracle timed on the
same workload, and, in the same line, the other two parts of the metric: the batched form
(512 uneven instances per graph replay, builds/s, autotuned against default launches and
against one build per launch) and the serving form (p50/p99 latency at 0.5x and 0.8x of
the saturated rate, against serial plain builds under the same arrivals). Batched and
served results are checked bitwise against plain builds before their rates are reported.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

# The request server runs each dispatch slot on its own stream, and each stream needs a
# hardware queue of its own: HIP shares GPU_MAX_HW_QUEUES queues (4 unless set) among all
# of a process's streams, torch's included, and two slots on one queue serialize. Raised
# here, before anything in the process initialises HIP.
SERVER_SLOTS = 8
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 2 * SERVER_SLOTS:
    os.environ["GPU_MAX_HW_QUEUES"] = str(2 * SERVER_SLOTS)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--batch", type=int, default=512, help="instances in the c4 batch")
    ap.add_argument("--requests", type=int, default=2200, help="c5: requests per replay (the first 200 warm up)")
    ap.add_argument("--max-batch", type=int, default=512, help="c5: requests one server dispatch groups")
    ap.add_argument("--streams", type=int, default=SERVER_SLOTS, help="c5: server dispatches in flight")
    ap.add_argument("--no-serial", action="store_true", help="c5: skip the serial plain-build comparison")
    ap.add_argument("--serial-requests", type=int, default=300,
                    help="c5: requests of the trace (from its start) replayed as serial plain builds")
    ap.add_argument("--no-c4", action="store_true", help="default run: leave out the batched (c4) summary")
    ap.add_argument("--no-c5", action="store_true", help="default run: leave out the serving (c5) summary")
    ap.add_argument("--c4-steps", type=int, default=5, help="default run: timed replays of the c4 batch")
    ap.add_argument("--fifo", action="store_true", help="c5: dispatch strictly in arrival order")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=0,
                    help="insertions of the oracle's build to time (0: all of them)")
    ap.add_argument("--rule", default="exact", choices=["exact", "paper", "corr"],
                    help="face rule: exact greedy, the paper's heap rule (Algorithm 2), or corr-tmfg "
                         "with a prefix size (Algorithm 1)")
    ap.add_argument("--prefix", type=int, default=1, help="corr-tmfg prefix size (1..16)")
    ap.add_argument("--dbht", action="store_true",
                    help="DBHT clustering on the host of the GPU-built TMFG (shortest paths, bubble "
                         "tree, complete linkage) and its ARI")
    ap.add_argument("--edge-sums", action="store_true",
                    help="edge-sum study: exact vs paper face rule on the single-build workloads")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run a 1 GiB device copy (the reference kernel for HBM counters)")
    return ap.parse_args()


HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "paper_2408_09399_amd", "csrc")
# source files whose text fixes each kernel's code; a traffic figure measured on other text is void
KERNEL_SOURCES = {
    "tmfg_loop": ["loop.hip", "facerule.h", "common.h", "internal.h"],
    "tmfg_corr": ["corr.hip", "facerule.h", "common.h", "internal.h"],
    "corr_gemm": ["pearson.hip", "common.h", "internal.h"],
    "sort_rows": ["sort.hip", "common.h", "internal.h"],
}
COPY_BYTES = 1 << 30


def source_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, config: str):
    """HBM bytes per build of `kernel` on `config` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE summed over the build's launches of the kernel, each scaled by
    what the same counter read for a copy of known size), or None when there is none or the
    kernel's source has changed since."""
    path = os.path.join(HERE, "profiles", f"{kernel}_{config}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv["source_sha256_16"] != source_digest(kernel):
            return None
        fetch = float(kv["fetch_kib_per_build"]) * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_build"]) * float(kv["write_scale"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0


def calibration_copy():
    """A plain elementwise copy of 1 GiB (read 1 GiB, write 1 GiB), three times."""
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    del x, y


def sweep_refresh(tm, plan, W, res, n, stream):
    """a6-sweep bulk refresh: the exact best vertex of all 2n-4 final faces by full sweeps,
    with the first n/2 vertices of the insertion order marked inserted."""
    import torch
    order = res.order.cpu().numpy()
    bits = np.zeros((n + 31) // 32, dtype=np.uint32)
    for v in order[: n // 2]:
        bits[v >> 5] |= np.uint32(1) << np.uint32(v & 31)
    ins = torch.from_numpy(bits.view(np.int32)).to(W.device)
    faces = res.faces.view(-1, 3)
    times = []
    for _ in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tm.face_sweep(W, faces, ins, plan=plan, stream=stream)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times[1:]))
    F = faces.shape[0]
    alg_bytes = F * (12.0 * n + (n + 7) // 8)
    return {"faces": F, "ms": round(ms, 3), "algorithmic_bytes": alg_bytes,
            "gbs": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
            "frac_hbm": round(alg_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def workload(name):
    from paper_2408_09399_amd import synth
    return {"c1": synth.config_c1, "c2": synth.config_c2, "c3": synth.config_c3}[name]()


def cpu_baseline(X: np.ndarray, W_gpu: np.ndarray, sample_steps: int) -> dict:
    """The CPU oracle on the host cores: float64 Pearson of all series (BLAS, all threads),
    float64 seed scores, and the oracle's lazy exact TMFG schedule (oracle.tmfg.tmfg_lazy,
    single thread) timed for its first `sample_steps` insertions (all of them when 0, the
    default) and for none; the difference is the loop's time for those insertions, scaled
    to n-4 when it is a sample."""
    import oracle
    from oracle import tmfg as otm
    try:
        from threadpoolctl import threadpool_info
        threads = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:
        threads = os.cpu_count() or 1
    n = X.shape[0]
    t0 = time.perf_counter()
    oracle.pearson64(X)
    t_pearson = time.perf_counter() - t0
    k = n - 4 if sample_steps <= 0 else min(sample_steps, n - 4)
    t0 = time.perf_counter()
    otm.tmfg_lazy(W_gpu, max_steps=0)          # checks, seed scores and the four seed faces
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    otm.tmfg_lazy(W_gpu, max_steps=k)
    t_loop = max(time.perf_counter() - t0 - t_setup, 1e-9)
    t_total = t_pearson + t_setup + t_loop * (n - 4) / k
    if k == n - 4:
        what = f"all {n - 4} insertions ({t_loop:.2f}s, 1 thread): the whole build, not a sample"
    else:
        what = (f"its first {k} of {n - 4} insertions ({t_loop:.2f}s, 1 thread) scaled linearly to all "
                f"insertions (late insertions cost more, so this overstates the oracle's rate)")
    return {
        "value": (n - 4) / t_total, "unit": "insertions/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"float64 Pearson of all {n} series ({t_pearson:.2f}s, {threads} BLAS threads); the "
                   f"oracle's lazy exact schedule: checks, seed and seed faces ({t_setup:.2f}s), then " + what),
    }


def bench_batch(args, steps=None, warmup=None):
    """512 independent instances (n log-uniform in [64, 4096], L uniform in [64, 512]) in one
    graph replay with autotuned launch configurations, against the same batch with default
    configurations and against the same instances built one per launch. Every instance of
    the autotuned batch is checked bitwise against its plain build before rates are reported."""
    import torch
    import paper_2408_09399_amd as tm
    from paper_2408_09399_amd import synth
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    inst = synth.config_c4(args.batch)
    dev = torch.device("cuda:0")
    Xs = [torch.from_numpy(s.X).to(dev) for s in inst]
    stream = torch.cuda.current_stream()

    def timed(batch):
        for _ in range(warmup):
            batch.run(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.run(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        bad = [i for i, r in enumerate(batch.results) if int(r.status.item()) != 0]
        if bad:
            raise RuntimeError(f"batch instances failed: {bad[:5]}")
        return wall

    rule = rule_flags(tm, args.rule, args.prefix)
    default = tm.Batch([("X", x) for x in Xs], flags=rule)
    wall_default = timed(default)
    default.close()
    batch = tm.Batch([("X", x) for x in Xs], flags=tm.BATCH_AUTOTUNE | rule)
    tuned_cfg = batch.config()
    wall = timed(batch)
    # the same instances, one build (one launch sequence) each, back to back on one plan
    n_max = max(s.X.shape[0] for s in inst)
    L_max = max(s.X.shape[1] for s in inst)
    plan = tm.Plan(n_max, L_max, rule)
    outs = [tm.alloc_result(x.shape[0], dev) for x in Xs]
    for x, o in zip(Xs[:8], outs[:8]):
        tm.build(X=x, plan=plan, out=o, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x, o in zip(Xs, outs):
        tm.build(X=x, plan=plan, out=o, stream=stream)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    mismatched = [i for i, (g, o) in enumerate(zip(batch.results, outs))
                  if not all(torch.equal(getattr(g, k), getattr(o, k)) for k in ("order", "edges", "steps", "faces"))
                  or not torch.equal(g.step_gain.view(torch.int32), o.step_gain.view(torch.int32))]
    if mismatched:
        raise RuntimeError(f"batched results differ from plain builds: {mismatched[:5]}")
    insertions = sum(s.X.shape[0] - 4 for s in inst)
    per = wall / steps
    out = {
        "metric": "batched builds/s (512 uneven instances per graph replay)",
        "value": round(len(inst) / per, 2), "unit": "builds/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(per * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(inst)} planted-cluster instances, n log-uniform in [64, 4096], "
                               f"L uniform in [64, 512]", "instances": len(inst),
                   "sum_n": int(sum(s.X.shape[0] for s in inst)), "rule": rule_name(args)},
        "insertions_per_s": round(insertions / per, 1),
        "autotuned": tuned_cfg,
        "default_launch": {"ms_per_step": round(wall_default / steps * 1e3, 3),
                           "builds_per_s": round(len(inst) * steps / wall_default, 2)},
        "plain_one_per_launch": {"seconds": round(plain, 3), "builds_per_s": round(len(inst) / plain, 2)},
        "speedup_vs_plain": round(plain / per, 2),
        "checked": f"all {len(inst)} autotuned results bitwise equal to their plain builds",
    }
    plan.close()
    batch.close()
    return out


def _percentile(v, p):
    """Nearest-rank percentile."""
    v = np.sort(np.asarray(v, dtype=np.float64))
    return float(v[min(len(v) - 1, max(0, int(np.ceil(p / 100.0 * len(v))) - 1))])


def _replay(srv, Xs, t_unit, qps, warm):
    """Submit every request at its arrival time (all at once when qps is None) while a
    second thread collects results in order; latencies of the requests after `warm`."""
    import queue
    import threading
    q = queue.Queue()
    out = [None] * len(Xs)

    def collect():
        for _ in range(len(Xs)):
            i, t = q.get()
            out[i] = srv.poll(t, wait_ms=-1)

    th = threading.Thread(target=collect)
    th.start()
    t0 = srv.now_ns() + 20_000_000
    for i, X in enumerate(Xs):
        arrival = 0
        if qps is not None:
            arrival = t0 + int(t_unit[i] / qps * 1e9)
            while True:
                d = arrival - srv.now_ns()
                if d <= 0:
                    break
                if d > 2_000_000:
                    time.sleep((d - 1_000_000) * 1e-9)
        q.put((i, srv.submit(X, arrival)))
    th.join()
    bad = [i for i, r in enumerate(out) if r["status"] != 0]
    if bad:
        raise RuntimeError(f"requests failed: {bad[:5]}")
    meas = out[warm:]
    lat = [(r["done_ns"] - r["arrival_ns"]) * 1e-6 for r in meas]
    span = (max(r["done_ns"] for r in meas) - min(r["arrival_ns"] for r in meas)) * 1e-9
    return {"p50_ms": round(_percentile(lat, 50), 2), "p99_ms": round(_percentile(lat, 99), 2),
            "mean_ms": round(float(np.mean(lat)), 2), "builds_per_s": round(len(meas) / span, 1),
            "requests": len(meas)}, out


def _serial_replay(tm, plan, Xs, t_unit, qps, dev):
    """Plain builds of the requests one at a time in arrival order (each waits for its arrival
    and for the one before): copy in, build, copy out; latencies observed on the host clock."""
    import torch
    outs = []
    lat = []
    t0 = time.perf_counter() + 0.02
    busy = 0.0
    for i, X in enumerate(Xs):
        arrival = t0 + t_unit[i] / qps
        d = arrival - time.perf_counter()
        if d > 0:
            time.sleep(d)
        s0 = time.perf_counter()
        res = tm.build(X=torch.from_numpy(X).to(dev), plan=plan)
        got = res.to_numpy()
        done = time.perf_counter()
        busy += done - s0
        lat.append((done - arrival) * 1e3)
        outs.append(got)
    return {"p50_ms": round(_percentile(lat, 50), 2), "p99_ms": round(_percentile(lat, 99), 2),
            "requests": len(Xs), "builds_per_s": round(len(Xs) / busy, 1)}, outs


def bench_serve(args):
    """Serving: Poisson arrivals of rolling-window requests (n log-uniform in [100, 8000],
    L = 256) from host memory through the request server; p50/p99 latency (done - arrival,
    queueing included) at 0.5x and 0.8x of the saturated rate, against serial plain builds of
    the start of the same arrival trace at the same rates, observed the same way. The serial
    builds' results are checked bitwise against the server's before rates are reported."""
    import torch
    import paper_2408_09399_amd as tm
    from paper_2408_09399_amd import synth
    warm = min(200, args.requests // 10)
    trace = synth.serving_trace(1.0, args.requests)          # arrival times at 1 request/s
    Xs = [r.series.X for r in trace]
    t_unit = np.array([r.t_arrival for r in trace])
    n_max = max(X.shape[0] for X in Xs)
    rule = rule_flags(tm, args.rule, args.prefix)
    srv = tm.Server(hbm_budget=96 << 30, host_budget=4 << 30, max_batch=args.max_batch, n_streams=args.streams,
                    n_max=n_max, L_max=256, flags=(tm.SERVER_FIFO if args.fifo else 0) | rule)
    _replay(srv, Xs[: warm], t_unit, None, 0)                # first use: code paths, caches
    sat, _ = _replay(srv, Xs, t_unit, None, 0)               # everything at once
    rates = {}
    served = {}
    for f in (0.5, 0.8):
        qps = f * sat["builds_per_s"]
        r, got = _replay(srv, Xs, t_unit, qps, warm)
        r["qps"] = round(qps, 1)
        rates[f"{f}x"] = r
        served[f"{f}x"] = got
    srv.close()
    out = {
        "metric": "p50/p99 latency at fixed QPS (request server, continuous batching)",
        "value": rates["0.5x"]["p99_ms"], "unit": "ms (p99 at 0.5x saturated QPS)", "n_gpus": 1,
        "steps": len(Xs) - warm, "warmup": warm, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals of {len(Xs)} rolling-window requests, n log-uniform in "
                               f"[100, 8000], L=256, from host memory", "requests": len(Xs),
                   "server": {"max_batch": args.max_batch, "n_streams": args.streams,
                              "policy": "fifo" if args.fifo else "size classes"}, "rule": rule_name(args)},
        "saturated": sat, "at_rate": rates,
    }
    if args.no_serial:
        return out
    # serial plain builds of the first requests of the trace, at the same rates
    k = min(args.serial_requests, len(Xs))
    dev = torch.device("cuda:0")
    plan = tm.Plan(n_max, 256, rule)
    serial = {}
    for key, r in rates.items():
        res, outs = _serial_replay(tm, plan, Xs[:k], t_unit, r["qps"], dev)
        for i, (a, b) in enumerate(zip(outs, served[key][:k])):
            if b["status"] != 0 or a["status"] != 0 or any(not np.array_equal(a[x], b[x])
                                                          for x in ("order", "edges", "steps", "faces")) \
                    or a["step_gain"].tobytes() != b["step_gain"].tobytes():
                raise RuntimeError(f"request {i}: served result differs from its plain build")
        serial[key] = res
    plan.close()
    out["serial_plain"] = {"requests": k, "at_rate": serial,
                           "note": f"the first {k} requests of the trace, one plain build at a time; "
                                   f"each result bitwise equal to the server's"}
    return out


def rule_name(args) -> str:
    return f"corr p={args.prefix}" if args.rule == "corr" else args.rule


def edge_sum(W, edges) -> float:
    """Sum of W over the TMFG's 3n-6 edges, in float64 (a quality diagnostic, Section 5.2)."""
    import torch
    e = edges.long()
    return float(W[e[:, 0], e[:, 1]].double().sum().item())


def rule_run(tm, X, steps, flags):
    """Builds X with the given plan flags; returns (result, median loop ms, stats)."""
    import torch
    n, L = X.shape
    plan = tm.Plan(n, L, tm.TIMING | flags)
    res = tm.alloc_result(n, X.device, keep_w=True)
    tm.build(X=X, plan=plan, out=res)
    loops = []
    for _ in range(steps):
        tm.build(X=X, plan=plan, out=res)
        loops.append(plan.phase_ms()[3])
    torch.cuda.synchronize()
    status = int(res.status.item())
    if status != 0:
        raise RuntimeError(f"build failed: {tm.STATUS.get(status)}")
    plan.close()
    return res, float(np.median(loops)), loop_counters(tm, X, flags)


def loop_counters(tm, X, flags):
    """The insertion loop's counters, from one more build on a plan that records them (outside
    any timed region: recording them costs the loop about a tenth of its time)."""
    import torch
    n, L = X.shape
    plan = tm.Plan(n, L, tm.STATS | flags)
    res = tm.build(X=X, plan=plan)
    torch.cuda.synchronize()
    if int(res.status.item()) != 0:
        raise RuntimeError("counter build failed")
    stats = plan.stats()
    plan.close()
    return stats


def rule_flags(tm, rule: str, prefix: int) -> int:
    return {"exact": 0, "paper": tm.RULE_PAPER, "corr": tm.rule_corr_prefix(prefix)}[rule]


def rule_summary(tm, X, res_exact, loop_ms_exact, steps, rule: str, prefix: int = 1) -> dict:
    """Another face rule on the same input (the paper's heap rule, Algorithm 2, or corr-tmfg
    with a prefix size, Algorithm 1): loop rate, counters, and its edge sum against the exact
    rule's."""
    n = X.shape[0]
    res, loop_ms, st = rule_run(tm, X, steps, rule_flags(tm, rule, prefix))
    es_p, es_e = edge_sum(res.W, res.edges), edge_sum(res_exact.W, res_exact.edges)
    oe = res_exact.order.cpu().numpy()
    op = res.order.cpu().numpy()
    diff = np.flatnonzero(oe != op)
    out = {"rule": rule if rule != "corr" else f"corr p={prefix}",
           "loop_ms": round(loop_ms, 3), "loop_insertions_per_s": round((n - 4) / (loop_ms * 1e-3), 1),
           "exact_loop_ms": round(loop_ms_exact, 3),
           "edge_sum": round(es_p, 6), "exact_edge_sum": round(es_e, 6),
           "edge_sum_rel_diff": float(f"{(es_p - es_e) / abs(es_e):.4e}"),
           "first_order_difference": int(diff[0]) if diff.size else None}
    if rule == "paper":
        out["stats"] = {"stale_recomputes": st[0], "row_scans": st[1], "phases": st[3],
                        "stale_top_phases": st[20], "work_overflow_phases": st[21],
                        "chunk_overflow_phases": st[22], "not_committed": st[23]}
    else:
        out["stats"] = {"recomputes": st[0], "row_scans": st[1], "extra_passes": st[2], "rounds": st[3],
                        "us": {"scan": st[5], "pairs": st[6], "publish": st[7], "rebuild": st[8],
                               "select": st[9]}}
    return out


def bench_edge_sums(args):
    """Edge-sum study (Section 5.2, Figure 7 analogue): exact greedy against the paper's heap
    rule and corr-tmfg with prefix sizes 1, 4 and 16."""
    import torch
    import paper_2408_09399_amd as tm
    rows = []
    for name in ("c1", "c2", "c3"):
        s = workload(name)
        X = torch.from_numpy(s.X).to(torch.device("cuda:0"))
        res_e, ms_e, _ = rule_run(tm, X, args.steps, 0)
        for rule, prefix in [("paper", 1), ("corr", 1), ("corr", 4), ("corr", 16)]:
            row = rule_summary(tm, X, res_e, ms_e, args.steps, rule, prefix)
            row["workload"] = f"{s.name}: n={s.X.shape[0]}, L={s.X.shape[1]}"
            rows.append(row)
            print(json.dumps(row), flush=True)
        del X, res_e
        torch.cuda.empty_cache()
    print(json.dumps({"edge_sums": rows}))


def bench_dbht(args):
    """DBHT (Section 2; ARI of Section 5) of the TMFG the GPU builds for the workload: the host
    library's time and ARI against the planted labels, and the oracle's time for the same."""
    import torch
    import paper_2408_09399_amd as tm
    from sklearn.metrics import adjusted_rand_score
    s = workload(args.config)
    n, L = s.X.shape
    X = torch.from_numpy(s.X).to(torch.device("cuda:0"))
    plan = tm.Plan(n, L, rule_flags(tm, args.rule, args.prefix))
    res = tm.alloc_result(n, X.device, keep_w=True)
    tm.build(X=X, plan=plan, out=res)
    torch.cuda.synchronize()
    got = res.to_numpy()
    plan.close()
    k = len(set(s.labels.tolist()))
    threads = min(os.cpu_count() or 1, 16)
    times = []
    for _ in range(max(args.steps, 1)):
        t0 = time.perf_counter()
        lib = tm.dbht(got["W"], got["order"], got["edges"], got["steps"], k, n_threads=threads)
        times.append(time.perf_counter() - t0)
    t_lib = float(np.median(times))
    out = {"metric": "DBHT clustering of the TMFG on the host (seconds per build)", "value": round(t_lib, 3),
           "unit": "s", "higher_is_better": False, "steps": len(times), "threads": threads,
           "config": {"workload": f"{s.name}: n={n}, L={L}, {k} ground-truth classes", "rule": rule_name(args)},
           "ari": round(float(adjusted_rand_score(s.labels, lib["labels"])), 4),
           "converging_bubbles": int(len(set(lib["group"].tolist())))}
    if not args.no_cpu_baseline:
        from oracle import dbht as dh
        t0 = time.perf_counter()
        ref = dh.dbht(got["W"], got, k)
        out["cpu_baseline"] = {"value": round(time.perf_counter() - t0, 3), "unit": "s", "cores": 1,
                               "kind": "oracle", "sample": "the whole DBHT of the same TMFG (numpy/scipy)",
                               "same_result": bool(all(np.array_equal(np.asarray(ref[x]), np.asarray(lib[x]))
                                                       for x in ("labels", "group", "bubble", "linkage")))}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library builds on one GPU per process (no multi-GPU path); use --gpus 1"}))
        sys.exit(2)
    if args.calibration_copy:
        calibration_copy()
    if args.config == "c4":
        print(json.dumps(bench_batch(args)))
        return
    if args.config == "c5":
        print(json.dumps(bench_serve(args)))
        return
    if args.edge_sums:
        return bench_edge_sums(args)
    if args.dbht:
        return bench_dbht(args)
    import torch
    import paper_2408_09399_amd as tm

    s = workload(args.config)
    n, L = s.X.shape
    dev = torch.device("cuda:0")
    X = torch.from_numpy(s.X).to(dev)
    plan = tm.Plan(n, L, tm.TIMING | rule_flags(tm, args.rule, args.prefix))
    res = tm.alloc_result(n, dev, keep_w=True)
    stream = torch.cuda.current_stream()

    def step():
        tm.build(X=X, plan=plan, out=res, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        phases.append(plan.phase_ms())      # waits for the last event of the TMFG build above
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = int(res.status.item())
    if status != 0:
        print(json.dumps({"error": f"build failed: {tm.STATUS.get(status)}"}))
        sys.exit(1)
    ms_per_step = wall * 1e3 / args.steps
    ph = np.median(np.asarray(phases), axis=0)          # [corr, seed, sort, loop, total]
    stats = loop_counters(tm, X, rule_flags(tm, args.rule, args.prefix))

    gemm_flops = float(n) * (n + 1) * L
    sort_bytes = 4.0 * n * n + 2.0 * n * (n - 1)
    gemm_tflops = gemm_flops / (ph[0] * 1e-3) / 1e12
    sort_gbs = sort_bytes / (ph[2] * 1e-3) / 1e9
    loop_ins_s = (n - 4) / (ph[3] * 1e-3)
    # Dominant kernel by time. The insertion loop is a serial chain of dependent steps; its
    # bandwidth figure counts the bytes each step must read (three 64-entry list windows and
    # their candidate gathers for the three new faces, per walk round actually taken).
    kernels = {
        "corr_gemm": ("mfma", gemm_tflops, PEAK_FP32_MFMA_TFLOPS, "TFLOP/s", ph[0]),
        "sort_rows": ("hbm", sort_gbs, PEAK_HBM_GBS, "GB/s", ph[2]),
    }
    # per walk round: 64 list entries (2-byte id + 4-byte value) from each of the three
    # lists; plus every similarity a walk had to read from W
    walk_rounds, gathers = stats[1], stats[11]
    loop_bytes = walk_rounds * 3 * 64 * 6 + gathers * 4
    loop_gbs = loop_bytes / (ph[3] * 1e-3) / 1e9
    kernels["tmfg_loop"] = ("latency", None, None, None, ph[3])
    dom = max(kernels, key=lambda k: kernels[k][4])
    floor = latency_floor(tm)
    if dom == "tmfg_loop":
        # The loop is a serial chain of dependent trips to memory on one CU. Per build it takes
        # at least: one trip per selection phase (the records of the queued chunks), one per
        # insertion (the new vertex's row position, advanced during the selection), and two per
        # round of each phase's deepest walk (list entries, then the similarities they name;
        # stats[12] sums those rounds). Its roofline is that count of trips against the measured
        # latency of one: a 64-line gather that hits the L2 (the floor) and one from HBM.
        trips = stats[3] + (n - 4) + 2 * stats[12]
        loop_us = ph[3] * 1e3
        lat = floor["l2_gather_ns"]
        roofline = {"kernel": "tmfg_loop", "bound": "latency", "achieved": round(trips / loop_us, 4),
                    "peak": round(1e3 / lat, 4), "unit": "dependent trips/us",
                    "frac": round(trips * lat * 1e-3 / loop_us, 5),
                    "traffic": None if (t := measured_traffic("tmfg_loop", args.config)) is None else round(t),
                    "trips": int(trips), "floor_ms_l2": round(trips * lat * 1e-6, 3),
                    "floor_ms_hbm": round(trips * floor["hbm_gather_ns"] * 1e-6, 3),
                    "us_per_phase": round(loop_us / stats[3], 3), "us_per_insertion": round(loop_us / (n - 4), 3),
                    "trips_per_phase": round(trips / stats[3], 3),
                    "hbm": {"achieved": round(loop_gbs, 3), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": round(loop_gbs / PEAK_HBM_GBS, 6)},
                    "per": f"build ({stats[24] + 1} launches, {stats[24]} row compactions between)"}
    else:
        b, ach, peak, unit, _ = kernels[dom]
        traffic = measured_traffic(dom, args.config)
        roofline = {"kernel": dom, "bound": b, "achieved": round(ach, 3), "peak": peak, "unit": unit,
                    "frac": round(ach / peak, 5), "traffic": None if traffic is None else round(traffic)}

    out = {
        "metric": "TMFG insertions/s at n=20k; batched builds/s; p50/p99 latency at fixed QPS",
        "value": round(args.steps * (n - 4) / wall, 1),
        "unit": "insertions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"single TMFG build from planted-cluster random-walk series, "
                               f"n={n}, L={L} ({s.name})", "n": n, "L": L, "rule": rule_name(args)},
        "phases_ms": {"similarity": round(ph[0], 3), "seed_scores": round(ph[1], 3),
                      "row_sort": round(ph[2], 3), "insertion_loop": round(ph[3], 3),
                      "total": round(ph[4], 3)},
        "loop_insertions_per_s": round(loop_ins_s, 1),
        "builds_per_s": round(1e3 / ms_per_step, 3),
        "corr_gemm_tflops": round(gemm_tflops, 2),
        "row_sort_gbs": round(sort_gbs, 1),
        "loop_stats": {"stale_recomputes": stats[0], "walk_rounds": stats[1], "sweeps": stats[2],
                       "phases": stats[3], "walk_batches": stats[4], "w_reads": stats[11],
                       "critical_rounds": stats[12], "walks_ge4": stats[13], "walks_ge16": stats[14],
                       "skip_scans": stats[15], "stale_top_phases": stats[20],
                       "work_overflow_phases": stats[21], "chunk_overflow_phases": stats[22],
                       "row_compactions": stats[24],
                       "from": "one more build on a plan with TMFG_STATS, outside the timed steps",
                       "us_with_counters": {"select": stats[5], "load": stats[6], "walk": stats[7],
                                            "sweep": stats[8], "publish": stats[9], "kernel": stats[10]}},
        "roofline": roofline,
        "latency_floor": floor,
        "face_sweep_refresh": sweep_refresh(tm, plan, res.W, res, n, stream),
    }
    if args.rule == "exact":
        k = min(args.steps, 3)
        out["paper_rule"] = rule_summary(tm, X, res, float(ph[3]), k, "paper")
        out["corr_rule"] = [rule_summary(tm, X, res, float(ph[3]), k, "corr", p) for p in (1, 16)]
    if not args.no_cpu_baseline and args.rule == "exact":
        out["cpu_baseline"] = cpu_baseline(s.X, res.W.cpu().numpy(), args.cpu_sample_steps)
    plan.close()
    del X, res
    torch.cuda.empty_cache()
    if args.config == "c3" and not args.no_c4:
        out["batched_c4"] = bench_batch(args, steps=args.c4_steps, warmup=2)
        print(json.dumps({"progress": "c4 done", "builds_per_s": out["batched_c4"]["value"]}), file=sys.stderr,
              flush=True)
    if args.config == "c3" and not args.no_c5:
        out["serving_c5"] = bench_serve(args)
    print(json.dumps(out))


def latency_floor(tm) -> dict:
    """Latency of one dependent trip to memory from one wave (tmfg_probe_load_latency): one line
    or a 64-line gather, from a chain that sits in the L2 and from one that is read from HBM."""
    kw = dict(steps=20000)
    return {"l2_line_ns": round(tm.load_latency_ns(1 << 20, lanes=1, **kw), 1),
            "l2_gather_ns": round(tm.load_latency_ns(1 << 20, lanes=64, **kw), 1),
            "hbm_line_ns": round(tm.load_latency_ns(4 << 30, lanes=1, **kw), 1),
            "hbm_gather_ns": round(tm.load_latency_ns(4 << 30, lanes=64, **kw), 1),
            "method": "one wave, pointer chase, 20000 dependent trips; L2: 1 MiB chain read once untimed "
                      "first; HBM: 4 GiB chain, every line read once"}


if __name__ == "__main__":
    main()
