"""Benchmark: vegas+ iterations on one MI355X at D=8, N_ev=1e8 per iteration.

A step is one full iteration of the hot path (allocation scan, fused
sampling / map / integrand / sums / training data, estimate, reallocation,
refinement) on the D=8 three-diagonal-Gaussian workload with N_g=1000,
alpha=0.5, beta=0.75.  The value is integrand samples per second (samples
actually drawn, sum of n_h) over the timed steps, with all state resident in
HBM.  Prints one JSON line.

Beside it, outside the timed steps:
  precision_split  the same workload with FP32 map and integrand (FP64 or
                   compensated-FP32 accumulation): samples/s and estimates;
  serving.batch    a batch of Gaussian-mixture requests (D 2..16, N_ev
                   log-uniform 1e4..1e6, 10 iterations, N_g=500) all submitted
                   at once to the continuous-batching server, against the plain
                   path (vp_integrate, one request after another): makespan,
                   samples/s and p50/p99 latency;
  serving.stream   Poisson arrivals of correlated-Gaussian requests (D 3..21,
                   N_ev log-uniform 1e5..1e7, 5..20 iterations, N_g=1000) at a
                   fixed rate, served live; the plain path is a first-come
                   first-served queue whose service times are measured one by
                   one.

    python bench.py [--gpus 1] [--steps 20] [--warmup 10] [--precision fp64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "integrand samples/sec/GPU (D=8, 1e8/iter) + p50/p99 solve latency vs plain"
PEAK_VALU_SLOTS = 256 * 64 * 2.4e9  # full-rate VALU lane-operations per second: 256 CUs x 64 lanes x 2.4 GHz
# Algorithmic VALU slots per sample of the fused sampling kernel at D=8 with
# three Gaussian terms: the minimal operation list of each stage (Philox
# blocks x 10 rounds x (2 multiplies + 2 xors), u -> t, the map, the
# integrand, the sums and training-data values), priced with the issue costs an
# instruction-rate microbenchmark measured on this device: a 32x32->64-bit
# multiply-add issues at the FP64-FMA rate (one slot), the FP32 exponential
# costs about three slots, an FP64 exponential about 25 operations.
#   FP64:   4 blocks 160 + u->t 72 + map 72 + integrand 48+6+3x25 + sums 16 = 449
#   FP32:   2 blocks  80 + u->t 32 + map 64 + integrand 24+6+3x3  + sums 16 = 231
#   compensated FP32: + 3 slots for each of the 2 + D compensated additions = 261
SLOTS_PER_SAMPLE = {"fp64": 449.0, "fp32_acc64": 231.0, "fp32_neumaier": 231.0 + 3 * (2 + 8)}
COUNTERS = os.path.join(ROOT, "profiles", "k_sample_d8_counters.md")


def measured_traffic(precision):
    """HBM bytes per sampling launch from the committed counter summary, or
    None when that summary is for other kernel sources (or another path)."""
    import hashlib
    if precision != "fp64" or not os.path.exists(COUNTERS):
        return None
    vals = {}
    for line in open(COUNTERS):
        line = line.strip()
        for key in ("traffic_bytes_per_launch:", "sources_sha256:", "sources:"):
            if line.startswith(key):
                vals[key] = line[len(key):].strip()
    if len(vals) != 3:
        return None
    h = hashlib.sha256()
    for f in vals["sources:"].split():
        path = os.path.join(ROOT, f)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    if h.hexdigest() != vals["sources_sha256:"]:
        return None
    return float(vals["traffic_bytes_per_launch:"])


def cpu_threads():
    """Host threads for the oracle's all-core leg: the cores this process may
    use, at most the OMP_NUM_THREADS share the host gives a GPU job."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n, cap) if cap > 0 else n)


def cpu_baseline(p, f, budget_s=10.0):
    """The CPU oracle on the same workload, timed on the host.

    All cores: one whole iteration (iteration 0: sampling of every hypercube,
    estimate, reallocation and refinement), the hypercubes split into one
    contiguous block per thread (the oracle's range call, run from that many
    threads; its sums are merged in block order).  The value is samples per
    second of that iteration.  Single core: the sampling of iteration 0 over
    leading hypercubes, about budget_s seconds."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    op = oracle.Problem(p, f)
    fmap = op.map_init()
    n_h = op.alloc_init()
    threads = cpu_threads()
    edges = [op.n_hc * t // threads for t in range(threads + 1)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda t: op.sample_range(fmap, n_h, 0, edges[t], edges[t + 1]), range(threads)))
    t_sample = time.perf_counter() - t0
    S1 = np.concatenate([q["S1"] for q in parts])
    S2 = np.concatenate([q["S2"] for q in parts])
    H = parts[0]["H"].copy()
    Wt = parts[0]["W"].copy()
    for q in parts[1:]:
        H += q["H"]
        Wt += q["W"]
    I, V = op.reduce(n_h, S1, S2)
    op.realloc(S1, S2, n_h)
    op.refine(H, Wt, fmap)
    dt = time.perf_counter() - t0
    samples = int(np.asarray(n_h, dtype=np.int64).sum())
    assert sum(q["n_samples"] for q in parts) == samples
    # single core, bounded
    c0 = time.perf_counter()
    op.sample_range(fmap, n_h, 0, 0, 20000)
    per_hc = max((time.perf_counter() - c0) / 20000, 1e-9)
    n = int(min(op.n_hc, max(20000, budget_s / per_hc)))
    c0 = time.perf_counter()
    out = op.sample_range(fmap, n_h, 0, 0, n)
    c1 = time.perf_counter() - c0
    s1 = int(np.asarray(n_h[:n], dtype=np.int64).sum())
    assert out["n_samples"] == s1
    return {"value": samples / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"one whole iteration (iteration 0) of the D=8 N_ev=1e8 workload: sampling of all "
                      f"{op.n_hc} hypercubes ({samples} samples) in {threads} contiguous blocks on {threads} "
                      f"threads ({t_sample:.1f} s), then the estimate, reallocation and refinement "
                      f"({dt - t_sample:.1f} s, one thread); {dt:.1f} s in all",
            "iteration_estimate": I,
            "single_core": {"value": s1 / c1, "unit": "samples/s", "cores": 1,
                            "sample": f"sampling of iteration 0 over hypercubes [0, {n}) ({s1} samples, "
                                      f"{c1:.1f} s)"}}


def pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x, dtype=float), q)) if len(x) else None


def lat_summary(lat):
    return {"p50_s": pct(lat, 50), "p99_s": pct(lat, 99), "mean_s": sum(lat) / max(len(lat), 1)}


def run_split(B, W, ctx, n_ev, steps):
    """FP64 and the two split precisions on the headline workload."""
    out = {}
    for prec in ("fp64", "fp32_acc64", "fp32_neumaier"):
        p, f = W.cfg_diag_d8(n_ev=n_ev, precision=prec)
        gp = B.Problem(ctx, p.with_(n_iter=steps + 2), f)
        gp.iterate(2)
        r0 = gp.result()
        gp.profile(True)
        gp.sync()
        t0 = time.perf_counter()
        gp.iterate(steps)
        gp.sync()
        dt = time.perf_counter() - t0
        r1 = gp.result()
        k_ms, k_n = gp.kernel_time(0)
        gp.close()
        samples = r1["n_evals"] - r0["n_evals"]
        k_s = k_ms / max(k_n, 1) / 1e3
        frac = SLOTS_PER_SAMPLE[prec] * (samples / max(k_n, 1)) / k_s / PEAK_VALU_SLOTS
        out[prec] = {"samples_per_s": samples / dt, "kernel_ms": 1e3 * k_s, "roofline_frac": frac,
                     "mean": r1["mean"], "sdev": r1["sdev"], "pull_vs_exact": (r1["mean"] - 1.0) / r1["sdev"]}
    ref = out["fp64"]
    for prec in ("fp32_acc64", "fp32_neumaier"):
        o = out[prec]
        o["speedup_vs_fp64"] = o["samples_per_s"] / ref["samples_per_s"]
        o["diff_vs_fp64_in_sdev"] = (o["mean"] - ref["mean"]) / ref["sdev"]
    return out


def run_batch_path(B, W, ctx, n_ev, steps):
    """The D=8 workload through the batched-integrand path: the library
    writes the points as structure-of-arrays buffers, the example library's
    Gaussian mixture (same arithmetic as the built-in kind) fills f."""
    p, f = W.cfg_diag_d8(n_ev=n_ev)
    bf = B.example_gauss_mix(f)
    try:
        gp = B.Problem(ctx, p.with_(n_iter=steps + 2), bf)
        gp.iterate(2)
        r0 = gp.result()
        gp.profile(True)
        gp.sync()
        t0 = time.perf_counter()
        gp.iterate(steps)
        gp.sync()
        dt = time.perf_counter() - t0
        r1 = gp.result()
        gp.close()
    finally:
        B.examples().vp_example_free_user(bf.user)
    n = r1["n_evals"] - r0["n_evals"]
    return {"workload": "D=8 three-Gaussian workload, N_ev=1e8, FP64, integrand evaluated by a user function "
                        "over structure-of-arrays points (example library)",
            "samples_per_s": n / dt, "ms_per_step": 1e3 * dt / steps, "mean": r1["mean"], "sdev": r1["sdev"],
            "bytes_per_sample_moved": 8 * 8 + 8 + 8 + 2 * 8 + 8 * 8 + 8 + 8 + 2 * 8}


def run_plain(B, ctx, reqs):
    """vp_integrate one request after another; per-request service times (the
    requests' C structures are built beforehand, as for the served batch)."""
    prepared = [B.marshal(r.params, r.integrand) for r in reqs]
    svc, res = [], []
    for r, pr in zip(reqs, prepared):
        t0 = time.perf_counter()
        res.append(B.integrate(ctx, r.params, r.integrand, prepared=pr))
        svc.append(time.perf_counter() - t0)
    return svc, res


def agreement(served, plain):
    """Largest |served - plain| over requests, in units of the plain sdev."""
    worst = 0.0
    for a, b in zip(served, plain):
        if b["sdev"] > 0:
            worst = max(worst, abs(a["mean"] - b["mean"]) / b["sdev"])
    return worst


def run_batch(B, W, ctx, n_req, plain_too=True):
    reqs = W.served_batch(n_req=n_req)
    # warm-up outside the timed run: one iteration of one request of every
    # (dimension, terms) shape, so that each sampling kernel the batch uses has
    # been loaded and its occupancy queried once in this process
    shapes = {}
    for r in reqs:
        shapes.setdefault((r.params.dim, r.integrand.n_terms), r)
    warm = B.Server(ctx, max_slots=len(shapes))
    for t in warm.submit_many([(r.params.with_(n_iter=1), r.integrand) for r in shapes.values()]):
        warm.wait(t)
    warm.close()
    srv = B.Server(ctx, max_slots=n_req)
    prepared = srv.prepare([(r.params, r.integrand) for r in reqs])
    t0 = srv.now()
    tickets = srv.submit_many(prepared)  # one call: every request arrives at once
    served = [srv.wait(t) for t in tickets]
    times = [srv.times(t) for t in tickets]
    st = srv.stats()
    srv.close()
    makespan = max(t[2] for t in times) - t0
    lat = [t[2] - t[0] for t in times]
    samples = sum(r["n_evals"] for r in served)
    served_out = {"makespan_s": makespan, "samples_per_s": samples / makespan, **lat_summary(lat),
                  "steps": st["steps"], "graph_launches": st["graph_launches"],
                  "graph_captures": st["graph_captures"], "peak_active": st["peak_active"],
                  "mem_peak_bytes": st["mem_peak"],
                  "scheduler_s": {k: st[k] for k in ("t_admit", "t_plan", "t_step", "t_retire")}}
    if not plain_too:
        return {"samples": samples, "served": served_out}
    svc, plain = run_plain(B, ctx, reqs)
    import numpy as np
    plain_lat = list(np.cumsum(svc))  # all submitted at time 0, served in order
    return {
        "workload": f"{n_req} Gaussian-mixture requests, D 2..16, N_ev 1e4..1e6 log-uniform, 1-4 terms, "
                    "10 iterations, N_g=500, fp64, all submitted at t=0 in one call (after a warm-up of one "
                    "iteration per kernel shape)",
        "samples": samples,
        "served": served_out,
        "plain": {"makespan_s": float(sum(svc)), "samples_per_s": samples / sum(svc), **lat_summary(plain_lat)},
        "max_diff_in_sdev": agreement(served, plain),
    }


def run_stream(B, W, ctx, n_req, loads, n_cal=300):
    """Poisson arrivals of the stream workload at fixed rates, run live twice
    per rate: submitted in real time to the continuous-batching server, and
    to the plain path (a worker that solves the requests with vp_integrate
    one at a time in arrival order, as they arrive).  The rates are the
    loads[0], loads[1], ... fractions of the plain path's capacity, 1 / (mean
    service time), measured beforehand on the first n_cal requests one by
    one; loads[0] is the headline, the others are summarised under by_load."""
    import threading

    import numpy as np
    reqs = W.served_stream(n_req=n_req, rate=1.0)
    unit = np.array([r.arrival for r in reqs])  # arrivals at rate 1
    cal, _ = run_plain(B, ctx, reqs[:n_cal])
    mean_svc = float(np.mean(cal))

    def serve(arr):
        srv = B.Server(ctx, max_slots=n_req)
        tickets = [None] * n_req

        def producer():
            t0 = time.perf_counter()
            for i, r in enumerate(reqs):
                d = arr[i] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(r.params, r.integrand)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        served = [srv.wait(t) for t in tickets]
        times = [srv.times(t) for t in tickets]
        st = srv.stats()
        srv.close()
        return served, [t[2] - t[0] for t in times], times, st

    def plain_live(arr):
        """One worker, first come first served, each request started when it
        has arrived and the previous one is done."""
        res, lat = [], []
        t0 = time.perf_counter()
        busy = 0.0
        for i, r in enumerate(reqs):
            d = arr[i] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            a = time.perf_counter()
            res.append(B.integrate(ctx, r.params, r.integrand))
            e = time.perf_counter()
            busy += e - a
            lat.append((e - t0) - arr[i])
        return res, lat, busy

    out = {}
    by = {}
    for k, load in enumerate(loads):
        rate = load / mean_svc
        arr = unit / rate
        print(f"  stream at {100 * load:.0f}% load ({rate:.0f}/s): served ...", file=sys.stderr, flush=True)
        served, lat, times, st = serve(arr)
        print(f"  stream at {100 * load:.0f}% load: plain ...", file=sys.stderr, flush=True)
        plain, plain_lat, busy = plain_live(arr)
        samples = sum(r["n_evals"] for r in served)
        span = max(t[2] for t in times) - min(t[0] for t in times)
        entry = {"rate_per_s": rate,
                 "served": {**lat_summary(lat), "span_s": span, "samples_per_s": samples / span,
                            "steps": st["steps"], "graph_launches": st["graph_launches"],
                            "graph_captures": st["graph_captures"], "peak_active": st["peak_active"],
                            "mem_peak_bytes": st["mem_peak"],
                            "scheduler_s": {q: st[q] for q in ("t_admit", "t_plan", "t_step", "t_retire")}},
                 "plain": {**lat_summary(plain_lat), "busy_s": busy, "utilisation": busy / (arr[-1] + plain_lat[-1])},
                 "max_diff_in_sdev": agreement(served, plain), "samples": samples}
        if k == 0:
            out = {"workload": f"{n_req} correlated-Gaussian requests (cond 100, scale 0.05), D 3..21, N_ev 1e5..1e7 "
                               f"log-uniform, 5-20 iterations, N_g=1000, fp64; Poisson arrivals at {rate:.1f}/s "
                               f"(plain path {100 * load:.0f}% busy at the mean service time of the first "
                               f"{n_cal} requests, {1e3 * mean_svc:.2f} ms); served and plain both run live",
                   **entry}
        else:
            by[f"{load:g}"] = entry
    if by:
        out["by_load"] = by
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=list(SLOTS_PER_SAMPLE))
    ap.add_argument("--n-ev", type=int, default=100_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the precision split and serving sections")
    ap.add_argument("--sections", default="split,batchfn,batch,stream",
                    help="extra sections to run after the headline steps (comma list of split, batchfn "
                         "(batched-integrand path), batch (served batch), stream)")
    ap.add_argument("--batch", type=int, default=4096, help="requests in the served batch")
    ap.add_argument("--stream", type=int, default=2000, help="requests in the Poisson stream")
    ap.add_argument("--no-plain", action="store_true",
                    help="served batch only, without the plain path's one-after-another comparison (for profiling)")
    ap.add_argument("--loads", default="0.8,0.5,0.95",
                    help="plain-path utilisations that set the stream rates (comma list; the first is the headline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the method's per-iteration "
              "state is sharded across GPUs only in the design notes, not built", file=sys.stderr)
        sys.exit(2)

    from paper_2009_05112_amd import _binding as B
    from paper_2009_05112_amd import workloads as W

    p, f = W.cfg_diag_d8(n_ev=args.n_ev, precision=args.precision)
    ctx = B.Context(0)
    gp = B.Problem(ctx, p.with_(n_iter=args.warmup + args.steps), f)
    gp.iterate(args.warmup)
    r0 = gp.result()
    gp.profile(True)
    gp.sync()
    # the K timed steps run as five consecutive runs (as equal as K allows),
    # each bracketed by stream synchronisation; value = all K steps' samples
    # over their summed time, beside the median of the five runs' rates
    n_runs = min(5, args.steps)
    bounds = [args.steps * r // n_runs for r in range(n_runs + 1)]
    wall, runs, prev = 0.0, [], r0["n_evals"]
    for r in range(n_runs):
        t0 = time.perf_counter()
        gp.iterate(bounds[r + 1] - bounds[r])
        gp.sync()
        dt_run = time.perf_counter() - t0
        wall += dt_run
        ev = gp.result()["n_evals"]
        runs.append((ev - prev) / dt_run)
        prev = ev
    r1 = gp.result()
    k_ms, k_n = gp.kernel_time(0)
    it_ms, it_n = gp.kernel_time(1)
    samples = r1["n_evals"] - r0["n_evals"]
    value = samples / wall
    per_launch = samples / max(k_n, 1)
    k_avg_s = k_ms / max(k_n, 1) / 1e3
    achieved = SLOTS_PER_SAMPLE[args.precision] * per_launch / k_avg_s
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "vegas+ D=8, three diagonal Gaussians exp(-100|x-c|^2), c=0.23/0.39/0.74, "
                               "normalised; N_ev=1e8 per iteration, N_g=1000, alpha=0.5, beta=0.75",
                   "dim": 8, "n_ev": args.n_ev, "n_g": 1000, "n_hc": gp.n_hc, "precision": args.precision},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / PEAK_VALU_SLOTS,
                     "traffic": measured_traffic(args.precision),
                     "kernel": "k_sample (fused sampling)", "kernel_ms": 1e3 * k_avg_s,
                     "slots_per_sample": SLOTS_PER_SAMPLE[args.precision]},
        "runs": {"count": n_runs, "steps_each": [bounds[r + 1] - bounds[r] for r in range(n_runs)],
                 "samples_per_s": runs, "median_samples_per_s": sorted(runs)[n_runs // 2]},
        "iteration_ms_device": it_ms / max(it_n, 1),
        "estimate": {"mean": r1["mean"], "sdev": r1["sdev"], "chi2_dof": r1["chi2"] / max(r1["dof"], 1),
                     "exact": 1.0},
    }
    gp.close()
    sections = set() if args.no_extra else set(x for x in args.sections.split(",") if x)
    if "split" in sections:
        print("precision split ...", file=sys.stderr, flush=True)
        line["precision_split"] = run_split(B, W, ctx, args.n_ev, 10)
    if "batchfn" in sections:
        print("batched-integrand path ...", file=sys.stderr, flush=True)
        line["batched_integrand"] = run_batch_path(B, W, ctx, args.n_ev, 5)
    serving, latency = {}, {}
    if "batch" in sections:
        print("served batch ...", file=sys.stderr, flush=True)
        serving["batch"] = b = run_batch(B, W, ctx, args.batch, plain_too=not args.no_plain)
        latency.update({"batch_p50_s": b["served"]["p50_s"], "batch_p99_s": b["served"]["p99_s"]})
        if "plain" in b:
            latency.update({"batch_plain_p50_s": b["plain"]["p50_s"], "batch_plain_p99_s": b["plain"]["p99_s"]})
    if "stream" in sections:
        print("served stream ...", file=sys.stderr, flush=True)
        serving["stream"] = t = run_stream(B, W, ctx, args.stream, [float(x) for x in args.loads.split(",") if x])
        latency.update({"stream_p50_s": t["served"]["p50_s"], "stream_p99_s": t["served"]["p99_s"],
                        "stream_plain_p50_s": t["plain"]["p50_s"], "stream_plain_p99_s": t["plain"]["p99_s"]})
    if serving:
        line["serving"] = serving
        line["latency"] = latency
    ctx.close()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, f)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
