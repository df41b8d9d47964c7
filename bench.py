#!/usr/bin/env python3
"""Throughput of the TIMEST hot path on one MI355X.

Default (the default line): the large workload.  One step is one pass of
the whole path, starting from edge arrays already resident in device memory:
  graph build (sorts + lists) -> for each motif: weights -> 10^8 samples
  (draw, validate, complete) -> reduction to the estimate.
Workload: 2,000,000 vertices, 100,000,000 edges (90M Chung-Lu gamma 2.0 +
10M reciprocated at +U{1..600} s, bursty Pareto(1.5) per-source times over
3e7 s, drawn on the device); scatter-gather and 6-chain at delta 86,400 s;
10^8 samples per motif, seed 1 (the 6-chain's weights need 128 bits).

The same JSON line carries: the roofline of the dominant kernel (the
sampler: its access-model bytes per launch over the average launch from HIP
events in the timed region) and of the level kernels of the weight builds,
the graph build and the root draws; the oracle's single-thread CPU throughput on
a bounded slice of the same workload; the batched-queue against one job per
launch (64 jobs); the serving loop's p50/p99 latency on a short Poisson
stream; and the medium workload's rate and sampler roofline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
STAGES = ["graph", "weights", "sample", "reduce", "roots", "levels"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-slice-days", type=float, default=1.0,
                    help="large: length (in delta) of the time slice the CPU baseline runs on")
    ap.add_argument("--cpu-samples", type=int, default=1_000_000,
                    help="oracle samples per motif in the CPU baseline (0: skip it)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="before timing, run a plain device copy of BYTES (3 times) so that "
                         "hardware counters can be scaled by a kernel of known traffic")
    ap.add_argument("--workload", choices=["medium", "large", "batched", "serving", "weights", "ablation", "trees",
                                           "family", "partial"],
                    default="large",
                    help="large: the 1e8-edge single-job path with every side leg (default); medium: "
                         "the 2e6-edge path alone; batched: 64 heterogeneous jobs, one launch per job "
                         "against the batched pass; serving: a Poisson query stream against the server; "
                         "partial: partial-order motifs")
    ap.add_argument("--legs", default="cpu,batched,serving,tiny,medium",
                    help="large: side legs to run after the timed steps (comma list of cpu, batched, "
                         "serving, tiny, medium; 'none' for profiling runs)")
    ap.add_argument("--large-traffic", default=os.path.join(ROOT, "profiles", "large_kernel_traffic.json"),
                    help="HBM bytes per launch of the large workload's kernels (JSON), if present")
    ap.add_argument("--weights-graph", choices=["medium", "serving"], default="serving",
                    help="weights: the medium graph, or the 5e8-edge serving graph")
    ap.add_argument("--weights-deltas", default="3600,86400")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="serving: size of the large resident graph relative to 5e8 edges")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="queries per second")
    ap.add_argument("--serve-budget-gb", type=float, default=0.0,
                    help="server budget; 0: free device memory after the graphs, less 4 GiB")
    ap.add_argument("--serve-cold", action="store_true",
                    help="serving: start the stream with an empty weight cache (default: every "
                         "(graph, motif, delta) set the stream uses is built first)")
    ap.add_argument("--serve-rates", default="",
                    help="serving: after the main stream, shorter open-loop streams at these rates "
                         "(queries/s, comma-separated) on a warm cache, for the server's capacity")
    ap.add_argument("--serve-sweep-seconds", type=float, default=10.0,
                    help="serving: length of each --serve-rates stream")
    ap.add_argument("--serve-check", type=int, default=12,
                    help="served queries re-run alone with tm_estimate and compared")
    ap.add_argument("--traffic-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the traffic file (--traffic) from two rocprofv3 --pmc runs of this "
                         "bench with --copy-calibration: FETCH_SIZE, then WRITE_SIZE")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "medium_kernel_traffic.json"),
                    help="HBM bytes per launch from rocprofv3 counters (JSON), if present")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.traffic_summarize:
        out = args.large_traffic if args.workload == "large" else args.traffic
        what = ("large (bench.py --workload large, one step)" if args.workload == "large"
                else "medium (bench.py --workload medium, one step)")
        return summarize_traffic(args.traffic_summarize[0], args.traffic_summarize[1], out,
                                 args.copy_calibration or (1 << 30), what)
    if args.workload == "batched":
        return batched(args)
    if args.workload == "serving":
        return serving(args)
    if args.workload == "weights":
        return weights_only(args)
    if args.workload == "large":
        return large(args)
    if args.workload == "ablation":
        return ablation(args)
    if args.workload == "trees":
        return trees(args)
    if args.workload == "family":
        return family(args)
    if args.workload == "partial":
        return partial(args)

    print(json.dumps(medium_run(args, args.steps, args.warmup, args.cpu_samples)), flush=True)


def medium_run(args, steps, warmup, cpu_samples):
    """The medium workload: one step is graph build + per motif weights,
    1e7 samples and the reduction; returns the JSON line as a dict."""
    import ctypes as C

    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    L = T.lib()
    L.tm_profile_enable.argtypes = [C.c_int]
    L.tm_profile_enable.restype = None

    class Profile(C.Structure):
        _fields_ = [("ms", C.c_double * len(STAGES)), ("launches", C.c_uint64 * len(STAGES))]

    L.tm_profile_read.argtypes = [C.POINTER(Profile), C.c_int]
    L.tm_sample_model_bytes.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64,
                                        C.c_void_p, C.POINTER(C.c_uint64)]

    log("generating the medium workload")
    g = W.medium_graph()
    cfg = W.MEDIUM
    k, seed = cfg["k"], cfg["seed"]
    motifs = [(name, T.make_motif(W.MOTIFS[name], delta)) for name, delta in cfg["motifs"]]
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    tt = torch.from_numpy(g.t).cuda()
    torch.cuda.synchronize()

    def step():
        # per motif one tm_estimate: weight build, sampling and reduction in
        # one call
        G = T.Graph(src, dst, tt, g.n)
        out = []
        for _, mo in motifs:
            res = T.estimate(G, mo, k, seed)
            out.append((res.estimate, res.std_error, res.n_valid, res.W.value))
        G.close()
        return out

    if args.copy_calibration > 0:
        a = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"warmup x{warmup}")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    prof = Profile()
    L.tm_profile_read(C.byref(prof), 1)
    # inside the timed region only the sampling kernel is bracketed by events
    # (its average launch is the roofline's denominator)
    L.tm_profile_stages(1 << STAGES.index("sample"))
    L.tm_profile_enable(1)
    log(f"timing x{steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        results = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    L.tm_profile_enable(0)
    L.tm_profile_read(C.byref(prof), 1)
    samples = len(motifs) * k * steps
    value = samples / elapsed
    sample_ms = prof.ms[STAGES.index("sample")] / steps
    sample_launches = prof.launches[STAGES.index("sample")] / steps
    # the stage breakdown: the same steps again with every stage timed
    # (outside the timed region)
    L.tm_profile_stages((1 << len(STAGES)) - 1)
    L.tm_profile_enable(1)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    L.tm_profile_enable(0)
    L.tm_profile_read(C.byref(prof), 1)
    stage_ms = {STAGES[i]: prof.ms[i] / steps for i in range(len(STAGES))}
    level_launches = prof.launches[STAGES.index("levels")] / steps
    log("stage ms per step", stage_ms)

    # Access-model bytes of the sampling kernel's launches in one step
    # (counting pass, outside the timed region: same draws).
    Gm = T.Graph(src, dst, tt, g.n)
    model_bytes = 0
    per_motif = []
    for (name, mo), r in zip(motifs, results):
        Wt = T.Weights(Gm, mo)
        b = C.c_uint64()
        rc = L.tm_sample_model_bytes(Wt.h, seed, 0, k, T._stream(), C.byref(b))
        assert rc == 0, L.tm_last_error()
        model_bytes += b.value
        est, se, nvalid, Wv = r
        per_motif.append(dict(motif=name, estimate=est, std_error=se,
                              rel_ci95=(1.96 * se / est) if est else None, valid=nvalid, W=Wv,
                              model_bytes=b.value))
        Wt.close()
    # ... and of the level kernels of one step's weight builds
    level_bytes = sum(T.weights_model_bytes(Gm, mo) for _, mo in motifs)
    Gm.close()
    # counter-measured bytes, valid only for the kernel source they were taken on
    traffic = load_traffic(args.traffic, "sample_kernel")
    level_traffic = load_traffic(args.traffic, "level_kernel")
    roofline = roofline_of("sample_kernel", model_bytes / sample_launches, sample_ms / sample_launches, traffic)
    # the weight builds' level kernels (times from the untimed stage run)
    level_ms = stage_ms["levels"]
    weights_roofline = roofline_of("level_kernel", level_bytes / level_launches if level_launches else 0,
                                   level_ms / level_launches if level_launches else None, level_traffic)

    cpu = None
    if cpu_samples > 0:
        cpu = cpu_baseline(g, cfg, cpu_samples)

    line = {
        "metric": "samples/s at <=5% rel. err; batched-queue vs one-job-per-launch; p99 latency",
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(elapsed * 1e3 / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "medium: 100000 vertices, 2000000 edges (Chung-Lu 2.1, bursty Pareto 1.5 "
                        "times over 1e7 s), 4-cycle and 4-star at delta 3600, 1e7 samples each, "
                        "seed 1; graph build + weights + sampling + reduction per step",
            "m": g.m, "n": g.n, "k_per_motif": k,
        },
        "stages_ms_per_step": {s: round(v, 3) for s, v in stage_ms.items()},
        "estimates": per_motif,
        "roofline": roofline,
        "weights_roofline": weights_roofline,
        "cpu_baseline": cpu,
    }
    return line


def batched(args):
    """64 estimation jobs of uneven graph size, motif, delta and budget, from
    resident graphs: one launch per job (tm_estimate each, the job's whole
    weights -> samples -> reduction) against one batched pass
    (tm_estimate_batch) with the autotuned schedule, and against the same
    pipeline recorded once into a HIP graph and replayed (tm_batch_plan_run,
    the reported value).  Same results required."""
    import torch

    from paper_2507_20441_amd import autotune
    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    jobs = W.batched_jobs()
    log(f"generating {len(jobs)} graphs")
    graphs = []
    for j in jobs:
        g = W.batched_graph(j)
        graphs.append(T.Graph(g.src, g.dst, g.t, g.n))
    motifs = [T.make_motif(W.MOTIFS[j["motif"]], j["delta"]) for j in jobs]
    ks = [j["k"] for j in jobs]
    seeds = [j["seed"] for j in jobs]
    total = sum(ks)

    def per_job():
        return [T.estimate(g, mo, k, s) for g, mo, k, s in zip(graphs, motifs, ks, seeds)]

    def batch():
        return T.estimate_batch(graphs, motifs, ks, seeds)

    log("tuning the batched schedule")
    ws = [T.Weights(g, mo) for g, mo in zip(graphs, motifs)]
    choice, times = autotune.tune(ws, ks, seeds, cus)
    for w in ws:
        w.close()
    log(f"schedule {choice}; timings ms {times}")
    log("recording the pipeline into a graph")
    t0 = time.perf_counter()
    plan = T.BatchPlan(graphs, motifs, ks, seeds)
    record_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(max(1, args.warmup)):
        ref = per_job()
        got = batch()
        rep = plan.run()

    def same_all(xs, ys):
        return all(a.acc2.value == b.acc2.value and a.n_valid == b.n_valid and a.estimate == b.estimate
                   for a, b in zip(xs, ys))

    same = same_all(ref, got) and same_all(ref, rep)
    assert same, "batched or replayed results differ from one-job-per-launch results"
    t_job, t_batch, t_graph = [], [], []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_job()
        torch.cuda.synchronize()
        t_job.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        batch()
        torch.cuda.synchronize()
        t_batch.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        rep = plan.run()
        torch.cuda.synchronize()
        t_graph.append(time.perf_counter() - t0)
        assert same_all(ref, rep), "a replay differs"
    plan.close()
    tj, tb, tgr = min(t_job), min(t_batch), min(t_graph)
    wide = sum(1 for r in got if r.flags & T.TM_F_WIDE)
    rel = [1.96 * r.std_error / r.estimate for r in got if r.estimate > 0]
    line = {
        "metric": "samples/s at <=5% rel. err; batched-queue vs one-job-per-launch; p99 latency",
        "value": round(total / tgr, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tgr * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "batched: 64 jobs, graphs log-uniform 1e4..5e6 edges (medium shape), "
                        "motifs uniform over 5, delta log-uniform 600..86400, k log-uniform 1e5..1e7; "
                        "resident graphs; weights + samples + reduction per job",
            "jobs": len(jobs), "edges_total": sum(j["m"] for j in jobs), "samples_total": total,
        },
        "one_job_per_launch": {"ms": round(tj * 1e3, 3), "samples_per_s": round(total / tj, 1)},
        "batched": {"ms": round(tb * 1e3, 3), "samples_per_s": round(total / tb, 1),
                    "schedule": {"tile": choice[0], "blocks": choice[1], "root_lds": choice[2]}},
        "graph_replay": {"ms": round(tgr * 1e3, 3), "samples_per_s": round(total / tgr, 1),
                         "record_ms": round(record_ms, 1)},
        "speedup": round(tj / tgr, 3),
        "speedup_eager_batch": round(tj / tb, 3),
        "bit_identical": same,
        "jobs_128bit": wide,
        "rel_ci95_max": max(rel) if rel else None,
        "autotune_ms": {",".join(str(x) for x in key): round(v, 3) for key, v in times.items()},
    }
    print(json.dumps(line), flush=True)


def serving(args):
    """Open-loop serving: Poisson arrivals submitted at their times to one
    server holding every graph resident; latency is measured by the server
    from submit to result.  A closed-loop pass over the first queries then
    compares the server's saturated throughput with one tm_estimate per
    query, and sampled served results are re-run alone for identity."""
    import threading

    import numpy as np
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    specs = W.serving_graph_specs(args.serve_scale)
    graphs = []
    t0 = time.perf_counter()
    for sp in specs:
        u, v, t = W.device_graph(sp["n"], sp["m"], 2.1, sp["seed"])
        torch.cuda.synchronize()
        graphs.append(T.Graph(u, v, t, sp["n"]))
        del u, v, t
        torch.cuda.empty_cache()
        log(f"graph n={sp['n']} m={sp['m']} built, {time.perf_counter() - t0:.1f} s")
    T.release_cached()  # the builds' temporaries go back to HIP before the budget is taken
    free = torch.cuda.mem_get_info()[0]
    budget = int(args.serve_budget_gb * 2**30) if args.serve_budget_gb > 0 else int(free - 4 * 2**30)
    queries = W.serving_queries(args.serve_seconds, args.serve_rate, len(graphs))
    motifs = {(q["motif"], q["delta"]): T.make_motif(W.MOTIFS[q["motif"]], q["delta"]) for q in queries}
    log(f"{len(queries)} queries over {args.serve_seconds} s; budget {budget / 2**30:.1f} GiB")

    def run(qs, open_loop, warm=False):
        srv = T.Server(budget)
        gids = [srv.add_graph(g) for g in graphs]
        warm_s = 0.0
        if warm:
            # resident weight tables: one zero-sample query per set the stream uses
            t_w = time.perf_counter()
            sets = sorted({(q["graph"], q["motif"], q["delta"]) for q in qs})
            for gi, name, delta in sets:
                srv.wait(srv.submit(gids[gi], motifs[(name, delta)], 0, 1))
            warm_s = time.perf_counter() - t_w
            log(f"{len(sets)} weight sets built in {warm_s:.1f} s")
        tickets = [None] * len(qs)
        ready = threading.Semaphore(0)
        res = [None] * len(qs)

        def collect():
            for i in range(len(qs)):
                ready.acquire()
                try:
                    res[i] = srv.wait(tickets[i])
                except T.TimestError as e:
                    res[i] = (None, str(e))
                if (i + 1) % 250 == 0:
                    log(f"{i + 1} results")

        th = threading.Thread(target=collect)
        th.start()
        start = time.perf_counter()
        for i, q in enumerate(qs):
            if open_loop:
                delay = start + q["at"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            tickets[i] = srv.submit(gids[q["graph"]], motifs[(q["motif"], q["delta"])], q["k"], q["seed"])
            ready.release()
        th.join()
        wall = time.perf_counter() - start
        st = srv.stats()
        st["warmup_s"] = round(warm_s, 3)
        srv.close()
        return res, st, wall

    log("open loop")
    res, st, wall = run(queries, True, warm=not args.serve_cold)
    errors = sorted({info for r, info in res if r is None})
    ok = [(r, info) for r, info in res if r is not None]
    if errors:
        log(f"{len(res) - len(ok)} queries failed: {errors[:3]}")
    lat = np.array([info.latency_ms for _, info in ok])
    qd = np.array([info.queued_ms for _, info in ok])
    total = sum(q["k"] for q, (r, _) in zip(queries, res) if r is not None)
    # closed loop: the same first queries all at once, then one tm_estimate each
    n_cl = min(len(queries), 400)
    cl = queries[:n_cl]
    cl_res, cl_st, cl_wall = run(cl, False)
    cl_total = sum(q["k"] for q in cl)
    log("one tm_estimate per query")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    alone = [T.estimate(graphs[q["graph"]], motifs[(q["motif"], q["delta"])], q["k"], q["seed"]) for q in cl]
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t1
    same_cl = all(r is not None and a.acc2.value == r.acc2.value and a.n_valid == r.n_valid
                  and a.estimate == r.estimate for a, (r, _) in zip(alone, cl_res))
    rng = np.random.default_rng(7)
    served = [i for i, (r, _) in enumerate(res) if r is not None]
    pick = rng.choice(served, size=min(args.serve_check, len(served)), replace=False)
    same_open = True
    for i in pick:
        q = queries[i]
        a = T.estimate(graphs[q["graph"]], motifs[(q["motif"], q["delta"])], q["k"], q["seed"])
        r = res[i][0]
        same_open &= a.acc2.value == r.acc2.value and a.n_valid == r.n_valid and a.estimate == r.estimate
    assert same_cl and same_open, "served results differ from tm_estimate alone"
    rel = [1.96 * r.std_error / r.estimate for r, _ in ok if r.estimate > 0]
    # capacity: the offered rate raised until the served rate falls behind it
    sweep = []
    for rate in [float(x) for x in args.serve_rates.split(",") if x.strip()]:
        qs = W.serving_queries(args.serve_sweep_seconds, rate, len(graphs), seed=5000 + int(rate))
        for q in qs:
            key = (q["motif"], q["delta"])
            if key not in motifs:
                motifs[key] = T.make_motif(W.MOTIFS[q["motif"]], q["delta"])
        log(f"capacity: {len(qs)} queries at {rate}/s for {args.serve_sweep_seconds} s")
        s_res, s_st, s_wall = run(qs, True, warm=True)
        s_ok = [info for r, info in s_res if r is not None]
        s_lat = np.array([info.latency_ms for info in s_ok]) if s_ok else np.zeros(1)
        s_total = sum(q["k"] for q, (r, _) in zip(qs, s_res) if r is not None)
        offered = sum(q["k"] for q in qs) / args.serve_sweep_seconds
        sweep.append({"rate_qps": rate, "queries": len(qs), "failed": len(qs) - len(s_ok),
                      "offered_samples_per_s": round(offered, 1),
                      "served_samples_per_s": round(s_total / s_wall, 1),
                      "served_over_offered": round(s_total / s_wall / offered, 4) if offered else None,
                      "latency_ms": {"p50": float(np.percentile(s_lat, 50)),
                                     "p99": float(np.percentile(s_lat, 99)), "max": float(s_lat.max())},
                      "passes": s_st["passes"]})
        log(f"capacity: {json.dumps(sweep[-1])}")
    keeping_up = [x["rate_qps"] for x in sweep if x["failed"] == 0 and (x["served_over_offered"] or 0) >= 0.95]
    line = {
        "metric": "samples/s at <=5% rel. err; batched-queue vs one-job-per-launch; p99 latency",
        "value": round(total / wall, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(wall * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"serving: resident graphs {[(sp['n'], sp['m']) for sp in specs]}; Poisson "
                        f"{args.serve_rate}/s for {args.serve_seconds} s; motif uniform over 5, delta "
                        "uniform over {3600, 86400} on the large graph and over 8 values 600..86400 "
                        "on the others, k log-uniform 1e5..1e7",
            "queries": len(queries), "samples_total": total, "budget_bytes": budget,
            "weight_cache": "cold" if args.serve_cold else "warm (every set built before the stream)",
        },
        "failed_queries": len(res) - len(ok),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "max": float(lat.max())},
        "queued_ms": {"p50": float(np.percentile(qd, 50)), "p99": float(np.percentile(qd, 99))},
        "offered_samples_per_s": round(total / args.serve_seconds, 1),
        "server": st,
        "closed_loop": {"queries": n_cl, "served_samples_per_s": round(cl_total / cl_wall, 1),
                        "one_job_per_launch_samples_per_s": round(cl_total / seq_wall, 1),
                        "speedup": round(seq_wall / cl_wall, 3), "server": cl_st},
        "identical_alone_vs_mix": bool(same_cl and same_open),
        "rel_ci95_max": max(rel) if rel else None,
        "rel_ci95_median": float(np.median(rel)) if rel else None,
    }
    if sweep:
        line["capacity_sweep"] = {"seconds_per_rate": args.serve_sweep_seconds, "points": sweep,
                                  "highest_rate_kept_up_qps": max(keeping_up) if keeping_up else None}
    print(json.dumps(line), flush=True)
    for g in graphs:
        g.close()


def host_info():
    """The host the CPU baseline ran on: logical CPUs and the CPU model."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def load_traffic(path, key):
    """HBM bytes per launch of kernel `key` from a counter summary, or None
    when the kernel's sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    try:
        tr = json.load(open(path))
    except (OSError, ValueError):
        return None
    k = tr.get("kernels", {}).get(key)
    if not k or k.get("source_sha") != kernel_source_sha(k.get("source", "sample.hip")):
        return None
    return k.get("hbm_bytes_per_launch")


def roofline_of(kernel, bytes_per_launch, avg_ms, traffic):
    ach = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms and avg_ms > 0 else 0.0
    out = dict(bound="hbm", kernel=kernel, achieved=round(ach, 2), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(ach / HBM_PEAK_GBS, 5), traffic=traffic, bytes_per_launch=bytes_per_launch,
               avg_launch_ms=avg_ms)
    if traffic is not None and avg_ms:
        # the counter-measured HBM bytes over the same launch time
        out["traffic_frac"] = round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)
    return out


def large(args):
    """The large workload: 2e6 vertices, 1e8 edges (drawn on the device),
    scatter-gather and 6-chain at delta 86400, 1e8 samples each; a step is
    the graph build, both weight sets, both sampling runs and reductions.
    Inside the timed steps only the sampling kernels (the dominant kernel)
    and the level kernels are bracketed by HIP events; the full stage
    breakdown comes from a second, untimed run of the same steps."""
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    legs = set() if args.legs == "none" else set(x for x in args.legs.split(",") if x)
    log("generating the large workload on the device")
    u, v, t = W.large_graph_device()
    torch.cuda.synchronize()
    n = 2_000_000
    m = int(u.numel())
    motifs = [(name, T.make_motif(W.MOTIFS[name], d)) for name, d in W.LARGE["motifs"]]
    k, seed = W.LARGE["k"], W.LARGE["seed"]

    def step():
        g = T.Graph(u, v, t, n)
        out = []
        for name, mo in motifs:
            w = T.Weights(g, mo)
            r, _ = w.sample(seed, k)
            out.append((name, r, w.W, w.info()["wide"]))
            w.close()
        g.close()
        return out

    if args.copy_calibration > 0:
        a = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    T.profile_read(reset=True)
    T.profile_stages(["levels", "sample"])
    T.profile_enable(True)
    log(f"timing x{args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    T.profile_enable(False)
    prof = T.profile_read(reset=True)
    li, si = T.STAGES.index("levels"), T.STAGES.index("sample")
    level_ms = prof["ms"][li] / args.steps
    level_launches = prof["launches"][li] / args.steps
    sample_ms = prof["ms"][si] / args.steps
    sample_launches = prof["launches"][si] / args.steps
    # the stage breakdown: the same steps again with every stage timed
    nb = max(1, min(3, args.steps))
    T.profile_stages(None)
    T.profile_enable(True)
    for _ in range(nb):
        step()
    torch.cuda.synchronize()
    T.profile_enable(False)
    bd = T.profile_read(reset=True)
    stage_ms = {T.STAGES[i]: bd["ms"][i] / nb for i in range(len(T.STAGES))}
    stage_n = {T.STAGES[i]: bd["launches"][i] / nb for i in range(len(T.STAGES))}
    log("stage ms per step", {a: round(b, 3) for a, b in stage_ms.items()})
    # access-model bytes of one step's level kernels and sampling kernels
    # (counting variants, outside the timed region)
    g = T.Graph(u, v, t, n)
    level_bytes = sum(T.weights_model_bytes(g, mo) for _, mo in motifs)
    sample_bytes = 0
    for _, mo in motifs:
        w = T.Weights(g, mo)
        sample_bytes += T.sample_model_bytes(w, seed, k)
        w.close()
    g.close()
    traffic = args.large_traffic
    # the sampling kernels take the largest share of the step: the line's
    # roofline; the level kernels' is reported beside it
    roof = roofline_of("sample_kernel", sample_bytes / sample_launches if sample_launches else 0,
                       sample_ms / sample_launches if sample_launches else None,
                       load_traffic(traffic, "sample_kernel"))
    weights_roof = roofline_of("level_kernel", level_bytes / level_launches if level_launches else 0,
                               level_ms / level_launches if level_launches else None,
                               load_traffic(traffic, "level_kernel"))
    # graph build: the 76 B per edge the path must move (16 read: the edge;
    # about 60 written: eid order, out- and in-lists, multi-edge runs), over
    # the whole graph stage (its sorts are implementation bytes on top)
    g_n = stage_n["graph"]
    graph_roof = roofline_of("graph build (all kernels)", 76.0 * m, stage_ms["graph"] / g_n if g_n else None,
                             load_traffic(traffic, "graph_build"))
    graph_roof["bytes_per_edge"] = 76
    # root draws: per draw two 16 B guide entries and the 4 B key written;
    # the stage also holds the sort by root (reported in sort_bytes)
    r_n = stage_n["roots"]
    draws = len(motifs) * k
    roots_roof = roofline_of("root draws + sort", 36.0 * draws / r_n if r_n else 0,
                             stage_ms["roots"] / r_n if r_n else None, load_traffic(traffic, "root_kernel"))
    roots_roof["bytes_per_draw"] = 36
    roots_roof["root_kernel_traffic"] = roots_roof.pop("traffic")
    roots_roof.pop("traffic_frac", None)
    total = len(motifs) * k * args.steps
    line = {
        "metric": "samples/s at <=5% rel. err; batched-queue vs one-job-per-launch; p99 latency",
        "value": round(total / el, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "large: 2e6 vertices, 1e8 edges (90M Chung-Lu 2.0 + 10M reciprocated, bursty "
                               "times over 3e7 s, drawn on the device), scatter-gather and 6-chain at delta "
                               "86400, 1e8 samples each, seed 1; graph build + weights + sampling + reduction "
                               "per step",
                   "m": m, "n": n, "k_per_motif": k},
        "stages_ms_per_step": {a: round(b, 3) for a, b in stage_ms.items()},
        "estimates": [dict(motif=a, estimate=r.estimate, std_error=r.std_error,
                           rel_ci95=(1.96 * r.std_error / r.estimate) if r.estimate else None,
                           valid=r.n_valid, W=str(Wv), wide=wide) for a, r, Wv, wide in res],
        "roofline": roof,
        "weights_roofline": weights_roof,
        "graph_roofline": graph_roof,
        "roots_roofline": roots_roof,
    }
    cpu = None
    if "cpu" in legs and args.cpu_samples > 0:
        cpu = cpu_baseline_large(u, v, t, n, motifs, k, seed, args.cpu_slice_days, min(args.cpu_samples, 4000))
    line["cpu_baseline"] = cpu
    del u, v, t
    torch.cuda.empty_cache()
    if "batched" in legs:
        line["batched"] = batched_leg(args)
    if "serving" in legs:
        line["serving"] = serving_leg(args)
    if "tiny" in legs:
        line["tiny"] = tiny_leg()
    if "medium" in legs:
        med = medium_run(args, 10, 2, 0)
        line["medium"] = {"value": med["value"], "ms_per_step": med["ms_per_step"],
                          "stages_ms_per_step": med["stages_ms_per_step"], "roofline": med["roofline"],
                          "weights_roofline": med["weights_roofline"],
                          "estimates": [dict(motif=e["motif"], rel_ci95=e["rel_ci95"]) for e in med["estimates"]],
                          "workload": med["config"]["workload"]}
    print(json.dumps(line), flush=True)


def tiny_leg(reps=50):
    """The tiny configuration as a latency: one estimate call (graph build
    from device-resident edges, weights, 1e5 samples, reduction) on 1,000
    vertices and 20,000 edges, the 3-cycle at delta 1,000; p50/p99 over reps
    calls after 5 warm-ups, and the samples/s that p50 gives."""
    import numpy as np
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    g = W.tiny_graph()
    u, v, t = (torch.from_numpy(x).cuda() for x in (g.src, g.dst, g.t))
    name, delta = W.TINY["motifs"][0]
    mo = T.make_motif(W.MOTIFS[name], delta)
    k, seed = W.TINY["k"], W.TINY["seed"]

    def call():
        G = T.Graph(u, v, t, g.n)
        r = T.estimate(G, mo, k, seed)
        G.close()
        return r

    for _ in range(5):
        call()
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        a = time.perf_counter()
        r = call()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    lat = np.array(lat)
    p50 = float(np.percentile(lat, 50))
    return {"workload": f"tiny: {g.n} vertices, {g.m} edges, {name} at delta {delta}, {k} samples, seed {seed}; "
                        "graph build from device-resident edges + weights + sampling + reduction per call",
            "latency_ms": {"p50": round(p50, 3), "p99": round(float(np.percentile(lat, 99)), 3),
                           "calls": reps},
            "samples_per_s_at_p50": round(k / (p50 / 1e3), 1), "estimate": r.estimate,
            "rel_ci95": (1.96 * r.std_error / r.estimate) if r.estimate else None}


def cpu_baseline_large(u, v, t, n, motifs, k, seed, slice_days, n_samples):
    """The oracle, single-threaded, on a time slice of the large graph: the
    edges with time in [t0, t0 + slice_days * delta) (t0 at the middle of the
    span), its graph build, the weights of both motifs and n_samples samples
    each.  Scaled to the whole workload: the graph build by edges, the
    weights by intervals (the slice's weights cover one interval's share; the
    whole graph has q), the sampling by samples.  A slice's windows near its
    end hold fewer candidates than in the whole graph, so the scaled figure
    favours the oracle."""
    import numpy as np
    import torch

    import oracle as O

    delta = motifs[0][1].delta
    tmax = int(t.max().item())
    t0 = (tmax // 2 // delta) * delta
    t1 = t0 + int(slice_days * delta)
    sel = (t >= t0) & (t < t1)
    su, sv, st = (x[sel].cpu().numpy() for x in (u, v, t))
    ms = len(su)
    q = tmax // delta + 1
    log(f"cpu baseline: oracle on a {slice_days}-delta slice ({ms} edges), {n_samples} samples per motif")
    a = time.perf_counter()
    og = O.Graph(su, sv, st, n)
    t_graph = (time.perf_counter() - a) * (len(t) / max(1, ms))
    total = t_graph
    parts = []
    for name, mo in motifs:
        omo = O.make_motif([(mo.src[p], mo.dst[p]) for p in range(mo.l)], mo.delta)
        a = time.perf_counter()
        P = O.Prep(og, omo)
        b = time.perf_counter()
        P.sample(seed, k, j0=0, count=n_samples)
        c = time.perf_counter()
        # the slice's weights: one interval's share when slice_days <= 2
        share = max(1.0, slice_days / 2.0)
        w_est = (b - a) / share * q
        s_est = (c - b) * (k / n_samples)
        parts.append(dict(motif=name, weights_s_measured=round(b - a, 3), weights_s_scaled=round(w_est, 1),
                          samples_s_measured=round(c - b, 3), samples_s_scaled=round(s_est, 1)))
        total += w_est + s_est
        del P
    value = len(motifs) * k / total
    return dict(value=round(value, 3), unit="samples/s", cores=1, kind="oracle",
                sample=f"single-threaded oracle on the edges with time in [{t0}, {t1}) ({ms} of {len(t)} edges, "
                       f"{slice_days} delta at mid-span): graph build, weights of both motifs, {n_samples} of "
                       f"{k} samples each; scaled to the workload (graph by edges, weights by the {q} "
                       "intervals, sampling by samples); favours the oracle (truncated windows at the "
                       "slice's end)",
                host=host_info(), parts=parts, seconds_scaled=round(total, 1))


def batched_leg(args):
    """The batched workload's 64 jobs (graphs drawn on the device): one
    tm_estimate per job against the eager batch (tm_estimate_batch, autotuned
    schedule) and the recorded pipeline's replay; identical results required."""
    import torch

    from paper_2507_20441_amd import autotune
    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    jobs = W.batched_jobs()
    log(f"batched leg: {len(jobs)} graphs on the device")
    graphs = []
    for j in jobs:
        uu, vv, tt = W.device_graph(j["n"], j["m"], 2.1, j["graph_seed"])
        graphs.append(T.Graph(uu, vv, tt, j["n"]))
        del uu, vv, tt
    motifs = [T.make_motif(W.MOTIFS[j["motif"]], j["delta"]) for j in jobs]
    ks = [j["k"] for j in jobs]
    seeds = [j["seed"] for j in jobs]
    total = sum(ks)
    ws = [T.Weights(g, mo) for g, mo in zip(graphs, motifs)]
    choice, times = autotune.tune(ws, ks, seeds, cus)
    for w in ws:
        w.close()
    plan = T.BatchPlan(graphs, motifs, ks, seeds)

    def per_job():
        return [T.estimate(g, mo, kk, s) for g, mo, kk, s in zip(graphs, motifs, ks, seeds)]

    def same_all(xs, ys):
        return all(a.acc2.value == b.acc2.value and a.acc2_sq.value == b.acc2_sq.value and a.n_valid == b.n_valid
                   and a.estimate == b.estimate for a, b in zip(xs, ys))

    ref = per_job()
    got = T.estimate_batch(graphs, motifs, ks, seeds)
    rep = plan.run()
    same = same_all(ref, got) and same_all(ref, rep)
    tj, tb, tr = [], [], []
    for _ in range(3):
        for fn, acc in ((per_job, tj), (lambda: T.estimate_batch(graphs, motifs, ks, seeds), tb), (plan.run, tr)):
            torch.cuda.synchronize()
            a = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            acc.append(time.perf_counter() - a)
            same = same and same_all(ref, out)
    plan.close()
    for g in graphs:
        g.close()
    rel = [1.96 * r.std_error / r.estimate for r in got if r.estimate > 0]
    return {"workload": "batched: 64 jobs, graphs log-uniform 1e4..5e6 edges (medium shape, drawn on the device), "
                        "motifs uniform over 5, delta log-uniform 600..86400, k log-uniform 1e5..1e7",
            "samples_total": total, "edges_total": sum(j["m"] for j in jobs),
            "one_job_per_launch_samples_per_s": round(total / min(tj), 1),
            "eager_batch_samples_per_s": round(total / min(tb), 1),
            "replay_samples_per_s": round(total / min(tr), 1),
            "speedup_replay": round(min(tj) / min(tr), 3), "speedup_eager": round(min(tj) / min(tb), 3),
            "ms": {"one_job_per_launch": round(min(tj) * 1e3, 3), "eager_batch": round(min(tb) * 1e3, 3),
                   "replay": round(min(tr) * 1e3, 3)},
            "schedule": {"tile": choice[0], "samples_per_lane": choice[0] // 256, "blocks": choice[1],
                         "root_lds": choice[2]},
            "identical_to_one_job_per_launch": bool(same), "rel_ci95_max": max(rel) if rel else None}


def serving_leg(args, seconds=10.0, rate=200.0):
    """A short open-loop stream against the server: the eight 1e6-edge
    resident graphs of the serving workload, Poisson arrivals at `rate` for
    `seconds`, every weight set built first; latency is measured by the
    server from submit to result."""
    import threading

    import numpy as np
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    specs = W.serving_graph_specs()[1:]
    graphs = []
    for sp in specs:
        uu, vv, tt = W.device_graph(sp["n"], sp["m"], 2.1, sp["seed"])
        graphs.append(T.Graph(uu, vv, tt, sp["n"]))
        del uu, vv, tt
    torch.cuda.synchronize()
    qs = [dict(q, graph=q["graph"]) for q in W.serving_queries(seconds, rate, len(graphs))]
    motifs = {(q["motif"], q["delta"]): T.make_motif(W.MOTIFS[q["motif"]], q["delta"]) for q in qs}
    budget = int(torch.cuda.mem_get_info()[0] - 4 * 2**30)
    log(f"serving leg: {len(qs)} queries over {seconds} s on {len(graphs)} graphs")
    srv = T.Server(budget)
    gids = [srv.add_graph(g) for g in graphs]
    for gi, name, delta in sorted({(q["graph"], q["motif"], q["delta"]) for q in qs}):
        srv.wait(srv.submit(gids[gi], motifs[(name, delta)], 0, 1))
    tickets = [None] * len(qs)
    res = [None] * len(qs)
    ready = threading.Semaphore(0)

    def collect():
        for i in range(len(qs)):
            ready.acquire()
            try:
                res[i] = srv.wait(tickets[i])
            except T.TimestError:
                res[i] = None

    th = threading.Thread(target=collect)
    th.start()
    start = time.perf_counter()
    for i, q in enumerate(qs):
        delay = start + q["at"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets[i] = srv.submit(gids[q["graph"]], motifs[(q["motif"], q["delta"])], q["k"], q["seed"])
        ready.release()
    th.join()
    wall = time.perf_counter() - start
    st = srv.stats()
    srv.close()
    ok = [x for x in res if x is not None]
    lat = np.array([info.latency_ms for _, info in ok])
    served = sum(q["k"] for q, x in zip(qs, res) if x is not None)
    # a few served results against the same query alone
    same = True
    for i in range(0, len(qs), max(1, len(qs) // 8)):
        if res[i] is None:
            continue
        q = qs[i]
        a = T.estimate(graphs[q["graph"]], motifs[(q["motif"], q["delta"])], q["k"], q["seed"])
        same = same and a.acc2.value == res[i][0].acc2.value and a.estimate == res[i][0].estimate
    for g in graphs:
        g.close()
    return {"workload": f"serving (short): the eight 1e6-edge resident graphs of the serving workload, Poisson "
                        f"{rate}/s for {seconds} s, motif uniform over 5, delta over 8 values 600..86400, k "
                        "log-uniform 1e5..1e7, warm weight cache",
            "queries": len(qs), "failed": len(qs) - len(ok),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
            "served_samples_per_s": round(served / wall, 1), "offered_samples_per_s": round(served / seconds, 1),
            "passes": st["passes"], "identical_alone_vs_mix": bool(same)}


ABLATION_MODES = (("C1", 0), ("C1+2", 1), ("C1+3", 2), ("C1+2+3", 3))


def ablation(args):
    """Constraint ablation (the paper's Tab. "constraints" on synthetic data):
    per motif and constraint mode, the invalid-sample rate by cause, the
    valid rate, the estimate's error against the exact count (mean over five
    seeds; exact counts stored by tests/golden/make_ablation_counts.py), the
    95% half-width and the device time of weights + sampling; then the
    4-cycle on the medium graph (no exact count) at 1e7 samples."""
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    exact = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "ablation_counts.txt")):
        if line.startswith("count "):
            _, name, c = line.split()
            exact[name] = int(c)

    def run(tg, name, delta, k, seeds, c):
        mo = T.make_motif(W.MOTIFS[name], delta)
        out = []
        for seed in seeds:
            T.profile_read(reset=True)
            T.profile_enable(True)
            w = T.Weights(tg, mo, constraints=c)
            r, _ = w.sample(seed, k)
            torch.cuda.synchronize()
            T.profile_enable(False)
            ms = sum(T.profile_read(reset=True)["ms"])
            out.append((r, ms, w.W))
            w.close()
        return out

    def row(name, label, res, k, C=None):
        r0 = res[0][0]
        d = dict(motif=name, mode=label, W=str(res[0][2]),
                 invalid_vertex=r0.n_bad_vertex / k, invalid_delta=r0.n_bad_delta / k,
                 invalid_order=r0.n_bad_order / k, valid=r0.n_valid / k,
                 rel_ci95=(1.96 * r0.std_error / r0.estimate) if r0.estimate else None,
                 device_ms=round(sum(x[1] for x in res) / len(res), 3))
        if C is not None:
            d["exact"] = C
            d["mean_abs_rel_error"] = sum(abs(x[0].estimate - C) / C for x in res) / len(res)
        return d

    g = W.ablation_graph()
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    k, delta = W.ABLATION["k"], W.ABLATION["delta"]
    rows = []
    for name in W.ABLATION["motifs"]:
        for label, c in ABLATION_MODES:
            rows.append(row(name, label, run(tg, name, delta, k, range(1, 6), c), k, exact[name]))
            log(rows[-1])
    tg.close()
    mg = W.medium_graph()
    tm = T.Graph(mg.src, mg.dst, mg.t, mg.n)
    med = []
    for label, c in ABLATION_MODES:
        med.append(row("4cycle", label, run(tm, "4cycle", 3600, 10_000_000, (1,), c), 10_000_000))
        log(med[-1])
    tm.close()
    print(json.dumps({"workload": "constraint ablation: ablation graph (n=5000, m=200000, gamma 2.1, bursty "
                                  "over 3e6 s, delta 3600, 1e6 samples, 5 seeds) and the medium graph (4-cycle, "
                                  "delta 3600, 1e7 samples)", "ablation": rows, "medium": med}), flush=True)


def trees(args):
    """Tree choice (the paper's Tab. "SPTree" and Alg. 7 on synthetic data):
    for every (spanning tree, center) candidate of each ablation motif, its
    looseness, W, the error against the exact count (mean over five seeds)
    and the 95% half-width at 1e6 samples; and what tm_choose_tree picks from
    the first three candidates, with the time the choice takes."""
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    exact = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "ablation_counts.txt")):
        if line.startswith("count "):
            _, name, c = line.split()
            exact[name] = int(c)
    g = W.ablation_graph()
    tg = T.Graph(g.src, g.dst, g.t, g.n)
    k, delta = W.ABLATION["k"], W.ABLATION["delta"]
    out = []
    for name in W.ABLATION["motifs"]:
        mo = T.make_motif(W.MOTIFS[name], delta)
        C = exact[name]
        cands = []
        for tr, loose in T.tree_candidates(mo):
            w = T.Weights(tg, mo, tr)
            res = [w.sample(seed, k)[0] for seed in range(1, 6)]
            cands.append(dict(tree=list(tr.edge[:tr.n_edges]), center=tr.center, looseness=loose, W=str(w.W),
                              mean_abs_rel_error=sum(abs(r.estimate - C) / C for r in res) / len(res),
                              rel_ci95=(1.96 * res[0].std_error / res[0].estimate) if res[0].estimate else None))
            w.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        best, Ws = T.choose_tree(tg, mo, 3)
        torch.cuda.synchronize()
        choose_ms = (time.perf_counter() - t0) * 1e3
        out.append(dict(motif=name, exact=C, candidates=cands,
                        chosen=dict(tree=list(best.edge[:best.n_edges]), center=best.center),
                        choose_n_c=3, choose_ms=round(choose_ms, 3)))
        log(name, "chosen", out[-1]["chosen"], "in", round(choose_ms, 2), "ms")
    tg.close()
    print(json.dumps({"workload": "tree choice on the ablation graph (delta 3600, 1e6 samples, 5 seeds)",
                      "motifs": out}), flush=True)


FAMILY_TREE = ((0, 1), (1, 2), (2, 3))
FAMILY = (((0, 1), (1, 2), (2, 3), (3, 0)), ((0, 1), (1, 2), (2, 3), (3, 1)), ((0, 1), (1, 2), (2, 0), (2, 3)),
          ((3, 0), (0, 1), (1, 2), (2, 3)))


def family(args):
    """A family of four 4-vertex motifs sharing the path a->b->c->d as their
    tree (the paper counts its 4-vertex motifs at once): one weight build and
    one stream of 1e7 tree samples completed for all four (tm_sample_family)
    against one tm_estimate per motif with the same tree and seed; then
    random instance listing of 1e7 samples of the 4-cycle."""
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    mg = W.medium_graph()
    g = T.Graph(mg.src, mg.dst, mg.t, mg.n)
    delta, k, seed = 3600, 10_000_000, 1
    mos = [T.make_motif(e, delta) for e in FAMILY]
    trees = []
    for e in FAMILY:
        idx = [list(e).index(x) for x in FAMILY_TREE]
        trees.append(T.make_tree(idx, idx[1]))
    tree_motif = T.make_motif(FAMILY_TREE, delta)

    def fam():
        w = T.Weights(g, tree_motif, T.make_tree([0, 1, 2], 1))
        out = T.sample_family(w, mos, seed, k)
        w.close()
        return out

    def sep():
        return [T.estimate(g, mo, k, seed, tr) for mo, tr in zip(mos, trees)]

    a, b = fam(), sep()
    same = all(x.acc2.value == y.acc2.value and x.n_valid == y.n_valid and x.estimate == y.estimate
               for x, y in zip(a, b))
    assert same, "family results differ from separate runs"
    tf, ts = [], []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fam()
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        sep()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    w = T.Weights(g, T.make_motif(W.MOTIFS["4cycle"], delta))
    T.list_instances(w, seed, 1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows, recs = T.list_instances(w, seed, k)
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    listed = int((rows[:, 0] >= 0).sum())
    w.close()
    g.close()
    line = {
        "workload": "motif family on the medium graph: 4 motifs on the tree a->b->c->d, delta 3600, 1e7 samples",
        "family_ms": round(min(tf) * 1e3, 3), "separate_ms": round(min(ts) * 1e3, 3),
        "speedup": round(min(ts) / min(tf), 3), "identical": same,
        "estimates": [dict(motif=[list(x) for x in e], estimate=r.estimate,
                           rel_ci95=(1.96 * r.std_error / r.estimate) if r.estimate else None)
                      for e, r in zip(FAMILY, a)],
        "listing": {"samples": k, "listed": listed, "ms_incl_host_copy": round(tl * 1e3, 3)},
    }
    print(json.dumps(line), flush=True)


def partial(args):
    """Partial-order motifs on the medium graph (1e7 samples each, delta
    3600): per motif, the weight build and the sampling timed with the
    library's stage events, the samples/s of the whole estimate, the
    sampler's access-model roofline and the 95% half-width; next to each,
    the same edges under their listed total order."""
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    mg = W.medium_graph()
    g = T.Graph(mg.src, mg.dst, mg.t, mg.n)
    k, seed, delta = 10_000_000, 1, 3600
    rows = []
    for name in ("po_fan3", "po_cycle3", "po_sg", "po_free2", "po_diamond"):
        edges, before = W.PO_MOTIFS[name]
        for order, mo in (("partial", T.make_motif(edges, delta, before=before)),
                          ("total", T.make_motif(edges, delta))):
            for _ in range(max(1, args.warmup)):
                T.estimate(g, mo, k, seed)
            torch.cuda.synchronize()
            T.profile_read(reset=True)
            T.profile_enable(True)
            best = None
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                a = time.perf_counter()
                r = T.estimate(g, mo, k, seed)
                torch.cuda.synchronize()
                dt = time.perf_counter() - a
                best = dt if best is None else min(best, dt)
            T.profile_enable(False)
            pr = T.profile_read(reset=True)
            si = T.STAGES.index("sample")
            w = T.Weights(g, mo)
            mb = T.sample_model_bytes(w, seed, k)
            W_ = w.W
            w.close()
            s_ms = pr["ms"][si] / max(1, pr["launches"][si])
            rows.append(dict(motif=name, order=order, samples_per_s=round(k / best, 1), ms=round(best * 1e3, 3),
                             weights_ms=round(pr["ms"][T.STAGES.index("weights")] / max(1, args.steps), 3),
                             sample_roofline=roofline_of("sample_kernel", mb, s_ms, None),
                             W=str(W_), valid=r.n_valid / k, estimate=r.estimate,
                             rel_ci95=(1.96 * r.std_error / r.estimate) if r.estimate else None))
            log(rows[-1])
    g.close()
    print(json.dumps({"workload": "partial-order motifs on the medium graph (delta 3600, 1e7 samples each); "
                                  "each next to its edges under the listed total order", "motifs": rows}),
          flush=True)


def weights_only(args):
    """Weight builds alone (tm_weights_create) for every motif at each delta,
    timed with the library's stage events, plus 1e6 samples each as a check."""
    import torch

    from paper_2507_20441_amd import timest as T
    from paper_2507_20441_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    torch.cuda.set_device(0)
    if args.weights_graph == "serving":
        sp = W.serving_graph_specs(args.serve_scale)[0]
        u, v, t = W.device_graph(sp["n"], sp["m"], 2.1, sp["seed"])
        g = T.Graph(u, v, t, sp["n"])
        del u, v, t
        torch.cuda.empty_cache()
    else:
        mg = W.medium_graph()
        g = T.Graph(mg.src, mg.dst, mg.t, mg.n)
    T.profile_enable(True)
    rows = []
    for delta in [int(x) for x in args.weights_deltas.split(",")]:
        for name in W.MOTIFS:
            mo = T.make_motif(W.MOTIFS[name], delta)
            best = None
            for _ in range(max(1, args.steps)):
                T.profile_read(reset=True)
                w = T.Weights(g, mo)
                ms = T.profile_read(reset=True)["ms"][1]
                info = w.info()
                r, _ = w.sample(1, 1_000_000)
                w.close()
                best = ms if best is None else min(best, ms)
            rows.append(dict(motif=name, delta=delta, ms=round(best, 3), bytes=info["bytes"],
                             wide=info["wide"], W=str(info["W"]), valid_of_1e6=int(r.n_valid)))
            log(f"{name} delta={delta}: {best:.2f} ms, {info['bytes'] / 2**30:.2f} GiB, wide {info['wide']}")
    print(json.dumps({"workload": f"weights on the {args.weights_graph} graph (m={g.m})", "builds": rows}),
          flush=True)
    g.close()


# Kernels whose HBM traffic the summaries record: a name test on the demangled
# kernel name and the source file whose hash keys the figure.  Counting
# variants (second template argument true) are left out.
def _targs(name):
    a = name.find("<")
    b = name.rfind(">")
    return [x.strip() for x in name[a + 1:b].split(",")] if a >= 0 and b > a else []


TRAFFIC_KERNELS = {
    "sample_kernel": (lambda nm: "sample_kernel<" in nm and "batch_" not in nm and _targs(nm)[1:2] == ["false"],
                      "sample.hip"),
    "root_kernel": (lambda nm: "root_kernel<" in nm and "batch_" not in nm, "sample.hip"),
    "level_kernel": (lambda nm: "level_kernel<" in nm and _targs(nm)[1:2] == ["false"], "weights.hip"),
}


def summarize_traffic(fetch_dir, write_dir, out_path, calib_bytes, workload):
    """HBM bytes per launch of the main kernels from rocprofv3 counter CSVs:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the same
    counter reads for a device copy of calib_bytes in the same run; a key's
    figure is the mean over every launch of the kernels it covers."""
    import csv
    import glob
    import statistics

    def rows(d):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        assert f, f"no counter file under {d}"
        return list(csv.DictReader(open(f[0])))

    def per_kernel(rs):
        out = {}
        for r in rs:
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fk, wk = per_kernel(rows(fetch_dir)), per_kernel(rows(write_dir))
    copy = [n for n in fk if "copyBuffer" in n]
    assert copy, "no copy kernel: run the bench with --copy-calibration"
    # the calibration copies are the largest copies of the run (the library's
    # own device copies, and PyTorch's when it draws a graph on the device,
    # run the same kernel on fewer bytes)
    f_cal = max(fk[copy[0]])
    w_cal = max(wk[copy[0]])
    f_scale = calib_bytes / 1024.0 / f_cal
    w_scale = calib_bytes / 1024.0 / w_cal
    kernels = {}
    for key, (test, src) in TRAFFIC_KERNELS.items():
        fv = [x for nm, vs in fk.items() if test(nm.replace("(anonymous namespace)::", "")) for x in vs]
        wv = [x for nm, vs in wk.items() if test(nm.replace("(anonymous namespace)::", "")) for x in vs]
        if not fv or not wv:
            continue
        names = sorted({nm.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
                        for nm in fk if test(nm.replace("(anonymous namespace)::", ""))})
        fb = statistics.mean(fv) * 1024 * f_scale
        wb = statistics.mean(wv) * 1024 * w_scale
        kernels[key] = dict(names=names, source=src, source_sha=kernel_source_sha(src), launches=len(fv),
                            fetch_bytes_per_launch=round(fb), write_bytes_per_launch=round(wb),
                            hbm_bytes_per_launch=round(fb + wb))
    # the graph build as a whole: every kernel only it launches, summed over
    # a build (builds counted by the validation kernel); the digit counts,
    # shared with the root sorts by name, are left out (a few percent)
    def graph_test(nm):
        nm = nm.replace("(anonymous namespace)::", "")
        return any(k in nm for k in ("validate_kernel(", "validate_reduce_kernel(", "canon_keys_kernel(",
                                     "decode_packed_kernel(", "decode_split_kernel(", "tpos_kernel(",
                                     "n_order_fix_kernel(", "offsets_kernel(")) or \
            ("sort_pass_kernel<" in nm and "sort_pass_kernel<unsigned int, unsigned int," not in nm)
    builds = sum(len(vs) for nm, vs in fk.items() if "validate_kernel(" in nm.replace("(anonymous namespace)::", ""))
    if builds:
        fb = sum(x for nm, vs in fk.items() if graph_test(nm) for x in vs) * 1024 * f_scale / builds
        wb = sum(x for nm, vs in wk.items() if graph_test(nm) for x in vs) * 1024 * w_scale / builds
        kernels["graph_build"] = dict(names=sorted({nm.replace("(anonymous namespace)::", "").replace("void ", "")
                                                    .split("(")[0] for nm in fk if graph_test(nm)}),
                                      source="csr.hip", source_sha=kernel_source_sha("csr.hip"), launches=builds,
                                      per="build", fetch_bytes_per_launch=round(fb), write_bytes_per_launch=round(wb),
                                      hbm_bytes_per_launch=round(fb + wb))
    doc = {
        "workload": workload,
        "copy_calibration": {"bytes": calib_bytes, "fetch_kib": f_cal, "write_kib": w_cal,
                             "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
        "kernels": kernels,
        "commands": [
            "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch> -o fetch "
            "-- python3 <repo>/bench.py --workload <w> --steps 1 --warmup 0 --cpu-samples 0 --legs none "
            "--copy-calibration 1073741824",
            "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write> -o write "
            "-- python3 <repo>/bench.py --workload <w> --steps 1 --warmup 0 --cpu-samples 0 --legs none "
            "--copy-calibration 1073741824",
            "python3 bench.py --workload <w> --traffic-summarize <fetch> <write>",
        ],
    }
    with open(out_path, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps({k: v["hbm_bytes_per_launch"] for k, v in kernels.items()}))


def kernel_source_sha(main="sample.hip"):
    """Hash of the sampling kernel's sources (the counters' validity key)."""
    import hashlib
    h = hashlib.sha256()
    for f in (main, "tm_common.h", "tm_primitives.h", "tm_internal.h"):
        with open(os.path.join(ROOT, "paper_2507_20441_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(g, cfg, n_samples):
    """The oracle, single-threaded, on the same workload: full graph build and
    weights, then n_samples of the k samples per motif; the sampling time is
    scaled linearly to k (samples are independent)."""
    import oracle as O
    from paper_2507_20441_amd import workloads as W
    log(f"cpu baseline: oracle, {n_samples} samples per motif")
    t0 = time.perf_counter()
    og = O.Graph(g.src, g.dst, g.t, g.n)
    t_graph = time.perf_counter() - t0
    total = t_graph
    k = cfg["k"]
    for name, delta in cfg["motifs"]:
        t1 = time.perf_counter()
        P = O.Prep(og, O.make_motif(W.MOTIFS[name], delta))
        t2 = time.perf_counter()
        P.sample(cfg["seed"], k, j0=0, count=n_samples)
        t3 = time.perf_counter()
        total += (t2 - t1) + (t3 - t2) * (k / n_samples)
    value = len(cfg["motifs"]) * k / total
    return dict(value=round(value, 1), unit="samples/s", cores=1, kind="oracle",
                sample=f"full graph build and weights for both motifs, {n_samples} of {k} samples "
                       f"per motif; sampling time scaled linearly to {k}")


if __name__ == "__main__":
    main()
