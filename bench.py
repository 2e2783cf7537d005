"""Benchmark: applied SSA events per second on one MI355X.

Headline workload (one "step" = the whole hot path over one batch): the
batched parameter sweep -- the gene-regulation model (two compartments, 10
species, 20 rules, four across the nuclear membrane) in 4096 instances whose
kinetic constants are scaled by a per-instance factor 10^U(-1,1), 64
replicas each (262144 trajectories, ~100x spread of events per trajectory),
simulated to t = 100 with 201 sample points and reduced on line into
per-instance, per-sample mean/variance.  Inputs are resident on the device
before the timed region.  `value` is the batched persistent form (resident
grid, lane refill from a longest-first work queue, replayed as a HIP graph,
autotuned launch shape); the plain one-lane-per-trajectory launch is timed
on the same inputs beside it.  Also reported: the 16384-replica
gene-regulation run in both forms, the 32-cell multi-compartment run, the
serving trace (continuous batching, p50/p99 latency), the VALU roofline of
the headline kernel and the CPU oracle on the host cores.

Prints one JSON line.  ``--gpus`` above 1 is refused: the benchmark runs
on one GPU.
"""
import argparse
import json
import re
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSA events/sec on 1 GPU (batched persistent vs plain launch); p99 job latency"
PEAK_VALU_SLOTS = 256 * 4 * 16 * 2.4e9     # CUs x SIMDs x lanes x clock = 3.93e13/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_form(ctx, model, run, mode, steps, warmup, stream, tuning=None, e2e=False):
    """Warm up, then time exactly `steps` launches bracketed by device
    synchronisation; per-launch simulation time from the library's HIP events
    on the launch stream.  With e2e, also one untimed-for-`value` cycle from
    host tables to host statistics (submission with table upload, the run,
    mean/variance/n copied back), wall clock."""
    import torch
    from paper_1010_2438_amd import Run
    r = Run(ctx, model, run, mode=mode, stream=stream, tuning=tuning)
    r.wait()
    for _ in range(warmup):
        r.relaunch(stream)
        r.wait()
    events = int(r.counters()["events"].sum())
    torch.cuda.synchronize()
    sims = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r.relaunch(stream)
        r.wait()
        sims.append(r.elapsed_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mean, var, n = r.stats()
    kernel = r.kernel_name()
    r.close()
    sim_ms = sum(s[0] for s in sims) / len(sims)
    tot_ms = sum(s[1] for s in sims) / len(sims)
    out = {"kernel": kernel, "events_per_step": events, "ms_per_step": 1e3 * wall / steps,
           "events_per_s": events * steps / wall, "kernel_ms": sim_ms,
           "launch_ms": tot_ms, "finite_mean": bool((mean == mean).all())}
    if e2e:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = Run(ctx, model, run, mode=mode, stream=stream, tuning=tuning)
        r.wait()
        mean, var, n = r.stats()
        wall = time.perf_counter() - t0
        r.close()
        out["host_to_host_ms"] = 1e3 * wall
        out["host_to_host_events_per_s"] = events / wall
    return out


def cpu_baseline(model, run, budget_s=15.0):
    """The oracle (plain C direct method) on the host cores over a bounded
    sample of the same workload: replica 0 of every s-th instance, s chosen
    for about `budget_s` seconds of work, the instances spread over the
    whole sweep (events per trajectory vary ~100x across it)."""
    import numpy as np
    import oracle
    threads = min(16, os.cpu_count() or 1)
    I, R = run["n_instances"], run["replicas"]
    fm = oracle.FlatModel(model)

    def sample(stride):
        ids = list(range(0, I, stride))
        t0 = time.perf_counter()
        import threading
        evs = [0] * len(ids)

        def work(k):
            for q in range(k, len(ids), threads):
                g = ids[q] * R
                r = oracle.simulate(model, run, g0=g, g1=g + 1, want_stats=False, flat=fm)
                evs[q] = int(r["events"][0])

        ts = [threading.Thread(target=work, args=(k,)) for k in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        return len(ids), sum(evs), time.perf_counter() - t0

    n, ev, dt = sample(256)                                  # probe: 16 trajectories
    rate = ev / max(dt, 1e-6) * threads / min(threads, n)    # events/s with all threads busy
    n_want = budget_s * rate / max(ev / n, 1.0)
    stride = max(1, int(I / max(n_want, 1.0)))
    n, ev, dt = sample(stride)
    return {"value": ev / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": "replica 0 of every %d-th of %d instances (%d trajectories, %d events, "
                      "%.1f s)" % (stride, I, n, ev, dt)}


def serve_trace(ctx, n_jobs, time_scale, budget, slice_events=4096, max_active=64):
    """Replays the first n_jobs of the serving trace (Poisson arrivals, mixed
    configurations 0-3, 64..8192 replicas, t_end 5..100) against the
    continuous-batching server; arrival times are multiplied by time_scale.
    Returns latency percentiles (submit -> statistics ready) and rates."""
    import threading
    import numpy as np
    import workloads as W
    from paper_1010_2438_amd import Model, Server
    trace = W.arrival_trace()[:n_jobs]
    models = {0: W.lotka_volterra(), 1: W.gene_regulation(1), 3: W.multi_compartment(3)}
    models[2] = models[1]
    mo = {}
    for c, m in models.items():
        key = id(m)
        if key not in mo:
            mo[key] = Model(ctx, m)
    tab, _ = W.sweep_rate_table(models[1], 4096, 2)
    srv = Server(ctx, hbm_budget=budget, max_active=max_active, slice_events=slice_events)

    def run_of(job):
        c = job["config"]
        if c == 2:
            ni = (job["replicas"] + 63) // 64
            lo = (job["job"] * 37) % (4096 - ni)
            return W.make_run(seed=job["seed"], n_instances=ni, replicas=64, dt=job["dt"],
                              n_samples=job["n_samples"], rate_table=tab[lo:lo + ni],
                              count_cap=job["count_cap"])
        return W.make_run(seed=job["seed"], replicas=job["replicas"], dt=job["dt"],
                          n_samples=job["n_samples"], count_cap=job["count_cap"])

    runs = [run_of(j) for j in trace]
    ids = [None] * len(trace)
    t_start = time.perf_counter()
    err = []

    def submitter():
        try:
            for i, job in enumerate(trace):
                target = job["arrival_s"] * time_scale
                dt = target - (time.perf_counter() - t_start)
                if dt > 0:
                    time.sleep(dt)
                ids[i] = srv.submit(mo[id(models[job["config"]])], runs[i])
        except Exception as e:       # surfaced below
            err.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    infos = {}
    last = time.perf_counter()
    while len(infos) < len(trace):
        if err:
            raise err[0]
        for jid in srv.poll():
            infos[jid] = srv.info(jid)
            srv.release(jid)
        if time.perf_counter() - last > 10.0:
            last = time.perf_counter()
            log("  serving: %d/%d jobs done after %.0f s" % (len(infos), len(trace),
                                                          last - t_start))
        time.sleep(0.001)
    th.join()
    wall = time.perf_counter() - t_start
    st = srv.server_stats()
    srv.close()
    lat = np.array([infos[j]["t_done"] - infos[j]["t_submit"] for j in ids])
    ev = sum(infos[j]["events"] for j in ids)
    span = trace[-1]["arrival_s"] * time_scale
    return {"jobs": len(trace), "arrival_span_s": span,
            "offered_jobs_per_s": len(trace) / max(span, 1e-9),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "max_latency_s": float(lat.max()),
            "events": int(ev), "achieved_events_per_s": ev / wall,
            "offered_events_per_s": ev / max(span, 1e-9),
            "makespan_s": wall, "ticks": st["ticks"],
            "hbm_budget_bytes": st["pool_bytes"], "pool_peak_bytes": st["pool_peak"]}


def fnv1a64(text):
    h = 0xcbf29ce484222325
    for b in text.encode():
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return "%016x" % h


def measured_traffic(source, kernel):
    """HBM bytes per launch of the headline kernel from its committed counter
    summary (profiles/<kernel>_gene_regulation_sweep_i4096_r64.md), only if
    the counters were taken on this exact kernel (same generated source);
    else None."""
    path = os.path.join(ROOT, "profiles", "%s_gene_regulation_sweep_i4096_r64.md" % kernel)
    try:
        text = open(path).read()
    except OSError:
        return None
    fig = dict(re.findall(r"^(source_fnv1a64|traffic_bytes_per_launch): (\S+)$", text, re.M))
    if fig.get("source_fnv1a64") != fnv1a64(source) or "traffic_bytes_per_launch" not in fig:
        return None
    return int(fig["traffic_bytes_per_launch"])


def parse_tuning(text):
    """BLOCK,WAVES_PER_SIMD[,REFILL_CHUNK[,SLOTS[,LANES_PER_REPLICA]]]"""
    v = [int(x) for x in text.split(",")]
    return {"block_size": v[0], "waves_per_simd": v[1],
            "refill_chunk": v[2] if len(v) > 2 else 0,
            "sample_slots": v[3] if len(v) > 3 else 0,
            "lanes_per_replica": v[4] if len(v) > 4 else 1}


def single_workload(ctx, stream, args):
    """One workload's persistent form alone (autotuned unless --tuning is
    given), with the roofline of its kernel, as one JSON line."""
    import workloads as W
    from paper_1010_2438_amd import Model
    m, run = W.config(args.workload)
    model = Model(ctx, m)
    alg = model.info["alg_slots_per_event"]
    tun = parse_tuning(args.tuning) if args.tuning else \
        model.autotune(run, "persistent", budget_s=2.0)
    res = time_form(ctx, model, run, "persistent", args.steps, args.warmup, stream, tun)
    achieved = res["events_per_step"] * alg / (res["kernel_ms"] * 1e-3)
    print(json.dumps({
        "workload": W.CONFIG_NAMES[args.workload], "form": "persistent",
        "events_per_s": res["events_per_s"], "ms_per_step": res["ms_per_step"],
        "kernel_ms": res["kernel_ms"], "events_per_step": res["events_per_step"],
        "steps": args.steps, "warmup": args.warmup, "tuning": tun,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": PEAK_VALU_SLOTS / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_VALU_SLOTS, "kernel": res["kernel"],
                     "work_unit": "%.1f VALU issue slots per applied event" % alg}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=150)
    ap.add_argument("--only-headline", action="store_true",
                    help="time only the headline kernel (for profiler runs)")
    ap.add_argument("--tuning", default="",
                    metavar="BLOCK,WAVES_PER_SIMD[,REFILL_CHUNK[,SLOTS[,LANES_PER_REPLICA]]]",
                    help="pin the launch shape (of the headline, or of --workload) instead of autotuning it")
    ap.add_argument("--workload", type=int, default=0, choices=(0, 1, 3),
                    help="time only the persistent form of workload 1 (gene regulation, "
                         "16384 replicas) or 3 (multi-compartment, 2048 replicas) and print "
                         "its own line (for profiler runs); 0 = the full benchmark")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="copy BYTES device-to-device 5 times and exit (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes_per_launch": args.copy_calibration}))
        return
    if args.only_headline:
        args.no_extra = args.no_serve = args.no_cpu = True
    if args.gpus != 1:
        print("bench.py: the simulator runs on one GPU; --gpus %d is not supported "
              "(a multi-GPU run would shard trajectories by id across GPUs)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1010_2438_amd import Context, Model
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.Stream()
    ctx = Context(0)

    if args.workload:
        single_workload(ctx, stream, args)
        return

    # ---- headline: the batched sweep, persistent vs plain
    m2, run2 = W.config(2)
    model2 = Model(ctx, m2)
    alg2 = model2.info["alg_slots_per_event"]
    if args.tuning:
        t2p = parse_tuning(args.tuning)
        t2q = dict(t2p)
    else:
        t2p = model2.autotune(run2, "persistent", budget_s=5.0)
        t2q = model2.autotune(run2, "plain", budget_s=1.0)
    log("sweep: %s, %.1f algorithmic VALU slots/event; tuned persistent %s plain %s"
        % (model2.info, alg2, t2p, t2q))
    pers = time_form(ctx, model2, run2, "persistent", args.steps, args.warmup, stream, t2p,
                     e2e=True)
    log("sweep persistent", pers)
    plain = None
    if not args.only_headline:
        plain = time_form(ctx, model2, run2, "plain", max(1, args.steps // 2), 1, stream, t2q)
        log("sweep plain", plain)

    # ---- the plain method at GPU scale and the multi-compartment model
    extra = {}
    if not args.no_extra:
        m1, run1 = W.config(1)
        model1 = Model(ctx, m1)
        t1p = model1.autotune(run1, "persistent", budget_s=2.0)
        t1q = model1.autotune(run1, "plain", budget_s=1.0)
        g1p = time_form(ctx, model1, run1, "persistent", args.steps, args.warmup, stream, t1p)
        g1q = time_form(ctx, model1, run1, "plain", args.steps, args.warmup, stream, t1q)
        log("gene regulation persistent", g1p, "plain", g1q)
        extra[W.CONFIG_NAMES[1]] = {
            "persistent_events_per_s": g1p["events_per_s"], "plain_events_per_s": g1q["events_per_s"],
            "events_per_step": g1p["events_per_step"], "tuning_persistent": t1p,
            "tuning_plain": t1q}
        m3, run3 = W.config(3)
        model3 = Model(ctx, m3)
        t3p = model3.autotune(run3, "persistent", budget_s=2.0)
        g3p = time_form(ctx, model3, run3, "persistent", max(1, args.steps // 2), 1, stream, t3p)
        g3q = time_form(ctx, model3, run3, "plain", max(1, args.steps // 2), 1, stream, None)
        log("multi-compartment persistent", g3p, "plain", g3q)
        extra[W.CONFIG_NAMES[3]] = {
            "persistent_events_per_s": g3p["events_per_s"], "plain_events_per_s": g3q["events_per_s"],
            "events_per_step": g3p["events_per_step"], "layout": "wavefront per trajectory",
            "tuning_persistent": t3p}

    serving = None
    if not args.no_serve:
        sat = serve_trace(ctx, args.serve_jobs, 1.0, 16 << 30)
        log("serving (trace rate)", sat)
        # a labelled sub-saturation run: arrivals stretched so the offered
        # load is about 70% of the achieved rate above
        scale = max(1.0, sat["offered_events_per_s"] / (0.7 * sat["achieved_events_per_s"]))
        sub = serve_trace(ctx, args.serve_jobs, scale, 16 << 30)
        log("serving (sub-saturation)", sub)
        small = serve_trace(ctx, args.serve_jobs, scale, 2 << 30)
        log("serving (sub-saturation, 2 GiB budget)", small)
        serving = {"trace": "first %d jobs of %s" % (args.serve_jobs, W.CONFIG_NAMES[4]),
                   "at_trace_rate": sat, "sub_saturation": dict(sub, time_scale=scale),
                   "sub_saturation_2GiB": small,
                   "p50_latency_s": sub["p50_latency_s"], "p99_latency_s": sub["p99_latency_s"]}

    achieved = pers["events_per_step"] * alg2 / (pers["kernel_ms"] * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_VALU_SLOTS,
                "traffic": measured_traffic(model2.source(), pers["kernel"]),
                "kernel": pers["kernel"],
                "work_unit": "%.1f VALU issue slots per applied event" % alg2}
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(m2, run2)
        log("cpu", cpu)

    out = {
        "metric": METRIC, "value": pers["events_per_s"], "unit": "events/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": pers["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+i32",
        "data": "synthetic",
        "config": {"workload": W.CONFIG_NAMES[2], "instances": run2["n_instances"],
                   "replicas_per_instance": run2["replicas"],
                   "trajectories": run2["n_instances"] * run2["replicas"],
                   "t_end": (run2["n_samples"] - 1) * run2["dt"],
                   "sample_points": run2["n_samples"], "form": "persistent",
                   "events_per_step": pers["events_per_step"], "tuning": t2p,
                   "host_to_host_events_per_s": pers.get("host_to_host_events_per_s"),
                   "host_to_host_ms": pers.get("host_to_host_ms")},
        "plain": None if plain is None else {
            "events_per_s": plain["events_per_s"], "ms_per_step": plain["ms_per_step"],
            "tuning": t2q, "persistent_over_plain": pers["events_per_s"] / plain["events_per_s"]},
        "other_workloads": extra,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
