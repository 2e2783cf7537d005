"""Benchmark: applied SSA events per second on one MI355X.

Workload (one "step" = the whole hot path over one batch): the
gene-regulation model (two compartments, 10 species, 20 rules, four of them
across the nuclear membrane), 16384 replicas simulated to t = 100 with 201
sample points and the on-line reduction into per-sample mean/variance.
Inputs are resident on the device before the timed region.  The headline
value is the persistent form (lane refill from a work queue, replayed as a
HIP graph); the plain one-lane-per-replica launch is timed on the same
inputs beside it, as is the 4096-instance x 64-replica parameter sweep.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build runs on
one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSA events/sec on 1 GPU (batched persistent vs plain launch); p99 job latency"
PEAK_VALU_SLOTS = 256 * 4 * 16 * 2.4e9     # CUs x SIMDs x lanes x clock = 3.93e13/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_form(ctx, model, run, mode, steps, warmup, stream):
    """Warm up, then time exactly `steps` launches bracketed by device
    synchronisation; per-launch simulation time from the library's HIP events
    on the launch stream."""
    import torch
    from paper_1010_2438_amd import Run
    r = Run(ctx, model, run, mode=mode, stream=stream)
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
    r.close()
    sim_ms = sum(s[0] for s in sims) / len(sims)
    tot_ms = sum(s[1] for s in sims) / len(sims)
    return {"events_per_step": events, "ms_per_step": 1e3 * wall / steps,
            "events_per_s": events * steps / wall, "kernel_ms": sim_ms,
            "launch_ms": tot_ms, "finite_mean": bool((mean == mean).all())}


def cpu_baseline(model, run, budget_s=15.0):
    """The oracle (plain C direct method, one trajectory per call) on the
    host cores: trajectories 0..n-1 of the same workload, n sized for about
    `budget_s` seconds of work."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    probe = oracle.simulate(model, run, g0=0, g1=threads, want_stats=False, threads=threads)
    t0 = time.perf_counter()
    probe = oracle.simulate(model, run, g0=0, g1=threads, want_stats=False, threads=threads)
    dt = time.perf_counter() - t0
    n = max(threads, int(threads * budget_s / max(dt, 1e-3)))
    n = min(n, run["n_instances"] * run["replicas"])
    t0 = time.perf_counter()
    res = oracle.simulate(model, run, g0=0, g1=n, want_stats=True, threads=threads)
    dt = time.perf_counter() - t0
    ev = int(res["events"].sum())
    return {"value": ev / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d trajectories of the same workload (%d events, %.1f s, "
                      "with the on-line moments)" % (n, run["n_instances"] * run["replicas"], ev, dt)}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=150)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build simulates on one GPU only; --gpus %d is not supported "
              "(trajectories shard by id across GPUs, see DESIGN.md)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1010_2438_amd import Context, Model
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.Stream()
    ctx = Context(0)
    m1, run1 = W.config(1)
    model1 = Model(ctx, m1)
    alg = model1.info["alg_slots_per_event"]
    log("config 1 model: %s, %.1f algorithmic VALU slots/event" % (model1.info, alg))
    pers = time_form(ctx, model1, run1, "persistent", args.steps, args.warmup, stream)
    log("persistent", pers)
    plain = time_form(ctx, model1, run1, "plain", args.steps, args.warmup, stream)
    log("plain", plain)

    sweep = None
    if not args.no_sweep:
        m2, run2 = W.config(2)
        model2 = Model(ctx, m2)
        sw_steps = max(1, args.steps // 4)
        sp = time_form(ctx, model2, run2, "persistent", sw_steps, 1, stream)
        sq = time_form(ctx, model2, run2, "plain", sw_steps, 1, stream)
        log("sweep persistent", sp, "plain", sq)
        sweep = {"workload": W.CONFIG_NAMES[2], "trajectories": 4096 * 64,
                 "events_per_step": sp["events_per_step"],
                 "persistent_events_per_s": sp["events_per_s"],
                 "plain_events_per_s": sq["events_per_s"],
                 "persistent_over_plain": sp["events_per_s"] / sq["events_per_s"]}

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

    achieved = pers["events_per_step"] * alg / (pers["kernel_ms"] * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12,
                "unit": "TOP/s", "frac": achieved / PEAK_VALU_SLOTS, "traffic": None,
                "work_unit": "%.1f VALU issue slots per applied event" % alg}
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(m1, run1)
        log("cpu", cpu)

    out = {
        "metric": METRIC, "value": pers["events_per_s"], "unit": "events/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": pers["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+i32",
        "data": "synthetic",
        "config": {"workload": W.CONFIG_NAMES[1], "replicas": run1["replicas"],
                   "t_end": (run1["n_samples"] - 1) * run1["dt"],
                   "sample_points": run1["n_samples"], "form": "persistent",
                   "events_per_step": pers["events_per_step"]},
        "plain": {"events_per_s": plain["events_per_s"], "ms_per_step": plain["ms_per_step"],
                  "persistent_over_plain": pers["events_per_s"] / plain["events_per_s"]},
        "sweep": sweep,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
