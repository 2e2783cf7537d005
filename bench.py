"""Benchmark: applied SSA events per second on one MI355X.

Headline workload (one "step" = the whole hot path over one batch): the
batched parameter sweep -- the gene-regulation model (two compartments, 10
species, 20 rules, four across the nuclear membrane) in 4096 instances whose
kinetic constants are scaled by a per-instance factor 10^U(-1,1), 64
replicas each (262144 trajectories, ~100x spread of events per trajectory),
simulated to t = 100 with 201 sample points and reduced on line into
per-instance, per-sample mean/variance.  Inputs are resident on the device
before the timed region.  `value` is the batched persistent form: instances
taken longest-first (predicted by their total propensity at t = 0), two
lanes per trajectory, replayed as a HIP graph, at the launch shape in
LAUNCH (the autotuner's choice on MI355X; its grid holds every trajectory,
so the hardware dispatcher, starting blocks as others finish, is the
queue).  Timed beside it on the same inputs: the plain launch with one lane
per trajectory in natural order, and the plain launch at the headline's own
layout (two lanes per trajectory, natural order), which isolates the gain
of the longest-first order.  Also reported: the 16384-replica
gene-regulation run, the 32-cell multi-compartment run, the serving trace
(continuous batching, p50/p99 latency), the VALU roofline of each kernel and
the CPU oracle on the host cores.

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

# Launch shapes the benchmark times: for each workload's persistent form the
# shape the autotuner chose on MI355X (``--autotune`` searches again
# instead), and the two plain launches of the sweep.  The full-size parity
# tests run exactly these shapes.
LAUNCH = {
    # sweep: two lanes per trajectory, block 256, 16 requested waves per
    # SIMD (a grid that holds every trajectory: the queue-free kernel)
    "sweep": {"block_size": 256, "waves_per_simd": 16, "lanes_per_replica": 2},
    # the plain per-trajectory launch: one lane each, natural order
    "sweep_plain": {"block_size": 256, "lanes_per_replica": 1},
    # the plain launch at the headline's layout: only the order differs
    "sweep_plain_pair": {"block_size": 256, "lanes_per_replica": 2},
    # 16384 replicas of one model: four lanes per trajectory, one wave/SIMD
    1: {"block_size": 256, "waves_per_simd": 1, "lanes_per_replica": 4},
    # the 32-cell model: one wavefront per trajectory
    3: {"block_size": 256, "waves_per_simd": 8, "lanes_per_replica": 64},
    # the general-term cell colony: one wavefront per trajectory
    5: {"block_size": 256, "waves_per_simd": 8},
}


# streamed run of the sweep: sample points per window
STREAM_WINDOW = 20
# serving policy of the predictive replays: slices of at most 64 sample
# points (constant simulation time) and 16384 draws, predictive order
SERVE_PREDICTED = {"slice_events": 16384, "slice_samples": 64, "predicted": True}
# a pool small enough that admission waits for memory on the trace prefix
SERVE_SMALL_POOL = 48 << 20


# the general-term workload: the cell colony (compartments created and
# deleted at run time), 2048 trajectories
GENERAL_NAME = "cell_colony_general_r2048"


def general_workload():
    """The cell colony in a fed nutrient bath at a settled size (about 28 of
    its 64 slots live; biomass spent, cells dying), 2048 trajectories to
    t = 100, 201 sample points."""
    import workloads as W
    m = W.cell_colony(nutrient=0, k_feed=100.0, k_up=0.05, k_div=0.05, k_die=0.3, k_decay=0.5)
    return m, W.make_run(seed=0, replicas=2048, dt=0.5, n_samples=201)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_form(ctx, model, run, mode, steps, warmup, stream, tuning=None, e2e=False,
              want_traj=False):
    """Warm up, then time exactly `steps` launches bracketed by device
    synchronisation; per-launch simulation time from the library's HIP events
    on the launch stream.  With e2e, also one untimed-for-`value` cycle from
    host tables to host statistics (submission with table upload, the run,
    mean/variance/n copied back), wall clock."""
    import torch
    from paper_1010_2438_amd import Run
    r = Run(ctx, model, run, mode=mode, stream=stream, tuning=tuning, want_traj=want_traj)
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


def time_stream(ctx, model, run, window, stream, run_bytes):
    """The run streamed in windows of `window` sample points (bounded device
    memory, statistics handed out per window while the next one runs), one
    pass after one untimed pass: wall time from opening to the last window's
    statistics on the host, events/s, and the device memory held against
    the whole run's."""
    import torch
    from paper_1010_2438_amd import Stream
    for timed in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = Stream(ctx, model, run, window, stream=stream)
        sim_ms = 0.0
        rows = 0
        for k0, mean, var, n in s:
            rows += mean.shape[1]
            sim_ms += s.info()["last_window_ms"]
        wall = time.perf_counter() - t0
        info = s.info()
        events = int(s.counters()["events"].sum())
        s.close()
    assert rows == run["n_samples"]
    return {"window": info["window"], "windows": info["n_windows"], "kernel": info["kernel"],
            "events": events, "wall_s": wall, "events_per_s": events / wall,
            "sum_window_kernel_ms": sim_ms, "device_bytes": info["device_bytes"],
            "whole_run_device_bytes": run_bytes}


def run_device_bytes(model, run, want_traj=False):
    """Device bytes cwc_run_submit allocates for `run` (the buffers listed
    in run.cpp: tables, per-trajectory outputs, moments, histogram, n and
    mean/variance)."""
    I, R, K1 = run["n_instances"], run["replicas"], run["n_samples"]
    C, NR = model.info["n_cells"], model.info["n_rules"]
    G, mom = I * R, I * K1 * C
    b = (I if run.get("rate_table") is not None else 1) * NR * 8
    b += (I if run.get("init_table") is not None else 1) * C * 4
    b += G * (4 * C + 8 + 8 + 8 + 1 + 4)
    b += (G * K1 * C * 4) if want_traj else 0
    b += mom * 8 * 3 + I * (K1 + 1) * 8 + 8 + I * 4 + I * K1 * 8 + mom * 8 * 2
    return b


def host_cpu():
    """(model name, usable host threads).  Threads: the CPUs this process
    may run on, at most 16 -- the host share of one GPU on the MI355X boxes
    this runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, max(1, min(16, n))


def oracle_rate(model, run, ids, threads):
    """The oracle over trajectories `ids` (one call per trajectory, spread
    over `threads` host threads): (events, seconds)."""
    import threading
    import oracle
    fm = oracle.FlatModel(model)
    evs = [0] * len(ids)

    def work(k):
        for q in range(k, len(ids), threads):
            g = int(ids[q])
            r = oracle.simulate(model, run, g0=g, g1=g + 1, want_stats=False, flat=fm)
            evs[q] = int(r["events"][0])

    t0 = time.perf_counter()
    ts = [threading.Thread(target=work, args=(k,)) for k in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    return sum(evs), time.perf_counter() - t0


def cpu_baseline(budget_s=10.0):
    """The oracle (plain C direct method, full propensity recomputation per
    event) on the host cores over bounded samples of the benchmark's
    workloads.  Headline (`value`): the sweep, replica 0 of every s-th
    instance (s chosen for about `budget_s` seconds of work on all threads;
    the instances spread over the whole sweep, whose events per trajectory
    vary ~100x), on every usable thread; beside it the same sample's first
    trajectories on one thread, and prefixes of the other workloads'
    trajectories on all threads.  Rates are events/s of the sample (a
    prefix's rate scales linearly to the full workload: trajectories are
    independent)."""
    import workloads as W
    cpu, threads = host_cpu()
    m2, run2 = W.config(2)
    I, R = run2["n_instances"], run2["replicas"]
    probe = [i * R for i in range(0, I, 256)]                  # 16 trajectories
    ev, dt = oracle_rate(m2, run2, probe, threads)
    rate = ev / max(dt, 1e-6) * threads / min(threads, len(probe))
    n_want = budget_s * rate / max(ev / len(probe), 1.0)
    stride = max(1, int(I / max(n_want, 1.0)))
    ids = [i * R for i in range(0, I, stride)]
    ev, dt = oracle_rate(m2, run2, ids, threads)
    # one thread: an evenly spread subset of that sample sized for about a
    # third of the budget
    per_traj = dt * min(threads, len(ids)) / len(ids)
    n1 = max(1, min(len(ids), int(budget_s / 3.0 / max(per_traj, 1e-9))))
    ids1 = ids[::max(1, len(ids) // n1)][:n1]
    ev1, dt1 = oracle_rate(m2, run2, ids1, 1)
    out = {"value": ev / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu,
           "sample": "sweep: replica 0 of every %d-th of %d instances (%d trajectories, %d "
                     "events, %.1f s on %d threads)" % (stride, I, len(ids), ev, dt, threads),
           "single_thread": {"value": ev1 / dt1, "unit": "events/s", "cores": 1,
                             "sample": "%d of those trajectories (%d events, %.1f s)"
                                       % (len(ids1), ev1, dt1)},
           "other_workloads": {}}
    gm_dict, grun = general_workload()
    gids = list(range(4 * threads))
    t0 = time.perf_counter()
    import oracle as _oracle
    gres = _oracle.gsimulate(gm_dict, grun, g0=0, g1=len(gids), want_stats=False, threads=threads)
    gdt = time.perf_counter() - t0
    out["other_workloads"][GENERAL_NAME] = {
        "value": float(gres["events"].sum()) / gdt, "unit": "events/s", "cores": threads,
        "sample": "trajectories 0..%d of 2048 (%d events, %.2f s)"
                  % (len(gids) - 1, int(gres["events"].sum()), gdt)}
    for c, n in ((0, 64), (1, 8 * threads), (3, 4 * threads)):
        m, run = W.config(c)
        G = run["n_instances"] * run["replicas"]
        ids = list(range(min(n, G)))
        e, d = oracle_rate(m, run, ids, threads)
        out["other_workloads"][W.CONFIG_NAMES[c]] = {
            "value": e / d, "unit": "events/s", "cores": threads,
            "sample": "trajectories 0..%d of %d (%d events, %.2f s)" % (len(ids) - 1, G, e, d)}
    return out


def chain_seconds_per_event(ctx, stream):
    """The shortest per-event time of one trajectory's dependent chain:
    64 Lotka-Volterra trajectories (the smallest model of the trace) to
    t = 20 in one plain launch with two lanes per trajectory, a wavefront
    or two on an otherwise idle GPU, so the launch lasts as long as its
    longest trajectory; kernel time / that trajectory's events."""
    import workloads as W
    from paper_1010_2438_amd import Model, Run
    model = Model(ctx, W.lotka_volterra())
    run = W.make_run(seed=0, replicas=64, dt=0.05, n_samples=401)
    best = None
    for lanes in (1, 2):
        r = Run(ctx, model, run, mode="plain", stream=stream,
                tuning={"block_size": 64, "lanes_per_replica": lanes})
        r.wait()
        r.relaunch(stream)
        r.wait()
        sec = r.elapsed_ms()[0] * 1e-3 / int(r.counters()["events"].max())
        r.close()
        best = sec if best is None else min(best, sec)
    model.close()
    return best


def serve_trace(ctx, n_jobs, time_scale, budget, slice_events=4096, max_active=64,
                slice_samples=0, predicted=False, chain_s_per_event=None, resident=False,
                detail=False):
    """Replays the first n_jobs of the serving trace (Poisson arrivals, mixed
    configurations 0-3, 64..8192 replicas, t_end 5..100) against the
    continuous-batching server; arrival times are multiplied by time_scale.
    Returns latency percentiles (submit -> statistics ready) and rates; with
    chain_s_per_event, also each job's latency floor (its longest
    trajectory's events x that time)."""
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
    srv.set_policy(slice_samples, predicted, resident)

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
    config_of = {}
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
                config_of[ids[i]] = job["config"]
        except Exception as e:       # surfaced below
            err.append(e)

    th = threading.Thread(target=submitter)
    th.start()
    infos = {}
    longest = {}            # per job: events of its longest trajectory
    # Lotka-Volterra jobs carry a count cap (prey explode once predators die
    # out): how many of their trajectories end in OVERFLOW
    overflow = {"lotka_volterra_jobs": 0, "trajectories": 0, "overflow_trajectories": 0,
                "jobs_with_overflow": 0}
    last = time.perf_counter()
    while len(infos) < len(trace):
        if err:
            raise err[0]
        for jid in srv.poll():
            infos[jid] = srv.info(jid)
            cnt = srv.counters(jid)
            longest[jid] = int(cnt["events"].max())
            if config_of[jid] == 0:
                st = cnt["status"]
                no = int((st == 2).sum())
                overflow["lotka_volterra_jobs"] += 1
                overflow["trajectories"] += int(st.size)
                overflow["overflow_trajectories"] += no
                overflow["jobs_with_overflow"] += int(no > 0)
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
    out = {"jobs": len(trace), "arrival_span_s": span,
           "offered_jobs_per_s": len(trace) / max(span, 1e-9),
           "p50_latency_s": float(np.percentile(lat, 50)),
           "p99_latency_s": float(np.percentile(lat, 99)),
           "max_latency_s": float(lat.max()),
           "events": int(ev), "achieved_events_per_s": ev / wall,
           "offered_events_per_s": ev / max(span, 1e-9),
           "makespan_s": wall, "ticks": st["ticks"],
           "policy": {"slice_events": slice_events, "slice_samples": slice_samples,
                      "order": "resident" if resident else
                      ("predicted" if predicted else "fifo")},
           "hbm_budget_bytes": st["pool_bytes"], "pool_peak_bytes": st["pool_peak"],
           "lotka_volterra_count_cap": {"cap": 100000, **overflow}}
    if detail:
        out["per_job"] = [{"config": trace[i]["config"], "replicas": trace[i]["replicas"],
                           "t_submit": infos[j]["t_submit"], "t_admit": infos[j]["t_admit"],
                           "t_done": infos[j]["t_done"], "longest": longest[j],
                           "events": infos[j]["events"]} for i, j in enumerate(ids)]
    if chain_s_per_event:
        # no schedule finishes a job before its longest trajectory's events
        # have run one after another at the fastest per-event chain
        floor = np.array([longest[j] * chain_s_per_event for j in ids])
        out["latency_floor"] = {
            "chain_us_per_event": chain_s_per_event * 1e6,
            "p50_s": float(np.percentile(floor, 50)), "p99_s": float(np.percentile(floor, 99)),
            "max_s": float(floor.max()),
            "longest_trajectory_events_max": int(max(longest.values()))}
    return out


def fnv1a64(text):
    h = 0xcbf29ce484222325
    for b in text.encode():
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return "%016x" % h


def measured_traffic(source, kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from its committed
    counter summary (profiles/<kernel>_<workload>.md), only if the counters
    were taken on this exact kernel (same generated source); else None."""
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload))
    try:
        text = open(path).read()
    except OSError:
        return None
    fig = dict(re.findall(r"^(source_fnv1a64|traffic_bytes_per_launch): (\S+)$", text, re.M))
    if fig.get("source_fnv1a64") != fnv1a64(source) or "traffic_bytes_per_launch" not in fig:
        return None
    return int(fig["traffic_bytes_per_launch"])


def algorithmic_output_bytes(I, K1, C, G):
    """Bytes the path must write per launch: the exact moments (S1, S2 as
    two 64-bit halves) per (instance, sample, cell), the contributor count
    per (instance, sample), mean and variance per (instance, sample, cell),
    and per trajectory its final counts, events, final time, digest, status
    and recorded-sample count."""
    return I * K1 * C * (3 * 8 + 2 * 8) + I * K1 * 8 + G * (4 * C + 8 + 8 + 8 + 1 + 4)


def roofline_of(res, alg, model, workload, run):
    """The VALU roofline of one timed form: algorithmic issue slots per
    applied event x events per launch / the kernel's HIP-event time."""
    achieved = res["events_per_step"] * alg / (res["kernel_ms"] * 1e-3)
    I, R, K1 = run["n_instances"], run["replicas"], run["n_samples"]
    C = model.info["n_cells"]
    traffic = measured_traffic(model.source(), res["kernel"], workload)
    alg_bytes = algorithmic_output_bytes(I, K1, C, I * R)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12,
            "unit": "TOP/s", "frac": achieved / PEAK_VALU_SLOTS, "traffic": traffic,
            "kernel": res["kernel"], "kernel_ms": res["kernel_ms"],
            "algorithmic_output_bytes": alg_bytes,
            "traffic_over_algorithmic": None if traffic is None else traffic / alg_bytes,
            "work_unit": "%.1f VALU issue slots per applied event" % alg}


def parse_tuning(text):
    """BLOCK,WAVES_PER_SIMD[,REFILL_CHUNK[,SLOTS[,LANES_PER_REPLICA]]]"""
    v = [int(x) for x in text.split(",")]
    return {"block_size": v[0], "waves_per_simd": v[1],
            "refill_chunk": v[2] if len(v) > 2 else 0,
            "sample_slots": v[3] if len(v) > 3 else 0,
            "lanes_per_replica": v[4] if len(v) > 4 else 1}


def single_workload(ctx, stream, args):
    """One workload's persistent form alone (at its LAUNCH shape unless
    --tuning or --autotune is given), with the roofline of its kernel, as
    one JSON line."""
    import workloads as W
    from paper_1010_2438_amd import GModel, Model
    if args.workload == 5:
        m, run = general_workload()
        model = GModel(ctx, m)
        name = GENERAL_NAME
    else:
        m, run = W.config(args.workload)
        model = Model(ctx, m)
        name = W.CONFIG_NAMES[args.workload]
    alg = model.info["alg_slots_per_event"]
    if args.tuning:
        tun = parse_tuning(args.tuning)
    elif args.autotune:
        tun = model.autotune(run, "persistent", budget_s=2.0)
    else:
        tun = dict(LAUNCH[args.workload])
    res = time_form(ctx, model, run, "persistent", args.steps, args.warmup, stream, tun)
    print(json.dumps({
        "workload": name, "form": "persistent",
        "events_per_s": res["events_per_s"], "ms_per_step": res["ms_per_step"],
        "kernel_ms": res["kernel_ms"], "events_per_step": res["events_per_step"],
        "steps": args.steps, "warmup": args.warmup, "tuning": tun,
        "roofline": roofline_of(res, alg, model, name, run)}),
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
                    help="time this launch shape (of the headline, or of --workload) instead "
                         "of the one in LAUNCH")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner for each persistent form instead of using LAUNCH")
    ap.add_argument("--workload", type=int, default=0, choices=(0, 1, 3, 5),
                    help="time only the persistent form of workload 1 (gene regulation, "
                         "16384 replicas), 3 (multi-compartment, 2048 replicas) or 5 (the "
                         "general-term cell colony, 2048 replicas) and print its own line "
                         "(for profiler runs); 0 = the full benchmark")
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
    t2q = dict(LAUNCH["sweep_plain"])
    t2s = dict(LAUNCH["sweep_plain_pair"])
    if args.tuning:
        t2p = parse_tuning(args.tuning)
    elif args.autotune:
        t2p = model2.autotune(run2, "persistent", budget_s=5.0)
    else:
        t2p = dict(LAUNCH["sweep"])
    log("sweep: %s, %.1f algorithmic VALU slots/event; persistent %s"
        % (model2.info, alg2, t2p))
    pers = time_form(ctx, model2, run2, "persistent", args.steps, args.warmup, stream, t2p,
                     e2e=True)
    log("sweep persistent", pers)
    plain = None
    if not args.only_headline:
        q_steps = max(1, args.steps // 2)
        plain1 = time_form(ctx, model2, run2, "plain", q_steps, 1, stream, t2q)
        log("sweep plain, one lane per trajectory", plain1)
        plain2 = time_form(ctx, model2, run2, "plain", q_steps, 1, stream, t2s)
        log("sweep plain, headline layout", plain2)
        plain = {
            # the plain launch: one lane per trajectory, natural order
            "events_per_s": plain1["events_per_s"], "ms_per_step": plain1["ms_per_step"],
            "kernel": plain1["kernel"], "tuning": t2q,
            "persistent_over_plain": pers["events_per_s"] / plain1["events_per_s"],
            "roofline": roofline_of(plain1, alg2, model2, W.CONFIG_NAMES[2], run2),
            # the plain launch at the persistent form's own layout: the
            # longest-first order alone
            "same_layout": {
                "events_per_s": plain2["events_per_s"], "ms_per_step": plain2["ms_per_step"],
                "kernel": plain2["kernel"], "tuning": t2s,
                "persistent_over_plain": pers["events_per_s"] / plain2["events_per_s"]}}

    # ---- the plain method at GPU scale and the multi-compartment model
    extra = {}
    if not args.no_extra:
        for c in (1, 3):
            m, run = W.config(c)
            mo = Model(ctx, m)
            alg = mo.info["alg_slots_per_event"]
            tp = mo.autotune(run, "persistent", budget_s=2.0) if args.autotune else dict(LAUNCH[c])
            tq = {"block_size": 256, "lanes_per_replica": 1 if mo.info["layout"] == 0 else 64}
            steps = args.steps if c == 1 else max(1, args.steps // 2)
            gp = time_form(ctx, mo, run, "persistent", steps, 1, stream, tp)
            gq = time_form(ctx, mo, run, "plain", steps, 1, stream, tq)
            log(W.CONFIG_NAMES[c], "persistent", gp, "plain", gq)
            extra[W.CONFIG_NAMES[c]] = {
                "persistent_events_per_s": gp["events_per_s"],
                "plain_events_per_s": gq["events_per_s"],
                "events_per_step": gp["events_per_step"], "ms_per_step": gp["ms_per_step"],
                "tuning_persistent": tp, "tuning_plain": tq, "kernel_plain": gq["kernel"],
                "roofline": roofline_of(gp, alg, mo, W.CONFIG_NAMES[c], run)}
            if c == 1:
                # the same launch keeping every sampled state: [K+1][C][G]
                # int32 written in place by the kernel
                gt = time_form(ctx, mo, run, "persistent", steps, 1, stream, tp, want_traj=True)
                tb = run["replicas"] * run["n_instances"] * run["n_samples"] * mo.info["n_cells"] * 4
                extra[W.CONFIG_NAMES[c]]["with_trajectories"] = {
                    "events_per_s": gt["events_per_s"], "kernel_ms": gt["kernel_ms"],
                    "kernel": gt["kernel"], "trajectory_bytes": tb,
                    "trajectory_write_GB_per_s": tb / (gt["kernel_ms"] * 1e-3) / 1e9,
                    "over_stats_only_ms": gt["kernel_ms"] / gp["kernel_ms"]}
                log(W.CONFIG_NAMES[c], "with trajectories", extra[W.CONFIG_NAMES[c]]["with_trajectories"])

    # ---- a general CWC model: the cell colony (cells divide, die, take up
    # nutrients; up to 64 compartments per term), 2048 trajectories
    if not args.no_extra:
        from paper_1010_2438_amd import GModel
        gm_dict, grun = general_workload()
        gmo = GModel(ctx, gm_dict)
        gr = time_form(ctx, gmo, grun, "persistent", args.steps, 1, stream,
                       {"block_size": 256, "waves_per_simd": 8})
        log(GENERAL_NAME, gr)
        extra[GENERAL_NAME] = {
            "persistent_events_per_s": gr["events_per_s"], "events_per_step": gr["events_per_step"],
            "ms_per_step": gr["ms_per_step"], "kernel": gr["kernel"],
            "roofline": roofline_of(gr, gmo.info["alg_slots_per_event"], gmo, GENERAL_NAME, grun)}
        gmo.close()

    # ---- the sweep streamed in windows (bounded device memory)
    streamed = None
    if not args.no_extra:
        streamed = time_stream(ctx, model2, run2, STREAM_WINDOW, stream,
                               run_device_bytes(model2, run2))
        log("sweep streamed", streamed)

    serving = None
    if not args.no_serve:
        chain = chain_seconds_per_event(ctx, stream)
        log("one trajectory's event chain: %.3f us per event" % (chain * 1e6))
        sat = serve_trace(ctx, args.serve_jobs, 1.0, 16 << 30)
        log("serving (trace rate)", sat)
        # labelled sub-saturation runs: arrivals stretched so the offered
        # load is about 70% of the achieved rate above; draw-bounded slices
        # in FIFO order, then slices of a few sample points (constant
        # simulation time) with the predictive order, then the latter in a
        # pool small enough that admission waits for memory
        scale = max(1.0, sat["offered_events_per_s"] / (0.7 * sat["achieved_events_per_s"]))
        sub = serve_trace(ctx, args.serve_jobs, scale, 16 << 30, chain_s_per_event=chain)
        log("serving (sub-saturation, FIFO)", sub)
        pred = serve_trace(ctx, args.serve_jobs, scale, 16 << 30, **SERVE_PREDICTED)
        log("serving (sub-saturation, predicted)", pred)
        small = serve_trace(ctx, args.serve_jobs, scale, SERVE_SMALL_POOL, **SERVE_PREDICTED)
        log("serving (sub-saturation, predicted, small pool)", small)
        res = serve_trace(ctx, args.serve_jobs, scale, 16 << 30, resident=True)
        log("serving (sub-saturation, resident kernels)", res)
        best = min((sub, pred, res), key=lambda r: r["p99_latency_s"])
        serving = {"trace": "first %d jobs of %s" % (args.serve_jobs, W.CONFIG_NAMES[4]),
                   "at_trace_rate": sat, "sub_saturation": dict(sub, time_scale=scale),
                   "sub_saturation_predicted": dict(pred, time_scale=scale),
                   "sub_saturation_resident": dict(res, time_scale=scale),
                   "sub_saturation_small_pool": dict(small, time_scale=scale),
                   "p50_latency_s": best["p50_latency_s"], "p99_latency_s": best["p99_latency_s"],
                   "p_latency_policy": best["policy"]}

    roofline = roofline_of(pers, alg2, model2, W.CONFIG_NAMES[2], run2)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()
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
        "plain": plain,
        "other_workloads": extra,
        "streamed": streamed,
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
