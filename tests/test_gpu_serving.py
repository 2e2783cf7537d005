"""Serving (continuous batching): a job's results are the same alone and in
a mix of concurrently admitted jobs of different models, however often its
trajectories are suspended and resumed; admission respects the HBM budget."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import compare_trajectories, gpu_run, same_float

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_2438_amd import Context
    c = Context(0)
    yield c
    c.close()


def job_specs():
    gene = W.gene_regulation(1)
    tab, _ = W.sweep_rate_table(gene, 4096, 2)
    mc = W.multi_compartment(3, n_cells_=6)
    return [
        (W.lotka_volterra(), W.make_run(seed=11, replicas=100, dt=0.05, n_samples=21)),
        (gene, W.make_run(seed=12, replicas=300, dt=0.5, n_samples=41)),
        (gene, W.make_run(seed=13, n_instances=8, replicas=16, dt=0.5, n_samples=21,
                          rate_table=tab[100:108])),
        (mc, W.make_run(seed=14, replicas=20, dt=0.5, n_samples=11)),
        (W.lotka_volterra(), W.make_run(seed=15, replicas=70, dt=0.05, n_samples=21,
                                        max_events=5000)),
        (W.receptor_binding(), W.make_run(seed=16, replicas=50, dt=0.25, n_samples=17)),
    ]


def same_stats(a, b):
    for x, y in zip(a, b):
        x, y = np.asarray(x), np.asarray(y)
        if x.dtype.kind == "f":
            assert same_float(np.nan_to_num(x, nan=-1.0), np.nan_to_num(y, nan=-1.0))
        else:
            assert np.array_equal(x, y)


@pytest.mark.parametrize("slice_samples,predicted,resident",
                         [(0, False, False), (3, True, False), (5, False, False),
                          (0, False, True)])
def test_alone_vs_mix(ctx, slice_samples, predicted, resident):
    """Every job of the mix equals the job run alone, with slices bounded by
    draws only, with slices of a few sample points (constant simulation
    time) under the predictive and the FIFO dispatch order, and with
    resident kernels draining per-model queues of items."""
    from paper_1010_2438_amd import Model, Server
    print("case serving mix slice_samples", slice_samples, "predicted", predicted,
          "resident", resident, flush=True)
    specs = job_specs()
    models = {}
    for m, _ in specs:
        if repr(m) not in models:
            models[repr(m)] = Model(ctx, m)
    alone = []
    for m, run in specs:
        g = gpu_run(ctx, models[repr(m)], run, mode="plain", want_traj=False, want_digest=True)
        alone.append(g)
    # oracle check of one job alone
    orc = oracle.simulate(specs[0][0], specs[0][1], threads=8)
    compare_trajectories(alone[0], orc)
    # the mix: every job admitted at once, sliced every 997 draws
    srv = Server(ctx, hbm_budget=256 << 20, max_active=16, slice_events=997)
    srv.set_policy(slice_samples, predicted, resident)
    ids = [srv.submit(models[repr(m)], run, want_digest=True) for m, run in specs]
    srv.wait_idle(300)
    done = set(srv.poll())
    assert done == set(ids)
    for jid, g in zip(ids, alone):
        info = srv.info(jid)
        assert info["state"] == 2 and info["t_done"] >= info["t_admit"] >= info["t_submit"]
        c = srv.counters(jid)
        for key in ("events", "status", "digest", "n_recorded", "final_counts"):
            assert np.array_equal(c[key], g[key]), (jid, key)
        assert same_float(c["t_final"], g["t_final"])
        same_stats(srv.stats(jid), (g["mean"], g["var"], g["n"]))
        assert info["events"] == int(g["events"].sum())
    if not resident:
        assert max(srv.info(j)["n_ticks"] for j in ids) > 3     # really sliced
    if slice_samples:
        # a job of K+1 sample points needs at least ceil((K+1) / slice) slices
        for jid, (m, run) in zip(ids, specs):
            if srv.info(jid)["events"] and run["max_events"] == 0:
                assert srv.info(jid)["n_ticks"] >= -(-run["n_samples"] // slice_samples)
    st = srv.server_stats()
    assert st["jobs_done"] == len(ids) and st["pool_peak"] <= st["pool_bytes"]
    for j in ids:
        srv.release(j)
    assert srv.server_stats()["pool_used"] == 0
    srv.close()


@pytest.mark.parametrize("slice_samples,predicted,resident",
                         [(0, False, False), (4, True, False), (0, False, True)])
def test_general_jobs_in_mix(ctx, slice_samples, predicted, resident):
    """General models (compartments created, dissolved, deleted) served
    beside a fixed-tree job: each job's counters, statistics and final terms
    equal the job run alone, with the terms checkpointed between slices; one
    job is also checked against the general oracle."""
    from paper_1010_2438_amd import CwcError, GModel, Model, Run, Server
    print("case serving general mix slice_samples", slice_samples, "predicted", predicted,
          "resident", resident, flush=True)
    colony = W.cell_colony(n0=4, nutrient=300, max_comp=24)
    tab = np.tile(np.array([r["k"] for r in colony["rules"]]), (3, 1)) * \
        np.array([0.5, 1.0, 2.0])[:, None]
    specs = [
        (colony, W.make_run(seed=31, replicas=40, dt=0.5, n_samples=21)),
        (W.cell_dissolution(release_wrap=True), W.make_run(seed=32, replicas=77, dt=0.25,
                                                           n_samples=17)),
        (colony, W.make_run(seed=33, n_instances=3, replicas=10, dt=0.5, n_samples=21,
                            rate_table=tab)),
        (W.nested_export(), W.make_run(seed=34, replicas=64, dt=0.25, n_samples=17,
                                       max_events=300)),
    ]
    gms = {}
    for m, _ in specs:
        if repr(m) not in gms:
            gms[repr(m)] = GModel(ctx, m)
    alone = []
    for m, run in specs:
        r = Run(ctx, gms[repr(m)], run, mode="plain", want_digest=True)
        r.wait()
        g = r.counters()
        g["stats"] = r.stats()
        g["term"] = r.term()
        r.close()
        alone.append(g)
    orc = oracle.gsimulate(specs[1][0], specs[1][1], want_term=True, threads=8)
    for key in ("events", "status", "digest", "n_recorded", "final_counts"):
        assert np.array_equal(alone[1][key], orc[key]), key
    assert np.array_equal(alone[1]["term"], orc["term"])
    lv = Model(ctx, W.lotka_volterra())
    lv_run = W.make_run(seed=35, replicas=100, dt=0.05, n_samples=21)
    srv = Server(ctx, hbm_budget=256 << 20, max_active=16, slice_events=97)
    srv.set_policy(slice_samples, predicted, resident)
    ids = [srv.submit(gms[repr(m)], run, want_digest=True) for m, run in specs]
    lv_id = srv.submit(lv, lv_run)
    srv.wait_idle(300)
    assert set(srv.poll()) == set(ids) | {lv_id}
    for jid, g in zip(ids, alone):
        c = srv.counters(jid)
        for key in ("events", "status", "digest", "n_recorded", "final_counts"):
            assert np.array_equal(c[key], g[key]), (jid, key)
        assert same_float(c["t_final"], g["t_final"])
        same_stats(srv.stats(jid), g["stats"])
        assert np.array_equal(srv.term(jid), g["term"]), jid
    if not resident:
        assert max(srv.info(j)["n_ticks"] for j in ids) > 3     # really sliced
    with pytest.raises(CwcError):
        srv.term(lv_id)                                     # a fixed-tree job has no term
    for j in ids + [lv_id]:
        srv.release(j)
    assert srv.server_stats()["pool_used"] == 0
    srv.close()
    for gm in gms.values():
        gm.close()


@pytest.mark.parametrize("resident", [False, True])
def test_admission_within_budget(ctx, resident):
    """A pool that holds two jobs at a time: the client fetches and releases
    finished jobs, queued jobs are admitted FIFO as memory frees up, the pool
    never overflows, and results match a solo run (resident: the job slots
    and pool memory of released jobs are reused while the kernels stay)."""
    import time
    from paper_1010_2438_amd import Model, Server
    print("case serving admission resident", resident, flush=True)
    m = W.gene_regulation(1)
    mo = Model(ctx, m)
    runs = [W.make_run(seed=100 + i, replicas=20000, dt=0.5, n_samples=11) for i in range(6)]
    srv = Server(ctx, hbm_budget=10 << 20, max_active=8, slice_events=2048)
    srv.set_policy(0, False, resident)
    ids = [srv.submit(mo, r) for r in runs]
    kept, infos = {}, {}
    t0 = time.time()
    while len(infos) < len(ids) and time.time() - t0 < 120:
        for j in srv.poll():
            infos[j] = srv.info(j)
            if j == ids[4]:
                kept = srv.counters(j)
            srv.release(j)
        time.sleep(0.002)
    assert set(infos) == set(ids)
    one = infos[ids[0]]["bytes"]
    st = srv.server_stats()
    assert 2 * one <= st["pool_bytes"] < 3 * one
    assert st["pool_peak"] <= 2 * one
    admits = [infos[j]["t_admit"] for j in ids]
    assert admits == sorted(admits)
    # the third job could only start after one of the first two was released
    assert infos[ids[2]]["t_admit"] >= min(infos[ids[0]]["t_done"], infos[ids[1]]["t_done"])
    solo = gpu_run(ctx, mo, runs[4], mode="plain", want_traj=False)
    assert np.array_equal(kept["final_counts"], solo["final_counts"])
    assert np.array_equal(kept["events"], solo["events"])
    srv.close()


def test_resident_slot_reuse_and_policy_switch(ctx):
    """Resident kernels with one job slot: every job reuses the slot (and
    the parameters the kernels copy from it) while the kernels may stay on
    the device; each result equals the job run alone.  The policy can change
    to or from resident only while no job is queued or active."""
    import time
    from paper_1010_2438_amd import CwcError, Model, Server
    print("case serving resident slot reuse", flush=True)
    m = W.lotka_volterra()
    mo = Model(ctx, m)
    runs = [W.make_run(seed=200 + i, replicas=64 * (i + 1), dt=0.05, n_samples=21,
                       count_cap=100000) for i in range(5)]
    srv = Server(ctx, hbm_budget=64 << 20, max_active=1, slice_events=4096)
    srv.set_policy(0, False, True)
    ids = [srv.submit(mo, r, want_digest=True) for r in runs]
    with pytest.raises(CwcError):
        srv.set_policy(0, False, False)            # jobs queued: no switch
    got, t0 = {}, time.time()
    while len(got) < len(ids) and time.time() - t0 < 120:
        for j in srv.poll():
            got[j] = (srv.counters(j), srv.stats(j))
            srv.release(j)
        time.sleep(0.002)
    assert set(got) == set(ids)
    for jid, run in zip(ids, runs):
        g = gpu_run(ctx, mo, run, mode="plain", want_traj=False, want_digest=True)
        c, st = got[jid]
        for key in ("events", "status", "digest", "n_recorded", "final_counts"):
            assert np.array_equal(c[key], g[key]), (jid, key)
        assert same_float(c["t_final"], g["t_final"])
        same_stats(st, (g["mean"], g["var"], g["n"]))
    srv.set_policy(0, False, False)                # idle: the switch is allowed
    srv.close()


def test_policy_validation(ctx):
    from paper_1010_2438_amd import CwcError, Server
    srv = Server(ctx, hbm_budget=2 << 20, max_active=4, slice_events=1024)
    with pytest.raises(CwcError):
        srv.set_policy(-1, False)
    srv.close()


def test_job_larger_than_pool_is_rejected(ctx):
    from paper_1010_2438_amd import CwcError, Model, Server
    mo = Model(ctx, W.gene_regulation(1))
    srv = Server(ctx, hbm_budget=2 << 20, max_active=4, slice_events=1024)
    with pytest.raises(CwcError) as e:
        srv.submit(mo, W.make_run(seed=1, replicas=100000, dt=0.5, n_samples=201))
    assert e.value.code == -3
    srv.close()
