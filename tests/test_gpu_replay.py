"""Relaunches and concurrency through the C ABI: the persistent form replays
its captured HIP graph (accumulator reset, simulation, n_k, finalisation);
every replay, with unrelated eager work and synchronisations in between,
must give the first launch's results exactly (which equal the oracle's).
Runs on two streams at once must each equal the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import compare_stats, compare_trajectories, per_trajectory

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


def results(r, want_traj=True):
    out = r.counters()
    out["mean"], out["var"], out["n"] = r.stats()
    out["s1"], out["s2_hi32"], out["s2_lo32"], _ = r.moments()
    if want_traj:
        out["samples"] = per_trajectory(r.trajectories())
    return out


def same(a, b):
    for k in ("events", "status", "digest", "n_recorded", "final_counts", "s1", "s2_hi32",
              "s2_lo32", "n", "samples"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    for k in ("t_final", "mean", "var"):
        x = np.asarray(a[k], np.float64).view(np.uint64)
        y = np.asarray(b[k], np.float64).view(np.uint64)
        assert np.array_equal(x, y), k


def sweep_case():
    """More trajectories than resident lanes at one wave per SIMD, so the
    replays also exercise the queue cursor's reset."""
    m = W.isomerisation(k1=1.0, k2=3.0, a0=12, b0=0)
    tab, _ = W.sweep_rate_table(m, 2800, 5)
    run = W.make_run(seed=31, n_instances=2800, replicas=37, dt=0.2, n_samples=11,
                     rate_table=tab)
    return m, run


@pytest.mark.parametrize("mode,tuning", [
    ("persistent", {"block_size": 64, "waves_per_simd": 1}),
    ("persistent", {"block_size": 64, "waves_per_simd": 1, "lanes_per_replica": 2}),
    ("plain", {"block_size": 128}),
])
def test_replays_equal_first_launch(ctx, mode, tuning):
    import torch
    from paper_1010_2438_amd import Model, Run
    m, run = sweep_case()
    print("case replay", mode, tuning, flush=True)
    mo = Model(ctx, m)
    stream = torch.cuda.Stream()
    r = Run(ctx, mo, run, mode=mode, stream=stream.cuda_stream, want_traj=True,
            want_digest=True, tuning=tuning)
    r.wait()
    first = results(r)
    orc = oracle.simulate(m, run, want_samples=True, threads=8)
    compare_trajectories(first, orc)
    compare_stats(first, orc)
    x = torch.ones(1 << 20, device="cuda")
    for i in range(3):
        # unrelated eager work on the same stream and a full synchronisation
        with torch.cuda.stream(stream):
            x.mul_(1.0001).add_(1.0)
        torch.cuda.synchronize()
        r.relaunch(stream.cuda_stream)
        r.wait()
        same(results(r), first)
    r.close()


def test_concurrent_runs_on_two_streams(ctx):
    import torch
    from paper_1010_2438_amd import Model, Run
    m1, run1 = sweep_case()
    m2, run2 = W.config(1, replicas=700)
    run2 = dict(run2, n_samples=21)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    mo1, mo2 = Model(ctx, m1), Model(ctx, m2)
    ra = Run(ctx, mo1, run1, mode="persistent", stream=s1.cuda_stream, want_traj=True,
             want_digest=True, tuning={"block_size": 64, "waves_per_simd": 1})
    rb = Run(ctx, mo2, run2, mode="plain", stream=s2.cuda_stream, want_traj=True,
             want_digest=True)
    for r in (ra, rb):
        r.relaunch(s1.cuda_stream if r is ra else s2.cuda_stream)
    ra.wait()
    rb.wait()
    for r, m, run in ((ra, m1, run1), (rb, m2, run2)):
        g = results(r)
        orc = oracle.simulate(m, run, want_samples=True, threads=8)
        compare_trajectories(g, orc)
        compare_stats(g, orc)
        r.close()


def test_wait_with_timeout(ctx):
    """The host-side watchdog: a launch still running after the timeout
    reports "not ready" (and keeps running); a later wait sees it end."""
    from paper_1010_2438_amd import Model, Run
    m, run = W.config(2)
    run = dict(run, n_instances=512, rate_table=run["rate_table"][:512])
    r = Run(ctx, Model(ctx, m), run, mode="persistent")
    assert r.wait_for(0.0) is False          # hundreds of milliseconds of work
    assert r.wait_for(120.0) is True
    assert r.wait() is r                     # chains, as the smoke check uses it
    assert int(r.counters()["events"].sum()) > 0
    r.close()


def test_context_closed_before_its_model_and_run(ctx):
    """A context closed while a model and a run still use it stays alive
    until they are destroyed; the run's results stay readable, and no error
    is left behind for the next caller."""
    from paper_1010_2438_amd import Context, Model, Run
    m, run = W.config(0, replicas=64)
    run = dict(run, n_samples=11)
    c = Context(0)
    mo = Model(c, m)
    r = Run(c, mo, run, mode="persistent", want_digest=True)
    c.close()
    r.wait()
    got = r.counters()
    r.close()
    mo.close()
    orc = oracle.simulate(m, run, threads=4)
    assert np.array_equal(got["digest"], orc["digest"])
    # the next user of the device sees a clean state
    r2 = Run(ctx, Model(ctx, m), run, mode="plain", want_digest=True).wait()
    assert np.array_equal(r2.counters()["digest"], orc["digest"])
    r2.close()
