"""GPU: streamed runs (paper Sec. 5.2 schemas ii and iii) -- the run cut into
windows of sample points, each window one time-sliced launch that stops
every trajectory at the window's end, its statistics handed out while the
next window runs.  Every window's mean, variance and contributor counts
must equal the oracle's rows (exact moments, so bit for bit in practice;
1e-12 relative is the bar), and every trajectory's counters must equal the
oracle's bit for bit, for the two-lane, one-lane and wavefront kernels,
ragged last windows, rate and initial-state tables, and a 10,001-point
horizon whose device memory does not grow with the horizon."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import RESULT_KEYS, same_float

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


def close_rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    both_nan = np.isnan(a) & np.isnan(b)
    ok = both_nan | (np.abs(a - b) <= 1e-12 * np.maximum(np.abs(a), np.abs(b)))
    return bool(ok.all())


def check_stream(ctx, m, run, window, lanes=0, kernel=None):
    from paper_1010_2438_amd import Model, Stream
    print("case stream", m["name"], "window", window, "lanes", lanes,
          "G", run["n_instances"] * run["replicas"], "K1", run["n_samples"], flush=True)
    orc = oracle.simulate(m, run, want_samples=False, threads=8)
    mo = Model(ctx, m)
    s = Stream(ctx, mo, run, window, want_digest=True, lanes_per_replica=lanes)
    info = s.info()
    if kernel:
        assert info["kernel"].startswith(kernel), info["kernel"]
    K1 = run["n_samples"]
    seen = 0
    for k0, mean, var, n in s:
        assert k0 == seen
        rows = mean.shape[1]
        assert rows == min(info["window"], K1 - k0)
        assert np.array_equal(n, orc["n"][:, k0:k0 + rows].astype(np.int64)), k0
        assert close_rel(mean, orc["mean"][:, k0:k0 + rows]), k0
        assert close_rel(var, orc["var"][:, k0:k0 + rows]), k0
        seen += rows
    assert seen == K1
    assert s.info()["windows_done"] == info["n_windows"]
    got = s.counters()
    for key in RESULT_KEYS:
        assert np.array_equal(got[key], orc[key]), key
    assert same_float(got["t_final"], orc["t_final"])
    s.close()
    return info


@pytest.mark.parametrize("lanes,kernel", [(0, "cwc_pair_slice"), (1, "cwc_lane_slice")])
def test_stream_gene_regulation(ctx, lanes, kernel):
    m = W.gene_regulation()
    run = W.make_run(seed=13, n_instances=3, replicas=111, dt=0.5, n_samples=41)
    check_stream(ctx, m, run, window=7, lanes=lanes, kernel=kernel)   # 6 windows, last 6 rows


def test_stream_sweep_tables_and_statuses(ctx):
    m = W.gene_regulation()
    tab, _ = W.sweep_rate_table(m, 24, 5)
    init = np.tile(np.asarray(W.gene_regulation()["init"][0] + W.gene_regulation()["init"][1],
                              np.int32), (24, 1))
    init[::3] //= 2
    run = W.make_run(seed=2, n_instances=24, replicas=5, dt=0.5, n_samples=21,
                     rate_table=tab, init_table=init)
    check_stream(ctx, m, run, window=4)
    # event cap and count cap end trajectories mid-window
    check_stream(ctx, m, dict(run, max_events=3000), window=5)
    check_stream(ctx, m, dict(run, count_cap=260), window=3)


def test_stream_absorbing_and_one_point_windows(ctx):
    check_stream(ctx, W.pure_decay(2.0, 5), W.make_run(replicas=65, dt=0.5, n_samples=30),
                 window=1)
    check_stream(ctx, W.birth_death(), W.make_run(seed=4, replicas=70, dt=0.25, n_samples=9),
                 window=100)   # one window holds the whole run


def test_stream_wavefront_layout(ctx):
    m = W.transport()
    run = W.make_run(seed=8, n_instances=2, replicas=40, dt=0.25, n_samples=33)
    check_stream(ctx, m, run, window=8, lanes=64, kernel="cwc_wave_slice")


def test_stream_long_horizon_bounded_memory(ctx):
    """10,001 sample points in windows of 100: the statistics equal the
    oracle's on every row, and the stream holds exactly as much device
    memory as the same run with 201 points."""
    from paper_1010_2438_amd import Model, Stream
    m = W.birth_death(lam=20.0, mu=1.0, n0=5)
    run = W.make_run(seed=6, replicas=256, dt=0.01, n_samples=10001)
    info = check_stream(ctx, m, run, window=100)
    assert info["n_windows"] == 101
    short = Stream(ctx, Model(ctx, m), dict(run, n_samples=201), 100)
    assert short.info()["device_bytes"] == info["device_bytes"]
    short.close()


def test_stream_confidence_bands_match_run(ctx):
    """The confidence half-widths of the streamed rows equal those of the
    same statistics from one uninterrupted run."""
    from paper_1010_2438_amd import Model, Run, Stream, confidence
    m = W.gene_regulation()
    run = W.make_run(seed=3, n_instances=2, replicas=64, dt=0.5, n_samples=25)
    mo = Model(ctx, m)
    r = Run(ctx, mo, run, mode="persistent")
    r.wait()
    mean, var, n = r.stats()
    r.close()
    s = Stream(ctx, mo, run, 6)
    for k0, wm, wv, wn in s:
        rows = wm.shape[1]
        assert np.array_equal(wn, n[:, k0:k0 + rows])
        assert same_float(wm, mean[:, k0:k0 + rows]) and same_float(wv, var[:, k0:k0 + rows])
        a = confidence(wv, wn)
        b = confidence(var[:, k0:k0 + rows], n[:, k0:k0 + rows])
        assert same_float(a, b)
    s.close()


def check_gstream(ctx, m, run, window):
    """A general model streamed: every window's rows and every trajectory's
    counters and final term against the general oracle."""
    from paper_1010_2438_amd import GModel, Stream
    print("case general stream", m["name"], "window", window,
          "G", run["n_instances"] * run["replicas"], "K1", run["n_samples"], flush=True)
    orc = oracle.gsimulate(m, run, want_term=True, threads=8)
    gm = GModel(ctx, m)
    s = Stream(ctx, gm, run, window, want_digest=True)
    assert s.info()["kernel"].startswith("cwc_gen_slice"), s.info()["kernel"]
    K1, seen = run["n_samples"], 0
    for k0, mean, var, n in s:
        assert k0 == seen
        rows = mean.shape[1]
        assert np.array_equal(n, orc["n"][:, k0:k0 + rows].astype(np.int64)), k0
        assert close_rel(mean, orc["mean"][:, k0:k0 + rows]), k0
        assert close_rel(var, orc["var"][:, k0:k0 + rows]), k0
        seen += rows
    assert seen == K1
    got = s.counters()
    for key in RESULT_KEYS:
        assert np.array_equal(got[key], orc[key]), key
    assert same_float(got["t_final"], orc["t_final"])
    assert np.array_equal(s.term(), orc["term"])
    s.close()
    gm.close()


def test_stream_general_models(ctx):
    """Compartments created, dissolved and deleted across window ends: the
    term is checkpointed between windows; rate tables and the pool-full
    OVERFLOW end trajectories mid-window."""
    check_gstream(ctx, W.cell_colony(n0=3, nutrient=40, max_comp=16, k_up=0.2, k_div=0.4,
                                     k_die=0.1),
                  W.make_run(seed=21, replicas=150, dt=0.25, n_samples=37), window=5)
    check_gstream(ctx, W.cell_dissolution(release_wrap=True),
                  W.make_run(seed=22, replicas=97, dt=0.25, n_samples=17), window=3)
    check_gstream(ctx, W.nested_export(), W.make_run(seed=23, replicas=64, dt=0.25, n_samples=17),
                  window=16)
    m = W.cell_colony(n0=4, nutrient=300, max_comp=24)
    tab = np.tile(np.array([r["k"] for r in m["rules"]]), (4, 1)) * \
        np.array([0.5, 1.0, 2.0, 3.0])[:, None]
    check_gstream(ctx, m, W.make_run(seed=24, n_instances=4, replicas=20, dt=0.5, n_samples=21,
                                     rate_table=tab), window=4)
    check_gstream(ctx, W.cell_birth_death(lam=20.0, mu=0.1, n0=0, max_comp=5),
                  W.make_run(seed=25, replicas=50, dt=0.1, n_samples=40), window=7)


def test_stream_errors(ctx):
    from paper_1010_2438_amd import CwcError, Model, Stream
    m = W.birth_death()
    mo = Model(ctx, m)
    run = W.make_run(replicas=8, n_samples=5)
    with pytest.raises(CwcError):
        Stream(ctx, mo, run, 0)
    with pytest.raises(CwcError):
        Stream(ctx, mo, run, 2, lanes_per_replica=4)
