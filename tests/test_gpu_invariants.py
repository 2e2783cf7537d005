"""Invariants of the GPU path that hold independently of the oracle, and
edge cases of the failure statuses.

* A trajectory depends only on (seed, trajectory id): running the first
  100 of 333 replicas alone, in any layout or form, gives the same bits.
* Scaling every rate by 2^m and dt by 2^-m dilates time exactly: the same
  fired leaves, counts and samples, every time scaled by 2^-m.
* Failure statuses at their edges (max_events = 1, a count starting at the
  cap, counts near INT32_MAX) agree with the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import compare_stats, compare_trajectories, gpu_run

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


_models = {}


def model(ctx, m):
    from paper_1010_2438_amd import Model
    key = repr(m)
    if key not in _models:
        _models[key] = Model(ctx, m)
    return _models[key]


KEYS = ("events", "status", "digest", "n_recorded", "final_counts")


@pytest.mark.parametrize("tuning", [None, {"lanes_per_replica": 2},
                                    {"block_size": 256, "waves_per_simd": 1}])
def test_prefix_of_a_batch(ctx, tuning):
    m, run = W.config(1, replicas=333)
    run = dict(run, n_samples=21)
    big = gpu_run(ctx, model(ctx, m), run, mode="persistent", tuning=tuning)
    small = gpu_run(ctx, model(ctx, m), dict(run, replicas=100), mode="plain")
    for k in KEYS:
        assert np.array_equal(np.asarray(big[k])[:100], np.asarray(small[k])), k
    assert np.array_equal(big["t_final"][:100].view(np.uint64),
                          small["t_final"].view(np.uint64))
    assert np.array_equal(big["samples"][:100], small["samples"])


@pytest.mark.parametrize("mexp", [1, -2])
def test_rate_scaling_dilates_time(ctx, mexp):
    base = W.lotka_volterra(x0=300, y0=300, k=(1.0, 0.005, 1.0))
    scaled = W.lotka_volterra(x0=300, y0=300, k=tuple(k * 2.0 ** mexp for k in (1.0, 0.005, 1.0)))
    run = W.make_run(seed=9, replicas=200, dt=0.25, n_samples=41)
    a = gpu_run(ctx, model(ctx, base), run, mode="plain")
    b = gpu_run(ctx, model(ctx, scaled), dict(run, dt=0.25 * 2.0 ** -mexp), mode="plain",
                tuning={"lanes_per_replica": 2})
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    assert np.array_equal(a["samples"], b["samples"])
    assert np.array_equal(a["t_final"] * 2.0 ** -mexp, b["t_final"])


def check(ctx, m, run, tuning=None):
    orc = oracle.simulate(m, run, want_samples=True, threads=8)
    for mode in ("plain", "persistent"):
        g = gpu_run(ctx, model(ctx, m), run, mode=mode, tuning=tuning)
        compare_trajectories(g, orc)
        compare_stats(g, orc)
    return orc


@pytest.mark.parametrize("tuning", [None, {"lanes_per_replica": 2}])
def test_status_edges(ctx, tuning):
    lv = W.lotka_volterra()
    run = W.make_run(seed=4, replicas=70, dt=0.05, n_samples=11)
    o = check(ctx, lv, dict(run, max_events=1), tuning)              # one event each
    assert (o["status"] == 3).all() and (o["events"] == 1).all()
    o = check(ctx, lv, dict(run, count_cap=1000), tuning)            # starts at the cap
    assert (o["status"] == 2).any()
    near = W.lotka_volterra(x0=2 ** 31 - 3, y0=0)                      # prey only, near INT32_MAX
    o = check(ctx, near, W.make_run(seed=5, replicas=65, dt=1e-9, n_samples=6), tuning)
    assert (o["status"] == 2).all() and (o["final_counts"][:, 0] <= 2 ** 31 - 1).all()


@pytest.mark.parametrize("bad", [
    {"replicas": 0}, {"n_instances": 0}, {"dt": 0.0}, {"dt": float("inf")},
    {"n_samples": 0}, {"count_cap": 0}, {"max_events": -1}, {"count_cap": 999},
])
def test_run_validation(ctx, bad):
    """Malformed run descriptors are refused with CWC_E_INVALID before any
    device work (count_cap 999 is below the model's initial 1000)."""
    from paper_1010_2438_amd import CwcError
    m, run = W.config(0)
    with pytest.raises(CwcError) as e:
        gpu_run(ctx, model(ctx, m), dict(run, **bad), mode="plain")
    assert e.value.code == -1


def test_rate_and_init_table_validation(ctx):
    from paper_1010_2438_amd import CwcError
    m, run = W.config(0)
    tab = np.array([[10.0, 0.01, 10.0], [10.0, 0.0, 10.0]])
    with pytest.raises(CwcError) as e:
        gpu_run(ctx, model(ctx, m), dict(run, n_instances=2, replicas=4, rate_table=tab))
    assert e.value.code == -1
    init = np.array([[10, 10], [-1, 3]], np.int32)
    with pytest.raises(CwcError) as e:
        gpu_run(ctx, model(ctx, m), dict(run, n_instances=2, replicas=4, init_table=init))
    assert e.value.code == -1
