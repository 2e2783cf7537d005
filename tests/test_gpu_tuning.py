"""Autotuner: returns a valid launch shape, stores it for later submissions,
and the tuned launch is bit-identical to the oracle."""
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


def test_autotune_lane_model(ctx):
    from paper_1010_2438_amd import Model
    m = W.gene_regulation(1)
    run = W.make_run(seed=21, replicas=1500, dt=0.5, n_samples=21)
    mo = Model(ctx, m)
    t = mo.autotune(run, "persistent", budget_s=2.0)
    assert t["block_size"] in (64, 128, 256) and t["waves_per_simd"] in (1, 2, 4, 8, 16)
    assert t["lanes_per_replica"] in (1, 2, 4, 64)
    if t["lanes_per_replica"] in (1, 2, 4):
        assert t["sample_slots"] in (0, 4, 64) and t["refill_chunk"] in (0, 1, 256)
    # a later submission without tuning picks the stored shape; results are
    # the oracle's regardless
    g = gpu_run(ctx, mo, run, mode="persistent")
    orc = oracle.simulate(m, run, want_samples=True, threads=8)
    compare_trajectories(g, orc)
    compare_stats(g, orc)


def test_autotune_wave_only_model(ctx):
    from paper_1010_2438_amd import Model
    m = W.multi_compartment(3, n_cells_=10)
    run = W.make_run(seed=22, replicas=64, dt=0.5, n_samples=11)
    mo = Model(ctx, m)
    t = mo.autotune(run, "plain", budget_s=1.0)
    assert t["lanes_per_replica"] == 64 or mo.info["layout"] == 0
    g = gpu_run(ctx, mo, run, mode="plain")
    orc = oracle.simulate(m, run, want_samples=True, threads=8)
    compare_trajectories(g, orc)
