"""GPU parity at full size, in the launch configurations the benchmark
times (bench.LAUNCH): each test pins the shape, asserts the name of the
kernel the run dispatches, compares an evenly spread sample of trajectories
one by one with the oracle (two-step procedure of Sec. 2.2, bit for bit:
counts, events, statuses, fired-leaf digests, final times, every recorded
sample), checks every sample of every trajectory against the model's
conservation laws and every moment against the exact integer sums of the
fetched samples, and runs the benchmark's other launches of the same
workload against the first, bit for bit, trajectory by trajectory; the
general-term colony is compared in full with the general oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from bench import LAUNCH
from tests.gpu_common import compare_trajectories, conservation_laws, gpu_run, oracle_ids

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


def kernel_of(ctx, mo, run, mode, tuning):
    from paper_1010_2438_amd import Run
    r = Run(ctx, mo, run, mode=mode, tuning=tuning)
    name = r.kernel_name()
    r.wait()
    r.close()
    return name


def check_moments_and_laws(m, g, I, R, K1):
    """Every sample keeps the model's conservation laws (an integer basis of
    the vectors orthogonal to every slot's net change); S1, S2 and n per
    (instance, sample) are the exact integer sums of the fetched samples."""
    S = g["samples"].reshape(I, R, K1, -1)
    Wl = conservation_laws(m)
    assert Wl.shape[1] > 0
    base = oracle.FlatModel(m).init.astype(np.int64) @ Wl
    assert ((g["final_counts"].astype(np.int64) @ Wl) == base).all()
    nr = g["n_recorded"].reshape(I, R)
    step = max(1, 2000000 // (R * K1))
    for i0 in range(0, I, step):
        blk = S[i0:i0 + step].astype(np.int64)
        rec = np.arange(K1)[None, None, :] < nr[i0:i0 + step, :, None]
        assert ((blk @ Wl)[rec] == base).all()
        blk = blk * rec[..., None]
        assert np.array_equal(g["s1"][i0:i0 + step], blk.sum(axis=1).astype(np.uint64))
        sq = (blk * blk).sum(axis=1)
        got = g["s2_hi32"][i0:i0 + step].astype(np.int64) * 2 ** 32 + \
            g["s2_lo32"][i0:i0 + step].astype(np.int64)
        assert np.array_equal(got, sq)
        assert np.array_equal(g["n"][i0:i0 + step], rec.sum(axis=1))


def same_results(a, b):
    for k in ("events", "status", "digest", "n_recorded", "final_counts", "s1", "s2_hi32",
              "s2_lo32", "n"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["t_final"].view(np.uint64), b["t_final"].view(np.uint64))
    assert np.array_equal(a["mean"].view(np.uint64), b["mean"].view(np.uint64))


def test_sweep_full_size_benchmark_launches(ctx):
    """The sweep (4096 instances x 64 replicas, t_end 100, 201 samples) in
    the benchmark's persistent launch (two lanes per trajectory, block 256,
    16 requested waves per SIMD: the queue-free pair kernel over the
    longest-first order): 1024 trajectories spread over the id range against
    the oracle one by one, laws and moments over all 262,144; then the
    benchmark's two plain launches (one lane per trajectory; two lanes in
    natural order) bit-identical to it."""
    from paper_1010_2438_amd import Model
    m, run = W.config(2)
    I, R, K1 = run["n_instances"], run["replicas"], run["n_samples"]
    mo = Model(ctx, m)
    assert kernel_of(ctx, mo, run, "persistent", LAUNCH["sweep"]) == "cwc_pair_plain_table"
    print("case sweep full size, persistent pair", flush=True)
    g = gpu_run(ctx, mo, run, mode="persistent", tuning=LAUNCH["sweep"])
    assert (g["status"] == 0).all() and (g["n_recorded"] == K1).all()
    ids = np.linspace(0, I * R - 1, 1024).astype(np.int64)
    orc = oracle_ids(m, run, ids)
    compare_trajectories(g, orc, g_index=ids)
    check_moments_and_laws(m, g, I, R, K1)
    samples = g.pop("samples")
    del samples
    for key, name in (("sweep_plain", "cwc_lane_plain_table"),
                      ("sweep_plain_pair", "cwc_pair_plain_table")):
        assert kernel_of(ctx, mo, run, "plain", LAUNCH[key]) == name
        print("case sweep full size,", key, flush=True)
        q = gpu_run(ctx, mo, run, mode="plain", tuning=LAUNCH[key], want_traj=False)
        same_results(q, g)


def test_gene_regulation_full_size_benchmark_launch(ctx):
    """Configuration 1 (16384 replicas, t_end 100) in the benchmark's
    persistent launch (four lanes per trajectory, block 256, one wave per
    SIMD: the queue-free quad kernel): 1024 trajectories against the oracle
    one by one, laws and moments over all; the plain one-lane launch
    bit-identical to it."""
    from paper_1010_2438_amd import Model
    m, run = W.config(1)
    R, K1 = run["replicas"], run["n_samples"]
    mo = Model(ctx, m)
    assert kernel_of(ctx, mo, run, "persistent", LAUNCH[1]) == "cwc_quad_plain_shared"
    print("case gene regulation full size, persistent quad", flush=True)
    g = gpu_run(ctx, mo, run, mode="persistent", tuning=LAUNCH[1])
    assert (g["status"] == 0).all() and (g["n_recorded"] == K1).all()
    ids = np.linspace(0, R - 1, 1024).astype(np.int64)
    compare_trajectories(g, oracle_ids(m, run, ids), g_index=ids)
    check_moments_and_laws(m, g, 1, R, K1)
    print("case gene regulation full size, plain lane", flush=True)
    q = gpu_run(ctx, mo, run, mode="plain", want_traj=False,
                tuning={"block_size": 256, "lanes_per_replica": 1})
    same_results(q, g)


def test_multi_compartment_full_size_benchmark_launch(ctx):
    """Configuration 3 (32 cells, 2048 replicas, t_end 50) in the
    benchmark's persistent launch (one wavefront per trajectory, block 256,
    8 requested waves per SIMD): 128 trajectories spread over the id range
    against the oracle one by one (its full tree rebuild over 2048 leaves
    per event makes more too slow for a test), laws and moments over all."""
    from paper_1010_2438_amd import Model
    m, run = W.config(3)
    R, K1 = run["replicas"], run["n_samples"]
    mo = Model(ctx, m)
    assert kernel_of(ctx, mo, run, "persistent", LAUNCH[3]) == "cwc_wave_plain_shared"
    print("case multi-compartment full size, persistent wave", flush=True)
    g = gpu_run(ctx, mo, run, mode="persistent", tuning=LAUNCH[3])
    assert (g["status"] == 0).all() and (g["n_recorded"] == K1).all()
    ids = np.linspace(0, R - 1, 128).astype(np.int64)
    compare_trajectories(g, oracle_ids(m, run, ids), g_index=ids)
    check_moments_and_laws(m, g, 1, R, K1)


def test_cell_colony_full_size_benchmark_launch(ctx):
    """The general-term cell colony (compartments created and deleted at run
    time; 2048 replicas, t_end 100, 201 samples) in the benchmark's
    persistent launch (one wavefront per trajectory, block 256, 8 requested
    waves per SIMD: the queue-free general kernel): every trajectory against
    the general oracle bit for bit (events, statuses, fired-leaf digests,
    final times, final observables, whole final terms) and the exact
    moments equal."""
    from bench import general_workload
    from paper_1010_2438_amd import GModel, Run
    from tests.gpu_common import RESULT_KEYS, compare_stats, same_float
    m, run = general_workload()
    gm = GModel(ctx, m)
    print("case cell colony full size, persistent general", flush=True)
    r = Run(ctx, gm, run, mode="persistent", tuning=LAUNCH[5], want_digest=True)
    assert r.kernel_name() == "cwc_gen_plain_shared"
    r.wait()
    g = r.counters()
    g["s1"], g["s2_hi32"], g["s2_lo32"], _ = r.moments()
    g["mean"], g["var"], g["n"] = r.stats()
    g["term"] = r.term()
    r.close()
    gm.close()
    orc = oracle.gsimulate(m, run, want_term=True, threads=16)
    for key in RESULT_KEYS:
        assert np.array_equal(g[key], orc[key]), key
    assert same_float(g["t_final"], orc["t_final"])
    assert np.array_equal(g["term"], orc["term"])
    compare_stats(g, orc)
