"""The no-allocation entry point (cwc_run_into) through the C ABI: two calls
in a row on one stream -- the second smaller, so it runs on what the first
left in the shared scratch array -- each bit-identical to cwc_run_submit's
results for the same run (statistics, contributor counts and every
per-trajectory output); a run too large for the scratch array is refused
with CWC_E_NOMEM."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import same_float

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


def outputs(mo, run):
    import torch
    I, R, K1, C = run["n_instances"], run["replicas"], run["n_samples"], mo.info["n_cells"]
    G = I * R
    dev = "cuda"
    return {"mean": torch.empty((I, K1, C), dtype=torch.float64, device=dev),
            "var": torch.empty((I, K1, C), dtype=torch.float64, device=dev),
            "n": torch.empty((I, K1), dtype=torch.int64, device=dev),
            "events": torch.empty(G, dtype=torch.int64, device=dev),
            "status": torch.empty(G, dtype=torch.uint8, device=dev),
            "digest": torch.empty(G, dtype=torch.int64, device=dev),
            "t_final": torch.empty(G, dtype=torch.float64, device=dev),
            "n_recorded": torch.empty(G, dtype=torch.int32, device=dev),
            "final_counts": torch.empty((G, C), dtype=torch.int32, device=dev)}


def reference(ctx, mo, run, mode, tuning):
    from paper_1010_2438_amd import Run
    r = Run(ctx, mo, run, mode=mode, want_digest=True, tuning=tuning).wait()
    out = r.counters()
    out["mean"], out["var"], out["n"] = r.stats()
    r.close()
    return out


def check_equal(got, ref):
    for k in ("events", "status", "n_recorded", "final_counts", "n"):
        assert np.array_equal(got[k].cpu().numpy(), ref[k]), k
    assert np.array_equal(got["digest"].cpu().numpy().view(np.uint64), ref["digest"])
    for k in ("t_final", "mean", "var"):
        assert same_float(got[k].cpu().numpy(), ref[k]), k


@pytest.mark.parametrize("which", ["lane", "wave"])
def test_run_into_two_calls_match_submit(ctx, which):
    import torch
    from paper_1010_2438_amd import Model, run_into
    if which == "lane":
        m = W.gene_regulation(1)
        tab, _ = W.sweep_rate_table(m, 40, 2)
        big = W.make_run(seed=7, n_instances=40, replicas=50, dt=0.5, n_samples=41,
                         rate_table=tab)
        small = W.make_run(seed=8, n_instances=3, replicas=33, dt=0.5, n_samples=21,
                           rate_table=tab[5:8])
        mode, tuning = "persistent", {"lanes_per_replica": 2, "block_size": 128,
                                      "waves_per_simd": 1}
    else:
        m = W.multi_compartment(3, n_cells_=8)
        big = W.make_run(seed=7, replicas=70, dt=0.5, n_samples=21)
        small = W.make_run(seed=9, replicas=20, dt=0.5, n_samples=11)
        mode, tuning = "plain", None
    mo = Model(ctx, m)
    stream = torch.cuda.Stream()
    res = []
    for run in (big, small):
        print("case run_into", which, run["n_instances"], run["replicas"], flush=True)
        out = outputs(mo, run)
        rate = None
        if run["rate_table"] is not None:
            rate = torch.from_numpy(run["rate_table"]).to("cuda")
        run_into(ctx, mo, run, out, mode=mode, want_digest=True, tuning=tuning,
                 rate_table=rate, stream=stream)
        res.append((run, out))
    stream.synchronize()
    for run, out in res:
        check_equal(out, reference(ctx, mo, run, mode, tuning))


def test_run_into_refuses_oversized_runs(ctx):
    from paper_1010_2438_amd import CwcError, Model, run_into
    m, run = W.config(2)
    mo = Model(ctx, m)
    with pytest.raises(CwcError) as e:
        run_into(ctx, mo, run, {k: None for k in ("mean",)})
    assert e.value.code == -1                   # missing outputs are checked first
    import torch
    run = W.make_run(seed=0, n_instances=2048, replicas=1, dt=0.5, n_samples=201)
    out = outputs(mo, W.make_run(n_instances=1, replicas=1, n_samples=1))
    with pytest.raises(CwcError) as e:
        run_into(ctx, mo, run, out)            # 2048 x 201 x 20 x 24 B > 32 MiB
    assert e.value.code == -3
    torch.cuda.synchronize()
