"""GPU: general CWC models (compartments created, dissolved and deleted at
run time; patterns two levels deep) through the C ABI against the general
oracle on the same seeded inputs.  Per trajectory bit for bit: applied
events, status, fired-leaf digest, recorded samples, final time, final
observables, every sampled observable, and the whole final term (each
slot's liveness, label, parent, wrap and content); exact moments equal and
mean/variance within 1e-12 relative.  Models without structural actions
must also give the fixed-tree kernels' trajectories."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.gpu_common import RESULT_KEYS, compare_stats, per_trajectory, same_float

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


def run_gpu(ctx, gm, run, mode, tuning=None):
    from paper_1010_2438_amd import Run
    r = Run(ctx, gm, run, mode=mode, want_traj=True, want_digest=True, tuning=tuning)
    r.wait()
    out = r.counters()
    out["mean"], out["var"], out["n"] = r.stats()
    out["s1"], out["s2_hi32"], out["s2_lo32"], _ = r.moments()
    out["samples"] = per_trajectory(r.trajectories())
    out["term"] = r.term()
    out["kernel"] = r.kernel_name()
    r.close()
    return out


def check(ctx, m, run, modes=("plain", "persistent"), tuning=None):
    from paper_1010_2438_amd import GModel
    orc = oracle.gsimulate(m, run, want_samples=True, want_term=True, threads=8)
    gm = GModel(ctx, m)
    for mode in modes:
        print("case general", m["name"], "mode", mode, "G",
              run["n_instances"] * run["replicas"], flush=True)
        g = run_gpu(ctx, gm, run, mode, tuning)
        assert g["kernel"].startswith("cwc_gen_")
        for key in RESULT_KEYS:
            assert np.array_equal(g[key], orc[key]), (key, np.argwhere(g[key] != orc[key])[:4])
        assert same_float(g["t_final"], orc["t_final"])
        assert np.array_equal(g["term"], orc["term"])
        for i, nr in enumerate(orc["n_recorded"]):
            assert np.array_equal(g["samples"][i, :nr], orc["samples"][i, :nr]), i
        compare_stats(g, orc)
    gm.close()
    return orc


DYNAMIC = {
    "cell_birth_death": lambda: W.cell_birth_death(lam=3.0, mu=1.0, n0=2, max_comp=12),
    "dissolution_release_wrap": lambda: W.cell_dissolution(release_wrap=True),
    "dissolution_drop_wrap": lambda: W.cell_dissolution(release_wrap=False),
    "nested_export_depth2": lambda: W.nested_export(),
    "receptor_internalisation": lambda: W.receptor_internalisation(),
    "colony_small": lambda: W.cell_colony(n0=2, nutrient=4, k_feed=0.0, max_comp=6,
                                          k_up=0.3, k_div=0.5, k_die=0.1),
}


@pytest.mark.parametrize("name", sorted(DYNAMIC))
def test_dynamic_models(ctx, name):
    check(ctx, DYNAMIC[name](), W.make_run(seed=5, replicas=333, dt=0.25, n_samples=17))


def test_cell_colony_64_slots(ctx):
    """The colony at its full pool (64 slots, one per lane): division
    creates cells until the pool is full, deaths free slots for reuse."""
    orc = check(ctx, W.cell_colony(), W.make_run(seed=7, replicas=96, dt=0.5, n_samples=41))
    assert (orc["term"][:, :, 0].sum(axis=1) > 9).any()          # the colony grew


def test_rate_table_and_statuses(ctx):
    m = W.cell_colony(n0=4, nutrient=300, max_comp=24)
    tab = np.tile(np.array([r["k"] for r in m["rules"]]), (6, 1)) * \
        np.array([0.5, 1.0, 2.0, 0.7, 1.3, 3.0])[:, None]
    run = W.make_run(seed=3, n_instances=6, replicas=20, dt=0.5, n_samples=21, rate_table=tab)
    check(ctx, m, run)
    check(ctx, m, dict(run, max_events=400))                   # EVENT_CAP
    check(ctx, m, dict(run, count_cap=320))                    # OVERFLOW by count
    o = check(ctx, W.cell_birth_death(lam=20.0, mu=0.1, n0=0, max_comp=5),
              W.make_run(seed=1, replicas=50, dt=0.1, n_samples=40))
    assert (o["status"] == 2).all()                             # OVERFLOW: pool full


@pytest.mark.parametrize("which", ["lotka_volterra", "transport", "multi_compartment"])
def test_fixed_tree_models_as_general(ctx, which):
    """Without structural actions the general engine gives the fixed-tree
    oracle's and the fixed-tree kernels' trajectories."""
    from tests.gpu_common import gpu_run
    from paper_1010_2438_amd import Model
    fixed = {"lotka_volterra": (W.lotka_volterra(), W.make_run(seed=2, replicas=70, dt=0.05, n_samples=21)),
             "transport": (W.transport(), W.make_run(seed=3, replicas=70, dt=0.25, n_samples=21)),
             "multi_compartment": (W.multi_compartment(3, n_cells_=8),
                                   W.make_run(seed=4, replicas=16, dt=0.5, n_samples=11))}[which]
    m, run = fixed
    orc = check(ctx, W.general_from_fixed(m), run, modes=("persistent",))
    mo = Model(ctx, m)
    f = gpu_run(ctx, mo, run, mode="plain", want_traj=False)
    for key in ("events", "digest", "status", "n_recorded"):
        assert np.array_equal(f[key], orc[key]), key
    assert same_float(f["t_final"], orc["t_final"])


def test_general_model_errors(ctx):
    from paper_1010_2438_amd import CwcError, GModel, Run, Server, Stream
    m = W.cell_dissolution()
    gm = GModel(ctx, m)
    run = W.make_run(replicas=8, n_samples=5)
    with pytest.raises(CwcError) as e:
        Run(ctx, gm, run, tuning={"lanes_per_replica": 2})
    assert e.value.code == -2
    with pytest.raises(CwcError):
        Run(ctx, gm, dict(run, init_table=np.zeros((1, gm.info["n_cells"]), np.int32)))
    with pytest.raises(CwcError) as e:
        Stream(ctx, gm, run, 2, lanes_per_replica=2)          # one wavefront per trajectory
    assert e.value.code == -2
    srv = Server(ctx, hbm_budget=8 << 20, max_active=2, slice_events=1024)
    with pytest.raises(CwcError):
        srv.submit(gm, dict(run, init_table=np.zeros((1, gm.info["n_cells"]), np.int32)))
    srv.close()
    gm.close()
