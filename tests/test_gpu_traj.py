"""GPU: sampled trajectories in the library's layout [sample][cell][trajectory]
(trajectory fastest), fetched to host and device memory, against the
oracle's samples of the same trajectories, for every lane layout (one,
two and four lanes per trajectory, one wavefront per trajectory) and both
forms.  Paper Sec. 3: states at fixed simulation times are the simulator's
output beside the on-line statistics."""
import numpy as np
import pytest

import oracle
import workloads as W

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


CASES = [
    ("gene_regulation", 1, "cwc_lane"),
    ("gene_regulation", 2, "cwc_pair"),
    ("gene_regulation", 4, "cwc_quad"),
    ("transport", 64, "cwc_wave"),
]


@pytest.mark.parametrize("name,lanes,family", CASES)
@pytest.mark.parametrize("mode", ["plain", "persistent"])
def test_trajectory_layout(ctx, name, lanes, family, mode):
    import torch
    from paper_1010_2438_amd import Model, Run
    m = getattr(W, name)()
    # 333 trajectories: several wavefronts of every layout and a ragged tail
    run = W.make_run(seed=21, n_instances=3, replicas=111, dt=0.5, n_samples=17)
    tuning = {"lanes_per_replica": lanes, "block_size": 64, "waves_per_simd": 1}
    print("case traj layout", name, lanes, mode, flush=True)
    orc = oracle.simulate(m, run, want_samples=True, threads=8)
    mo = Model(ctx, m)
    r = Run(ctx, mo, run, mode=mode, want_traj=True, tuning=tuning)
    r.wait()
    assert r.kernel_name().startswith(family)
    K1, C, G = run["n_samples"], mo.info["n_cells"], 333
    t = r.trajectories()
    assert t.shape == (K1, C, G) and t.flags["C_CONTIGUOUS"]
    dev = torch.full((K1, C, G), -7, dtype=torch.int32, device="cuda")
    r.trajectories(out=dev)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), t)
    flat = t.ravel()
    nrec = orc["n_recorded"]
    assert np.array_equal(r.counters()["n_recorded"], nrec)
    r.close()
    for g in range(G):
        for k in range(int(nrec[g])):
            # element (k, c, g) at offset (k * C + c) * G + g
            got = flat[(k * C + np.arange(C)) * G + g]
            assert np.array_equal(got, orc["samples"][g, k]), (g, k)
