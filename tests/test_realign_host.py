"""Host: cwc_realign (a trajectory recorded at its own times onto the fixed
sample grid, right-continuous) against its definition written out by brute
force, and against the oracle: the oracle's trajectory sampled on a grid
four times finer, realigned, is the oracle's run on the coarse grid bit for
bit (the random stream does not depend on the sampling grid)."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_1010_2438_amd as P
    P.load()
    return P


def brute(times, values, dt, K1, fill):
    out = np.full((K1, values.shape[1]), fill, np.int32)
    for k in range(K1):
        tk = float(k) * dt
        idx = [i for i in range(len(times)) if times[i] <= tk]
        if idx:
            out[k] = values[max(idx)]
    return out


def test_realign_matches_definition(P):
    rng = np.random.default_rng(7)
    for trial in range(200):
        n = int(rng.integers(0, 30))
        t = np.sort(rng.uniform(-0.5, 6.0, n))
        if n > 3:
            t[2] = t[1]                           # a tie: the later record wins
            t[3] = float(int(rng.integers(0, 20))) * 0.25   # exactly on the grid
            t = np.sort(t)
        v = rng.integers(0, 1000, (n, 3)).astype(np.int32)
        K1 = int(rng.integers(0, 25))
        got = P.realign(t, v, 0.25, K1, fill=-9)
        assert np.array_equal(got, brute(t, v, 0.25, K1, -9)), trial


def test_realign_fine_oracle_grid_equals_coarse_run(P):
    m = W.gene_regulation()
    fine = W.make_run(seed=5, replicas=12, dt=2.0 ** -3, n_samples=4 * 40 + 1)
    coarse = W.make_run(seed=5, replicas=12, dt=2.0 ** -1, n_samples=40 + 1)
    of = oracle.simulate(m, fine, want_samples=True, threads=4)
    oc = oracle.simulate(m, coarse, want_samples=True, threads=4)
    assert (of["status"] == 0).all() and (oc["status"] == 0).all()
    tf = np.arange(fine["n_samples"]) * fine["dt"]
    for g in range(12):
        got = P.realign(tf, of["samples"][g], coarse["dt"], coarse["n_samples"])
        assert np.array_equal(got, oc["samples"][g]), g
    # the trajectories themselves are the same
    assert np.array_equal(of["events"], oc["events"])
    assert np.array_equal(of["final_counts"], oc["final_counts"])


def test_realign_errors(P):
    with pytest.raises(P.CwcError):
        P.realign([1.0, 0.5], np.zeros((2, 1)), 0.1, 5)      # decreasing times
    with pytest.raises(P.CwcError):
        P.realign([0.0], np.zeros((1, 1)), 0.0, 5)           # dt = 0
    with pytest.raises(P.CwcError):
        P.realign([float("nan")], np.zeros((1, 1)), 0.1, 5)
