"""The oracle's trajectories follow the CTMC the paper defines (Sec. 2.2):
compared with closed forms and with brute-force CTMC solutions whose rates
come from enumerating reactant combinations (tests/ctmc.py)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W
from tests import ctmc


def run_oracle(model, R, dt, K1, seed=0, **kw):
    run = W.make_run(seed=seed, replicas=R, dt=dt, n_samples=K1, **kw)
    return oracle.simulate(model, run, want_samples=True, threads=4)


def check_against_ctmc(model, R, dt, K1, max_count=60, zmax=5.5, seed=0,
                       chi_at=None):
    times = [k * dt for k in range(K1)]
    states, dists = ctmc.solve(model, times, max_count=max_count)
    vals = ctmc.cell_values(model, states)
    lost = 1.0 - dists.sum(axis=1)
    assert lost.max() < 1e-9, "truncated probability mass %.3g" % lost.max()
    res = run_oracle(model, R, dt, K1, seed=seed)
    S = res["samples"].astype(np.float64)          # [R][K1][C]
    assert (res["n_recorded"] == K1).all()
    for k in range(K1):
        mu = dists[k] @ vals
        var = dists[k] @ (vals - mu) ** 2
        m4 = dists[k] @ (vals - mu) ** 4
        emp = S[:, k, :]
        em, ev = emp.mean(axis=0), emp.var(axis=0, ddof=1)
        for c in range(vals.shape[1]):
            if var[c] < 1e-14:
                assert np.all(emp[:, c] == mu[c]), (k, c)
                continue
            z = (em[c] - mu[c]) / math.sqrt(var[c] / R)
            assert abs(z) < zmax, ("mean", k, c, em[c], mu[c], z)
            se_v = math.sqrt(max(m4[c] - var[c] ** 2, 1e-30) / R)
            zv = (ev[c] - var[c]) / se_v
            assert abs(zv) < zmax + 1, ("var", k, c, ev[c], var[c], zv)
    if chi_at is not None:
        # chi-square on the full joint distribution at one sample time
        k = chi_at
        idx = {tuple(v): i for i, v in enumerate(vals.astype(np.int64))}
        obs = np.zeros(len(states))
        for row in S[:, k, :].astype(np.int64):
            obs[idx[tuple(row)]] += 1
        exp = dists[k] * R
        big = exp >= 5
        o = np.append(obs[big], obs[~big].sum())
        e = np.append(exp[big], exp[~big].sum())
        if e[-1] < 5:
            o[-2] += o[-1]; e[-2] += e[-1]
            o, e = o[:-1], e[:-1]
        chi2 = ((o - e) ** 2 / e).sum()
        p = stats.chi2.sf(chi2, len(o) - 1)
        assert p > 1e-6, (chi2, len(o), p)
    return res


def test_paper_example_ctmc():
    """a a b b with a b X -> c X: rate 4k, then 1k after one firing."""
    check_against_ctmc(W.paper_example(k=0.5), R=20000, dt=0.25, K1=9, chi_at=3)


def test_dimerisation_binomial_2_not_n_squared():
    """A + A -> 0 uses C(n,2) combinations: separates C(n,2), n(n-1), n^2."""
    model = W.dimerisation(k=0.05, n0=30)
    res = check_against_ctmc(model, R=20000, dt=0.2, K1=11, chi_at=5)
    # the same test fails for a law with twice the rate (n(n-1) instead of C(n,2))
    wrong = W.dimerisation(k=0.10, n0=30)
    states, dists = ctmc.solve(wrong, [0.2 * 5])
    mu_wrong = dists[0] @ ctmc.cell_values(wrong, states)
    em = res["samples"][:, 5, 0].mean()
    assert abs(em - mu_wrong[0]) > 10 * res["samples"][:, 5, 0].std() / math.sqrt(20000)


def test_isomerisation_transient_binomial():
    """A <-> B from (N,0): A(t) ~ Binomial(N, p(t)),
    p(t) = k2/(k1+k2) + k1/(k1+k2) exp(-(k1+k2) t)."""
    k1, k2, N = 1.0, 3.0, 40
    R, dt, K1 = 20000, 0.1, 21
    res = run_oracle(W.isomerisation(k1, k2, N, 0), R, dt, K1)
    S = res["samples"]
    assert (S.sum(axis=2) == N).all()                       # conservation
    for k in range(K1):
        t = k * dt
        p = k2 / (k1 + k2) + k1 / (k1 + k2) * math.exp(-(k1 + k2) * t)
        a = S[:, k, 0]
        assert abs(a.mean() - N * p) < 5 * math.sqrt(max(N * p * (1 - p), 1e-12) / R) + 1e-12
    # full law at t = 1: chi-square against Binomial(N, p)
    t = 1.0
    p = k2 / (k1 + k2) + k1 / (k1 + k2) * math.exp(-(k1 + k2) * t)
    a = S[:, 10, 0]
    exp = stats.binom.pmf(np.arange(N + 1), N, p) * R
    obs = np.bincount(a, minlength=N + 1)
    big = exp >= 5
    chi2 = ((obs[big] - exp[big]) ** 2 / exp[big]).sum()
    assert stats.chi2.sf(chi2, big.sum() - 1) > 1e-6


def test_pure_decay_binomial():
    """A -> 0: A(t) ~ Binomial(n0, exp(-k t)); absorbed once all decayed."""
    k, n0 = 0.7, 50
    R, dt, K1 = 20000, 0.5, 21
    res = run_oracle(W.pure_decay(k, n0), R, dt, K1)
    S = res["samples"][:, :, 0]
    for kk in range(K1):
        p = math.exp(-k * kk * dt)
        assert abs(S[:, kk].mean() - n0 * p) < 5 * math.sqrt(n0 * p * (1 - p) / R) + 1e-12
    # replicas that reached 0 before t_end are absorbed, with all samples filled
    done = res["final_counts"][:, 0] == 0
    assert (res["status"][done] == 1).all() and (res["status"][~done] == 0).all()
    assert (res["n_recorded"] == K1).all()
    assert (res["events"][done] == n0).all()


def test_birth_death_poisson():
    """0 -> A (lam), A -> 0 (mu): from 0, A(t) ~ Poisson(lam/mu (1-e^{-mu t}));
    stationary Poisson(lam/mu)."""
    lam, mu = 20.0, 1.0
    R, dt, K1 = 20000, 0.5, 21
    res = run_oracle(W.birth_death(lam, mu, 0), R, dt, K1)
    S = res["samples"][:, :, 0]
    for k in range(K1):
        m = lam / mu * (1 - math.exp(-mu * k * dt))
        assert abs(S[:, k].mean() - m) < 5 * math.sqrt(max(m, 1e-12) / R) + 1e-12
        if m > 1:
            assert abs(S[:, k].var(ddof=1) - m) < 6 * math.sqrt((m + 2 * m * m) / R)
    a = S[:, -1]
    m = lam / mu * (1 - math.exp(-mu * 10.0))
    xs = np.arange(0, 60)
    exp = stats.poisson.pmf(xs, m) * R
    obs = np.bincount(a, minlength=60)[:60]
    big = exp >= 5
    chi2 = ((obs[big] - exp[big]) ** 2 / exp[big]).sum()
    assert stats.chi2.sf(chi2, big.sum() - 1) > 1e-6


def test_transport_stationary_multinomial():
    """x moves into each of m children at k_in per outer atom and out at
    k_out per inner atom: stationary p_outer = k_out / (k_out + m k_in)."""
    k_in, k_out, m, n = 2.0, 1.0, 3, 30
    model = W.transport(k_in, k_out, m, n)
    R, dt, K1 = 10000, 2.0, 6
    res = run_oracle(model, R, dt, K1)
    S = res["samples"]
    assert (S.sum(axis=2) == n).all()                        # atoms conserved
    p_out = k_out / (k_out + m * k_in)
    outer = S[:, -1, 0]
    assert abs(outer.mean() - n * p_out) < 5 * math.sqrt(n * p_out * (1 - p_out) / R)
    for j in range(1, m + 1):
        pj = k_in / (k_out + m * k_in)
        assert abs(S[:, -1, j].mean() - n * pj) < 5 * math.sqrt(n * pj * (1 - pj) / R)


def test_transport_transient_ctmc():
    check_against_ctmc(W.transport(2.0, 1.0, 2, 6), R=20000, dt=0.1, K1=11, chi_at=4)


def test_receptor_binding_wrap_ctmc():
    """Patterns over a parent's content and a child's wrap; rewrite of wrap
    and content across the membrane."""
    model = W.receptor_binding(k_on=0.2, k_off=0.5, k_int=0.3, n_lig=5, n_rec=2,
                               n_cells_=2)
    check_against_ctmc(model, R=20000, dt=0.5, K1=9, chi_at=4)


def test_gene_regulation_like_ctmc():
    """Two compartments with local and membrane-crossing rules (a reduced,
    bounded version of the gene-regulation workload's structure)."""
    m = W.gene_regulation(1)
    # keep nucleus gene switching, mRNA export, mRNA decay; tiny counts
    keep = [0, 2, 3, 6, 10, 16, 18]
    m["rules"] = [dict(m["rules"][i]) for i in keep]
    for r, k in zip(m["rules"], [0.5, 0.3, 0.8, 0.4, 0.6, 1.0, 0.7]):
        r["k"] = k
    z = [0] * 10
    m["init"] = [list(z), list(z)]
    m["init"][1][0] = 1       # one G1 gene in the nucleus
    m["init"][0][8] = 2       # two D1 in the cytoplasm
    m["init"][1][9] = 2       # two D2 in the nucleus
    check_against_ctmc(m, R=20000, dt=0.5, K1=9, max_count=12, chi_at=6)


def test_time_dilation_invariance():
    """Scaling every rate by 2^m and dt by 2^-m gives the same fired-slot
    sequence and samples; times scale exactly by 2^-m."""
    model, run = W.config(0, replicas=16)
    run["n_samples"] = 11
    base = oracle.simulate(model, run, want_samples=True)
    for m in (-3, 2):
        mm = W.lotka_volterra(k=tuple(k * 2.0 ** m for k in (10.0, 0.01, 10.0)))
        rr = dict(run, dt=run["dt"] * 2.0 ** -m)
        sc = oracle.simulate(mm, rr, want_samples=True)
        assert (sc["digest"] == base["digest"]).all()
        assert (sc["samples"] == base["samples"]).all()
        assert (sc["t_final"] == base["t_final"] * 2.0 ** -m).all()


def test_thread_count_invariance():
    model, run = W.config(0, replicas=24)
    run["n_samples"] = 21
    a = oracle.simulate(model, run, threads=1)
    b = oracle.simulate(model, run, threads=5)
    for key in ("digest", "events", "t_final", "n", "s1", "s2_lo", "s2_hi"):
        assert (a[key] == b[key]).all(), key
    assert np.array_equal(a["mean"], b["mean"]) and np.array_equal(a["var"], b["var"])


@pytest.mark.parametrize("name", ["gene_regulation", "multi_compartment", "transport",
                                  "receptor_binding"])
def test_trajectories_keep_conservation_laws(name):
    """Every sample of every oracle trajectory keeps each conservation law of
    the model, the laws taken from the net changes that the brute-force
    chain (tests/ctmc.py) enumerates from the model itself, in a state where
    every rule can fire in every context."""
    from tests.gpu_common import integer_null_space
    m = {"gene_regulation": lambda: W.config(1)[0],
         "multi_compartment": lambda: W.multi_compartment(3, n_cells_=4),
         "transport": W.transport, "receptor_binding": W.receptor_binding}[name]()
    rich = dict(m, init=[[5] * len(r) for r in m["init"]],
                init_wrap=[None if w is None else [5] * len(w)
                           for w in (m.get("init_wrap") or [None] * len(m["init"]))])
    s0 = ctmc.initial_state(rich)
    base = ctmc.cell_values(rich, [s0])[0]
    rows = [ctmc.cell_values(rich, [nxt])[0] - base for _, nxt in ctmc.transitions(rich, s0)]
    C = len(base)
    Wl = integer_null_space([[int(x) for x in r] for r in rows], C)
    assert Wl.shape[1] > 0
    run = W.make_run(seed=17, replicas=12, dt=0.5, n_samples=21)
    res = oracle.simulate(m, run, want_samples=True, want_stats=False)
    init = oracle.FlatModel(m).init.astype(np.int64)
    assert ((res["samples"].astype(np.int64) @ Wl) == init @ Wl).all()
    assert ((res["final_counts"].astype(np.int64) @ Wl) == init @ Wl).all()
