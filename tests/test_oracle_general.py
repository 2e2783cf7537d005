"""The general-CWC oracle (oracle/gcwc.c: compartments created, dissolved and
deleted at run time; patterns two levels deep), pinned three ways:

* on models without structural actions it is the fixed-tree oracle, bit
  for bit (events, fired-leaf digests, final times, statuses, every count);
* the number of cells of a cell birth-death model follows its closed form,
  Binomial(n0, e^-mu t) + Poisson(lam/mu (1 - e^-mu t));
* the observables of models with creation, dissolution (with and without
  released wraps), deletion, wrap patterns and depth-2 patterns follow the
  distribution of a brute-force chain over nested terms written directly
  from the calculus (tests/ctmc_terms.py), checked by chi-square at
  several times, overflow of the compartment pool included;
plus conservation laws and a hand-computed first event."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W
from tests import ctmc_terms


def cells_from_term(term, fm, ns):
    out = np.zeros((term.shape[0], fm.n_cells), np.int32)
    for i in range(fm.n_comp):
        out[:, fm.content_base[i]:fm.content_base[i] + ns] = term[:, i, 3 + ns:3 + 2 * ns]
        if fm.wrap_base[i] >= 0:
            out[:, fm.wrap_base[i]:fm.wrap_base[i] + ns] = term[:, i, 3:3 + ns]
    return out


FIXED = {
    "lotka_volterra": lambda: (W.lotka_volterra(), W.make_run(seed=1, replicas=24, dt=0.05, n_samples=41)),
    "gene_regulation_sweep": lambda: (W.gene_regulation(), W.make_run(
        seed=2, n_instances=6, replicas=4, dt=0.5, n_samples=21,
        rate_table=W.sweep_rate_table(W.gene_regulation(), 6, 9)[0])),
    "multi_compartment": lambda: (W.multi_compartment(3, n_cells_=8), W.make_run(seed=3, replicas=6, dt=0.5, n_samples=11)),
    "transport": lambda: (W.transport(), W.make_run(seed=4, replicas=60, dt=0.25, n_samples=21)),
    "receptor_binding": lambda: (W.receptor_binding(), W.make_run(seed=5, replicas=60, dt=0.25, n_samples=21)),
    "paper_example": lambda: (W.paper_example(), W.make_run(seed=6, replicas=60, dt=0.25, n_samples=21)),
    "statuses": lambda: (W.lotka_volterra(), W.make_run(seed=7, replicas=30, dt=0.05, n_samples=41,
                                                        count_cap=1050, max_events=4000)),
}


@pytest.mark.parametrize("name", sorted(FIXED))
def test_fixed_tree_models_equal_the_fixed_tree_oracle(name):
    m, run = FIXED[name]()
    a = oracle.simulate(m, run, threads=4)
    b = oracle.gsimulate(W.general_from_fixed(m), run, want_term=True, threads=4)
    for key in ("events", "digest", "status", "n_recorded"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["t_final"].view(np.uint64), b["t_final"].view(np.uint64))
    assert np.array_equal(cells_from_term(b["term"], a["flat"], len(m["species"])), a["final_counts"])
    assert (b["term"][:, :, 0] == 1).all()                    # nothing created or removed


def chi_square_p(obs_rows, states, P, model, zero_ok=1e-12):
    """p-value of the empirical distribution of observable tuples (None =
    not recorded: overflow) against the chain's distribution P."""
    dist = {}
    for s, p in zip(states, P):
        key = "OVF" if s == ctmc_terms.OVERFLOW else ctmc_terms.observables(model, s)
        dist[key] = dist.get(key, 0.0) + p
    n = len(obs_rows)
    counts = {}
    for row in obs_rows:
        key = "OVF" if row is None else tuple(int(x) for x in row)
        assert key in dist and dist[key] > zero_ok, ("impossible observation", key)
        counts[key] = counts.get(key, 0) + 1
    keys = sorted(dist, key=lambda k: -dist[k])
    o = np.array([counts.get(k, 0) for k in keys], float)
    e = np.array([dist[k] * n for k in keys])
    big = e >= 5
    o2 = np.append(o[big], o[~big].sum())
    e2 = np.append(e[big], e[~big].sum())
    if e2[-1] < 5 and len(e2) > 1:
        o2[-2] += o2[-1]
        e2[-2] += e2[-1]
        o2, e2 = o2[:-1], e2[:-1]
    if len(o2) < 2:
        return 1.0
    chi2 = ((o2 - e2) ** 2 / e2).sum()
    return stats.chi2.sf(chi2, len(o2) - 1)


DYNAMIC = {
    "cell_birth_death": lambda: W.cell_birth_death(lam=3.0, mu=1.0, n0=2, max_comp=12),
    "dissolution_release_wrap": lambda: W.cell_dissolution(release_wrap=True),
    "dissolution_drop_wrap": lambda: W.cell_dissolution(release_wrap=False),
    "nested_export_depth2": lambda: W.nested_export(),
    "receptor_internalisation": lambda: W.receptor_internalisation(),
    "colony_division": lambda: W.cell_colony(n0=2, nutrient=4, k_feed=0.0, max_comp=6,
                                             k_up=0.3, k_div=0.5, k_die=0.1),
}


@pytest.mark.parametrize("name", sorted(DYNAMIC))
def test_dynamic_models_follow_the_term_chain(name):
    m = DYNAMIC[name]()
    R, dt, K1 = 20000, 0.5, 7
    run = W.make_run(seed=11, replicas=R, dt=dt, n_samples=K1)
    res = oracle.gsimulate(m, run, want_samples=True, want_stats=False, threads=8)
    times = [k * dt for k in range(K1)]
    states, P = ctmc_terms.transient(m, times)
    for k in (1, 3, 6):
        rows = [res["samples"][g, k] if k < res["n_recorded"][g] else None for g in range(R)]
        p = chi_square_p(rows, states, P[k], m)
        assert p > 1e-5, (name, k, p)


def test_cell_count_closed_form():
    lam, mu, n0 = 3.0, 1.0, 2
    m = W.cell_birth_death(lam=lam, mu=mu, n0=n0, max_comp=40)
    R, dt, K1 = 40000, 0.4, 9
    res = oracle.gsimulate(m, W.make_run(seed=3, replicas=R, dt=dt, n_samples=K1),
                           want_samples=True, want_stats=False, threads=8)
    assert (res["n_recorded"] == K1).all()
    cnt = res["samples"][:, :, -1]                     # cell.count, the last observable
    for k in range(1, K1):
        t = k * dt
        q = math.exp(-mu * t)
        pois = lam / mu * (1 - q)
        pmf = np.convolve(stats.binom.pmf(np.arange(n0 + 1), n0, q),
                          stats.poisson.pmf(np.arange(40), pois))[:40]
        obs = np.bincount(cnt[:, k], minlength=40)[:40].astype(float)
        e = pmf * R
        big = e >= 5
        o2, e2 = np.append(obs[big], obs[~big].sum()), np.append(e[big], e[~big].sum())
        chi2 = ((o2 - e2) ** 2 / np.maximum(e2, 1e-300)).sum()
        assert stats.chi2.sf(chi2, len(o2) - 1) > 1e-5, k
        mean = n0 * q + pois
        assert abs(cnt[:, k].mean() - mean) < 5 * math.sqrt(mean / R) + 1e-9


def test_conservation_laws():
    # dissolution releasing the wrap: w is never made or destroyed
    m = W.cell_dissolution(release_wrap=True, n_cells_=4)
    gm = oracle.GModel(m)
    res = oracle.gsimulate(m, W.make_run(seed=2, replicas=500, dt=0.25, n_samples=21),
                           want_samples=True, want_stats=False, threads=4, gm=gm)
    names = gm.obs_names
    w = res["samples"][:, :, names.index("top.w")] + res["samples"][:, :, names.index("cell.w")] + \
        res["samples"][:, :, names.index("cell.wrap.w")]
    assert (w == 4).all()
    # receptor internalisation: ligand + every bound receptor, and receptors
    m = W.receptor_internalisation()
    gm = oracle.GModel(m)
    res = oracle.gsimulate(m, W.make_run(seed=3, replicas=500, dt=0.25, n_samples=21),
                           want_samples=True, want_stats=False, threads=4, gm=gm)
    S = res["samples"]
    names = gm.obs_names
    col = {n: S[:, :, i] for i, n in enumerate(names)}
    rl = sum(col[n] for n in names if n.endswith(".RL"))
    r = sum(col[n] for n in names if n.endswith(".R"))
    assert (col["top.L"] + rl == 4).all()
    assert (r + rl == 2 * 3).all()
    # vesicles exist only while their receptor has not been released
    assert (col["ves.count"] == col["ves.wrap.RL"]).all()


def test_pool_overflow_and_final_term():
    """Cells appear faster than they go in a pool of 5 slots: the event that
    needs a sixth slot ends the trajectory (OVERFLOW), its later samples are
    not recorded, and the final term holds five live compartments."""
    m = W.cell_birth_death(lam=20.0, mu=0.1, n0=0, max_comp=5)
    res = oracle.gsimulate(m, W.make_run(seed=1, replicas=50, dt=0.1, n_samples=40),
                           want_samples=True, want_term=True, threads=4)
    assert (res["status"] == 2).all()
    assert (res["n_recorded"] < 40).all()
    assert (res["term"][:, :, 0].sum(axis=1) == 5).all()
    assert (res["final_counts"][:, -1] == 4).all()            # four cells below the top
    for g in range(50):
        nr = res["n_recorded"][g]
        assert (res["samples"][g, :nr, -1] <= 4).all()


def test_first_event_by_hand():
    """One cell deleted at rate 2 from a top with no other rule: the first
    event happens at -ln(u_tau)/2 with u_tau of draw 0, then the state is
    absorbing (no cell, no rule)."""
    m = W.cell_birth_death(lam=1.0, mu=2.0, n0=1, max_comp=4)
    m["rules"] = m["rules"][1:]                              # deletion only
    res = oracle.gsimulate(m, W.make_run(seed=9, replicas=5, dt=10.0, n_samples=2),
                           want_term=True)
    for g in range(5):
        u_tau, _ = oracle.draw(9, g, 0)
        assert res["t_final"][g] == (-oracle.ssa_log(u_tau)) / 2.0
        assert res["events"][g] == 1 and res["status"][g] == 1
        assert res["term"][g, 1, 0] == 0 and res["term"][g, 0, 0] == 1
