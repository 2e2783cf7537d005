"""Hand-worked cases for the oracle: the paper's propensity example, first
events computed by hand from the Philox stream with a 60-digit logarithm,
the selection rule on exact trees, terminal statuses and the statistics."""
import itertools
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W
from tests import ctmc

mpmath.mp.dps = 60


def close_ulps(a, b, n=4):
    return abs(a - b) <= n * math.ulp(max(abs(a), abs(b)))


def first_time(seed, g, e, a0):
    u, _ = oracle.draw(seed, g, e)
    return float(-mpmath.log(mpmath.mpf(u)) / a0)


def test_paper_example_combination_count():
    """Sec. 2.2: rule a b X -> c X on the term a a b b has 4 reactant
    combinations, so rate 4k; both by enumeration and in the oracle."""
    k = 0.5
    model = W.paper_example(k)
    st = ctmc.initial_state(model)
    (rate, _), = ctmc.transitions(model, st)
    assert rate == 4 * k
    # the oracle's first waiting time uses a0 = 4k
    run = W.make_run(replicas=50, dt=1e9, n_samples=2, max_events=1)
    res = oracle.simulate(model, run)
    for g in range(50):
        assert close_ulps(res["t_final"][g], first_time(0, g, 0, 4 * k))
        assert res["final_counts"][g].tolist() == [1, 1, 1]


def test_decay_two_molecules_by_hand():
    """A -> 0 (k = 1) from n0 = 2: t1 = -ln u0 / 2, t2 = t1 - ln u1 / 1,
    then absorbed."""
    model = W.pure_decay(1.0, 2)
    run = W.make_run(seed=99, replicas=40, dt=1e9, n_samples=2)
    res = oracle.simulate(model, run)
    one = oracle.simulate(model, dict(run, max_events=1))
    for g in range(40):
        t1 = first_time(99, g, 0, 2.0)
        t2 = t1 + first_time(99, g, 1, 1.0)
        assert close_ulps(one["t_final"][g], t1)
        assert one["status"][g] == 3 and one["events"][g] == 1
        assert close_ulps(res["t_final"][g], t2, 8)
        assert res["status"][g] == 1 and res["events"][g] == 2


def test_two_channel_choice_by_hand():
    """A -> B (k=1) vs A -> C (k=3) with one A: leaves [1, 3]; B iff
    u_sel * 4 < 1."""
    model = {"name": "split", "species": ["A", "B", "C"],
             "types": [{"name": "top", "wrap": False}],
             "compartments": [{"type": 0, "parent": -1}],
             "init": [[1, 0, 0]], "init_wrap": [None],
             "rules": [{"parent": 0, "child": -1, "lhs": {"p": {0: 1}},
                        "rhs": {"p": {1: 1}}, "k": 1.0},
                       {"parent": 0, "child": -1, "lhs": {"p": {0: 1}},
                        "rhs": {"p": {2: 1}}, "k": 3.0}]}
    run = W.make_run(seed=7, replicas=4000, dt=1e9, n_samples=2)
    res = oracle.simulate(model, run)
    nb = 0
    for g in range(4000):
        _, us = oracle.draw(7, g, 0)
        want_b = us * 4.0 < 1.0
        assert res["final_counts"][g].tolist() == ([0, 1, 0] if want_b else [0, 0, 1])
        nb += want_b
    assert abs(nb / 4000 - 0.25) < 5 * math.sqrt(0.25 * 0.75 / 4000)


def test_lotka_volterra_first_event_by_hand():
    """Config 0 at t = 0: a = [10*1000, 0.01*1000*1000, 10*1000] =
    [10000, 10000, 10000]; tree (20000, 10000), a0 = 30000."""
    model, run = W.config(0)
    run = dict(run, max_events=1, n_samples=2, dt=1e9)
    res = oracle.simulate(model, run)
    for g in range(64):
        us = oracle.draw(0, g, 0)[1]
        x = us * 30000.0
        if x < 20000.0:
            want = [1001, 1000] if x < 10000.0 else [999, 1001]
        else:
            want = [1000, 999]
        assert res["final_counts"][g].tolist() == want
        assert close_ulps(res["t_final"][g], first_time(0, g, 0, 30000.0))


def _interval_leaf(leaves, x):
    """Exact definition: the leaf j with prefix_j <= x < prefix_{j+1} over
    exact rational prefix sums; if x is at or beyond the total, the last
    positive leaf."""
    acc = Fraction(0)
    xq = Fraction(x)
    for j, v in enumerate(leaves):
        nxt = acc + Fraction(v)
        if v > 0 and acc <= xq < nxt:
            return j
        acc = nxt
    return max(j for j, v in enumerate(leaves) if v > 0)


def test_selection_exact_trees():
    """With integer leaves every tree sum is exact, so the descent must pick
    exactly the half-open interval containing x -- ties go right, a zero
    leaf is never chosen, x >= a0 falls back to the last positive leaf."""
    rng = np.random.default_rng(11)
    for P in (1, 2, 4, 8, 32, 64):
        for _ in range(40):
            leaves = rng.integers(0, 5, size=P).astype(np.float64)
            leaves[rng.random(P) < 0.3] = 0.0
            if leaves.sum() == 0:
                leaves[rng.integers(P)] = 1.0
            tot = leaves.sum()
            xs = set(np.cumsum(leaves)[:-1].tolist())            # boundaries
            xs |= {0.0, tot, float(np.nextafter(tot, 0))}
            xs |= set((rng.random(10) * tot).tolist())
            for x in xs:
                if x < 0:
                    continue
                j, a0 = oracle.select(leaves, x)
                assert a0 == tot
                assert leaves[j] > 0
                assert j == _interval_leaf(leaves, x), (leaves, x, j)


def test_selection_inexact_trees_within_rounding():
    """Arbitrary doubles: the chosen leaf is positive and its exact interval
    contains x up to the rounding of the tree (relative 2^-45)."""
    rng = np.random.default_rng(12)
    for _ in range(300):
        P = 32
        leaves = 10.0 ** rng.uniform(-3, 3, size=P)
        leaves[rng.random(P) < 0.3] = 0.0
        if leaves.sum() == 0:
            leaves[0] = 1.0
        x = rng.random() * leaves.sum()
        j, a0 = oracle.select(leaves, x)
        assert leaves[j] > 0
        pre = [Fraction(0)]
        for v in leaves:
            pre.append(pre[-1] + Fraction(v))
        tol = Fraction(a0) * Fraction(1, 2 ** 45)
        assert pre[j] - tol <= Fraction(x) < pre[j + 1] + tol


def test_statuses():
    model, run = W.config(0, replicas=8)
    # event cap
    r = oracle.simulate(model, dict(run, max_events=5), want_samples=True)
    assert (r["status"] == 3).all() and (r["events"] == 5).all()
    # samples recorded strictly before the stop time only
    for g in range(8):
        n = r["n_recorded"][g]
        assert all((k * run["dt"]) <= r["t_final"][g] for k in range(n))
    # overflow: cap at the initial 1000; the first birth event must stop it
    r = oracle.simulate(model, dict(run, count_cap=1000), want_samples=True)
    assert (r["status"] == 2).all()
    assert (r["final_counts"] <= 1000).all()
    # absorbing: pure decay reaches 0 and fills all remaining samples
    r = oracle.simulate(W.pure_decay(5.0, 3), W.make_run(replicas=8, dt=1.0, n_samples=50),
                        want_samples=True)
    assert (r["status"] == 1).all() and (r["n_recorded"] == 50).all()
    assert (r["samples"][:, -1, 0] == 0).all()


def test_stats_match_exact_rationals():
    """mean = S1/n and unbiased var from exact rationals over the recorded
    samples, including samples missing after OVERFLOW/EVENT_CAP stops."""
    model, run = W.config(0, replicas=40)
    run = dict(run, n_samples=31, max_events=30000)
    r = oracle.simulate(model, run, want_samples=True)
    S, nrec = r["samples"], r["n_recorded"]
    assert (r["status"] == 3).any()
    for k in range(0, 31, 3):
        rows = [g for g in range(40) if nrec[g] > k]
        assert r["n"][0, k] == len(rows)
        for c in range(2):
            xs = [int(S[g, k, c]) for g in rows]
            n = len(xs)
            if n == 0:
                assert math.isnan(r["mean"][0, k, c])
                continue
            mean = Fraction(sum(xs), n)
            assert abs(r["mean"][0, k, c] - float(mean)) <= math.ulp(float(mean))
            if n < 2:
                assert math.isnan(r["var"][0, k, c])
                continue
            var = sum((Fraction(x) - mean) ** 2 for x in xs) / (n - 1)
            assert abs(r["var"][0, k, c] - float(var)) <= 2 * math.ulp(float(var))


def test_sweep_instances_use_their_rate_rows():
    """Instance i of a sweep runs with rate row i; trajectories of instance
    i equal a single-instance run with that row's rates and the same g."""
    model = W.lotka_volterra()
    tab, f = W.sweep_rate_table(model, 3, 9)
    run = W.make_run(n_instances=3, replicas=4, dt=0.05, n_samples=11, rate_table=tab)
    r = oracle.simulate(model, run)
    for i in range(3):
        mi = W.lotka_volterra(k=tuple(tab[i]))
        ri = W.make_run(n_instances=3, replicas=4, dt=0.05, n_samples=11)
        ri["rate_table"] = np.repeat(tab[i:i + 1], 3, axis=0)
        s = oracle.simulate(mi, ri, g0=4 * i, g1=4 * i + 4)
        assert (s["digest"] == r["digest"][4 * i:4 * i + 4]).all()
