"""The paper's printed worked examples, read from text fixtures in
tests/golden/ (each cites its section), against the oracle's flattening,
propensities and rewriting."""
import math
import os

import mpmath
import numpy as np

import oracle
from tests import ctmc

mpmath.mp.dps = 60
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_fixture(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = (s.strip() for s in line.split("=", 1))
                out[key] = val
    return out


def multiset(species, atoms):
    """Count vector over `species` of a space-separated list of atoms."""
    v = [0] * len(species)
    for a in atoms.split():
        v[species.index(a)] += 1
    return v


def test_term_example_cells():
    """Sec. 2.1: the term a b (c d | e f)^l as count cells."""
    fx = read_fixture("term_example_sec2_1.txt")
    sp = fx["species"].split()
    model = {"name": "term_example", "species": sp,
             "types": [{"name": "top", "wrap": False},
                       {"name": fx["comp_type"], "wrap": True}],
             "compartments": [{"type": 0, "parent": -1}, {"type": 1, "parent": 0}],
             "init": [multiset(sp, fx["top_content"]), multiset(sp, fx["comp_content"])],
             "init_wrap": [None, multiset(sp, fx["comp_wrap"])],
             "rules": []}
    want = [int(x) for x in fx["cells"].split()]
    flat = oracle.FlatModel(model)
    assert flat.n_cells == len(want) == 3 * len(sp)
    assert flat.init.tolist() == want
    # the brute-force chain's state of the same term, in the same cell order
    assert ctmc.cell_values(model, [ctmc.initial_state(model)])[0].tolist() == want


def rule_model(fx, k, counts):
    sp = fx["species"].split()
    lhs = {i: m for i, m in enumerate(multiset(sp, fx["lhs"])) if m}
    rhs = {i: m for i, m in enumerate(multiset(sp, fx["rhs"])) if m}
    return {"name": "rate_example", "species": sp,
            "types": [{"name": "l", "wrap": False}],
            "compartments": [{"type": 0, "parent": -1}],
            "init": [list(counts)], "init_wrap": [None],
            "rules": [{"parent": 0, "child": -1, "lhs": {"p": lhs}, "rhs": {"p": rhs},
                       "k": float(k)}]}


def exp_time(seed, g, e, a0):
    u, _ = oracle.draw(seed, g, e)
    return float(-mpmath.log(mpmath.mpf(u)) / a0)


def close_ulps(a, b, n):
    return abs(a - b) <= n * math.ulp(max(abs(a), abs(b)))


def test_rate_example_combinations():
    """Sec. 2.2: 4 combinations of a b in a a b b, so rate 4k; the counts
    of every state of the rewriting sequence by enumeration."""
    fx = read_fixture("rate_example_sec2_2.txt")
    sp = fx["species"].split()
    k = 0.375
    states = [multiset(sp, s) for s in fx["states"].split(";")]
    combos = [int(x) for x in fx["combinations_per_state"].split()]
    assert states[0] == multiset(sp, fx["term"])
    assert combos[0] == int(fx["combinations"])
    for st, n in zip(states, combos):
        tr = ctmc.transitions(rule_model(fx, k, st), ctmc.initial_state(rule_model(fx, k, st)))
        assert sum(r for r, _ in tr) == n * k
    # each state's successor is the next state of the sequence
    for a, b in zip(states, states[1:]):
        m = rule_model(fx, k, a)
        (_, nxt), = ctmc.transitions(m, ctmc.initial_state(m))
        assert ctmc.cell_values(m, [nxt])[0].tolist() == b


def test_rate_example_oracle_sequence():
    """The oracle walks the fixture's rewriting sequence: after e events it
    holds state e, its waiting times use a0 = combinations x k, and it ends
    absorbed in the last state."""
    fx = read_fixture("rate_example_sec2_2.txt")
    sp = fx["species"].split()
    k, seed, R = 0.375, 7, 48
    states = [multiset(sp, s) for s in fx["states"].split(";")]
    combos = [int(x) for x in fx["combinations_per_state"].split()]
    model = rule_model(fx, k, states[0])
    base = {"seed": seed, "n_instances": 1, "replicas": R, "dt": 1e9, "n_samples": 2,
            "rate_table": None, "init_table": None, "count_cap": 2**31 - 1}
    t_ref = np.zeros(R)
    for e in range(1, len(states)):
        res = oracle.simulate(model, dict(base, max_events=e))
        for g in range(R):
            t_ref[g] += exp_time(seed, g, e - 1, combos[e - 1] * k)
            assert res["final_counts"][g].tolist() == states[e]
            assert res["events"][g] == e
            assert close_ulps(res["t_final"][g], t_ref[g], 8)
    res = oracle.simulate(model, dict(base, max_events=0))
    assert combos[-1] == 0
    for g in range(R):
        assert res["final_counts"][g].tolist() == states[-1]
        assert oracle.STATUS[int(res["status"][g])] == "ABSORBED"
        assert res["events"][g] == len(states) - 1
