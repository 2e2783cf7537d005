"""Brute-force CTMC solution of small CWC models (test helper).

Independent of the oracle: contexts are found by walking the compartment
tree, and the number of reactant combinations of a pattern is obtained by
*enumerating* the distinct subsets of atom instances that match it (not by
a binomial formula).  The forward equation p(t) = p(0) exp(Q t) is solved
with scipy's matrix exponential on the reachable (truncated) state space.
"""
import itertools
from collections import deque

import numpy as np
import scipy.linalg


def _regions(model):
    """Per compartment: (content key, wrap key or None)."""
    out = []
    for i, c in enumerate(model["compartments"]):
        has_w = model["types"][c["type"]]["wrap"]
        out.append((("c", i), ("w", i) if has_w else None))
    return out


def initial_state(model):
    ns = len(model["species"])
    st = {}
    for i, c in enumerate(model["compartments"]):
        st[("c", i)] = tuple(int(x) for x in model["init"][i])
        if model["types"][c["type"]]["wrap"]:
            w = (model.get("init_wrap") or [None] * len(model["compartments"]))[i]
            st[("w", i)] = tuple(int(x) for x in (w if w is not None else [0] * ns))
    return tuple(sorted(st.items()))


def _count_subsets(n, m):
    return sum(1 for _ in itertools.combinations(range(n), m))


def transitions(model, state):
    """List of (rate, new_state) out of ``state``."""
    st = dict(state)
    comps = model["compartments"]
    out = []
    for rule in model["rules"]:
        ctxs = []
        for i, c in enumerate(comps):
            if rule["child"] < 0:
                if c["type"] == rule["parent"]:
                    ctxs.append({"p": ("c", i)})
            else:
                par = c["parent"]
                if (c["type"] == rule["child"] and par >= 0
                        and comps[par]["type"] == rule["parent"]):
                    ctxs.append({"p": ("c", par), "w": ("w", i), "c": ("c", i)})
        for ctx in ctxs:
            combos = 1
            for reg, atoms in rule["lhs"].items():
                for sp, m in atoms.items():
                    combos *= _count_subsets(st[ctx[reg]][int(sp)], int(m))
            if combos == 0:
                continue
            new = {k: list(v) for k, v in st.items()}
            for reg, atoms in rule["lhs"].items():
                for sp, m in atoms.items():
                    new[ctx[reg]][int(sp)] -= int(m)
            for reg, atoms in rule["rhs"].items():
                for sp, m in atoms.items():
                    new[ctx[reg]][int(sp)] += int(m)
            out.append((rule["k"] * combos,
                        tuple(sorted((k, tuple(v)) for k, v in new.items()))))
    return out


def solve(model, times, max_count=60, max_states=5000):
    """Exact distribution over reachable states at each time.

    States with any multiplicity above ``max_count`` are cut (their inflow
    becomes lost mass, reported so callers can bound it)."""
    s0 = initial_state(model)
    index = {s0: 0}
    states = [s0]
    edges = []
    q = deque([s0])
    while q:
        s = q.popleft()
        for rate, t in transitions(model, s):
            if max(max(v) for _, v in t) > max_count:
                edges.append((index[s], -1, rate))
                continue
            if t not in index:
                if len(states) >= max_states:
                    raise RuntimeError("state space too large")
                index[t] = len(states)
                states.append(t)
                q.append(t)
            edges.append((index[s], index[t], rate))
    n = len(states)
    Q = np.zeros((n, n))
    for a, b, r in edges:
        Q[a, a] -= r
        if b >= 0:
            Q[a, b] += r
    p = np.zeros(n)
    p[0] = 1.0
    dists = []
    prev_t = 0.0
    for t in times:
        if t > prev_t:
            p = p @ scipy.linalg.expm(Q * (t - prev_t))
        dists.append(p.copy())
        prev_t = t
    return states, np.array(dists)


def cell_values(model, states):
    """Matrix [state][cell] in the oracle/GPU output cell order
    (per compartment: content species, then wrap species)."""
    regs = _regions(model)
    rows = []
    for s in states:
        d = dict(s)
        row = []
        for ck, wk in regs:
            row.extend(d[ck])
            if wk is not None:
                row.extend(d[wk])
        rows.append(row)
    return np.array(rows, dtype=np.float64)
