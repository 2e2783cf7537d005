"""Brute-force continuous-time Markov chain over CWC *terms* (test helper).

An independent, direct reading of the calculus (paper Sec. 2.1-2.2) on
canonical nested terms, written without the oracle's slot pool, leaf
layout or update code: a compartment is (label, wrap counts, content
counts, children), children kept as a sorted tuple so equal terms are equal
values.  For every rule, every context compartment of its label, every
child (and grandchild) of the named labels is a match; its rate is k times
the product of binomial(n, m) over the pattern's atoms; applying it
rewrites the named regions and performs the structural action (create,
dissolve -- content and compartments to the parent, wrap atoms too if
released --, delete).  Matches that lead to the same term add their rates.
A transition that would hold more compartments than ``max_comp`` or a count
above ``cap`` leads to the absorbing state OVERFLOW.

transient(model, times) -> (states, P[len(times)][n_states]) from the
initial term, by scipy's expm_multiply on the sparse generator.
"""
from __future__ import annotations

from math import comb

import numpy as np

REG = ("c", "w1", "c1", "w2", "c2")
OVERFLOW = "OVERFLOW"


def comp(label, wrap, content, children=()):
    return (label, tuple(wrap), tuple(content), tuple(sorted(children)))


def initial_term(model):
    ns = len(model["species"])
    term = model["term"]
    kids = [[] for _ in term]

    def vec(v):
        return tuple(int(x) for x in (v if v is not None else [0] * ns))

    built = [None] * len(term)
    for i in range(len(term) - 1, -1, -1):       # children come after parents
        c = term[i]
        built[i] = comp(c["label"], vec(c.get("wrap")), vec(c.get("content")), kids[i])
        if c["parent"] >= 0:
            kids[c["parent"]].append(built[i])
    return built[0]


def n_comps(t):
    return 1 + sum(n_comps(c) for c in t[3])


def _vec(d, ns):
    v = [0] * ns
    for a, m in (d or {}).items():
        v[int(a)] += int(m)
    return v


def _with(c, wrap=None, content=None, children=None):
    return comp(c[0], c[1] if wrap is None else wrap, c[2] if content is None else content,
                c[3] if children is None else children)


def _rate(rule, regions, ns):
    h = 1
    for q, cnt in enumerate(regions):
        if cnt is None:
            continue
        for a, m in enumerate(_vec(rule["lhs"].get(REG[q]), ns)):
            if m:
                h *= comb(cnt[a], m)
    return rule["k"] * h


def _apply_regions(rule, regions, ns):
    out = []
    for q, cnt in enumerate(regions):
        if cnt is None:
            out.append(None)
            continue
        lhs = _vec(rule["lhs"].get(REG[q]), ns)
        rhs = _vec(rule["rhs"].get(REG[q]), ns)
        out.append(tuple(cnt[a] - lhs[a] + rhs[a] for a in range(ns)))
    return out


def _successors(model, t):
    """(rate, next term) for every match in term t (recursive over the term)."""
    ns = len(model["species"])
    res = []

    def in_context(c, rebuild):
        """Matches whose context is compartment c; rebuild(c') puts a new
        c' back into the whole term."""
        for r in model["rules"]:
            if r["context"] != c[0]:
                continue
            ch, gc = r.get("child", -1), r.get("grandchild", -1)
            act, lv = r.get("action", "none"), int(r.get("level", 0))
            if ch < 0:
                rate = _rate(r, [c[2]], ns)
                if rate > 0:
                    (ctx_c,) = _apply_regions(r, [c[2]], ns)
                    nc = _with(c, content=ctx_c)
                    if act == "create":
                        nw = r["new"]
                        nc = _with(nc, children=nc[3] + (comp(nw["label"], _vec_of(nw.get("wrap"), ns),
                                                              _vec_of(nw.get("content"), ns)),))
                    res.append((rate, rebuild(nc)))
                continue
            for i, d in enumerate(c[3]):
                if d[0] != ch:
                    continue
                others = c[3][:i] + c[3][i + 1:]
                gcs = [(None, None)] if gc < 0 else [(j, e) for j, e in enumerate(d[3]) if e[0] == gc]
                for j, e in gcs:
                    regs = [c[2], d[1], d[2]] + ([e[1], e[2]] if e is not None else [None, None])
                    rate = _rate(r, regs, ns)
                    if rate <= 0:
                        continue
                    nr = _apply_regions(r, regs, ns)
                    ne = None if e is None else _with(e, wrap=nr[3], content=nr[4])
                    d_kids = d[3] if e is None else d[3][:j] + d[3][j + 1:]
                    nd_parts = {"wrap": nr[1], "content": nr[2], "kids": list(d_kids)}
                    nc_parts = {"content": nr[0], "kids": list(others)}
                    # structural action
                    if act == "create":
                        nw = r["new"]
                        new = comp(nw["label"], _vec_of(nw.get("wrap"), ns), _vec_of(nw.get("content"), ns))
                        if lv == 0:
                            nc_parts["kids"].append(new)
                        elif lv == 1:
                            nd_parts["kids"].append(new)
                        else:
                            ne = _with(ne, children=ne[3] + (new,))
                    if act in ("dissolve", "delete") and lv == 2:
                        if act == "dissolve":
                            add = [ne[2][a] + (ne[1][a] if r.get("release_wrap") else 0) for a in range(ns)]
                            nd_parts["content"] = tuple(nd_parts["content"][a] + add[a] for a in range(ns))
                            nd_parts["kids"] += list(ne[3])
                        ne = None
                    if ne is not None:
                        nd_parts["kids"].append(ne)
                    nd = comp(d[0], nd_parts["wrap"], nd_parts["content"], nd_parts["kids"])
                    if act in ("dissolve", "delete") and lv == 1:
                        if act == "dissolve":
                            add = [nd[2][a] + (nd[1][a] if r.get("release_wrap") else 0) for a in range(ns)]
                            nc_parts["content"] = tuple(nc_parts["content"][a] + add[a] for a in range(ns))
                            nc_parts["kids"] += list(nd[3])
                        nd = None
                    if nd is not None:
                        nc_parts["kids"].append(nd)
                    nc = comp(c[0], c[1], nc_parts["content"], nc_parts["kids"])
                    res.append((rate, rebuild(nc)))
        # recurse into the children as contexts
        for i, d in enumerate(c[3]):
            others = c[3][:i] + c[3][i + 1:]
            in_context(d, lambda nd, c=c, others=others: rebuild(_with(c, children=others + (nd,))))

    in_context(t, lambda nc: nc)
    return res


def _vec_of(v, ns):
    if v is None:
        return tuple([0] * ns)
    if isinstance(v, dict):
        return tuple(_vec(v, ns))
    return tuple(int(x) for x in v)


def _too_big(model, t, cap):
    if n_comps(t) > model["max_comp"]:
        return True

    def big(c):
        return max(c[1] + c[2] + (0,)) > cap or any(big(d) for d in c[3])

    return big(t)


def transient(model, times, cap=2 ** 31 - 1, max_states=200000):
    from scipy.sparse import csr_matrix
    from scipy.sparse.linalg import expm_multiply
    t0 = initial_term(model)
    index = {t0: 0}
    states = [t0]
    rows, cols, vals = [], [], []
    q = 0
    while q < len(states):
        s = states[q]
        if s != OVERFLOW:
            out = {}
            for rate, nt in _successors(model, s):
                key = OVERFLOW if _too_big(model, nt, cap) else nt
                out[key] = out.get(key, 0.0) + rate
            for key, rate in out.items():
                if key == s:
                    continue
                if key not in index:
                    index[key] = len(states)
                    states.append(key)
                    if len(states) > max_states:
                        raise ValueError("state space too large")
                rows.append(q)
                cols.append(index[key])
                vals.append(rate)
        q += 1
    n = len(states)
    Q = csr_matrix((vals, (rows, cols)), shape=(n, n)).tolil()
    out_rate = np.asarray(Q.sum(axis=1)).ravel()
    Q.setdiag(-out_rate)
    Q = Q.tocsc()
    p0 = np.zeros(n)
    p0[0] = 1.0
    P = []
    for t in times:
        P.append(expm_multiply(Q.T * t, p0) if t > 0 else p0.copy())
    return states, np.maximum(np.array(P), 0.0)


def observables(model, t):
    """The oracle's observables of a term: per label, content totals, wrap
    totals (labels with a wrap), compartment count."""
    ns = len(model["species"])
    labels = model["labels"]
    tot = {l: ([0] * ns, [0] * ns, [0]) for l in range(len(labels))}

    def walk(c):
        cn, wr, k = tot[c[0]]
        for a in range(ns):
            cn[a] += c[2][a]
            wr[a] += c[1][a]
        k[0] += 1
        for d in c[3]:
            walk(d)

    walk(t)
    out = []
    for l, lab in enumerate(labels):
        cn, wr, k = tot[l]
        out += cn
        if lab["wrap"]:
            out += wr
        out += k
    return tuple(out)
