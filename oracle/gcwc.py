"""CPU oracle, Python side, for general CWC models (gcwc.c): compartments
created, dissolved and deleted at run time, patterns two levels deep.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.

A general model dictionary (built in ``workloads``):

* ``species``: atom names; ``labels``: [{"name", "wrap"}] compartment types;
* ``max_comp``: compartment slots (<= 64) -- the term's capacity;
* ``term``: the initial compartments in preorder, each {"label", "parent",
  "content": [NS], "wrap": [NS] or None}; entry 0 is the top level;
* ``rules``: each {"context", "child", "grandchild" (labels, -1 = absent),
  "lhs"/"rhs": {region: {species: multiplicity}} with regions "c" (the
  context's content), "w1"/"c1" (the child's wrap / content), "w2"/"c2"
  (the grandchild's), "action": "none" | "create" | "dissolve" |
  "delete", "level" (create: 0 context, 1 child, 2 grandchild receives the
  new compartment; dissolve / delete: 1 child, 2 grandchild), "new":
  {"label", "wrap", "content"} (create), "release_wrap" (dissolve: the
  wrap atoms join the parent's content), "k"}.

The atoms of a region that the pattern does not name are its variable (x
for a wrap, X for a content) and are carried over unchanged; a dissolved
compartment's content, compartments included, passes to its parent
(paper Sec. 2.1: the substitution sigma applied to the right-hand side).
"""
from __future__ import annotations

import ctypes
import threading
from typing import Dict, Optional

import numpy as np

from . import cwc as _cwc

REGIONS = ("c", "w1", "c1", "w2", "c2")
ACTIONS = {"none": 0, "create": 1, "dissolve": 2, "delete": 3}


class _CGModel(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_labels", ctypes.c_int32),
                ("max_comp", ctypes.c_int32), ("has_wrap", ctypes.c_void_p),
                ("n_init", ctypes.c_int32), ("init_label", ctypes.c_void_p),
                ("init_parent", ctypes.c_void_p), ("init_wrap", ctypes.c_void_p),
                ("init_content", ctypes.c_void_p), ("n_rules", ctypes.c_int32),
                ("rule_depth", ctypes.c_void_p), ("rule_labels", ctypes.c_void_p),
                ("rule_lhs", ctypes.c_void_p), ("rule_rhs", ctypes.c_void_p),
                ("rule_action", ctypes.c_void_p), ("rule_level", ctypes.c_void_p),
                ("rule_new_label", ctypes.c_void_p), ("rule_new_wrap", ctypes.c_void_p),
                ("rule_new_content", ctypes.c_void_p),
                ("rule_release_wrap", ctypes.c_void_p), ("rule_k", ctypes.c_void_p)]


def _vec(d, ns):
    v = np.zeros(ns, np.int32)
    if d is None:
        return v
    if isinstance(d, dict):
        for sp, m in d.items():
            v[int(sp)] += int(m)
    else:
        v[:] = np.asarray(d, np.int32)
    return v


class GModel:
    """Array form of a general model, checked."""

    def __init__(self, model: Dict):
        ns = len(model["species"])
        labels = model["labels"]
        nl = len(labels)
        term, rules = model["term"], model["rules"]
        self.n_species, self.n_labels = ns, nl
        self.max_comp = int(model["max_comp"])
        if not 1 <= self.max_comp <= 64 or ns > 32 or len(term) > self.max_comp:
            raise ValueError("at most 64 compartment slots, 32 species, and the term must fit")
        if term[0]["parent"] != -1 or any(c["parent"] < 0 or c["parent"] >= i
                                          for i, c in enumerate(term) if i > 0):
            raise ValueError("term must be in preorder with the top level first")
        self.has_wrap = np.array([int(bool(l["wrap"])) for l in labels], np.int32)
        self.init_label = np.array([c["label"] for c in term], np.int32)
        self.init_parent = np.array([c["parent"] for c in term], np.int32)
        self.init_wrap = np.stack([_vec(c.get("wrap"), ns) for c in term]).astype(np.int32)
        self.init_content = np.stack([_vec(c.get("content"), ns) for c in term]).astype(np.int32)
        R = len(rules)
        self.n_rules = R
        self.depth = np.zeros(R, np.int32)
        self.labels = np.full((R, 3), -1, np.int32)
        self.lhs = np.zeros((R, 5, ns), np.int32)
        self.rhs = np.zeros((R, 5, ns), np.int32)
        self.action = np.zeros(R, np.int32)
        self.level = np.zeros(R, np.int32)
        self.new_label = np.full(R, -1, np.int32)
        self.new_wrap = np.zeros((R, ns), np.int32)
        self.new_content = np.zeros((R, ns), np.int32)
        self.release_wrap = np.zeros(R, np.int32)
        self.k = np.array([float(r["k"]) for r in rules], np.float64)
        for i, r in enumerate(rules):
            ch, gc = r.get("child", -1), r.get("grandchild", -1)
            d = 0 if ch < 0 else (1 if gc < 0 else 2)
            self.depth[i] = d
            self.labels[i] = (r["context"], ch, gc if d == 2 else -1)
            for side, arr in (("lhs", self.lhs), ("rhs", self.rhs)):
                for reg, atoms in r.get(side, {}).items():
                    q = REGIONS.index(reg)
                    if q > 2 * d:
                        raise ValueError("rule %d names region %s beyond its depth" % (i, reg))
                    arr[i, q] = _vec(atoms, ns)
            if self.lhs[i].sum() > 2:
                raise ValueError("rule %d: total reactant order above 2" % i)
            act = ACTIONS[r.get("action", "none")]
            self.action[i] = act
            lv = int(r.get("level", 0))
            self.level[i] = lv
            if act == 1:
                if not 0 <= lv <= d:
                    raise ValueError("rule %d creates below its pattern" % i)
                nw = r["new"]
                self.new_label[i] = nw["label"]
                self.new_wrap[i] = _vec(nw.get("wrap"), ns)
                self.new_content[i] = _vec(nw.get("content"), ns)
            elif act in (2, 3):
                if not 1 <= lv <= d:
                    raise ValueError("rule %d dissolves or deletes a compartment it does not name" % i)
                self.release_wrap[i] = int(bool(r.get("release_wrap", False)))
        # the observables: per label, content totals, wrap totals (if any),
        # compartment count
        names = []
        for l, lab in enumerate(labels):
            names += ["%s.%s" % (lab["name"], s) for s in model["species"]]
            if lab["wrap"]:
                names += ["%s.wrap.%s" % (lab["name"], s) for s in model["species"]]
            names.append("%s.count" % lab["name"])
        self.obs_names = names
        self.n_obs = len(names)
        self._c = _CGModel(ns, nl, self.max_comp, self.has_wrap.ctypes.data, len(term),
                           self.init_label.ctypes.data, self.init_parent.ctypes.data,
                           self.init_wrap.ctypes.data, self.init_content.ctypes.data, R,
                           self.depth.ctypes.data, self.labels.ctypes.data,
                           self.lhs.ctypes.data, self.rhs.ctypes.data,
                           self.action.ctypes.data, self.level.ctypes.data,
                           self.new_label.ctypes.data, self.new_wrap.ctypes.data,
                           self.new_content.ctypes.data, self.release_wrap.ctypes.data,
                           self.k.ctypes.data)

    def layout(self):
        """(PL, Np, rule_at [n_labels][PL]) of the leaf array."""
        L = _lib()
        PL, Np = ctypes.c_int(), ctypes.c_int()
        buf = np.zeros(self.n_labels * 64 + 1, np.int32)
        L.goracle_layout(ctypes.byref(self._c), ctypes.byref(PL), ctypes.byref(Np),
                         buf.ctypes.data)
        return PL.value, Np.value, buf[:self.n_labels * PL.value].reshape(self.n_labels, PL.value)


_glib = None


def _lib():
    global _glib
    if _glib is None:
        L = _cwc.lib()
        L.goracle_layout.argtypes = [ctypes.c_void_p] * 4
        L.goracle_layout.restype = ctypes.c_int
        L.goracle_n_obs.argtypes = [ctypes.c_void_p]
        L.goracle_n_obs.restype = ctypes.c_int
        L.goracle_simulate.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        L.goracle_simulate.restype = ctypes.c_int
        _glib = L
    return _glib


def gsimulate(model: Dict, run: Dict, g0: int = 0, g1: Optional[int] = None,
              want_samples: bool = False, want_stats: bool = True, want_term: bool = False,
              threads: int = 1, gm: Optional[GModel] = None) -> Dict:
    """Trajectories g0..g1-1 of a general model: per-trajectory results
    (final observables as ``final_counts``, events, final time, fired-leaf
    digest, status, recorded samples), optionally the observables' samples
    [g][K+1][C] and the final term [g][max_comp][alive, label, parent, wrap
    NS, content NS], and the exact moments and mean/var per (instance,
    sample, observable)."""
    gm = gm or GModel(model)
    L = _lib()
    I, R = run["n_instances"], run["replicas"]
    G = I * R
    g1 = G if g1 is None else g1
    n = g1 - g0
    C, K1 = gm.n_obs, run["n_samples"]
    if run.get("init_table") is not None:
        raise ValueError("general models take their initial term from the model")
    rate = run.get("rate_table")
    if rate is not None:
        rate = np.ascontiguousarray(rate, dtype=np.float64)
        assert rate.shape == (I, gm.n_rules)
    cr = _cwc._CRun(run["seed"], I, R, _cwc._ptr(rate), None, run["dt"], K1,
                    run["count_cap"], run["max_events"])
    res = {"final_counts": np.zeros((n, C), np.int32), "events": np.zeros(n, np.int64),
           "t_final": np.zeros(n, np.float64), "digest": np.zeros(n, np.uint64),
           "status": np.zeros(n, np.uint8), "n_recorded": np.zeros(n, np.int32)}
    if want_samples:
        res["samples"] = np.zeros((n, K1, C), np.int32)
    if want_term:
        res["term"] = np.zeros((n, gm.max_comp, 3 + 2 * gm.n_species), np.int32)
    threads = max(1, min(threads, n)) if n > 0 else 1
    bounds = [g0 + (n * t) // threads for t in range(threads + 1)]
    accs = []

    def work(t):
        a, b = bounds[t], bounds[t + 1]
        o = a - g0
        acc = None
        if want_stats:
            acc = {"n": np.zeros((I, K1), np.uint64), "s1": np.zeros((I, K1, C), np.uint64),
                   "s2_lo": np.zeros((I, K1, C), np.uint64),
                   "s2_hi": np.zeros((I, K1, C), np.uint64)}
        p = _cwc._ptr
        co = _cwc._COut(p(res["samples"][o:]) if want_samples else None,
                        p(res["final_counts"][o:]), p(res["events"][o:]),
                        p(res["t_final"][o:]), p(res["digest"][o:]), p(res["status"][o:]),
                        p(res["n_recorded"][o:]),
                        *([p(acc[k]) for k in ("n", "s1", "s2_lo", "s2_hi")] if acc
                          else [None] * 4))
        rc = L.goracle_simulate(ctypes.byref(gm._c), ctypes.byref(cr), a, b, ctypes.byref(co),
                                p(res["term"][o:]) if want_term else None)
        if rc != 0:
            raise MemoryError("goracle_simulate failed")
        accs.append(acc)

    if threads == 1:
        work(0)
    else:
        ts = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
        for th in ts:
            th.start()
        for th in ts:
            th.join()
    if want_stats:
        tot = accs[0]
        for acc in accs[1:]:
            L.oracle_merge_moments(*[_cwc._ptr(tot[k]) for k in ("n", "s1", "s2_lo", "s2_hi")],
                                   *[_cwc._ptr(acc[k]) for k in ("n", "s1", "s2_lo", "s2_hi")],
                                   I * K1, C)
        res.update(tot)
        res["mean"], res["var"] = _cwc.finalize(tot, C)
    res["gmodel"] = gm
    return res
