"""CPU oracle: CWC model flattening and the Python side of the plain
direct-method simulator in ssa.c.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library; both read the same model dictionaries (see ``workloads``).

Flattening (paper Sec. 2.1-2.3).  The Match routine of the paper's
simulator walks the term tree and, for every rule, records one weighted
match per context in which the rule's pattern occurs.  With a fixed
compartment tree the contexts of a rule are known in advance:

* a rule applied in compartments of label l that only rewrites their
  content has one context per compartment i of label l;
* a rule whose pattern also reaches a child compartment of label l' (its
  wrap and/or content, e.g. transport across the membrane) has one context
  per compartment i of label l' whose parent has label l.  Summing over
  those contexts is the paper's count_compartments factor.

A (rule, context) pair is a *slot*.  Slots are laid out context-major: the
slot block of compartment i (preorder) lists the rules that apply at i in
ascending rule index.  Every block is padded with zero leaves to
P_local = next power of two of the largest block, and the compartment count
to P_comp = next power of two, so leaf index = i*P_local + position and the
total P = P_comp*P_local is a power of two.

The propensity of a slot is k times the product, over the pattern's atoms
(x, m), of binomial(n_x, m) where n_x is the multiplicity of x in the
region (parent content, child wrap or child content) the pattern names
(paper Sec. 2.2, the a a b b example; Match_Populations in Fig. "simd").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
LIB = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(BUILD, "libcwcoracle.so")
MAX_DELTA = 16
STATUS = {0: "OK", 1: "ABSORBED", 2: "OVERFLOW", 3: "EVENT_CAP"}


def build(force: bool = True) -> str:
    """Compile ssa.c and gcwc.c with gcc: -O2, no contraction of a*b+c into FMA, no
    fast-math, so every floating-point operation is one IEEE binary64
    rounding."""
    os.makedirs(BUILD, exist_ok=True)
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-o", tmp, os.path.join(HERE, "ssa.c"),
             os.path.join(HERE, "gcwc.c"), "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = ctypes.CDLL(LIB)
        L.oracle_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.oracle_u_tau.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_u_tau.restype = ctypes.c_double
        L.oracle_u_sel.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_u_sel.restype = ctypes.c_double
        L.oracle_ssa_log.argtypes = [ctypes.c_double]
        L.oracle_ssa_log.restype = ctypes.c_double
        L.oracle_simulate.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_void_p]
        L.oracle_simulate.restype = ctypes.c_int
        P = ctypes.c_void_p
        L.oracle_select.argtypes = [P, ctypes.c_int, ctypes.c_double, P]
        L.oracle_select.restype = ctypes.c_int
        L.oracle_merge_moments.argtypes = [P] * 8 + [ctypes.c_int64, ctypes.c_int]
        L.oracle_finalize.argtypes = [P] * 4 + [ctypes.c_int64, ctypes.c_int, P, P]
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# Flattening
# --------------------------------------------------------------------------

def _next_pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


class FlatModel:
    """Slot tables of a CWC model with a fixed compartment tree."""

    def __init__(self, model: Dict):
        ns = len(model["species"])
        types = model["types"]
        comps = model["compartments"]
        self.n_species = ns
        self.n_comp = len(comps)
        self.n_rules = len(model["rules"])
        # output cells: per compartment, content species then wrap species
        self.content_base, self.wrap_base = [], []
        c = 0
        for comp in comps:
            self.content_base.append(c)
            c += ns
            if types[comp["type"]]["wrap"]:
                self.wrap_base.append(c)
                c += ns
            else:
                self.wrap_base.append(-1)
        self.n_cells = c
        init = np.zeros(c, dtype=np.int32)
        for i, comp in enumerate(comps):
            init[self.content_base[i]:self.content_base[i] + ns] = model["init"][i]
            if self.wrap_base[i] >= 0:
                w = (model.get("init_wrap") or [None] * len(comps))[i]
                if w is not None:
                    init[self.wrap_base[i]:self.wrap_base[i] + ns] = w
        self.init = init
        self.k = np.array([r["k"] for r in model["rules"]], dtype=np.float64)

        # slots per compartment, context-major
        blocks = []
        for i, comp in enumerate(comps):
            par = comp["parent"]
            blk = []
            for r, rule in enumerate(model["rules"]):
                if rule["child"] < 0:
                    if rule["parent"] == comp["type"]:
                        blk.append(r)
                elif (rule["child"] == comp["type"] and par >= 0
                      and comps[par]["type"] == rule["parent"]):
                    blk.append(r)
            blocks.append(blk)
        self.blocks = blocks
        self.p_local = _next_pow2(max(1, max(len(b) for b in blocks)))
        self.p_comp = _next_pow2(self.n_comp)
        P = self.p_local * self.p_comp
        self.n_leaves = P
        self.leaf_rule = np.full(P, -1, dtype=np.int32)
        self.leaf_ctx = np.full(P, -1, dtype=np.int32)
        self.leaf_react = np.zeros((P, 2, 2), dtype=np.int32)
        self.leaf_delta = np.zeros((P, MAX_DELTA, 2), dtype=np.int32)
        self.leaf_ndelta = np.zeros(P, dtype=np.int32)
        for i, blk in enumerate(blocks):
            for pos, r in enumerate(blk):
                leaf = i * self.p_local + pos
                rule = model["rules"][r]
                self.leaf_rule[leaf] = r
                self.leaf_ctx[leaf] = i
                region_cell = self._regions(i, rule, comps)
                terms = []
                for reg, atoms in rule["lhs"].items():
                    for sp, m in atoms.items():
                        if int(m) > 0:
                            terms.append((region_cell[reg] + int(sp), int(m)))
                if len(terms) > 2 or sum(m for _, m in terms) > 2:
                    raise ValueError("oracle handles reactant order <= 2")
                for t, (cell, m) in enumerate(terms):
                    self.leaf_react[leaf, t] = (cell, m)
                net = {}
                for reg, atoms in rule["lhs"].items():
                    for sp, m in atoms.items():
                        cell = region_cell[reg] + int(sp)
                        net[cell] = net.get(cell, 0) - int(m)
                for reg, atoms in rule["rhs"].items():
                    for sp, m in atoms.items():
                        cell = region_cell[reg] + int(sp)
                        net[cell] = net.get(cell, 0) + int(m)
                nz = [(cell, d) for cell, d in sorted(net.items()) if d != 0]
                if len(nz) > MAX_DELTA:
                    raise ValueError("too many changed cells")
                for d, (cell, v) in enumerate(nz):
                    self.leaf_delta[leaf, d] = (cell, v)
                self.leaf_ndelta[leaf] = len(nz)

    def _regions(self, i, rule, comps):
        """Base cell of each pattern region for the slot (rule, context i)."""
        if rule["child"] < 0:
            return {"p": self.content_base[i]}
        par = comps[i]["parent"]
        return {"p": self.content_base[par], "w": self.wrap_base[i],
                "c": self.content_base[i]}


class _CModel(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("n_rules", ctypes.c_int32),
                ("leaf_rule", ctypes.c_void_p), ("leaf_react", ctypes.c_void_p),
                ("leaf_delta", ctypes.c_void_p), ("leaf_ndelta", ctypes.c_void_p),
                ("rule_k", ctypes.c_void_p), ("init_counts", ctypes.c_void_p)]


class _CRun(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_instances", ctypes.c_int64),
                ("replicas", ctypes.c_int64), ("rate_table", ctypes.c_void_p),
                ("init_table", ctypes.c_void_p), ("dt", ctypes.c_double),
                ("n_samples", ctypes.c_int32), ("count_cap", ctypes.c_int32),
                ("max_events", ctypes.c_int64)]


class _COut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("samples", "final_counts", "events", "t_final", "digest",
                 "status", "n_recorded", "n", "s1", "s2_lo", "s2_hi")]


def _ptr(a):
    return None if a is None else a.ctypes.data


def simulate(model: Dict, run: Dict, g0: int = 0, g1: Optional[int] = None,
             want_samples: bool = False, want_stats: bool = True,
             threads: int = 1, flat: Optional[FlatModel] = None) -> Dict:
    """Run trajectories g0..g1-1 (g = instance*R + replica) of ``run``.

    Returns per-trajectory arrays (final counts, applied events, final time,
    fired-slot digest, status, number of recorded samples, optionally the
    samples [g][K+1][C]) and, if ``want_stats``, the exact integer moments
    per (instance, sample[, cell]) over these trajectories plus mean/var."""
    fm = flat or FlatModel(model)
    L = lib()
    I, R = run["n_instances"], run["replicas"]
    G = I * R
    g1 = G if g1 is None else g1
    n = g1 - g0
    C, K1 = fm.n_cells, run["n_samples"]
    rate = run.get("rate_table")
    init = run.get("init_table")
    if rate is not None:
        rate = np.ascontiguousarray(rate, dtype=np.float64)
        assert rate.shape == (I, fm.n_rules)
    if init is not None:
        init = np.ascontiguousarray(init, dtype=np.int32)
        assert init.shape == (I, C)
    keep = [fm.leaf_rule, fm.leaf_react, fm.leaf_delta, fm.leaf_ndelta, fm.k, fm.init]
    cm = _CModel(C, fm.n_leaves, fm.n_rules, *[_ptr(a) for a in keep])
    cr = _CRun(run["seed"], I, R, _ptr(rate), _ptr(init), run["dt"], K1,
               run["count_cap"], run["max_events"])
    res = {
        "final_counts": np.zeros((n, C), np.int32),
        "events": np.zeros(n, np.int64),
        "t_final": np.zeros(n, np.float64),
        "digest": np.zeros(n, np.uint64),
        "status": np.zeros(n, np.uint8),
        "n_recorded": np.zeros(n, np.int32),
    }
    if want_samples:
        res["samples"] = np.zeros((n, K1, C), np.int32)
    threads = max(1, min(threads, n)) if n > 0 else 1
    bounds = [g0 + (n * t) // threads for t in range(threads + 1)]
    accs = []

    def work(t):
        a, b = bounds[t], bounds[t + 1]
        o = a - g0
        acc = None
        if want_stats:
            acc = {"n": np.zeros((I, K1), np.uint64),
                   "s1": np.zeros((I, K1, C), np.uint64),
                   "s2_lo": np.zeros((I, K1, C), np.uint64),
                   "s2_hi": np.zeros((I, K1, C), np.uint64)}
        co = _COut(
            _ptr(res["samples"][o:]) if want_samples else None,
            _ptr(res["final_counts"][o:]), _ptr(res["events"][o:]),
            _ptr(res["t_final"][o:]), _ptr(res["digest"][o:]),
            _ptr(res["status"][o:]), _ptr(res["n_recorded"][o:]),
            *([_ptr(acc[k]) for k in ("n", "s1", "s2_lo", "s2_hi")] if acc
              else [None] * 4))
        rc = L.oracle_simulate(ctypes.byref(cm), ctypes.byref(cr), a, b,
                               ctypes.byref(co))
        if rc != 0:
            raise MemoryError("oracle_simulate failed")
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
            L.oracle_merge_moments(*[_ptr(tot[k]) for k in ("n", "s1", "s2_lo", "s2_hi")],
                                   *[_ptr(acc[k]) for k in ("n", "s1", "s2_lo", "s2_hi")],
                                   I * K1, C)
        res.update(tot)
        res["mean"], res["var"] = finalize(tot, C)
    res["flat"] = fm
    return res


def finalize(acc: Dict, C: int):
    """mean = S1/n and unbiased var = (n S2 - S1^2)/(n(n-1)) per
    (instance, sample, cell) from exact integer moments."""
    n_rows = acc["n"].size
    mean = np.empty(acc["s1"].shape, np.float64)
    var = np.empty(acc["s1"].shape, np.float64)
    lib().oracle_finalize(*[_ptr(np.ascontiguousarray(acc[k])) for k in ("n", "s1", "s2_lo", "s2_hi")],
                          n_rows, C, _ptr(mean), _ptr(var))
    return mean, var


def philox(ctr, key):
    """One Philox4x32-10 block (4 x uint32) for a counter and a key."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return tuple(o)


def draw(seed: int, g: int, e: int):
    """(u_tau, u_sel) of draw e of trajectory g under run seed ``seed``."""
    x = philox((e & 0xFFFFFFFF, e >> 32, g & 0xFFFFFFFF, g >> 32),
               (seed & 0xFFFFFFFF, seed >> 32))
    return lib().oracle_u_tau(x[0], x[1]), lib().oracle_u_sel(x[2], x[3])


def select(leaves, x: float):
    """(leaf index, root sum) chosen by the selection descent for x."""
    lv = np.ascontiguousarray(leaves, dtype=np.float64)
    a0 = ctypes.c_double()
    j = lib().oracle_select(lv.ctypes.data, len(lv), float(x), ctypes.byref(a0))
    return j, a0.value


def ssa_log(u: float) -> float:
    return lib().oracle_ssa_log(u)
