"""Seeded synthetic workloads for bulk CWC stochastic simulation.

This module only *describes* inputs: CWC models (species, compartment tree,
rewrite rules with kinetic constants, initial multiplicities), run
descriptors (seed, replicas, sample grid, caps), parameter-sweep rate tables
and a serving arrival trace.  It holds none of the simulation arithmetic
(no propensities, no random streams, no sampling); both the CPU oracle and
the GPU library consume what it returns.

Model dictionaries (JSON-serialisable) follow the CWC formalism of the
paper (Sec. 2.1): a term is a multiset of atoms and compartments
``(wrap | content)^label``; a rewrite rule ``label: P -> O`` carries a
kinetic constant ``k`` (Sec. 2.2).  The compartment tree is fixed, so a
model lists its compartments in preorder and every rule names

* ``parent``: the label of the compartment whose *content* the rule is
  applied in (compartment 0 is the top level, label 0);
* ``child``:  ``-1`` for a rule that only rewrites that content, or the
  label of a child compartment whose wrap and/or content the pattern also
  reaches (a rule across a membrane, e.g. transport);
* ``lhs``/``rhs``: atom multiplicities per region, ``"p"`` = the parent
  content, ``"w"`` = the child's wrap, ``"c"`` = the child's content.

Initial multiplicities: ``init[i]`` is compartment i's content vector (one
int per species), ``init_wrap[i]`` its wrap vector (only for labels whose
``wrap`` flag is set).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "lotka_volterra", "gene_regulation", "multi_compartment",
    "birth_death", "isomerisation", "pure_decay", "dimerisation",
    "transport", "receptor_binding", "paper_example",
    "make_run", "sweep_rate_table", "arrival_trace", "config",
    "n_cells", "CONFIG_NAMES",
    "general_from_fixed", "cell_birth_death", "cell_dissolution", "nested_export",
    "receptor_internalisation", "cell_colony",
]

CONFIG_NAMES = {
    0: "lotka_volterra_r64",
    1: "gene_regulation_r16384",
    2: "gene_regulation_sweep_i4096_r64",
    3: "multi_compartment_c32_r2048",
    4: "serving_poisson_200jobs_per_s",
}


def _rule(parent, child, lhs, rhs, k):
    return {"parent": int(parent), "child": int(child),
            "lhs": {r: dict(v) for r, v in lhs.items()},
            "rhs": {r: dict(v) for r, v in rhs.items()},
            "k": float(k)}


def _local(label, lhs: Dict[int, int], rhs: Dict[int, int], k):
    return _rule(label, -1, {"p": lhs}, {"p": rhs}, k)


def n_cells(model) -> int:
    """Number of (region, species) count cells in a model's output layout.

    Cells are ordered by compartment (preorder); each compartment contributes
    its content species, then its wrap species if its label has a wrap."""
    ns = len(model["species"])
    tot = 0
    for c in model["compartments"]:
        tot += ns * (2 if model["types"][c["type"]]["wrap"] else 1)
    return tot


def _single(name, species, rules, init):
    return {"name": name, "species": list(species),
            "types": [{"name": "top", "wrap": False}],
            "compartments": [{"type": 0, "parent": -1}],
            "init": [list(map(int, init))], "init_wrap": [None],
            "rules": rules}


# ---------------------------------------------------------------------------
# Workload models
# ---------------------------------------------------------------------------

def lotka_volterra(x0=1000, y0=1000, k=(10.0, 0.01, 10.0)):
    """Prey-predator Lotka-Volterra, one compartment (the paper's Sec. 5
    test model family; rates and sizes are the workload's own):
    X -> 2X, X + Y -> 2Y, Y -> 0."""
    X, Y = 0, 1
    rules = [_local(0, {X: 1}, {X: 2}, k[0]),
             _local(0, {X: 1, Y: 1}, {Y: 2}, k[1]),
             _local(0, {Y: 1}, {}, k[2])]
    return _single("lotka_volterra", ["X", "Y"], rules, [x0, y0])


GENE_SPECIES = ["G1", "G1r", "G2", "G2r", "M1", "M2", "P1", "P2", "D1", "D2"]


def gene_regulation(model_seed=1):
    """Two-compartment gene-regulation network: a nucleus wrapped inside the
    cytoplasm (top level).  Ten species, twenty mass-action rules: eight in
    the nucleus, eight in the cytoplasm and four across the nuclear
    membrane.  Kinetic constants 10^U(-3,1), initial multiplicities
    U{0..200} for all 20 cells, both drawn once from ``model_seed``."""
    s = {n: i for i, n in enumerate(GENE_SPECIES)}
    rng = np.random.default_rng(model_seed)
    ks = 10.0 ** rng.uniform(-3.0, 1.0, size=20)
    init = rng.integers(0, 201, size=(2, 10))
    CYT, NUC = 0, 1
    g = lambda n: s[n]
    rules = [
        # nucleus-local
        _local(NUC, {g("G1"): 1}, {g("G1"): 1, g("M1"): 1}, ks[0]),
        _local(NUC, {g("G2"): 1}, {g("G2"): 1, g("M2"): 1}, ks[1]),
        _local(NUC, {g("G1"): 1, g("D2"): 1}, {g("G1r"): 1}, ks[2]),
        _local(NUC, {g("G1r"): 1}, {g("G1"): 1, g("D2"): 1}, ks[3]),
        _local(NUC, {g("G2"): 1, g("D1"): 1}, {g("G2r"): 1}, ks[4]),
        _local(NUC, {g("G2r"): 1}, {g("G2"): 1, g("D1"): 1}, ks[5]),
        _local(NUC, {g("D1"): 1}, {}, ks[6]),
        _local(NUC, {g("D2"): 1}, {}, ks[7]),
        # cytoplasm-local
        _local(CYT, {g("M1"): 1}, {g("M1"): 1, g("P1"): 1}, ks[8]),
        _local(CYT, {g("M2"): 1}, {g("M2"): 1, g("P2"): 1}, ks[9]),
        _local(CYT, {g("M1"): 1}, {}, ks[10]),
        _local(CYT, {g("M2"): 1}, {}, ks[11]),
        _local(CYT, {g("P1"): 1}, {}, ks[12]),
        _local(CYT, {g("P2"): 1}, {}, ks[13]),
        _local(CYT, {g("P1"): 2}, {g("D1"): 1}, ks[14]),
        _local(CYT, {g("P2"): 2}, {g("D2"): 1}, ks[15]),
        # across the nuclear membrane: mRNA export, dimer import
        _rule(CYT, NUC, {"c": {g("M1"): 1}}, {"p": {g("M1"): 1}}, ks[16]),
        _rule(CYT, NUC, {"c": {g("M2"): 1}}, {"p": {g("M2"): 1}}, ks[17]),
        _rule(CYT, NUC, {"p": {g("D1"): 1}}, {"c": {g("D1"): 1}}, ks[18]),
        _rule(CYT, NUC, {"p": {g("D2"): 1}}, {"c": {g("D2"): 1}}, ks[19]),
    ]
    return {"name": "gene_regulation", "species": GENE_SPECIES,
            "types": [{"name": "cytoplasm", "wrap": False},
                      {"name": "nucleus", "wrap": False}],
            "compartments": [{"type": CYT, "parent": -1},
                             {"type": NUC, "parent": 0}],
            "init": [list(map(int, init[0])), list(map(int, init[1]))],
            "init_wrap": [None, None],
            "rules": rules}


def multi_compartment(model_seed=3, n_cells_=32):
    """An outer compartment holding ``n_cells_`` sibling cells, 12 species
    per compartment.  Cells run 20 local rules (four isomerisations,
    two hetero- and one homo-dimerisation, synthesis/decay of s11, s11
    driven production of s6, decays); the outer compartment runs 4
    isomerisations; s0, s2 and s11 are imported into and exported from
    every cell (6 membrane-crossing rules).  Kinetic constants 10^U(-3,1),
    initial multiplicities Poisson(50) per (compartment, species), drawn
    once from ``model_seed``."""
    rng = np.random.default_rng(model_seed)
    ks = 10.0 ** rng.uniform(-3.0, 1.0, size=30)
    ncomp = 1 + n_cells_
    init = rng.poisson(50.0, size=(ncomp, 12))
    OUT, CELL = 0, 1
    rules = []
    ki = iter(ks)
    for a, b in [(0, 1), (2, 3), (4, 5), (6, 7)]:
        rules.append(_local(CELL, {a: 1}, {b: 1}, next(ki)))
        rules.append(_local(CELL, {b: 1}, {a: 1}, next(ki)))
    rules.append(_local(CELL, {0: 1, 2: 1}, {8: 1}, next(ki)))
    rules.append(_local(CELL, {8: 1}, {0: 1, 2: 1}, next(ki)))
    rules.append(_local(CELL, {1: 1, 3: 1}, {9: 1}, next(ki)))
    rules.append(_local(CELL, {9: 1}, {1: 1, 3: 1}, next(ki)))
    rules.append(_local(CELL, {4: 2}, {10: 1}, next(ki)))
    rules.append(_local(CELL, {10: 1}, {4: 2}, next(ki)))
    rules.append(_local(CELL, {}, {11: 1}, next(ki)))
    rules.append(_local(CELL, {11: 1}, {}, next(ki)))
    rules.append(_local(CELL, {11: 1}, {11: 1, 6: 1}, next(ki)))
    rules.append(_local(CELL, {6: 1}, {}, next(ki)))
    rules.append(_local(CELL, {7: 1}, {}, next(ki)))
    rules.append(_local(CELL, {10: 1}, {}, next(ki)))
    for a, b in [(0, 1), (2, 3)]:
        rules.append(_local(OUT, {a: 1}, {b: 1}, next(ki)))
        rules.append(_local(OUT, {b: 1}, {a: 1}, next(ki)))
    for s in (0, 2, 11):
        rules.append(_rule(OUT, CELL, {"p": {s: 1}}, {"c": {s: 1}}, next(ki)))
        rules.append(_rule(OUT, CELL, {"c": {s: 1}}, {"p": {s: 1}}, next(ki)))
    comps = [{"type": OUT, "parent": -1}] + \
        [{"type": CELL, "parent": 0} for _ in range(n_cells_)]
    return {"name": "multi_compartment",
            "species": ["s%d" % i for i in range(12)],
            "types": [{"name": "outer", "wrap": False},
                      {"name": "cell", "wrap": False}],
            "compartments": comps,
            "init": [list(map(int, r)) for r in init],
            "init_wrap": [None] * ncomp,
            "rules": rules}


# ---------------------------------------------------------------------------
# Small models with closed-form laws (test workloads)
# ---------------------------------------------------------------------------

def birth_death(lam=20.0, mu=1.0, n0=0):
    """0 -> A at rate lam, A -> 0 at rate mu per molecule."""
    return _single("birth_death", ["A"],
                   [_local(0, {}, {0: 1}, lam), _local(0, {0: 1}, {}, mu)],
                   [n0])


def isomerisation(k1=1.0, k2=3.0, a0=40, b0=0):
    """A -> B at k1, B -> A at k2."""
    return _single("isomerisation", ["A", "B"],
                   [_local(0, {0: 1}, {1: 1}, k1), _local(0, {1: 1}, {0: 1}, k2)],
                   [a0, b0])


def pure_decay(k=0.7, n0=50):
    return _single("pure_decay", ["A"], [_local(0, {0: 1}, {}, k)], [n0])


def dimerisation(k=0.05, n0=30):
    """A + A -> 0 (second order in one species)."""
    return _single("dimerisation", ["A"], [_local(0, {0: 2}, {}, k)], [n0])


def paper_example(k=0.5):
    """The paper's propensity example (Sec. 2.2): rule a b X -> c X applied
    to the term a a b b; a, b, c are species 0, 1, 2."""
    return _single("paper_example", ["a", "b", "c"],
                   [_local(0, {0: 1, 1: 1}, {2: 1}, k)], [2, 2, 0])


def transport(k_in=2.0, k_out=1.0, n_children=3, n_outer=30):
    """An outer compartment with ``n_children`` wrapped children; atom x
    enters every child at k_in per atom of the parent and leaves at k_out
    per atom of the child."""
    rules = [_rule(0, 1, {"p": {0: 1}}, {"c": {0: 1}}, k_in),
             _rule(0, 1, {"c": {0: 1}}, {"p": {0: 1}}, k_out)]
    comps = [{"type": 0, "parent": -1}] + \
        [{"type": 1, "parent": 0} for _ in range(n_children)]
    init = [[n_outer]] + [[0] for _ in range(n_children)]
    return {"name": "transport", "species": ["x"],
            "types": [{"name": "top", "wrap": False},
                      {"name": "cell", "wrap": False}],
            "compartments": comps, "init": init,
            "init_wrap": [None] * (1 + n_children), "rules": rules}


def receptor_binding(k_on=0.02, k_off=0.5, k_int=0.1, n_lig=40, n_rec=10,
                     n_cells_=2):
    """Wrap atoms: ligand L (outside) binds receptor R on a cell's wrap,
    forming LR on the wrap; LR releases L back outside or internalises it
    as L inside the cell (content), freeing R.  Exercises the wrap region
    and a two-region bimolecular pattern."""
    L, R, LR = 0, 1, 2
    rules = [
        _rule(0, 1, {"p": {L: 1}, "w": {R: 1}}, {"w": {LR: 1}}, k_on),
        _rule(0, 1, {"w": {LR: 1}}, {"p": {L: 1}, "w": {R: 1}}, k_off),
        _rule(0, 1, {"w": {LR: 1}}, {"w": {R: 1}, "c": {L: 1}}, k_int),
        _local(1, {L: 1}, {}, 0.05),
    ]
    comps = [{"type": 0, "parent": -1}] + \
        [{"type": 1, "parent": 0} for _ in range(n_cells_)]
    init = [[n_lig, 0, 0]] + [[0, 0, 0] for _ in range(n_cells_)]
    init_wrap = [None] + [[0, n_rec, 0] for _ in range(n_cells_)]
    return {"name": "receptor_binding", "species": ["L", "R", "LR"],
            "types": [{"name": "top", "wrap": False},
                      {"name": "cell", "wrap": True}],
            "compartments": comps, "init": init, "init_wrap": init_wrap,
            "rules": rules}


# ---------------------------------------------------------------------------
# General CWC models: compartments created, dissolved and deleted at run
# time; patterns that reach a grandchild compartment (paper Sec. 2.1)
# ---------------------------------------------------------------------------
#
# A general model lists ``labels`` (compartment types with a wrap flag), a
# slot capacity ``max_comp`` (<= 64), the initial ``term`` (compartments in
# preorder, each {"label", "parent", "content", "wrap"}; entry 0 is the top
# level) and ``rules``, each applied in the content of a compartment of
# label ``context``, naming optionally a ``child`` compartment of a label
# inside it and a ``grandchild`` inside that (-1 = none).  ``lhs``/``rhs``
# give atom multiplicities per region: "c" the context's content, "w1"/"c1"
# the child's wrap/content, "w2"/"c2" the grandchild's; unnamed atoms of a
# region are the pattern's variable (x / X) and are kept.  ``action``:
#   "create"   a compartment {"label", "wrap", "content"} (``new``) in the
#              context (level 0), the child (1) or the grandchild (2);
#   "dissolve" the child (level 1) or grandchild (2): its content (atoms and
#              compartments), and its wrap atoms if ``release_wrap``, pass to
#              its parent's content -- O = X in the pattern (x | X)^l -> X;
#   "delete"   the child or grandchild with everything in it.

def _grule(context, lhs, rhs, k, child=-1, grandchild=-1, action="none", level=0, new=None,
           release_wrap=False):
    return {"context": int(context), "child": int(child), "grandchild": int(grandchild),
            "lhs": {r: {int(a): int(m) for a, m in v.items()} for r, v in lhs.items()},
            "rhs": {r: {int(a): int(m) for a, m in v.items()} for r, v in rhs.items()},
            "action": action, "level": int(level), "new": new,
            "release_wrap": bool(release_wrap), "k": float(k)}


def general_from_fixed(model, max_comp=None):
    """A fixed-tree model written as a general one (same compartments as the
    initial term, same rules, no structural action): the general engine
    must simulate it exactly as the fixed-tree engine does."""
    comps = model["compartments"]
    iw = model.get("init_wrap") or [None] * len(comps)
    term = [{"label": c["type"], "parent": c["parent"], "content": list(model["init"][i]),
             "wrap": None if iw[i] is None else list(iw[i])} for i, c in enumerate(comps)]
    rules = []
    for r in model["rules"]:
        reg = {"p": "c", "w": "w1", "c": "c1"}
        lhs = {reg[q]: v for q, v in r["lhs"].items()}
        rhs = {reg[q]: v for q, v in r["rhs"].items()}
        rules.append(_grule(r["parent"], lhs, rhs, r["k"], child=r["child"]))
    return {"name": model["name"] + "_general", "species": list(model["species"]),
            "labels": [dict(t) for t in model["types"]],
            "max_comp": int(max_comp or len(comps)), "term": term, "rules": rules}


def cell_birth_death(lam=3.0, mu=1.0, n0=2, max_comp=32):
    """Cells appear in the top level at rate lam (an empty compartment is
    created) and each is removed at rate mu: the number of cells is a
    birth-death process, Binomial(n0, e^-mu t) + Poisson(lam/mu (1 - e^-mu t))."""
    term = [{"label": 0, "parent": -1, "content": [0], "wrap": None}]
    term += [{"label": 1, "parent": 0, "content": [0], "wrap": [0]} for _ in range(n0)]
    rules = [_grule(0, {}, {}, lam, action="create", level=0,
                    new={"label": 1, "wrap": [0], "content": [0]}),
             _grule(0, {}, {}, mu, child=1, action="delete", level=1)]
    return {"name": "cell_birth_death", "species": ["a"],
            "labels": [{"name": "top", "wrap": False}, {"name": "cell", "wrap": True}],
            "max_comp": max_comp, "term": term, "rules": rules}


def cell_dissolution(n_cells_=3, a_per_cell=2, w_per_cell=1, mu=0.7, k_out=0.5,
                     release_wrap=True, max_comp=8):
    """Cells holding atoms a (content) and w (wrap) dissolve at rate mu,
    releasing their content -- and their wrap atoms if ``release_wrap`` --
    into the top level, where a decays at rate k_out.  (x | X)^cell -> X."""
    A, Wd = 0, 1
    term = [{"label": 0, "parent": -1, "content": [0, 0], "wrap": None}]
    term += [{"label": 1, "parent": 0, "content": [a_per_cell, 0], "wrap": [0, w_per_cell]}
             for _ in range(n_cells_)]
    rules = [_grule(0, {}, {}, mu, child=1, action="dissolve", level=1,
                    release_wrap=release_wrap),
             _grule(0, {"c": {A: 1}}, {}, k_out)]
    return {"name": "cell_dissolution", "species": ["a", "w"],
            "labels": [{"name": "top", "wrap": False}, {"name": "cell", "wrap": True}],
            "max_comp": max_comp, "term": term, "rules": rules}


def nested_export(n_outer=2, n_inner=2, s0=2, k_mk=0.8, k_exp=1.3, k_deg=0.4, max_comp=16):
    """Two levels below the top: outer compartments hold inner ones.  Inner
    compartments turn s into b; a depth-2 pattern at the top moves b from an
    inner compartment's content to its outer's,
    (x | (y | b Y)^in X)^out -> (x | (y | Y)^in b X)^out; b decays in outers."""
    S, B = 0, 1
    term = [{"label": 0, "parent": -1, "content": [0, 0], "wrap": None}]
    for o in range(n_outer):
        po = len(term)
        term.append({"label": 1, "parent": 0, "content": [0, 0], "wrap": [0, 0]})
        for _ in range(n_inner):
            term.append({"label": 2, "parent": po, "content": [s0, 0], "wrap": [0, 0]})
    rules = [_grule(2, {"c": {S: 1}}, {"c": {B: 1}}, k_mk),
             _grule(0, {"c2": {B: 1}}, {"c1": {B: 1}}, k_exp, child=1, grandchild=2),
             _grule(1, {"c": {B: 1}}, {}, k_deg)]
    return {"name": "nested_export", "species": ["s", "b"],
            "labels": [{"name": "top", "wrap": False}, {"name": "out", "wrap": True},
                       {"name": "in", "wrap": True}],
            "max_comp": max_comp, "term": term, "rules": rules}


def receptor_internalisation(n_cells_=2, r0=3, l0=4, k_on=0.3, k_int=0.8, k_ves=0.6,
                             max_comp=16):
    """Wrap variables and creation below the context: a ligand L in the top
    binds a receptor R on a cell's wrap, L (R x | X)^cell -> (RL x | X)^cell;
    a bound receptor is internalised by creating a vesicle inside the cell,
    (RL x | X)^cell -> (x | (RL | )^ves X)^cell; vesicles dissolve into the
    cell's content, releasing RL there."""
    L, R, RL = 0, 1, 2
    term = [{"label": 0, "parent": -1, "content": [l0, 0, 0], "wrap": None}]
    term += [{"label": 1, "parent": 0, "content": [0, 0, 0], "wrap": [0, r0, 0]}
             for _ in range(n_cells_)]
    rules = [_grule(0, {"c": {L: 1}, "w1": {R: 1}}, {"w1": {RL: 1}}, k_on, child=1),
             _grule(0, {"w1": {RL: 1}}, {}, k_int, child=1, action="create", level=1,
                    new={"label": 2, "wrap": [0, 0, 1], "content": [0, 0, 0]}),
             _grule(1, {}, {}, k_ves, child=2, action="dissolve", level=1, release_wrap=True)]
    return {"name": "receptor_internalisation", "species": ["L", "R", "RL"],
            "labels": [{"name": "top", "wrap": False}, {"name": "cell", "wrap": True},
                       {"name": "ves", "wrap": True}],
            "max_comp": max_comp, "term": term, "rules": rules}


def cell_colony(n0=8, nutrient=2000, k_up=0.002, k_grow=1.0, k_div=0.05, k_die=0.02,
                k_feed=200.0, max_comp=64, model_seed=5, k_decay=0.0):
    """A colony of cells in a nutrient bath: nutrients N enter cells across
    the wrap, N (x | X)^cell -> (x | N X)^cell; inside, N becomes biomass A;
    a cell with two units of biomass divides, creating a new cell in the
    top level that takes one unit, (x | A A X)^cell -> (x | A X)^cell (| A)^cell;
    cells die (deleted with their content); nutrients are fed to the top.
    Initial cell contents are drawn once from ``model_seed``.  Feeding is
    left out with ``k_feed`` = 0.  With ``k_decay`` > 0 biomass is also spent, A -> 0 inside cells, so the colony
    can settle instead of filling its slots."""
    Nn, A = 0, 1
    rng = np.random.default_rng(model_seed)
    term = [{"label": 0, "parent": -1, "content": [nutrient, 0], "wrap": None}]
    for _ in range(n0):
        term.append({"label": 1, "parent": 0, "content": [0, int(rng.integers(1, 6))],
                     "wrap": [0, 0]})
    rules = [_grule(0, {"c": {Nn: 1}}, {"c1": {Nn: 1}}, k_up, child=1),
             _grule(1, {"c": {Nn: 1}}, {"c": {A: 1}}, k_grow),
             _grule(0, {"c1": {A: 2}}, {"c1": {A: 1}}, k_div, child=1, action="create",
                    level=0, new={"label": 1, "wrap": [0, 0], "content": [0, 1]}),
             _grule(0, {}, {}, k_die, child=1, action="delete", level=1)]
    if k_feed > 0:
        rules.append(_grule(0, {}, {"c": {Nn: 1}}, k_feed))
    if k_decay > 0:
        rules.append(_grule(1, {"c": {A: 1}}, {}, k_decay))
    return {"name": "cell_colony", "species": ["N", "A"],
            "labels": [{"name": "top", "wrap": False}, {"name": "cell", "wrap": True}],
            "max_comp": max_comp, "term": term, "rules": rules}


# ---------------------------------------------------------------------------
# Runs, sweeps, serving trace
# ---------------------------------------------------------------------------

def make_run(seed=0, n_instances=1, replicas=64, dt=0.05, n_samples=101,
             rate_table=None, init_table=None, count_cap=2**31 - 1,
             max_events=0):
    """Run descriptor.  ``n_samples`` = K+1 sample points t_k = k*dt,
    k = 0..K.  ``rate_table`` [n_instances][n_rules] float64 or None (use
    the model's k), ``init_table`` [n_instances][n_cells] int32 or None
    (use the model's initial multiplicities).  ``max_events`` 0 = no cap."""
    return {"seed": int(seed), "n_instances": int(n_instances),
            "replicas": int(replicas), "dt": float(dt),
            "n_samples": int(n_samples),
            "rate_table": None if rate_table is None else
            np.ascontiguousarray(rate_table, dtype=np.float64),
            "init_table": None if init_table is None else
            np.ascontiguousarray(init_table, dtype=np.int32),
            "count_cap": int(count_cap), "max_events": int(max_events)}


def sweep_rate_table(model, n_instances=4096, sweep_seed=2):
    """Parameter sweep: instance i scales every kinetic constant by one
    factor f_i = 10^U(-1,1) drawn from ``sweep_seed``; entry = RN(k_r*f_i)."""
    rng = np.random.default_rng(sweep_seed)
    f = 10.0 ** rng.uniform(-1.0, 1.0, size=n_instances)
    k = np.array([r["k"] for r in model["rules"]], dtype=np.float64)
    return (f[:, None] * k[None, :]).astype(np.float64), f


def arrival_trace(n_jobs=2000, mean_gap_s=0.005, seed=4):
    """Serving trace: Poisson arrivals (exponential gaps, mean 5 ms), each
    job draws a config in {0,1,2,3}, replicas round(exp(U(ln 64, ln 8192)))
    and t_end ~ U(5,100) snapped down to that config's sample grid; the job
    seed is the job index.  Lotka-Volterra jobs carry a count cap of 10^5:
    over horizons this long a replica's predators can die out, after which
    prey grow without bound (about 2^31 birth events to overflow int32); the
    cap ends such a replica with status OVERFLOW instead."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap_s, size=n_jobs)
    t_arr = np.cumsum(gaps)
    cfg = rng.integers(0, 4, size=n_jobs)
    reps = np.rint(np.exp(rng.uniform(math.log(64), math.log(8192), size=n_jobs))).astype(int)
    t_end = rng.uniform(5.0, 100.0, size=n_jobs)
    jobs = []
    for j in range(n_jobs):
        c = int(cfg[j])
        dt = 0.05 if c == 0 else 0.5
        K = int(math.floor(t_end[j] / dt + 1e-9))
        jobs.append({"job": j, "arrival_s": float(t_arr[j]), "config": c,
                     "replicas": int(reps[j]), "dt": dt, "n_samples": K + 1,
                     "seed": j, "count_cap": 100000 if c == 0 else 2**31 - 1})
    return jobs


def config(i: int, replicas: Optional[int] = None):
    """(model, run) for the benchmark configurations 0-3.

    0: Lotka-Volterra, 64 replicas, t_end 5 sampled every 0.05, seed 0.
    1: gene regulation, 16384 replicas, t_end 100, 201 samples.
    2: gene-regulation sweep, 4096 instances x 64 replicas.
    3: 32 cells in an outer compartment, 2048 replicas, t_end 50, 101 samples.
    ``replicas`` overrides the replica count (smaller parity cases)."""
    if i == 0:
        m = lotka_volterra()
        return m, make_run(seed=0, replicas=replicas or 64, dt=0.05, n_samples=101)
    if i == 1:
        m = gene_regulation(1)
        return m, make_run(seed=0, replicas=replicas or 16384, dt=0.5, n_samples=201)
    if i == 2:
        m = gene_regulation(1)
        tab, _ = sweep_rate_table(m, 4096, 2)
        return m, make_run(seed=0, n_instances=4096, replicas=replicas or 64,
                           dt=0.5, n_samples=201, rate_table=tab)
    if i == 3:
        m = multi_compartment(3)
        return m, make_run(seed=0, replicas=replicas or 2048, dt=0.5, n_samples=101)
    raise ValueError("config %r" % i)
