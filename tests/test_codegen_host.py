"""Generated model code checked on the host.  The per-leaf change table: the model's
CWC_APPLY macro and its table (as the library generates them) are compiled
with g++ around stand-ins for the two bit-field-extract builtins, every
leaf's change is applied to a known state, and the result must be the net
change the oracle's own flattening gives for that leaf (Sec. 2.1: the
rewrite replaces the matched reactants by the products).  Covers the byte
layout (signed and unsigned bytes and half-words, 1 to 4 words), the dense
layout, and the per-digit leaf-mask fallback on 32- and 64-leaf trees.  The
pair and quad layouts' per-lane counts: each lane's slots after the update,
undo and redo, the lanes' written rows together and the growth test, per
leaf, in both state forms (per-lane table, or every lane keeping every
cell).  The
selection descents (one lane; two lanes after the engine's root decision):
compiled the same way and compared with the oracle's selection (Sec. 2.2:
the reaction is chosen with probability proportional to its rate) on
random trees with zero leaves and on integer trees at every tie.  The
propensity trees: every leaf k x (double) prod C(n, m) and every node
left + right, bit for bit, and the pair and quad layouts' partial trees,
built from each lane's own slots, equal to them."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

import oracle
import workloads as W
from tests.test_gpu_parity import bursts, bursts_dense, bursts_wide

HARNESS = r"""
#include <cstdio>
typedef unsigned int u32;
typedef unsigned long long u64;
typedef int i32;
typedef long long i64;
struct uint2 { unsigned x, y; };
struct uint4 { unsigned x, y, z, w; };
#define __constant__
#define CWC_KEEP(v) ((void)0)
static inline int host_sbfe(int v, unsigned off, unsigned w) {
    return (int)((unsigned)v << (32u - off - w)) >> (32u - w);
}
static inline unsigned host_ubfe(unsigned v, unsigned off, unsigned w) {
    return (v >> off) & (w >= 32u ? 0xFFFFFFFFu : ((1u << w) - 1u));
}
#define __builtin_amdgcn_sbfe(v, o, w) host_sbfe((v), (o), (w))
#define __builtin_amdgcn_ubfe(v, o, w) host_ubfe((v), (o), (w))
%(table)s
%(apply)s
%(lds)s
int main() {
%(copy)s
    for (int j = 0; j < %(P)d; ++j) {
        for (int capcase = 0; capcase < 2; ++capcase) {
%(decl)s
            const unsigned cap_ = capcase ? %(base)du : 0xFFFFFFFFu;
            bool ovf_;
            { CWC_APPLY(j, cap_, o_); ovf_ = o_; }
            if (!capcase) {
                std::printf("%%d", j);
%(print)s
            } else {
                std::printf(" %%d\n", ovf_ ? 1 : 0);
            }
        }
    }
    return 0;
}
"""

BASE = 1 << 20


def macro(src, head):
    i = src.index("#define " + head)
    j = src.index("/* end */", i)
    return src[i:j] + "/* end */\n"


def applied_changes(model):
    """(P, C, {leaf: [change per cell]}, {leaf: overflow flag at cap = state})
    from the generated code."""
    from paper_1010_2438_amd import cwc_codegen
    src = cwc_codegen(model)
    C = int(re.search(r"#define CWC_C (\d+)", src).group(1))
    P = int(re.search(r"#define CWC_P (\d+)", src).group(1))
    dtw = int(re.search(r"#define CWC_DT_W (\d+)", src).group(1))
    table = lds = copy = ""
    if dtw:
        table = re.search(r"__constant__ unsigned int cwc_dtab_g\[\d+\] = \{[^}]*\};", src).group(0)
        ty = re.search(r"__shared__ (\w[\w ]*?) cwc_dtab\[", src).group(1)
        lds = "static %s cwc_dtab[%d];" % (ty, P)
        copy = ("    for (int i = 0; i < %d; ++i) ((unsigned *)cwc_dtab)[i] = cwc_dtab_g[i];"
                % (P * dtw))
    code = HARNESS % {
        "table": "#define CWC_DT_W %d\n%s" % (dtw, table),
        "apply": macro(src, "CWC_APPLY_MX(j, mx)") + macro(src, "CWC_APPLY(j, cap, ovf)"),
        "lds": lds, "copy": copy, "P": P,
        "base": BASE,
        "decl": "\n".join("            int n%d = %d;" % (c, BASE) for c in range(C)),
        "print": "\n".join('                std::printf(" %%d", n%d - %d);' % (c, BASE)
                           for c in range(C))}
    d = tempfile.mkdtemp(prefix="cwc_apply_")
    try:
        with open(os.path.join(d, "t.cpp"), "w") as f:
            f.write(code)
        subprocess.check_call(["g++", "-O1", "-w", "-o", os.path.join(d, "t"),
                               os.path.join(d, "t.cpp")])
        out = subprocess.check_output([os.path.join(d, "t")], text=True)
    finally:
        shutil.rmtree(d)
    changes, ovf = {}, {}
    for line in out.splitlines():
        v = [int(x) for x in line.split()]
        changes[v[0]] = v[1:1 + C]
        ovf[v[0]] = v[1 + C]
    return P, C, changes, ovf, src


def huge_burst():
    """One species made 1,000,000 at a time (the largest net change the
    library accepts) and lost one at a time: a 21-bit signed field, too
    wide for the byte layout."""
    return W._single("huge_burst", ["X"],
                     [W._local(0, {}, {0: 1_000_000}, 0.01), W._local(0, {0: 1}, {}, 1.0)],
                     [0])


MODELS = {
    "paper_example": W.paper_example,                  # byte layout, unsigned byte
    "receptor_binding": W.receptor_binding,            # byte layout, two words
    "transport7": lambda: W.transport(n_children=7),
    "gene_regulation": lambda: W.config(1)[0],         # byte layout, four words
    "bursts": bursts,                                  # signed and unsigned half-words
    "bursts_dense": bursts_dense,                      # dense fields + 32-bit leaf masks
    "bursts_wide": bursts_wide,                        # dense fields + 64-bit leaf masks
    "one_cell": lambda: W.multi_compartment(3, n_cells_=1),   # dense, 64 leaves
    "huge_burst": huge_burst,                          # dense, a 21-bit signed field
    "lotka_volterra": W.lotka_volterra,                # 4 leaves
    "transport": W.transport,                          # 8 leaves
}


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("name", sorted(MODELS))
def test_generated_change_table(name):
    model = MODELS[name]()
    P, C, changes, ovf, src = applied_changes(model)
    flat = oracle.FlatModel(model)
    assert (P, C) == (flat.n_leaves, flat.n_cells)
    for leaf in range(P):
        want = [0] * C
        for k in range(int(flat.leaf_ndelta[leaf])):
            cell, v = (int(x) for x in flat.leaf_delta[leaf, k])
            want[cell] += v
        assert changes[leaf] == want, "leaf %d" % leaf
        # with the cap at the current state, the event overflows exactly
        # when it raises some count
        assert ovf[leaf] == int(any(v > 0 for v in want)), "leaf %d" % leaf


def test_layouts_covered():
    """The models above reach every encoding of the table."""
    from paper_1010_2438_amd import cwc_codegen
    seen = set()
    for name, mk in MODELS.items():
        body = macro(cwc_codegen(mk()), "CWC_APPLY_MX(j, mx)")
        for key, pat in (("s8", "(signed char)"), ("u8", "(unsigned char)"),
                         ("s16", "(short)"), ("u16", "(unsigned short)"),
                         ("sbfe", "amdgcn_sbfe"), ("ubfe", "amdgcn_ubfe(dw"),
                         ("mask32", "amdgcn_ubfe(0x"), ("mask64", "(js_ & 32u)"),
                         ("w4", "uint4 dq_")):
            if pat in body:
                seen.add(key)
    assert seen == {"s8", "u8", "s16", "u16", "sbfe", "ubfe", "mask32", "mask64", "w4"}


GROUP_APPLY_HARNESS = r"""
#include <cstdio>
typedef unsigned int u32;
typedef int i32;
struct uint2 { unsigned x, y; };
struct uint4 { unsigned x, y, z, w; };
#define __constant__
#define CWC_KEEP(v) ((void)0)
static inline int host_sbfe(int v, unsigned off, unsigned w) {
    return (int)((unsigned)v << (32u - off - w)) >> (32u - w);
}
static inline unsigned host_ubfe(unsigned v, unsigned off, unsigned w) {
    return (v >> off) & (w >= 32u ? 0xFFFFFFFFu : ((1u << w) - 1u));
}
#define __builtin_amdgcn_sbfe(v, o, w) host_sbfe((v), (o), (w))
#define __builtin_amdgcn_ubfe(v, o, w) host_ubfe((v), (o), (w))
%(tables)s
%(macros)s
static void show(const char *tag, int h, int j, const int *v) {
    std::printf("%%s %%d %%d", tag, h, j);
    for (int c = 0; c < %(C)d; ++c) std::printf(" %%d", v[c]);
    std::printf("\n");
}
int main() {
%(copy)s
    for (int pass = 0; pass < 2; ++pass) {
        int N[%(C)d];
        for (int c = 0; c < %(C)d; ++c) N[c] = %(base)d + (pass ? 0 : 7 * c);
        for (int j = 0; j < %(P)d; ++j) {
            int own[%(C)d];
            for (int c = 0; c < %(C)d; ++c) own[c] = -1;
            unsigned mxs[%(G)d];
            for (int h = 0; h < %(G)d; ++h) {
%(ndecl)s
                %(X)s_STATE;
                %(X)s_LOAD_COUNTS(N, h);
%(tabh)s
                %(X)s_APPLY_MX(j, mx_);
                mxs[h] = mx_;
                int held[%(C)d];
                for (int c = 0; c < %(C)d; ++c) held[c] = -1;
                %(X)s_HELD(held, h);
                if (!pass) show("H", h, j, held);
                %(X)s_STORE_COUNTS(own, h);
                %(X)s_UNDO();
                for (int c = 0; c < %(C)d; ++c) held[c] = -1;
                %(X)s_HELD(held, h);
                if (!pass) show("U", h, j, held);
                %(X)s_REDO();
                for (int c = 0; c < %(C)d; ++c) held[c] = -1;
                %(X)s_HELD(held, h);
                if (!pass) show("R", h, j, held);
            }
            if (!pass) show("O", 0, j, own);
            else {
                unsigned mx = 0u;
                for (int h = 0; h < %(G)d; ++h) mx = mxs[h] > mx ? mxs[h] : mx;
                std::printf("M %%d %%u\n", j, mx);
            }
        }
    }
    return 0;
}
"""


GROUPS = {"pair": ("CWC_PAIR", 2, "cwc_ptab"), "quad": ("CWC_QUAD", 4, "cwc_qtab")}


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("group", sorted(GROUPS))
@pytest.mark.parametrize("name", sorted(MODELS))
def test_generated_group_change_table(name, group):
    """The pair and quad layouts' per-lane counts (Sec. 2.1 update, split
    over the two or four lanes of a trajectory): for every leaf, each lane's
    slots take the oracle's net change of the cells they hold, undo and redo
    restore and re-apply it exactly, the lanes' written rows together give
    every cell's new count, and the largest of the lanes' growth maxima
    exceeds the state exactly when the leaf raises some count.  Covers both
    the per-lane table and the fallback where every lane keeps every
    cell."""
    from paper_1010_2438_amd import cwc_codegen
    model = MODELS[name]()
    src = cwc_codegen(model)
    C = int(re.search(r"#define CWC_C (\d+)", src).group(1))
    P = int(re.search(r"#define CWC_P (\d+)", src).group(1))
    X, G, tab = GROUPS[group]
    if "#define %s_SPLIT" % X not in src:
        pytest.skip("too few leaves for this layout")
    split = int(re.search(r"#define %s_SPLIT (\d+)" % X, src).group(1))
    dtw = int(re.search(r"#define CWC_DT_W (\d+)", src).group(1))
    tables, copy, tabh = [], [], ""
    if dtw:
        tables.append(re.search(r"__constant__ unsigned int cwc_dtab_g\[\d+\] = \{[^}]*\};", src).group(0))
        ty = re.search(r"__shared__ (\w[\w ]*?) cwc_dtab\[", src).group(1)
        tables.append("static %s cwc_dtab[%d];" % (ty, P))
        copy.append("    for (int i = 0; i < %d; ++i) ((unsigned *)cwc_dtab)[i] = cwc_dtab_g[i];"
                    % (P * dtw))
    m = re.search(r"__constant__ unsigned int %s_g\[(\d+)\] = \{[^}]*\};" % tab, src)
    if split and m:
        tables.append(m.group(0))
        ty = re.search(r"__shared__ (\w[\w ]*?) %s\[" % tab, src).group(1)
        tables.append("static %s %s[%d];" % (ty, tab, G * P))
        copy.append("    for (int i = 0; i < %s; ++i) ((unsigned *)%s)[i] = %s_g[i];"
                    % (m.group(1), tab, tab))
        tabh = "                const %s *%s_h = %s + h * %d;" % (ty, tab, tab, P)
    heads = ["CWC_LOAD_COUNTS(ptr)", "CWC_STORE_COUNTS(ptr)", "CWC_APPLY_MX(j, mx)",
             "CWC_UNDO()", "CWC_REDO()", X + "_STATE", X + "_LOAD_COUNTS(ptr, h)",
             X + "_STORE_COUNTS(ptr, h)", X + "_HELD(ptr, h)"]
    macros = "".join(macro(src, hd) for hd in heads)
    for hd in (X + "_APPLY_MX(", X + "_UNDO(", X + "_REDO("):
        # one-line aliases of the lane macros, or multi-line macros
        i = src.index("#define " + hd)
        eol = src.index("\n", i)
        macros += src[i:eol + 1] if not src[:eol].endswith("\\") else \
            src[i:src.index("/* end */", i)] + "/* end */\n"
    code = GROUP_APPLY_HARNESS % {
        "tables": "\n".join(tables), "macros": macros, "copy": "\n".join(copy), "C": C, "P": P,
        "base": BASE, "tabh": tabh, "X": X, "G": G,
        "ndecl": "\n".join("                int n%d = 0; (void)n%d;" % (c, c) for c in range(C))}
    d = tempfile.mkdtemp(prefix="cwc_papply_")
    try:
        with open(os.path.join(d, "t.cpp"), "w") as f:
            f.write(code)
        subprocess.check_call(["g++", "-O1", "-w", "-o", os.path.join(d, "t"),
                               os.path.join(d, "t.cpp")])
        out = subprocess.check_output([os.path.join(d, "t")], text=True)
    finally:
        shutil.rmtree(d)
    flat = oracle.FlatModel(model)
    N = [BASE + 7 * c for c in range(C)]
    rows = {}
    for line in out.splitlines():
        f = line.split()
        rows[(f[0], int(f[1]), int(f[2]))] = [int(x) for x in f[3:]]
    n_held = [0] * G
    for leaf in range(P):
        want = [0] * C
        for k in range(int(flat.leaf_ndelta[leaf])):
            cell, v = (int(x) for x in flat.leaf_delta[leaf, k])
            want[cell] += v
        new = [N[c] + want[c] for c in range(C)]
        assert rows[("O", 0, leaf)] == new, "leaf %d: written rows" % leaf
        for h in range(G):
            held = rows[("H", h, leaf)]
            kept = [c for c in range(C) if held[c] != -1]
            n_held[h] = len(kept)
            assert all(held[c] == new[c] for c in kept), ("apply", leaf, h)
            assert rows[("R", h, leaf)] == held, ("redo", leaf, h)
            assert all(rows[("U", h, leaf)][c] == N[c] for c in kept), ("undo", leaf, h)
            assert all(rows[("U", h, leaf)][c] == -1 for c in range(C) if c not in kept)
    mx = {int(f[1]): int(f[2]) for f in (l.split() for l in out.splitlines()) if f[0] == "M"}
    for leaf in range(P):
        want = [0] * C
        for k in range(int(flat.leaf_ndelta[leaf])):
            cell, v = (int(x) for x in flat.leaf_delta[leaf, k])
            want[cell] += v
        assert (mx[leaf] > BASE) == any(v > 0 for v in want), "leaf %d: growth" % leaf
    if split:
        # the split leaves some lane with fewer cells than the model has
        assert min(n_held) < C


@pytest.mark.parametrize("group", sorted(GROUPS))
def test_group_split_covered(group):
    """The models above reach both state forms of the pair and quad
    layouts."""
    from paper_1010_2438_amd import cwc_codegen
    X = GROUPS[group][0]
    seen = {int(m.group(1)) for m in (re.search(r"#define %s_SPLIT (\d+)" % X, cwc_codegen(mk()))
                                      for mk in MODELS.values()) if m}
    assert seen == {0, 1}


def test_benchmark_model_lanes_keep_few_counts():
    """The benchmark's gene-regulation model (20 cells): its pair and quad
    kernels keep per-lane counts, ten slots per lane with two lanes and six
    with four."""
    from paper_1010_2438_amd import cwc_codegen
    src = cwc_codegen(W.config(1)[0])
    for X, slots in (("CWC_PAIR", 10), ("CWC_QUAD", 6)):
        assert re.search(r"#define %s_SPLIT 1" % X, src)
        assert len(re.findall(r"int z\d+ = 0;", macro(src, X + "_STATE"))) == slots


DESCENT_HARNESS = r"""
#include <cstdio>
%(macros)s
static int lane_descend(const double *A, double x) {
%(adecl)s
    int j = 0;
    CWC_DESCEND(x, j);
    return j;
}
%(pairfn)s
%(quadfn)s
int main() {
    int T, P, K;
    if (std::scanf("%%d %%d %%d", &T, &P, &K) != 3) return 1;
    static double A[2 * 4096], L[4096], X[4096];
    for (int t = 0; t < T; ++t) {
        for (int l = 0; l < P; ++l) std::scanf("%%lf", &L[l]);
        for (int k = 0; k < K; ++k) std::scanf("%%lf", &X[k]);
        for (int l = 0; l < P; ++l) A[P + l] = L[l];
        for (int i = P - 1; i >= 1; --i) A[i] = A[2 * i] + A[2 * i + 1];
        for (int k = 0; k < K; ++k) {
            std::printf("%%d %%d %%d\n", lane_descend(A, X[k]), %(paircall)s, %(quadcall)s);
        }
    }
    return 0;
}
"""

PAIR_FN = r"""
// the engine's root decision over the two half sums, then the chosen half
static int pair_descend(const double *L, int P, double x) {
    const int B = P / 2;
    static double Q[2][2 * 4096];
    for (int h = 0; h < 2; ++h) {
        for (int i = 0; i < B; ++i) Q[h][B + i] = L[h * B + i];
        for (int i = B - 1; i >= 1; --i) Q[h][i] = Q[h][2 * i] + Q[h][2 * i + 1];
    }
    const double L0 = Q[0][1], R0 = Q[1][1];
    const bool b0 = (x >= L0) && (R0 != 0.0);
    x = b0 ? x - L0 : x;
    const double *q = Q[b0 ? 1 : 0];
%(qdecl)s
    int jl = 0;
    CWC_PAIR_DESCEND(x, jl);
    return (b0 ? B : 0) + jl;
}
"""

QUAD_FN = r"""
// the engine's two top decisions over the four quarter sums, then the quarter
static int quad_descend(const double *L, int P, double x) {
    const int B = P / 4;
    static double R[4][2 * 4096];
    for (int h = 0; h < 4; ++h) {
        for (int i = 0; i < B; ++i) R[h][B + i] = L[h * B + i];
        for (int i = B - 1; i >= 1; --i) R[h][i] = R[h][2 * i] + R[h][2 * i + 1];
    }
    const double p0 = R[0][1], p1 = R[1][1], p2 = R[2][1], p3 = R[3][1];
    const double n1 = p0 + p1, n2 = p2 + p3;
    const bool b0 = (x >= n1) && (n2 != 0.0);
    x = b0 ? x - n1 : x;
    const double L1 = b0 ? p2 : p0, R1 = b0 ? p3 : p1;
    const bool b1 = (x >= L1) && (R1 != 0.0);
    x = b1 ? x - L1 : x;
    const int qq = (b0 ? 2 : 0) + (b1 ? 1 : 0);
    const double *r = R[qq];
%(rdecl)s
    int jl = 0;
    CWC_QUAD_DESCEND(x, jl);
    return qq * B + jl;
}
"""


DESCENT_MODELS = {
    "paper_example": W.paper_example,                       # 1 leaf of 1
    "lotka_volterra": W.lotka_volterra,                     # 4 leaves
    "dimerisation": W.dimerisation,                         # C(n, 2) factors
    "receptor_binding": W.receptor_binding,
    "transport7": lambda: W.transport(n_children=7),        # padding subtrees
    "gene_regulation": lambda: W.config(1)[0],              # 32 leaves
    "one_cell": lambda: W.multi_compartment(3, n_cells_=1),  # 64 leaves
}


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("name", sorted(DESCENT_MODELS))
def test_generated_descent(name):
    """The generated selection descents (one lane; two and four lanes with
    the engine's top decisions) pick the oracle's leaf for random trees with
    zero leaves, and for integer trees at every integer x (exact sums, so
    every tie x == L occurs and must go right)."""
    import numpy as np
    from paper_1010_2438_amd import cwc_codegen
    model = DESCENT_MODELS[name]()
    src = cwc_codegen(model)
    P = int(re.search(r"#define CWC_P (\d+)", src).group(1))
    flat = oracle.FlatModel(model)
    live = flat.leaf_rule >= 0
    pair = "#define CWC_PAIR_DESCEND" in src
    quad = "#define CWC_QUAD_DESCEND" in src
    macros = macro(src, "CWC_DESCEND(x, j)")
    if pair:
        macros += macro(src, "CWC_PAIR_DESCEND(x, j)")
    if quad:
        macros += macro(src, "CWC_QUAD_DESCEND(x, j)")
    B = P // 2
    code = DESCENT_HARNESS % {
        "macros": macros,
        "adecl": "\n".join("    const double a%d = A[%d]; (void)a%d;" % (i, i, i)
                           for i in range(1, 2 * P)),
        "pairfn": (PAIR_FN % {"qdecl": "\n".join("    const double q%d = q[%d]; (void)q%d;"
                                                  % (i, i, i) for i in range(1, 2 * B))})
        if pair else "",
        "paircall": "pair_descend(L, P, X[k])" if pair else "-1",
        "quadfn": (QUAD_FN % {"rdecl": "\n".join("    const double r%d = r[%d]; (void)r%d;"
                                                 % (i, i, i) for i in range(1, 2 * (P // 4)))})
        if quad else "",
        "quadcall": "quad_descend(L, P, X[k])" if quad else "-1"}
    rng = np.random.default_rng(11)
    trials = []
    for t in range(40):
        if t % 2:
            lv = rng.integers(0, 4, P).astype(np.float64)         # exact sums, ties
        else:
            lv = rng.uniform(0.0, 3.0, P) * (rng.random(P) < 0.8)  # some zeros
        lv[~live] = 0.0
        a0 = oracle.select(lv, 0.0)[1]
        if a0 == 0.0:
            continue
        if t % 2:
            xs = np.arange(0.0, a0)                                 # every integer below a0
        else:
            xs = np.concatenate([rng.uniform(0.0, a0, 60), [0.0, np.nextafter(a0, 0.0)]])
        trials.append((lv, xs))
    d = tempfile.mkdtemp(prefix="cwc_desc_")
    try:
        with open(os.path.join(d, "t.cpp"), "w") as f:
            f.write(code)
        subprocess.check_call(["g++", "-O1", "-w", "-o", os.path.join(d, "t"),
                               os.path.join(d, "t.cpp")])
        for lv, xs in trials:
            inp = "1 %d %d\n%s\n%s\n" % (P, len(xs), " ".join(repr(float(v)) for v in lv),
                                        " ".join(repr(float(x)) for x in xs))
            out = subprocess.check_output([os.path.join(d, "t")], input=inp, text=True)
            for x, line in zip(xs, out.splitlines()):
                jl, jp, jq = (int(v) for v in line.split())
                want = oracle.select(lv, float(x))[0]
                assert jl == want, (x, jl, want)
                if pair:
                    assert jp == want, (x, jp, want)
                if quad:
                    assert jq == want, (x, jq, want)
    finally:
        shutil.rmtree(d)


TREE_HARNESS = r"""
#include <cstdio>
#include <cstring>
static unsigned long long bits(double v) { unsigned long long b; std::memcpy(&b, &v, 8); return b; }
%(macros)s
int main() {
    int T;
    if (std::scanf("%%d", &T) != 1) return 1;
    for (int t = 0; t < T; ++t) {
        int N[%(C)d];
        double KR[%(NR)d];
        for (int c = 0; c < %(C)d; ++c) std::scanf("%%d", &N[c]);
        for (int r = 0; r < %(NR)d; ++r) std::scanf("%%lf", &KR[r]);
%(ndecl)s
%(kdecl)s
%(adecl)s
        CWC_TREE;
%(aprint)s
        std::printf("\n");
%(pair)s
%(quad)s
    }
    return 0;
}
"""

QUAD_TREE_PART = r"""
        for (int h = 0; h < 4; ++h) {
            CWC_QUAD_STATE;
            CWC_QUAD_LOAD_COUNTS(N, h);
            CWC_QUAD_DECL;
            CWC_QUAD_LOAD_K(KR, h);
            CWC_QUAD_TREE(h);
%(rprint)s
            std::printf("\n");
        }
"""

PAIR_TREE_PART = r"""
        for (int h = 0; h < 2; ++h) {
            CWC_PAIR_STATE;
            CWC_PAIR_LOAD_COUNTS(N, h);
            CWC_PAIR_DECL;
            CWC_PAIR_LOAD_K(KR, h);
            CWC_PAIR_TREE(h);
%(qprint)s
            std::printf("\n");
        }
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("name", sorted(DESCENT_MODELS))
def test_generated_trees(name):
    """The generated propensity tree (one lane) has, bit for bit, leaves
    k_r x (double)h with h the exact product of binomials C(n, m) of the
    slot's reactant counts (Sec. 2.2) and nodes left + right; the pair
    layout's half trees hold the same leaves and their roots are the tree's
    two level-1 nodes; the quad layout's quarter trees likewise, their roots
    the four level-2 nodes."""
    import math
    import numpy as np
    from paper_1010_2438_amd import cwc_codegen
    model = DESCENT_MODELS[name]()
    src = cwc_codegen(model)
    C = int(re.search(r"#define CWC_C (\d+)", src).group(1))
    P = int(re.search(r"#define CWC_P (\d+)", src).group(1))
    NR = int(re.search(r"#define CWC_NR (\d+)", src).group(1))
    pair = "#define CWC_PAIR_TREE" in src
    B = P // 2
    macros = macro(src, "CWC_TREE")
    qnames = set()
    if pair:
        for head in ("CWC_LOAD_COUNTS(ptr)", "CWC_PAIR_STATE", "CWC_PAIR_LOAD_COUNTS(ptr, h)",
                     "CWC_PAIR_DECL", "CWC_PAIR_LOAD_K(ptr, h)", "CWC_PAIR_TREE(h)"):
            macros += macro(src, head)
        # the half tree declares only the nodes that can be non-zero
        qnames = set(re.findall(r"double (q\d+) = ", macro(src, "CWC_PAIR_DECL")))
    quad = "#define CWC_QUAD_TREE" in src
    rnames = set()
    Q = P // 4
    if quad:
        if not pair:
            macros += macro(src, "CWC_LOAD_COUNTS(ptr)")
        for head in ("CWC_QUAD_STATE", "CWC_QUAD_LOAD_COUNTS(ptr, h)", "CWC_QUAD_DECL",
                     "CWC_QUAD_LOAD_K(ptr, h)", "CWC_QUAD_TREE(h)"):
            macros += macro(src, head)
        rnames = set(re.findall(r"double (r\d+) = ", macro(src, "CWC_QUAD_DECL")))
    code = TREE_HARNESS % {
        "macros": macros, "C": C, "NR": NR,
        "ndecl": "\n".join("        int n%d = N[%d]; (void)n%d;" % (c, c, c) for c in range(C)),
        "kdecl": "\n".join("        double k%d = KR[%d]; (void)k%d;" % (r, r, r) for r in range(NR)),
        "adecl": "\n".join("        double a%d = 0.0; (void)a%d;" % (i, i) for i in range(1, 2 * P)),
        "aprint": "\n".join('        std::printf("%%llu ", bits(a%d));' % i for i in range(1, 2 * P)),
        "pair": (PAIR_TREE_PART % {"qprint": "\n".join(
            '            std::printf("%%llu ", bits(%s));' % ("q%d" % i if "q%d" % i in qnames else "0.0")
            for i in range(1, 2 * B))})
        if pair else "",
        "quad": (QUAD_TREE_PART % {"rprint": "\n".join(
            '            std::printf("%%llu ", bits(%s));' % ("r%d" % i if "r%d" % i in rnames else "0.0")
            for i in range(1, 2 * Q))})
        if quad else ""}
    flat = oracle.FlatModel(model)
    rng = np.random.default_rng(5)
    trials = []
    for t in range(30):
        hi = [3, 50, 5000, 1_000_000][t % 4]
        n = rng.integers(0, hi + 1, C)
        n[rng.random(C) < 0.2] = 0
        n[rng.random(C) < 0.1] = 1
        k = rng.uniform(0.01, 10.0, NR)
        trials.append((n, k))
    inp = "%d\n" % len(trials) + "\n".join(
        " ".join(str(int(v)) for v in n) + " " + " ".join(repr(float(v)) for v in k)
        for n, k in trials)
    d = tempfile.mkdtemp(prefix="cwc_tree_")
    try:
        with open(os.path.join(d, "t.cpp"), "w") as f:
            f.write(code)
        subprocess.check_call(["g++", "-O1", "-w", "-ffp-contract=off", "-o",
                               os.path.join(d, "t"), os.path.join(d, "t.cpp")])
        out = subprocess.check_output([os.path.join(d, "t")], input=inp, text=True).splitlines()
    finally:
        shutil.rmtree(d)
    as_bits = lambda v: int(np.float64(v).view(np.uint64))
    per = 1 + (2 if pair else 0) + (4 if quad else 0)
    for t, (n, k) in enumerate(trials):
        got = [int(x) for x in out[per * t].split()]
        node = [0.0] * (2 * P)
        for leaf in range(P):
            if flat.leaf_rule[leaf] < 0:
                continue
            h = 1
            for cell, m in flat.leaf_react[leaf]:
                if m > 0:
                    h *= math.comb(int(n[cell]), int(m))
            node[P + leaf] = float(np.float64(k[flat.leaf_rule[leaf]]) * np.float64(float(h)))
        for i in range(P - 1, 0, -1):
            node[i] = float(np.float64(node[2 * i]) + np.float64(node[2 * i + 1]))
        assert got == [as_bits(node[i]) for i in range(1, 2 * P)], "trial %d" % t
        if pair:
            for h in range(2):
                q = [int(x) for x in out[per * t + 1 + h].split()]
                assert q[0] == as_bits(node[2 + h]), ("half root", t, h)
                assert q[B - 1:] == [as_bits(node[P + h * B + i]) for i in range(B)], ("leaves", t, h)
        if quad:
            base = per * t + 1 + (2 if pair else 0)
            for h in range(4):
                r = [int(x) for x in out[base + h].split()]
                assert r[0] == as_bits(node[4 + h]), ("quarter root", t, h)
                assert r[Q - 1:] == [as_bits(node[P + h * Q + i]) for i in range(Q)], ("quarter", t, h)
