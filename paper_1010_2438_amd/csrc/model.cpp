// Model compilation (host).  A CWC model with a fixed compartment tree
// (paper Sec. 2.1) is flattened once into slots: the paper's Match step
// (Fig. "simd") walks the term for every rule and records one weighted
// match per context; with a static tree the contexts of each rule are known
// up front, so the walk is done here and the device only re-evaluates the
// combination counts (Sec. 2.2) of a fixed slot list.
//
// Contexts: a rule of label l that rewrites only a content has one context
// per compartment of label l; a rule whose pattern also names a child of
// label l' has one context per compartment of label l' whose parent has
// label l (the sum over those contexts is the paper's count_compartments).
// Slot order is context-major (compartments in preorder, rules ascending
// inside a compartment); each compartment's block is padded to the next
// power of two of the largest block, the compartment count to a power of
// two, giving the leaf array of the propensity tree.
#include "model.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <functional>
#include <sstream>

namespace cwc {

static int next_pow2(int n)
{
    int p = 1;
    while (p < n) p *= 2;
    return p;
}

static cwc_status fail(std::string *err, cwc_status code, const std::string &msg)
{
    *err = msg;
    return code;
}

cwc_status flatten(const cwc_model_desc *d, Flat *f, std::string *err)
{
    if (!d) return fail(err, CWC_E_INVALID, "null model descriptor");
    if (d->n_species < 1 || d->n_types < 1 || d->n_comp < 1 || d->n_rules < 0)
        return fail(err, CWC_E_INVALID, "n_species, n_types, n_comp must be >= 1, n_rules >= 0");
    if (!d->type_has_wrap || !d->comp_type || !d->comp_parent || !d->init_counts ||
        (d->n_rules > 0 && !d->rules))
        return fail(err, CWC_E_INVALID, "null array in model descriptor");
    if (d->n_species > 4096 || d->n_comp > 65536 || d->n_rules > 65536)
        return fail(err, CWC_E_UNSUPPORTED, "model too large");
    f->n_species = d->n_species;
    f->n_types = d->n_types;
    f->n_comp = d->n_comp;
    f->n_rules = d->n_rules;
    const int ns = d->n_species;
    f->has_wrap.assign(d->type_has_wrap, d->type_has_wrap + d->n_types);
    for (int w : f->has_wrap)
        if (w != 0 && w != 1) return fail(err, CWC_E_INVALID, "type_has_wrap must be 0 or 1");
    f->comp_type.assign(d->comp_type, d->comp_type + d->n_comp);
    f->comp_parent.assign(d->comp_parent, d->comp_parent + d->n_comp);
    for (int i = 0; i < d->n_comp; ++i) {
        if (f->comp_type[i] < 0 || f->comp_type[i] >= d->n_types)
            return fail(err, CWC_E_INVALID, "compartment type out of range");
        if (i == 0 ? f->comp_parent[0] != -1
                   : (f->comp_parent[i] < 0 || f->comp_parent[i] >= i))
            return fail(err, CWC_E_INVALID,
                        "compartments must be in preorder: comp 0 is the top level "
                        "(parent -1), every other parent has a smaller index");
    }
    int c = 0;
    f->content_base.resize(d->n_comp);
    f->wrap_base.resize(d->n_comp);
    for (int i = 0; i < d->n_comp; ++i) {
        f->content_base[i] = c;
        c += ns;
        if (f->has_wrap[f->comp_type[i]]) {
            f->wrap_base[i] = c;
            c += ns;
        } else {
            f->wrap_base[i] = -1;
        }
    }
    f->n_cells = c;
    f->init.assign(d->init_counts, d->init_counts + c);
    for (int v : f->init)
        if (v < 0) return fail(err, CWC_E_INVALID, "negative initial count");

    // rules
    f->k.resize(d->n_rules);
    struct Pat {
        std::map<std::pair<int, int>, int> lhs, rhs;   // (region, species) -> mult
    };
    std::vector<Pat> pats(d->n_rules);
    for (int r = 0; r < d->n_rules; ++r) {
        const cwc_rule &R = d->rules[r];
        char where[64];
        std::snprintf(where, sizeof where, "rule %d: ", r);
        if (!(std::isfinite(R.k) && R.k > 0.0 && R.k <= 1e250))
            return fail(err, CWC_E_INVALID, std::string(where) + "kinetic constant must be finite, > 0, <= 1e250");
        if (R.parent_type < 0 || R.parent_type >= d->n_types)
            return fail(err, CWC_E_INVALID, std::string(where) + "parent_type out of range");
        if (R.child_type < -1 || R.child_type >= d->n_types)
            return fail(err, CWC_E_INVALID, std::string(where) + "child_type out of range");
        if (R.n_lhs < 0 || R.n_rhs < 0 || (R.n_lhs > 0 && !R.lhs) || (R.n_rhs > 0 && !R.rhs))
            return fail(err, CWC_E_INVALID, std::string(where) + "bad term arrays");
        f->k[r] = R.k;
        for (int side = 0; side < 2; ++side) {
            const cwc_term *T = side ? R.rhs : R.lhs;
            int nt = side ? R.n_rhs : R.n_lhs;
            auto &dst = side ? pats[r].rhs : pats[r].lhs;
            for (int t = 0; t < nt; ++t) {
                const cwc_term &x = T[t];
                if (x.species < 0 || x.species >= ns)
                    return fail(err, CWC_E_INVALID, std::string(where) + "species out of range");
                if (x.mult < 1)
                    return fail(err, CWC_E_INVALID, std::string(where) + "multiplicity must be >= 1");
                if (x.region < CWC_REGION_PARENT || x.region > CWC_REGION_CHILD)
                    return fail(err, CWC_E_INVALID, std::string(where) + "region out of range");
                if (x.region != CWC_REGION_PARENT && R.child_type < 0)
                    return fail(err, CWC_E_INVALID, std::string(where) +
                                "wrap/child region in a rule without a child compartment");
                if (x.region == CWC_REGION_WRAP && !f->has_wrap[R.child_type])
                    return fail(err, CWC_E_INVALID, std::string(where) + "child label has no wrap");
                dst[{x.region, x.species}] += x.mult;
            }
        }
        int order = 0, nterms = 0;
        for (auto &kv : pats[r].lhs) { order += kv.second; ++nterms; }
        if (order > 2)
            return fail(err, CWC_E_UNSUPPORTED, std::string(where) +
                        "reactant order > 2 (only mass action up to bimolecular is supported)");
        (void)nterms;
    }

    // slots, context-major
    std::vector<std::vector<int>> blocks(d->n_comp);
    size_t max_blk = 0;
    for (int i = 0; i < d->n_comp; ++i) {
        const int par = f->comp_parent[i];
        for (int r = 0; r < d->n_rules; ++r) {
            const cwc_rule &R = d->rules[r];
            bool applies = R.child_type < 0
                               ? R.parent_type == f->comp_type[i]
                               : (R.child_type == f->comp_type[i] && par >= 0 &&
                                  f->comp_type[par] == R.parent_type);
            if (applies) blocks[i].push_back(r);
        }
        max_blk = std::max(max_blk, blocks[i].size());
    }
    f->p_local = next_pow2(std::max<int>(1, (int)max_blk));
    f->p_comp = next_pow2(d->n_comp);
    if ((long long)f->p_local * f->p_comp > (1 << 22))
        return fail(err, CWC_E_UNSUPPORTED, "too many slots");
    f->n_leaves = f->p_local * f->p_comp;
    f->leaf_slot.assign(f->n_leaves, -1);
    for (int i = 0; i < d->n_comp; ++i) {
        for (size_t pos = 0; pos < blocks[i].size(); ++pos) {
            const int r = blocks[i][pos];
            const cwc_rule &R = d->rules[r];
            Slot s;
            s.rule = r;
            s.ctx = i;
            s.leaf = i * f->p_local + (int)pos;
            auto cell_of = [&](int region, int species) {
                if (R.child_type < 0) return f->content_base[i] + species;
                if (region == CWC_REGION_PARENT) return f->content_base[f->comp_parent[i]] + species;
                if (region == CWC_REGION_WRAP) return f->wrap_base[i] + species;
                return f->content_base[i] + species;
            };
            std::map<int, int> net;
            for (auto &kv : pats[r].lhs) {
                const int cell = cell_of(kv.first.first, kv.first.second);
                s.react_cell[s.n_react] = cell;
                s.react_mult[s.n_react] = kv.second;
                ++s.n_react;
                net[cell] -= kv.second;
            }
            for (auto &kv : pats[r].rhs) net[cell_of(kv.first.first, kv.first.second)] += kv.second;
            for (auto &kv : net)
                if (kv.second != 0) {
                    if (kv.second > 1000000 || kv.second < -1000000)
                        return fail(err, CWC_E_UNSUPPORTED, "net change too large");
                    s.delta.push_back(kv);
                }
            f->leaf_slot[s.leaf] = (int)f->slots.size();
            f->slots.push_back(s);
        }
    }
    f->layout = 0;
    return CWC_OK;
}

// ------------------------------------------------------ algorithmic work
// VALU issue slots (wave64 instruction = one slot per lane; quarter-rate
// instructions -- 32x32->64 multiplies, the f64 reciprocal inside a
// division -- count 4) that one applied event of the direct method needs,
// independent of how the kernels are organised:
//   draw:  Philox4x32-10, 10 rounds x (2 wide multiplies [4 each] and 4
//          xor) = 120 (the key schedule's two adds per round act on the run
//          seed, which is the same in every lane, so they are scalar work
//          and not counted); two 53-bit uniforms 14; ssa_log 45 (split,
//          fold, atanh series of 11 terms, one division); tau = -l/a0 and
//          t + tau 15; one sample-time compare 1                     = 195
//   select: x = u*a0, then 5 per tree level (compare, zero test, and,
//          subtract, select)                                  = 1 + 5 log2 P
//   update: 2 per changed cell (add, cap compare)
//   match:  only the slots whose reactants changed are re-evaluated (a
//          count conversion and a multiply per factor, an extra subtract
//          and halving for C(n,2)), plus one add per distinct tree node on
//          their paths to the root.
// The update/match terms are averaged uniformly over the model's slots.
double algorithmic_slots_per_event(const Flat &f)
{
    const int P = f.n_leaves;
    int D = 0;
    while ((1 << D) < P) ++D;
    double fixed = 195.0 + 1.0 + 5.0 * D;
    if (f.slots.empty()) return fixed;
    auto cost = [](const Slot &s) {
        if (s.n_react == 0) return 0.0;
        if (s.n_react == 2) return 4.0;
        return s.react_mult[0] == 2 ? 6.0 : 2.0;
    };
    double acc = 0.0;
    for (const Slot &j : f.slots) {
        double w = 2.0 * (double)j.delta.size();
        std::vector<char> changed(f.n_cells, 0);
        for (auto &dv : j.delta) changed[dv.first] = 1;
        std::vector<char> node(2 * P, 0);
        for (const Slot &s : f.slots) {
            bool dep = false;
            for (int t = 0; t < s.n_react; ++t) dep |= changed[s.react_cell[t]] != 0;
            if (!dep) continue;
            w += cost(s);
            for (int i = (P + s.leaf) / 2; i >= 1; i /= 2) node[i] = 1;
        }
        for (int i = 1; i < P; ++i) w += node[i];
        acc += w;
    }
    return fixed + acc / (double)f.slots.size();
}

// ------------------------------------------------------------------ codegen

static std::string dlit(double v)
{
    char b[64];
    std::snprintf(b, sizeof b, "%a", v);
    return b;
}

// Emits one macro per line group; every statement of a macro ends with a
// line continuation so the model section stays readable when dumped.
namespace {
struct MacroWriter {
    std::ostringstream &o;
    explicit MacroWriter(std::ostringstream &os) : o(os) {}
    void begin(const std::string &head) { o << "#define " << head << " \\\n"; }
    void line(const std::string &l) { o << "    " << l << " \\\n"; }
    void end() { o << "    /* end */\n"; }
};
}  // namespace

// Narrows the level-(d+1) node values `vals` (heap order, d = bits.size())
// to the pair (L, R) under the current node, given the decisions taken so
// far (bits[q] of depth q; "" = constant false), with two-way selects that
// never use a lane-varying index.  The decisions are applied most
// significant first (each select can start as soon as its decision is
// known) unless applying them least significant first needs fewer selects
// (padding subtrees then pair up with padding and cost nothing).  Emits the
// selects as `const double <pfx><n>_ = bit ? A : B;` lines when `w` is
// given; returns (L, R) and the number of selects.
struct Narrowed {
    std::string L, R;
    int selects;
};
static Narrowed narrow_pair(std::vector<std::string> vals, const std::vector<std::string> &bits,
                            const std::string &pfx, int &tmp, MacroWriter *w)
{
    auto run = [&](bool lsb, MacroWriter *out, int &t) {
        std::vector<std::string> v = vals;
        int n = 0;
        const int d = (int)bits.size();
        for (int k = 0; k < d; ++k) {
            const int q = lsb ? d - 1 - k : k;
            const size_t half = v.size() / 2;
            std::vector<std::string> nv(half);
            for (size_t r = 0; r < half; ++r) {
                size_t i0, i1;
                if (lsb) {   // decision q sits at bit 1 of the index
                    i0 = ((r >> 1) << 2) | (r & 1);
                    i1 = i0 | 2;
                } else {     // decision q is the most significant bit
                    i0 = r;
                    i1 = r + half;
                }
                const std::string &A = v[i1], &B = v[i0];
                if (bits[q].empty() || A == B) {
                    nv[r] = B;
                } else {
                    ++n;
                    const std::string tv = pfx + std::to_string(t++) + "_";
                    if (out) out->line("const double " + tv + " = " + bits[q] + " ? " + A + " : " + B + ";");
                    nv[r] = tv;
                }
            }
            v = nv;
        }
        return Narrowed{v[0], v[1], n};
    };
    int scratch = 0;
    const bool lsb = run(true, nullptr, scratch).selects < run(false, nullptr, scratch).selects;
    return run(lsb, w, tmp);
}

std::string codegen_lane(const Flat &f)
{
    std::ostringstream o;
    MacroWriter w(o);
    const int C = f.n_cells, P = f.n_leaves, NR = std::max(1, f.n_rules);
    int D = 0;
    while ((1 << D) < P) ++D;
    o << "// ---- generated model section (lane-per-replica layout)\n";
    o << "#define CWC_C " << C << "\n#define CWC_P " << P << "\n#define CWC_NR " << NR << "\n";

    // zero (padding-only) subtrees in heap order; a<i> holds heap node i
    std::vector<char> zero(2 * P, 1);
    for (int l = 0; l < P; ++l) zero[P + l] = f.leaf_slot[l] < 0;
    for (int i = P - 1; i >= 1; --i) zero[i] = zero[2 * i] && zero[2 * i + 1];
    auto val = [&](int i) -> std::string {
        return zero[i] ? std::string("0.0") : "a" + std::to_string(i);
    };
    auto I = [](int v) { return std::to_string(v); };

    w.begin("CWC_DECL_K");
    for (int r = 0; r < NR; ++r) w.line("double k" + I(r) + " = 0.0;");
    w.end();
    w.begin("CWC_LOAD_K(ptr)");
    for (int r = 0; r < f.n_rules; ++r) w.line("k" + I(r) + " = (ptr)[" + I(r) + "];");
    w.end();
    w.begin("CWC_DECL_STATE");
    for (int c = 0; c < C; ++c) w.line("int n" + I(c) + " = 0;");
    for (int i = 1; i < 2 * P; ++i)
        if (!zero[i]) w.line("double a" + I(i) + " = 0.0;");
    w.end();
    w.begin("CWC_LOAD_COUNTS(ptr)");
    for (int c = 0; c < C; ++c) w.line("n" + I(c) + " = (ptr)[" + I(c) + "];");
    w.end();
    w.begin("CWC_STORE_COUNTS(ptr)");
    for (int c = 0; c < C; ++c) w.line("(ptr)[" + I(c) + "] = n" + I(c) + ";");
    w.end();
    o << "#define CWC_ROOT " << val(1) << "\n";

    // --- leaves k * prod C(n, m) and internal sums.  h = prod C(n, m)
    // rounded once to binary64: the product of two exact integer-valued
    // doubles is the correctly rounded integer product; C(n,2) is
    // RN(n (n-1)) / 2 exactly.
    std::vector<char> need_c(C, 0), need_d(C, 0);
    for (auto &s : f.slots)
        for (int t = 0; t < s.n_react; ++t) {
            need_c[s.react_cell[t]] = 1;
            if (s.react_mult[t] == 2) need_d[s.react_cell[t]] = 1;
        }
    w.begin("CWC_TREE");
    w.line("{");
    for (int c = 0; c < C; ++c) {
        if (need_c[c]) w.line("const double c" + I(c) + "_ = (double)n" + I(c) + ";");
        if (need_d[c])
            w.line("const double m" + I(c) + "_ = (double)(n" + I(c) + " > 0 ? n" + I(c) + " - 1 : 0);");
    }
    for (auto &s : f.slots) {
        std::string h;
        if (s.n_react == 1 && s.react_mult[0] == 1) {
            h = "c" + I(s.react_cell[0]) + "_";
        } else if (s.n_react == 1 && s.react_mult[0] == 2) {
            const int c = s.react_cell[0];
            h = "((c" + I(c) + "_ * m" + I(c) + "_) * 0.5)";
        } else if (s.n_react == 2) {
            h = "(c" + I(s.react_cell[0]) + "_ * c" + I(s.react_cell[1]) + "_)";
        }
        w.line("a" + I(P + s.leaf) + " = k" + I(s.rule) + (h.empty() ? "" : " * " + h) + ";");
    }
    for (int i = P - 1; i >= 1; --i) {
        if (zero[i]) continue;
        if (!zero[2 * i] && !zero[2 * i + 1])
            w.line("a" + I(i) + " = a" + I(2 * i) + " + a" + I(2 * i + 1) + ";");
        else if (!zero[2 * i])
            w.line("a" + I(i) + " = a" + I(2 * i) + ";");
        else
            w.line("a" + I(i) + " = a" + I(2 * i + 1) + ";");
    }
    w.line("}");
    w.end();

    // --- selection descent.  At depth d the pair (L, R) under the current
    // node is picked from the level-(d+1) nodes with the decisions already
    // taken (narrow_pair), so no value is ever picked with a lane-varying
    // index and the temporaries of one level die before the next starts.
    w.begin("CWC_DESCEND(x, j)");
    w.line("{");
    w.line("int jj_ = 0;");
    std::vector<std::string> bits;   // decision of each depth ("" = constant false)
    int tmp = 0;
    for (int d = 0; d < D; ++d) {
        std::vector<std::string> vals;
        for (int m = 0; m < (2 << d); ++m) vals.push_back(val((2 << d) + m));
        const Narrowed nw = narrow_pair(vals, bits, "t", tmp, &w);
        const std::string L = nw.L, R = nw.R;
        if (R == "0.0") {
            w.line("jj_ = jj_ << 1;");
            bits.push_back("");
            continue;
        }
        const std::string b = "b" + I(d) + "_";
        if (L == "0.0")
            w.line("const bool " + b + " = (" + R + " != 0.0);");
        else
            w.line("const bool " + b + " = ((x) >= " + L + ") && (" + R + " != 0.0);");
        if (L != "0.0") w.line("(x) = " + b + " ? (x) - " + L + " : (x);");
        w.line("jj_ = (jj_ << 1) | (" + b + " ? 1 : 0);");
        bits.push_back(b);
    }
    w.line("(j) = jj_;");
    w.line("}");
    w.end();

    // --- net change of the chosen leaf.  Each cell's change over the
    // leaves is a small integer field (signed when the cell can decrease);
    // the fields of the cells are packed into 32-bit words per leaf (first
    // fit, a field never straddles a word), and the table of these words,
    // one entry per leaf, is copied to LDS when the block starts: an event
    // reads its leaf's entry once (one LDS load) and takes each cell's
    // change from it.  In the byte layout the fields are whole bytes or
    // half-words, so the extension of the field folds into the add of the
    // count (a sub-dword operand); in the dense layout they have their own
    // widths in at most two words and are taken with bit-field extracts.
    // Cells whose fields do not fit take the change from per-digit leaf
    // masks instead: d = sum_b ((M+_b >> j) & 1) << b - (...).  Nothing is
    // written if any count would exceed the cap.
    std::vector<std::vector<std::pair<int, int>>> per_cell(C);   // (leaf, delta)
    for (auto &s : f.slots)
        for (auto &dv : s.delta) per_cell[dv.first].push_back({s.leaf, dv.second});
    struct Field { int word = -1, off = 0, width = 0; bool sgn = false; };
    std::vector<Field> field(C);
    for (int c = 0; c < C; ++c) {
        if (per_cell[c].empty()) continue;
        int lo = 0, hi = 0;
        for (auto &ld : per_cell[c]) { lo = std::min(lo, ld.second); hi = std::max(hi, ld.second); }
        Field &fd = field[c];
        fd.sgn = lo < 0;
        fd.width = 1;
        if (fd.sgn) {
            while (!(-(1ll << (fd.width - 1)) <= lo && hi <= (1ll << (fd.width - 1)) - 1)) ++fd.width;
        } else {
            while (hi > (1ll << fd.width) - 1) ++fd.width;
        }
    }
    // Byte layout: every field widened to 8 or 16 bits at an offset that is
    // a multiple of its width, in up to four words, when the whole table
    // fits the static LDS reserved for it; a cell's change is then one add
    // of a sign- or zero-extended byte or half-word of the entry.  Otherwise
    // the dense layout: fields of their own width, at most two words.
    int n_words = 0;
    bool bytes = false;   // the byte layout was taken
    {
        std::vector<Field> bf = field;
        int used[4] = {0, 0, 0, 0}, nw = 0;
        bool ok = true;
        for (int c = 0; c < C && ok; ++c) {
            if (per_cell[c].empty()) continue;
            Field &fd = bf[c];
            if (fd.width > 16) { ok = false; break; }
            fd.width = fd.width <= 8 ? 8 : 16;
            fd.word = -1;
            for (int wd = 0; wd < 4 && fd.word < 0; ++wd) {
                const int off = (used[wd] + fd.width - 1) / fd.width * fd.width;
                if (off + fd.width <= 32) {
                    fd.word = wd;
                    fd.off = off;
                    used[wd] = off + fd.width;
                    nw = std::max(nw, wd + 1);
                }
            }
            if (fd.word < 0) ok = false;
        }
        if (nw == 3) nw = 4;   // a three-word entry is read as one 16-byte load
        if (ok && (size_t)P * (size_t)nw * 4u <= kLaneStaticLdsBytes) {
            field = bf;
            n_words = nw;
            bytes = nw > 0;
        } else {
            int used2[2] = {0, 0};
            for (int c = 0; c < C; ++c) {
                if (per_cell[c].empty()) continue;
                Field &fd = field[c];
                for (int wd = 0; wd < 2; ++wd)
                    if (used2[wd] + fd.width <= 32) {
                        fd.word = wd;
                        fd.off = used2[wd];
                        used2[wd] += fd.width;
                        n_words = std::max(n_words, wd + 1);
                        break;
                    }
            }
        }
    }
    o << "#define CWC_DT_W " << n_words << "\n";
    if (n_words > 0) {
        // table entry l: words 0..n_words-1 of leaf l
        o << "__constant__ unsigned int cwc_dtab_g[" << P * n_words << "] = {";
        for (int l = 0; l < P; ++l) {
            unsigned long long wv[4] = {0, 0, 0, 0};
            for (int c = 0; c < C; ++c) {
                if (field[c].word < 0) continue;
                long long d = 0;
                for (auto &ld : per_cell[c])
                    if (ld.first == l) d += ld.second;
                const unsigned long long bits =
                    (unsigned long long)d & ((1ull << field[c].width) - 1ull);
                wv[field[c].word] |= bits << field[c].off;
            }
            for (int k = 0; k < n_words; ++k) {
                char b[32];
                std::snprintf(b, sizeof b, "%s0x%llxu", (l || k) ? ", " : "", wv[k]);
                o << b;
            }
        }
        o << "};\n";
        // the block's copy in LDS (every thread of the block passes here
        // before any event)
        const char *ty = n_words == 1 ? "unsigned int" : n_words == 2 ? "uint2" : "uint4";
        w.begin("CWC_DT_SETUP");
        w.line(std::string("__shared__ ") + ty + " cwc_dtab[" + I(P) + "];");
        w.line("for (int i_ = (int)threadIdx.x; i_ < " + I(P * n_words) +
               "; i_ += (int)blockDim.x) ((unsigned int *)cwc_dtab)[i_] = cwc_dtab_g[i_];");
        w.line("__syncthreads();");
        w.end();
    } else {
        o << "#define CWC_DT_SETUP\n";
    }
    const bool wide = P > 32;
    auto mask_lit = [&](unsigned long long m) {
        char b[40];
        std::snprintf(b, sizeof b, wide ? "0x%llxull" : "0x%llxu", m);
        return std::string(b);
    };
    // CWC_APPLY adds the change d<c>_ of leaf j to the counts in place and
    // declares the changes and the overflow flag in the enclosing scope;
    // CWC_UNDO takes the change back (the slow path of an event that is
    // not, or not yet, applied) and CWC_REDO applies it again.  Counts are
    // added modulo 2^32, so an undo restores them exactly.  A rule only
    // fires with enough reactants, so no count goes below zero and the cap
    // test over the cells that can grow is one compare of their maximum.
    // CWC_APPLY_MX leaves the largest count that can grow in `mx` (the
    // pair layout takes the cap test across its two lanes).
    w.begin("CWC_APPLY_MX(j, mx)");
    w.line("const unsigned js_ = (unsigned)(j);");
    if (n_words == 1) {
        w.line("const unsigned dw0_ = cwc_dtab[js_];");
    } else if (n_words == 2) {
        w.line("const uint2 dq_ = cwc_dtab[js_];");
        w.line("const unsigned dw0_ = dq_.x, dw1_ = dq_.y;");
    } else if (n_words == 4) {
        w.line("const uint4 dq_ = cwc_dtab[js_];");
        w.line("const unsigned dw0_ = dq_.x, dw1_ = dq_.y, dw2_ = dq_.z, dw3_ = dq_.w;");
    }
    w.line("unsigned mx = 0u;");
    for (int c = 0; c < C; ++c) {
        if (per_cell[c].empty()) continue;
        bool pos = false;
        for (auto &ld : per_cell[c]) pos = pos || ld.second > 0;
        std::string e;
        const Field &fd = field[c];
        if (fd.word >= 0) {
            const std::string wv = "dw" + I(fd.word) + "_";
            const std::string sh = fd.off ? "(" + wv + " >> " + I(fd.off) + ")" : wv;
            if (bytes && fd.sgn)
                e = std::string("(unsigned)(int)(") + (fd.width == 8 ? "signed char" : "short") +
                    ")" + sh;
            else if (bytes)
                e = std::string("(unsigned)(") + (fd.width == 8 ? "unsigned char" : "unsigned short") +
                    ")" + sh;
            else if (fd.sgn)
                e = "(unsigned)__builtin_amdgcn_sbfe((int)" + wv + ", " + I(fd.off) + "u, " +
                    I(fd.width) + "u)";
            else
                e = "__builtin_amdgcn_ubfe(" + wv + ", " + I(fd.off) + "u, " + I(fd.width) + "u)";
        } else {
            e = "0u";
            for (int sign = 1; sign >= -1; sign -= 2) {
                for (int b = 0; b < 21; ++b) {
                    unsigned long long m = 0;
                    for (auto &ld : per_cell[c]) {
                        int v = ld.second * sign;
                        if (v > 0 && ((v >> b) & 1)) m |= 1ull << ld.first;
                    }
                    if (!m) continue;
                    std::string bit;
                    if (!wide) {
                        bit = "__builtin_amdgcn_ubfe(" + mask_lit(m) + ", js_, 1u)";
                    } else {
                        // 64-bit mask: extract from the half holding bit j
                        char hi[24], lo[24];
                        std::snprintf(hi, sizeof hi, "0x%llxu", m >> 32);
                        std::snprintf(lo, sizeof lo, "0x%llxu", m & 0xffffffffull);
                        bit = std::string("__builtin_amdgcn_ubfe((js_ & 32u) ? ") + hi + " : " + lo +
                              ", js_ & 31u, 1u)";
                    }
                    if (b) bit = "(" + bit + " << " + I(b) + ")";
                    e += (sign > 0 ? " + " : " - ") + bit;
                }
            }
        }
        w.line("const unsigned d" + I(c) + "_ = " + e + ";");
        w.line("n" + I(c) + " = (int)((unsigned)n" + I(c) + " + d" + I(c) + "_);");
        w.line("CWC_KEEP(n" + I(c) + ");");
        if (pos) w.line("mx = mx > (unsigned)n" + I(c) + " ? mx : (unsigned)n" + I(c) + ";");
    }
    w.end();
    w.begin("CWC_APPLY(j, cap, ovf)");
    w.line("CWC_APPLY_MX(j, mx_)");
    w.line("const bool ovf = mx_ > (cap);");
    w.end();
    w.begin("CWC_UNDO()");
    for (int c = 0; c < C; ++c)
        if (!per_cell[c].empty()) w.line("n" + I(c) + " = (int)((unsigned)n" + I(c) + " - d" + I(c) + "_);");
    w.end();
    w.begin("CWC_REDO()");
    for (int c = 0; c < C; ++c)
        if (!per_cell[c].empty()) w.line("n" + I(c) + " = (int)((unsigned)n" + I(c) + " + d" + I(c) + "_);");
    w.end();

    // --- stage the counts for the on-line reduction (see CWC_EMIT)
    w.begin("CWC_STAGE(ptr, stride)");
    for (int c = 0; c < C; ++c) w.line("(ptr)[" + I(c) + " * (stride)] = n" + I(c) + ";");
    w.end();

    // --- lane groups (pair and quad layouts below): the binomial factors of
    // a slot, (F1, F2) with h = F1 * F2.  Kinds: 'n' a count, 'd' n (n-1)
    // of a count, '1' one, 'h' one half.
    struct Fac {
        char kind;
        int cell;
        bool operator==(const Fac &o) const { return kind == o.kind && cell == o.cell; }
    };
    auto factors = [&](int si) -> std::pair<Fac, Fac> {
        const Fac one{'1', -1};
        if (si < 0) return {one, one};
        const Slot &sl = f.slots[si];
        if (sl.n_react == 1 && sl.react_mult[0] == 1) return {Fac{'n', sl.react_cell[0]}, one};
        if (sl.n_react == 1 && sl.react_mult[0] == 2)
            return {Fac{'d', sl.react_cell[0]}, Fac{'h', -1}};
        if (sl.n_react == 2) return {Fac{'n', sl.react_cell[0]}, Fac{'n', sl.react_cell[1]}};
        return {one, one};
    };

    // --- per-lane counts of a lane group (the pair and quad layouts below).
    // Lane h of a group of G lanes builds leaf positions i = 0..B-1, the
    // leaves h*B + i of the canonical tree (B = P/G), and keeps only the
    // counts those leaves read, in registers z0..z(S-1) ("slots"): slot k
    // holds cell cell_of[h][k] in lane h, or nothing.  The reactant cells
    // the G lanes read at the same leaf position are put in one slot
    // wherever the cells already placed allow it (a lane's two two-cell
    // factors may be swapped, the product being the same), so the factor is
    // that slot in every lane with no select.  Cells no lane reads are
    // shared out (a changing cell to the lane holding the fewest changing
    // cells, a constant one to the lane holding the fewest cells), so every
    // cell lives in some lane; a cell kept by several lanes is written out
    // by the lowest of them.  Each lane updates its slots from its own rows
    // of a per-slot change table (lane h: rows h*P + j, byte layout).  When
    // that table does not fit its LDS budget, every lane keeps every cell
    // (slot k = cell k: the lane layout's counts, table and update).
    std::vector<std::vector<long long>> dcl(C, std::vector<long long>(P, 0));
    for (int c = 0; c < C; ++c)
        for (auto &ld : per_cell[c]) dcl[c][ld.first] += ld.second;
    std::vector<char> changes(C, 0);
    for (int c = 0; c < C; ++c) changes[c] = !per_cell[c].empty();
    auto is_cell = [](const Fac &a) { return a.kind == 'n' || a.kind == 'd'; };
    struct GroupMaps {
        int G = 0, B = 0, S = 0, pw = 0;
        bool split = true;
        std::vector<std::vector<int>> slot_of, cell_of;      // [G][C], [G][S]
        std::vector<std::vector<std::pair<Fac, Fac>>> fac;   // [G][B] (after swaps)
        std::vector<Field> sf;                               // [S]
        std::vector<char> spos;                              // [S]: can grow
    };
    auto group_maps = [&](int G) -> GroupMaps {
        GroupMaps m;
        m.G = G;
        m.B = P / G;
        const int B = m.B;
        m.slot_of.assign(G, std::vector<int>(C, -1));
        m.cell_of.assign(G, std::vector<int>());
        m.fac.assign(G, std::vector<std::pair<Fac, Fac>>(B));
        for (int h = 0; h < G; ++h)
            for (int i = 0; i < B; ++i) m.fac[h][i] = factors(f.leaf_slot[h * B + i]);
        auto free_at = [&](int h, int k) { return k >= (int)m.cell_of[h].size() || m.cell_of[h][k] < 0; };
        auto take = [&](int h, int c, int k) {
            if ((int)m.cell_of[h].size() <= k) m.cell_of[h].resize(k + 1, -1);
            m.cell_of[h][k] = c;
            m.slot_of[h][c] = k;
        };
        // would cell a of lane ha and cell b of lane hb end up in one slot
        auto alignable = [&](int ha, int a, int hb, int b) {
            const int ka = m.slot_of[ha][a], kb = m.slot_of[hb][b];
            if (ka >= 0 && kb >= 0) return ka == kb;
            if (ka >= 0) return free_at(hb, ka);
            if (kb >= 0) return free_at(ha, kb);
            return true;
        };
        auto misaligned = [&](int ha, const Fac &l, int hb, const Fac &r) {
            if (l.kind != r.kind) return 1;
            if (!is_cell(l)) return 0;
            return alignable(ha, l.cell, hb, r.cell) ? 0 : 1;
        };
        // put the members' cells, (lane, cell), in one slot where possible:
        // the slot of the first member already placed, else the lowest slot
        // free in every member's lane
        auto align = [&](const std::vector<std::pair<int, int>> &mem) {
            int k = -1;
            for (auto &hc : mem)
                if (k < 0 && m.slot_of[hc.first][hc.second] >= 0) k = m.slot_of[hc.first][hc.second];
            if (k < 0) {
                k = 0;
                for (;;) {
                    bool ok = true;
                    for (auto &hc : mem) ok = ok && free_at(hc.first, k);
                    if (ok) break;
                    ++k;
                }
            }
            for (auto &hc : mem)
                if (m.slot_of[hc.first][hc.second] < 0 && free_at(hc.first, k)) take(hc.first, hc.second, k);
        };
        for (int i = 0; i < B; ++i) {
            int ref = -1, present = 0;
            for (int h = 0; h < G; ++h)
                if (f.leaf_slot[h * B + i] >= 0) {
                    ++present;
                    if (ref < 0) ref = h;
                }
            if (present < 2) continue;
            const std::pair<Fac, Fac> Rf = m.fac[ref][i];
            for (int h = ref + 1; h < G; ++h) {
                if (f.leaf_slot[h * B + i] < 0) continue;
                const std::pair<Fac, Fac> F = m.fac[h][i], Fs{F.second, F.first};
                if (is_cell(F.first) && is_cell(F.second) &&
                    misaligned(ref, Rf.first, h, Fs.first) + misaligned(ref, Rf.second, h, Fs.second) <
                        misaligned(ref, Rf.first, h, F.first) + misaligned(ref, Rf.second, h, F.second))
                    m.fac[h][i] = Fs;
            }
            for (int t = 0; t < 2; ++t) {
                const Fac &r = t ? Rf.second : Rf.first;
                if (!is_cell(r)) continue;
                std::vector<std::pair<int, int>> mem{{ref, r.cell}};
                for (int h = ref + 1; h < G; ++h) {
                    if (f.leaf_slot[h * B + i] < 0) continue;
                    const Fac &a = t ? m.fac[h][i].second : m.fac[h][i].first;
                    if (a.kind == r.kind) mem.push_back({h, a.cell});
                }
                if (mem.size() >= 2) align(mem);
            }
        }
        // the rest of each lane's reactants, then the cells no lane reads
        auto first_free = [&](int h) {
            int k = 0;
            while (!free_at(h, k)) ++k;
            return k;
        };
        for (int h = 0; h < G; ++h)
            for (int i = 0; i < B; ++i)
                for (const Fac &a : {m.fac[h][i].first, m.fac[h][i].second})
                    if (is_cell(a) && m.slot_of[h][a.cell] < 0) take(h, a.cell, first_free(h));
        auto held = [&](int h, bool changing) {
            int n = 0;
            for (int c = 0; c < C; ++c) n += m.slot_of[h][c] >= 0 && (!changing || changes[c]);
            return n;
        };
        for (int c = 0; c < C; ++c) {
            bool any = false;
            for (int h = 0; h < G; ++h) any = any || m.slot_of[h][c] >= 0;
            if (any) continue;
            int best = 0;
            for (int h = 1; h < G; ++h)
                if (held(h, changes[c]) < held(best, changes[c])) best = h;
            take(best, c, first_free(best));
        }
        int S = 0;
        for (int h = 0; h < G; ++h) S = std::max(S, (int)m.cell_of[h].size());
        for (int h = 0; h < G; ++h) m.cell_of[h].resize(S, -1);
        // per-slot change table, byte layout (as the lane layout's)
        m.sf.assign(S, Field{});
        m.spos.assign(S, 0);
        int used[4] = {0, 0, 0, 0};
        for (int k = 0; k < S && m.split; ++k) {
            long long lo = 0, hi = 0;
            for (int h = 0; h < G; ++h) {
                const int c = m.cell_of[h][k];
                if (c < 0) continue;
                for (int j = 0; j < P; ++j) {
                    lo = std::min(lo, dcl[c][j]);
                    hi = std::max(hi, dcl[c][j]);
                }
            }
            if (lo == 0 && hi == 0) continue;   // no field: never changes
            m.spos[k] = hi > 0;
            Field &fd = m.sf[k];
            fd.sgn = lo < 0;
            const bool b8 = fd.sgn ? (lo >= -128 && hi <= 127) : hi <= 255;
            const bool b16 = fd.sgn ? (lo >= -32768 && hi <= 32767) : hi <= 65535;
            if (!b16) {
                m.split = false;
                break;
            }
            fd.width = b8 ? 8 : 16;
            for (int wd = 0; wd < 4 && fd.word < 0; ++wd) {
                const int off = (used[wd] + fd.width - 1) / fd.width * fd.width;
                if (off + fd.width <= 32) {
                    fd.word = wd;
                    fd.off = off;
                    used[wd] = off + fd.width;
                    m.pw = std::max(m.pw, wd + 1);
                }
            }
            if (fd.word < 0) m.split = false;
        }
        if (m.pw == 3) m.pw = 4;
        if ((size_t)G * (size_t)P * (size_t)m.pw * 4u > (G == 2 ? kPairStaticLdsBytes : kQuadStaticLdsBytes))
            m.split = false;
        if (!m.split) {
            // every cell in every lane, slot k = cell k
            m.S = C;
            for (int h = 0; h < G; ++h) {
                m.cell_of[h].assign(C, -1);
                for (int c = 0; c < C; ++c) {
                    m.cell_of[h][c] = c;
                    m.slot_of[h][c] = c;
                }
            }
        } else {
            m.S = S;
        }
        return m;
    };
    // four-way select by the bits of h, folding equal operands
    auto sel4 = [&](const std::string v[4]) -> std::string {
        auto sel2 = [&](const std::string &bit, const std::string &a, const std::string &b) {
            return a == b ? a : "((" + bit + ") ? " + b + " : " + a + ")";
        };
        const std::string lo = sel2("(h) & 1", v[0], v[1]);
        const std::string hi = sel2("(h) & 1", v[2], v[3]);
        return sel2("(h) & 2", lo, hi);
    };
    // The group's state macros (X = CWC_PAIR or CWC_QUAD): X_SPLIT, the
    // slots (X_STATE), load from a count row, write the lane's cells to a
    // count row or to a staging column (stride 64), and (for the host
    // tests) write every cell the lane holds; the update X_APPLY_MX (the
    // change of leaf j added to the lane's slots, the largest count that
    // can grow left in `mx`), X_UNDO / X_REDO; the table in LDS (X_SETUP).
    auto emit_group_state = [&](const GroupMaps &m, const std::string &X, const std::string &tab) {
        const int G = m.G, S = m.S;
        auto sv = [&](int k) { return (m.split ? "z" : "n") + I(k); };
        auto owns = [&](int h, int k) {
            const int c = m.cell_of[h][k];
            if (c < 0) return false;
            for (int g = 0; g < h; ++g)
                if (m.slot_of[g][c] >= 0) return false;
            return true;
        };
        o << "#define " << X << "_SPLIT " << (m.split ? 1 : 0) << "\n";
        w.begin(X + "_STATE");
        if (m.split)
            for (int k = 0; k < S; ++k) w.line("int z" + I(k) + " = 0;");
        w.end();
        w.begin(X + "_LOAD_COUNTS(ptr, h)");
        if (m.split) {
            for (int k = 0; k < S; ++k) {
                std::string l[4];
                for (int h = 0; h < G; ++h) {
                    const int c = m.cell_of[h][k];
                    l[h] = c < 0 ? "0" : "(ptr)[" + I(c) + "]";
                }
                w.line("z" + I(k) + " = " + (G == 2 ? "(h) ? " + l[1] + " : " + l[0] : sel4(l)) + ";");
            }
        } else {
            w.line("CWC_LOAD_COUNTS(ptr);");
        }
        w.end();
        auto store_lines = [&](const std::string &dst, const std::string &stride, bool all) {
            if (!m.split) {
                w.line(all ? "{" : "if (!(h)) {");
                for (int c = 0; c < C; ++c)
                    w.line("(" + dst + ")[" + I(c) + stride + "] = n" + I(c) + ";");
                w.line("}");
                return;
            }
            for (int h = 0; h < G; ++h) {
                if (G == 2) w.line(h ? "} else {" : "if (!(h)) {");
                else w.line(h == 0 ? "if ((h) == 0) {" : h < G - 1 ? "} else if ((h) == " + I(h) + ") {" : "} else {");
                for (int k = 0; k < S; ++k)
                    if (all ? m.cell_of[h][k] >= 0 : owns(h, k))
                        w.line("(" + dst + ")[" + I(m.cell_of[h][k]) + stride + "] = z" + I(k) + ";");
            }
            w.line("}");
        };
        w.begin(X + "_STORE_COUNTS(ptr, h)");
        store_lines("ptr", "", false);
        w.end();
        w.begin(X + "_STAGE(col0, h)");
        store_lines("col0", " * 64", false);
        w.end();
        w.begin(X + "_HELD(ptr, h)");
        store_lines("ptr", "", true);
        w.end();
        if (!m.split) {
            o << "#define " << X << "_SETUP CWC_DT_SETUP\n";
            o << "#define " << X << "_APPLY_MX(j, mx) CWC_APPLY_MX(j, mx)\n";
            o << "#define " << X << "_UNDO() CWC_UNDO()\n";
            o << "#define " << X << "_REDO() CWC_REDO()\n";
            return;
        }
        const int pw = m.pw;
        const char *ty = pw == 1 ? "unsigned int" : pw == 2 ? "uint2" : "uint4";
        if (pw > 0) {
            o << "__constant__ unsigned int " << tab << "_g[" << G * P * pw << "] = {";
            for (int h = 0; h < G; ++h)
                for (int j = 0; j < P; ++j) {
                    unsigned long long wv[4] = {0, 0, 0, 0};
                    for (int k = 0; k < S; ++k) {
                        const int c = m.cell_of[h][k];
                        if (m.sf[k].word < 0 || c < 0) continue;
                        const unsigned long long bv =
                            (unsigned long long)dcl[c][j] & ((1ull << m.sf[k].width) - 1ull);
                        wv[m.sf[k].word] |= bv << m.sf[k].off;
                    }
                    for (int q = 0; q < pw; ++q) {
                        char b[32];
                        std::snprintf(b, sizeof b, "%s0x%llxu", (h || j || q) ? ", " : "", wv[q]);
                        o << b;
                    }
                }
            o << "};\n";
            // the block's copy in LDS; <tab>_h = this lane's rows
            w.begin(X + "_SETUP");
            w.line(std::string("__shared__ ") + ty + " " + tab + "[" + I(G * P) + "];");
            w.line("for (int i_ = (int)threadIdx.x; i_ < " + I(G * P * pw) +
                   "; i_ += (int)blockDim.x) ((unsigned int *)" + tab + ")[i_] = " + tab + "_g[i_];");
            w.line("__syncthreads();");
            if (G == 2)
                w.line(std::string("const ") + ty + " *const " + tab + "_h = " + tab +
                       " + ((threadIdx.x & 1u) ? " + I(P) + " : 0);");
            else
                w.line(std::string("const ") + ty + " *const " + tab + "_h = " + tab + " + (threadIdx.x & " +
                       I(G - 1) + "u) * " + I(P) + "u;");
            w.end();
        } else {
            o << "#define " << X << "_SETUP\n";
        }
        w.begin(X + "_APPLY_MX(j, mx)");
        if (pw == 1) {
            w.line("const unsigned dw0_ = " + tab + "_h[(unsigned)(j)];");
        } else if (pw == 2) {
            w.line("const uint2 dq_ = " + tab + "_h[(unsigned)(j)];");
            w.line("const unsigned dw0_ = dq_.x, dw1_ = dq_.y;");
        } else if (pw == 4) {
            w.line("const uint4 dq_ = " + tab + "_h[(unsigned)(j)];");
            w.line("const unsigned dw0_ = dq_.x, dw1_ = dq_.y, dw2_ = dq_.z, dw3_ = dq_.w;");
        }
        w.line("unsigned mx = 0u;");
        for (int k = 0; k < S; ++k) {
            const Field &fd = m.sf[k];
            if (fd.word < 0) continue;
            const std::string wv = "dw" + I(fd.word) + "_";
            const std::string sh = fd.off ? "(" + wv + " >> " + I(fd.off) + ")" : wv;
            const std::string e =
                fd.sgn ? std::string("(unsigned)(int)(") + (fd.width == 8 ? "signed char" : "short") + ")" + sh
                       : std::string("(unsigned)(") + (fd.width == 8 ? "unsigned char" : "unsigned short") +
                             ")" + sh;
            w.line("const unsigned d" + I(k) + "_ = " + e + ";");
            w.line("z" + I(k) + " = (int)((unsigned)z" + I(k) + " + d" + I(k) + "_);");
            w.line("CWC_KEEP(z" + I(k) + ");");
            if (m.spos[k]) w.line("mx = mx > (unsigned)z" + I(k) + " ? mx : (unsigned)z" + I(k) + ";");
        }
        w.end();
        w.begin(X + "_UNDO()");
        for (int k = 0; k < S; ++k)
            if (m.sf[k].word >= 0) w.line("z" + I(k) + " = (int)((unsigned)z" + I(k) + " - d" + I(k) + "_);");
        w.end();
        w.begin(X + "_REDO()");
        for (int k = 0; k < S; ++k)
            if (m.sf[k].word >= 0) w.line("z" + I(k) + " = (int)((unsigned)z" + I(k) + " + d" + I(k) + "_);");
        w.end();
    };
    // A factor of lane h in slot terms: the kind and the slot of its cell in
    // that lane.  Where the lanes' factors differ (kind or slot) h selects,
    // integer-valued factors as integers converted once (the conversion is
    // exact either way).  A lane whose position is empty has rate +0: any
    // finite factor gives +0 there, so it takes another lane's factors.
    struct SF {
        char kind;
        int slot;
        bool operator==(const SF &o) const { return kind == o.kind && slot == o.slot; }
    };
    auto sexpr = [&](const SF &a) -> std::string {
        switch (a.kind) {
        case 'n': return "y" + I(a.slot) + "_";
        case 'd': return "(y" + I(a.slot) + "_ * w" + I(a.slot) + "_)";
        case 'h': return "0.5";
        default: return "1.0";
        }
    };
    // the conversions a group's tree reads: y<k>_ of every slot and
    // w<k>_ = max(z<k> - 1, 0) of the slots some lane squares
    auto emit_group_conv = [&](const GroupMaps &m) {
        auto sv = [&](int k) { return (m.split ? "z" : "n") + I(k); };
        std::vector<char> s_need_d(m.S, 0);
        for (int h = 0; h < m.G; ++h)
            for (int i = 0; i < m.B; ++i)
                for (const Fac &a : {m.fac[h][i].first, m.fac[h][i].second})
                    if (a.kind == 'd') s_need_d[m.slot_of[h][a.cell]] = 1;
        for (int k = 0; k < m.S; ++k) {
            w.line("const double y" + I(k) + "_ = (double)" + sv(k) + ";");
            if (s_need_d[k])
                w.line("const double w" + I(k) + "_ = (double)(" + sv(k) + " > 0 ? " + sv(k) + " - 1 : 0);");
        }
    };
    // the factors of position i in each lane, in slot terms, an empty lane
    // taking those of a present lane (its partner first)
    auto group_factors = [&](const GroupMaps &m, int i, std::vector<std::pair<SF, SF>> &out) {
        const int G = m.G, B = m.B;
        out.assign(G, {SF{'1', -1}, SF{'1', -1}});
        std::vector<char> present(G, 0);
        for (int h = 0; h < G; ++h) {
            present[h] = f.leaf_slot[h * B + i] >= 0;
            if (!present[h]) continue;
            const Fac &a = m.fac[h][i].first, &b = m.fac[h][i].second;
            out[h] = {SF{a.kind, is_cell(a) ? m.slot_of[h][a.cell] : -1},
                      SF{b.kind, is_cell(b) ? m.slot_of[h][b.cell] : -1}};
        }
        for (int h = 0; h < G; ++h) {
            if (present[h]) continue;
            for (int d = 1; d < G; ++d)
                if (present[h ^ d]) {
                    out[h] = out[h ^ d];
                    break;
                }
        }
    };

    // --- pair layout: two lanes per trajectory.  Lane h (0 or 1) of a pair
    // holds leaves [h*B, (h+1)*B) of the same canonical tree (B = P/2): the
    // root is its half plus the partner's, the root decision is taken by
    // both lanes, the rest of the descent by the lane holding the chosen
    // half.  Leaf position i of a lane is the left slot i or the right slot
    // B + i, formed with the same operations as the lane layout's leaf
    // (k * h with h = product of the binomial factors) from the lane's
    // count slots, so the tree has the same bits; an empty side has rate 0
    // and gives +0, which leaves every sum unchanged.
    if (P >= 2) {
        const int B = P / 2;
        int DB = 0;
        while ((1 << DB) < B) ++DB;
        o << "#define CWC_PAIR 1\n#define CWC_PB " << B << "\n";
        std::vector<char> hz(2 * B, 1);
        for (int i = 0; i < B; ++i) hz[B + i] = (f.leaf_slot[i] < 0) && (f.leaf_slot[B + i] < 0);
        for (int i = B - 1; i >= 1; --i) hz[i] = hz[2 * i] && hz[2 * i + 1];
        auto hv = [&](int i) -> std::string { return hz[i] ? std::string("0.0") : "q" + I(i); };
        const GroupMaps m = group_maps(2);
        w.begin("CWC_PAIR_DECL");
        for (int i = 0; i < B; ++i)
            if (!hz[B + i]) w.line("double K" + I(i) + " = 0.0;");
        for (int i = 1; i < 2 * B; ++i)
            if (!hz[i]) w.line("double q" + I(i) + " = 0.0;");
        w.end();
        // per-lane rates of the lane's leaf positions from a rate row
        w.begin("CWC_PAIR_LOAD_K(ptr, h)");
        for (int i = 0; i < B; ++i) {
            if (hz[B + i]) continue;
            const int sl = f.leaf_slot[i], sr = f.leaf_slot[B + i];
            const std::string Ls = sl < 0 ? "0.0" : "(ptr)[" + I(f.slots[sl].rule) + "]";
            const std::string Rs = sr < 0 ? "0.0" : "(ptr)[" + I(f.slots[sr].rule) + "]";
            w.line("K" + I(i) + " = (h) ? " + Rs + " : " + Ls + ";");
        }
        w.end();
        emit_group_state(m, "CWC_PAIR", "cwc_ptab");
        auto ssel = [&](const SF &l, const SF &r) -> std::string {
            if (l == r) return sexpr(l);
            const bool li = l.kind == 'n' || l.kind == '1', ri = r.kind == 'n' || r.kind == '1';
            auto sv = [&](int k) { return (m.split ? "z" : "n") + I(k); };
            if (li && ri) {
                auto iexpr = [&](const SF &a) { return a.kind == 'n' ? sv(a.slot) : std::string("1"); };
                return "(double)((h) ? " + iexpr(r) + " : " + iexpr(l) + ")";
            }
            return "((h) ? " + sexpr(r) + " : " + sexpr(l) + ")";
        };
        w.begin("CWC_PAIR_TREE(h)");
        w.line("{");
        emit_group_conv(m);
        std::vector<std::pair<SF, SF>> fs;
        for (int i = 0; i < B; ++i) {
            if (hz[B + i]) continue;
            group_factors(m, i, fs);
            const std::string F1 = ssel(fs[0].first, fs[1].first);
            const std::string F2 = ssel(fs[0].second, fs[1].second);
            std::string H;
            if (F2 == "1.0") H = F1;
            else H = "(" + F1 + " * " + F2 + ")";
            w.line("q" + I(B + i) + " = " + (H == "1.0" ? "K" + I(i) : "K" + I(i) + " * " + H) + ";");
        }
        for (int i = B - 1; i >= 1; --i) {
            if (hz[i]) continue;
            if (!hz[2 * i] && !hz[2 * i + 1]) w.line("q" + I(i) + " = q" + I(2 * i) + " + q" + I(2 * i + 1) + ";");
            else if (!hz[2 * i]) w.line("q" + I(i) + " = q" + I(2 * i) + ";");
            else w.line("q" + I(i) + " = q" + I(2 * i + 1) + ";");
        }
        w.line("}");
        w.end();
        o << "#define CWC_PAIR_HALF " << hv(1) << "\n";
        // descent inside the lane's half (same narrowing as CWC_DESCEND)
        w.begin("CWC_PAIR_DESCEND(x, j)");
        w.line("{");
        w.line("int jj_ = 0;");
        std::vector<std::string> hbits;
        int htmp = 0;
        for (int d = 0; d < DB; ++d) {
            std::vector<std::string> vals;
            for (int q = 0; q < (2 << d); ++q) vals.push_back(hv((2 << d) + q));
            const Narrowed nw = narrow_pair(vals, hbits, "u", htmp, &w);
            const std::string Lv = nw.L, Rv = nw.R;
            if (Rv == "0.0") {
                w.line("jj_ = jj_ << 1;");
                hbits.push_back("");
                continue;
            }
            const std::string b = "e" + I(d) + "_";
            if (Lv == "0.0")
                w.line("const bool " + b + " = (" + Rv + " != 0.0);");
            else
                w.line("const bool " + b + " = ((x) >= " + Lv + ") && (" + Rv + " != 0.0);");
            if (Lv != "0.0") w.line("(x) = " + b + " ? (x) - " + Lv + " : (x);");
            w.line("jj_ = (jj_ << 1) | (" + b + " ? 1 : 0);");
            hbits.push_back(b);
        }
        w.line("(j) = jj_;");
        w.line("}");
        w.end();
    }

    // --- quad layout: four lanes per trajectory.  Lane h (0..3) of a quad
    // holds quarter h, leaves [h*B, (h+1)*B) of the canonical tree
    // (B = P/4); the two top levels (halves = quarter 0 + quarter 1 and
    // quarter 2 + quarter 3, root = left half + right half) are formed from
    // the four quarter sums in every lane.  Leaf position i of a lane is
    // slot h*B + i, formed from the lane's count slots; factors that differ
    // between the lanes are selected by the two bits of h.
    if (P >= 4) {
        const int B = P / 4;
        int DB = 0;
        while ((1 << DB) < B) ++DB;
        o << "#define CWC_QUAD 1\n#define CWC_QB " << B << "\n";
        std::vector<char> qz(2 * B, 1);
        for (int i = 0; i < B; ++i) {
            bool z = true;
            for (int k = 0; k < 4; ++k) z = z && f.leaf_slot[k * B + i] < 0;
            qz[B + i] = z;
        }
        for (int i = B - 1; i >= 1; --i) qz[i] = qz[2 * i] && qz[2 * i + 1];
        auto qv = [&](int i) -> std::string { return qz[i] ? std::string("0.0") : "r" + I(i); };
        const GroupMaps m = group_maps(4);
        w.begin("CWC_QUAD_DECL");
        for (int i = 0; i < B; ++i)
            if (!qz[B + i]) w.line("double KQ" + I(i) + " = 0.0;");
        for (int i = 1; i < 2 * B; ++i)
            if (!qz[i]) w.line("double r" + I(i) + " = 0.0;");
        w.end();
        w.begin("CWC_QUAD_LOAD_K(ptr, h)");
        for (int i = 0; i < B; ++i) {
            if (qz[B + i]) continue;
            std::string v[4];
            for (int k = 0; k < 4; ++k) {
                const int sl = f.leaf_slot[k * B + i];
                v[k] = sl < 0 ? "0.0" : "(ptr)[" + I(f.slots[sl].rule) + "]";
            }
            w.line("KQ" + I(i) + " = " + sel4(v) + ";");
        }
        w.end();
        emit_group_state(m, "CWC_QUAD", "cwc_qtab");
        auto fsel4 = [&](const SF g[4]) -> std::string {
            bool all_int = true, all_eq = true;
            for (int k = 0; k < 4; ++k) {
                all_int = all_int && (g[k].kind == 'n' || g[k].kind == '1');
                all_eq = all_eq && g[k] == g[0];
            }
            if (all_eq) return sexpr(g[0]);
            std::string v[4];
            if (all_int) {
                for (int k = 0; k < 4; ++k)
                    v[k] = g[k].kind == 'n' ? (m.split ? "z" : "n") + I(g[k].slot) : std::string("1");
                return "(double)" + sel4(v);
            }
            for (int k = 0; k < 4; ++k) v[k] = sexpr(g[k]);
            return sel4(v);
        };
        w.begin("CWC_QUAD_TREE(h)");
        w.line("{");
        emit_group_conv(m);
        std::vector<std::pair<SF, SF>> fs;
        for (int i = 0; i < B; ++i) {
            if (qz[B + i]) continue;
            group_factors(m, i, fs);
            SF g1[4], g2[4];
            for (int k = 0; k < 4; ++k) {
                g1[k] = fs[k].first;
                g2[k] = fs[k].second;
            }
            const std::string F1 = fsel4(g1), F2 = fsel4(g2);
            std::string H;
            if (F2 == "1.0") H = F1;
            else H = "(" + F1 + " * " + F2 + ")";
            w.line("r" + I(B + i) + " = " + (H == "1.0" ? "KQ" + I(i) : "KQ" + I(i) + " * " + H) + ";");
        }
        for (int i = B - 1; i >= 1; --i) {
            if (qz[i]) continue;
            if (!qz[2 * i] && !qz[2 * i + 1]) w.line("r" + I(i) + " = r" + I(2 * i) + " + r" + I(2 * i + 1) + ";");
            else if (!qz[2 * i]) w.line("r" + I(i) + " = r" + I(2 * i) + ";");
            else w.line("r" + I(i) + " = r" + I(2 * i + 1) + ";");
        }
        w.line("}");
        w.end();
        o << "#define CWC_QUAD_PART " << qv(1) << "\n";
        // descent inside the lane's quarter (same narrowing as CWC_DESCEND)
        w.begin("CWC_QUAD_DESCEND(x, j)");
        w.line("{");
        w.line("int jj_ = 0;");
        std::vector<std::string> qbits;
        int qtmp = 0;
        for (int d = 0; d < DB; ++d) {
            std::vector<std::string> vals;
            for (int q = 0; q < (2 << d); ++q) vals.push_back(qv((2 << d) + q));
            const Narrowed nw = narrow_pair(vals, qbits, "w", qtmp, &w);
            const std::string Lv = nw.L, Rv = nw.R;
            if (Rv == "0.0") {
                w.line("jj_ = jj_ << 1;");
                qbits.push_back("");
                continue;
            }
            const std::string b = "g" + I(d) + "_";
            if (Lv == "0.0")
                w.line("const bool " + b + " = (" + Rv + " != 0.0);");
            else
                w.line("const bool " + b + " = ((x) >= " + Lv + ") && (" + Rv + " != 0.0);");
            if (Lv != "0.0") w.line("(x) = " + b + " ? (x) - " + Lv + " : (x);");
            w.line("jj_ = (jj_ << 1) | (" + b + " ? 1 : 0);");
            qbits.push_back(b);
        }
        w.line("(j) = jj_;");
        w.line("}");
        w.end();
    }
    return o.str();
}

}  // namespace cwc

namespace cwc {

bool fits_lane(const Flat &f) { return f.n_leaves <= 64 && f.n_cells <= 64; }

bool fits_wave(const Flat &f)
{
    int ns_w = 0;
    for (int t = 0; t < f.n_types; ++t) ns_w |= f.has_wrap[t];
    return f.p_comp <= 64 && f.p_local <= 64 && f.n_species * (2 + ns_w) <= 96;
}

int choose_layout(const Flat &f)
{
    if (fits_lane(f)) return 0;
    if (fits_wave(f)) return 1;
    return -1;
}

// ------------------------------------------------------------ wave layout
// One wavefront per trajectory; lane q owns compartment q: its content
// counts nc<s>, its wrap counts nw<s>, a copy np<s> of its parent's
// content, and the P_local leaves of its slot block (a<P_local + pos>)
// with their local subtree (a<1..P_local-1>).  Lanes whose compartments
// run the same slot list share a "kind"; leaf formulas are selected per
// kind.  The selected slot is uniform across the wavefront, so the update
// is a scalar switch over (kind, position).
std::string codegen_wave(const Flat &f)
{
    std::ostringstream o;
    MacroWriter w(o);
    auto I = [](int v) { return std::to_string(v); };
    const int NS = f.n_species, PL = f.p_local, PC = f.p_comp;
    int LP = 0;
    while ((1 << LP) < PC) ++LP;
    int DL = 0;
    while ((1 << DL) < PL) ++DL;
    bool any_wrap = false;
    for (int t = 0; t < f.n_types; ++t) any_wrap |= f.has_wrap[t] != 0;
    const int NR = std::max(1, f.n_rules);

    // kinds: distinct slot lists (sequence of rules) among compartments
    std::vector<std::vector<int>> kinds;
    std::vector<int> kind_of(f.n_comp, -1);
    for (int q = 0; q < f.n_comp; ++q) {
        std::vector<int> lst;
        for (int l = 0; l < PL; ++l) {
            int si = f.leaf_slot[q * PL + l];
            lst.push_back(si < 0 ? -1 : f.slots[si].rule);
        }
        int k = -1;
        for (size_t i = 0; i < kinds.size(); ++i)
            if (kinds[i] == lst) k = (int)i;
        if (k < 0) {
            k = (int)kinds.size();
            kinds.push_back(lst);
        }
        kind_of[q] = k;
    }
    // region of a global cell relative to context q: 0 own content, 1 own
    // wrap, 2 parent content
    std::vector<int> cell_comp(f.n_cells), cell_wrap(f.n_cells), cell_sp(f.n_cells);
    for (int q = 0; q < f.n_comp; ++q)
        for (int s = 0; s < NS; ++s) {
            cell_comp[f.content_base[q] + s] = q;
            cell_wrap[f.content_base[q] + s] = 0;
            cell_sp[f.content_base[q] + s] = s;
            if (f.wrap_base[q] >= 0) {
                cell_comp[f.wrap_base[q] + s] = q;
                cell_wrap[f.wrap_base[q] + s] = 1;
                cell_sp[f.wrap_base[q] + s] = s;
            }
        }
    auto var_of = [&](int q, int cell) -> std::string {
        const int cq = cell_comp[cell], sp = cell_sp[cell];
        if (cq == q) return (cell_wrap[cell] ? "nw" : "nc") + std::to_string(sp);
        return "np" + std::to_string(sp);   // parent content
    };

    o << "// ---- generated model section (wavefront-per-replica layout)\n";
    o << "#define CWC_C " << f.n_cells << "\n#define CWC_NS " << NS << "\n#define CWC_PL " << PL
      << "\n#define CWC_PC " << PC << "\n#define CWC_LP " << LP << "\n#define CWC_NR " << NR
      << "\n#define CWC_HAS_WRAP " << (any_wrap ? 1 : 0) << "\n";
    auto table = [&](const char *name, std::vector<int> v) {
        v.resize(64, -1);
        o << "__constant__ int " << name << "[64] = {";
        for (int i = 0; i < 64; ++i) o << (i ? "," : "") << v[i];
        o << "};\n";
    };
    std::vector<int> kt(f.n_comp), par(f.comp_parent), cb(f.content_base), wb(f.wrap_base);
    for (int q = 0; q < f.n_comp; ++q) kt[q] = kind_of[q];
    table("cwc_kind", kt);
    table("cwc_parent", par);
    table("cwc_cbase", cb);
    table("cwc_wbase", wb);

    w.begin("CWC_DECL_STATE");
    for (int s = 0; s < NS; ++s) w.line("int nc" + I(s) + " = 0; int np" + I(s) + " = 0;");
    if (any_wrap)
        for (int s = 0; s < NS; ++s) w.line("int nw" + I(s) + " = 0;");
    for (int i = 1; i < 2 * PL; ++i) w.line("double a" + I(i) + " = 0.0;");
    w.end();
    // per-lane loads: own content/wrap and parent content from a cell row
    w.begin("CWC_LOAD_COUNTS(ptr, cb, wb, pb)");
    w.line("if ((cb) >= 0) {");
    for (int s = 0; s < NS; ++s) w.line("    nc" + I(s) + " = (ptr)[(cb) + " + I(s) + "];");
    w.line("}");
    if (any_wrap) {
        w.line("if ((wb) >= 0) {");
        for (int s = 0; s < NS; ++s) w.line("    nw" + I(s) + " = (ptr)[(wb) + " + I(s) + "];");
        w.line("}");
    }
    w.line("if ((pb) >= 0) {");
    for (int s = 0; s < NS; ++s) w.line("    np" + I(s) + " = (ptr)[(pb) + " + I(s) + "];");
    w.line("}");
    w.end();
    w.begin("CWC_STORE_COUNTS(ptr, cb, wb)");
    w.line("if ((cb) >= 0) {");
    for (int s = 0; s < NS; ++s) w.line("    (ptr)[(cb) + " + I(s) + "] = nc" + I(s) + ";");
    w.line("}");
    if (any_wrap) {
        w.line("if ((wb) >= 0) {");
        for (int s = 0; s < NS; ++s) w.line("    (ptr)[(wb) + " + I(s) + "] = nw" + I(s) + ";");
        w.line("}");
    }
    w.end();
    w.begin("CWC_STAGE(ptr, stride)");
    for (int s = 0; s < NS; ++s) w.line("(ptr)[" + I(s) + " * (stride)] = nc" + I(s) + ";");
    if (any_wrap)
        for (int s = 0; s < NS; ++s)
            w.line("(ptr)[" + I(NS + s) + " * (stride)] = nw" + I(s) + ";");
    w.end();

    // Leaves: a lane evaluates the formulas of its kind only.  Each
    // formula's rate is multiplied once per trajectory by the lane's kind
    // mask (1.0 for the formula's kind, else 0.0), into a masked rate
    // km<position>_<kind>: (k * 1) * h is k * h and (k * 0) * h is +0 (every
    // factor is finite and non-negative), so no per-leaf select by kind and
    // no per-event mask is needed; a leaf position that several kinds use
    // sums their formulas, of which at most one is non-zero.  The masked
    // rates differ between kinds, so they take vector registers; the
    // queue-draining form, which holds more state, keeps the rule rates
    // uniform instead and masks the first count factor of each formula per
    // event (k * (x * 1) is k * x, k * (x * 0) is +0): CWC_LEAVES_FREE.
    std::vector<char> used_c(NS, 0), used_d(NS, 0), used_p(NS, 0), used_pd(NS, 0), used_w(NS, 0),
        used_wd(NS, 0);
    std::vector<char> kind_used(kinds.size(), 0);
    std::vector<std::pair<std::string, int>> kmask;   // (masked rate, rule), kind in the name
    std::set<std::pair<int, std::string>> masked;     // (kind, count factor) masked per event
    // representative compartment of each kind, to resolve regions
    std::vector<int> rep(kinds.size(), -1);
    for (int q = 0; q < f.n_comp; ++q)
        if (rep[kind_of[q]] < 0) rep[kind_of[q]] = q;
    std::vector<std::vector<std::string>> form(PL, std::vector<std::string>(kinds.size(), "0.0"));
    std::vector<std::vector<std::string>> form_free = form;
    for (size_t kd = 0; kd < kinds.size(); ++kd) {
        const int q = rep[kd];
        for (int l = 0; l < PL; ++l) {
            int si = f.leaf_slot[q * PL + l];
            if (si < 0) continue;
            const Slot &s = f.slots[si];
            std::string h;
            auto cv = [&](int cell, bool dec) {
                std::string v = var_of(q, cell);
                std::string tag = v.substr(0, 2), sp = v.substr(2);
                int spi = std::stoi(sp);
                if (tag == "nc") (dec ? used_d : used_c)[spi] = 1;
                else if (tag == "np") (dec ? used_pd : used_p)[spi] = 1;
                else (dec ? used_wd : used_w)[spi] = 1;
                return (dec ? "m" : "x") + v + "_";
            };
            // the first count factor, masked by the kind (queue-draining form)
            auto cvm = [&](int cell) {
                const std::string v = cv(cell, false);
                masked.insert({(int)kd, v});
                return v + "k" + I((int)kd) + "_";
            };
            kind_used[kd] = 1;
            std::string hm;
            if (s.n_react == 1 && s.react_mult[0] == 1) {
                h = cv(s.react_cell[0], false);
                hm = cvm(s.react_cell[0]);
            } else if (s.n_react == 1 && s.react_mult[0] == 2) {
                h = "((" + cv(s.react_cell[0], false) + " * " + cv(s.react_cell[0], true) + ") * 0.5)";
                hm = "((" + cvm(s.react_cell[0]) + " * " + cv(s.react_cell[0], true) + ") * 0.5)";
            } else if (s.n_react == 2) {
                h = "(" + cv(s.react_cell[0], false) + " * " + cv(s.react_cell[1], false) + ")";
                hm = "(" + cvm(s.react_cell[0]) + " * " + cv(s.react_cell[1], false) + ")";
            } else {
                hm = "mk" + I((int)kd) + "_";   // order 0: the rate itself, masked
            }
            const std::string km = "km" + I(l) + "_" + I((int)kd);
            kmask.push_back({km, s.rule});
            form[l][kd] = h.empty() ? km : km + " * " + h;   // order 0: the masked rate itself
            form_free[l][kd] = "k" + I(s.rule) + " * " + hm;
        }
    }
    // rates: the rule rates of the trajectory's instance, and each
    // formula's rate masked by the lane's kind.  The masked rates are the
    // same in every lane of a kind, but in scalar registers they crowd out
    // the kernel's other uniform values and spill to lanes of a VGPR (a lane
    // read per use); kept in VGPRs instead (CWC_KEEP), they fit beside the
    // state.  The queue-draining form (CWC_LOAD_K_FREE) reloads them per
    // trajectory and holds more state: there the compiler's own placement
    // keeps two wavefronts per SIMD.
    w.begin("CWC_DECL_K");
    for (auto &km : kmask) w.line("double " + km.first + " = 0.0;");
    for (int r = 0; r < NR; ++r) w.line("double k" + I(r) + " = 0.0;");
    w.end();
    w.begin("CWC_LOAD_K(ptr, kind)");
    w.line("{");
    for (size_t kd = 0; kd < kinds.size(); ++kd)
        if (kind_used[kd])
            w.line("const double mk" + I((int)kd) + "_ = (kind) == " + I((int)kd) + " ? 1.0 : 0.0;");
    for (auto &km : kmask) {
        const std::string kd = km.first.substr(km.first.rfind('_') + 1);
        w.line(km.first + " = (ptr)[" + I(km.second) + "] * mk" + kd + "_; CWC_KEEP(" + km.first + ");");
    }
    w.line("}");
    w.end();
    w.begin("CWC_LOAD_K_FREE(ptr, kind)");
    for (int r = 0; r < f.n_rules; ++r) w.line("k" + I(r) + " = (ptr)[" + I(r) + "];");
    w.end();
    // leaves: per position, the formula of the lane's kind (0 if none)
    std::vector<char> zero(2 * PL, 1);
    for (int free_form = 0; free_form < 2; ++free_form) {
    w.begin(free_form ? "CWC_LEAVES_FREE(kind)" : "CWC_LEAVES(kind)");
    w.line("{");
    for (int s = 0; s < NS; ++s) {
        if (used_c[s] || used_d[s]) w.line("const double xnc" + I(s) + "_ = (double)nc" + I(s) + ";");
        if (used_d[s]) w.line("const double mnc" + I(s) + "_ = (double)(nc" + I(s) + " > 0 ? nc" + I(s) + " - 1 : 0);");
        if (used_p[s] || used_pd[s]) w.line("const double xnp" + I(s) + "_ = (double)np" + I(s) + ";");
        if (used_pd[s]) w.line("const double mnp" + I(s) + "_ = (double)(np" + I(s) + " > 0 ? np" + I(s) + " - 1 : 0);");
        if (used_w[s] || used_wd[s]) w.line("const double xnw" + I(s) + "_ = (double)nw" + I(s) + ";");
        if (used_wd[s]) w.line("const double mnw" + I(s) + "_ = (double)(nw" + I(s) + " > 0 ? nw" + I(s) + " - 1 : 0);");
    }
    if (free_form) {
        for (size_t kd = 0; kd < kinds.size(); ++kd)
            if (kind_used[kd])
                w.line("const double mk" + I((int)kd) + "_ = (kind) == " + I((int)kd) + " ? 1.0 : 0.0;");
        for (auto &mv : masked)
            w.line("const double " + mv.second + "k" + I(mv.first) + "_ = " + mv.second + " * mk" +
                   I(mv.first) + "_;");
    }
    const auto &fm = free_form ? form_free : form;
    for (int l = 0; l < PL; ++l) {
        bool any = false;
        for (size_t kd = 0; kd < kinds.size(); ++kd) any |= fm[l][kd] != "0.0";
        zero[PL + l] = !any;
        if (!any) continue;
        std::string e;
        for (size_t kd = 0; kd < kinds.size(); ++kd) {
            if (fm[l][kd] == "0.0") continue;
            e = e.empty() ? fm[l][kd] : "(" + e + ") + (" + fm[l][kd] + ")";
        }
        w.line("a" + I(PL + l) + " = " + e + ";");
    }
    for (int i = PL - 1; i >= 1; --i) {
        zero[i] = zero[2 * i] && zero[2 * i + 1];
        if (zero[i]) continue;
        if (!zero[2 * i] && !zero[2 * i + 1]) w.line("a" + I(i) + " = a" + I(2 * i) + " + a" + I(2 * i + 1) + ";");
        else if (!zero[2 * i]) w.line("a" + I(i) + " = a" + I(2 * i) + ";");
        else w.line("a" + I(i) + " = a" + I(2 * i + 1) + ";");
    }
    if (zero[1]) w.line("a1 = 0.0;");
    w.line("}");
    w.end();
    }

    // local descent inside lane b, uniform branches; node values read with
    // readlane.  The recursion emits one block per internal node.
    w.begin("CWC_LOCAL_DESCEND(x, b, jl)");
    w.line("{");
    std::function<void(int, int)> emit = [&](int i, int depth) {
        std::string ind(2 * depth + 2, ' ');
        if (i >= PL) {
            w.line(ind + "(jl) = " + I(i - PL) + ";");
            return;
        }
        const int L = 2 * i, R = 2 * i + 1;
        if (zero[R]) {
            emit(L, depth + 1);
            return;
        }
        // x >= L and R != 0 in lane b are bit b of ballots of those
        // comparisons in every lane (x is the same in all lanes); L is read
        // from lane b only when the descent goes right
        if (zero[L]) {
            w.line(ind + "{ const unsigned long long nz_ = __ballot(a" + I(R) + " != 0.0);");
            w.line(ind + "if ((x) >= 0.0 && ((nz_ >> (b)) & 1ull)) {");
        } else {
            w.line(ind + "{ const unsigned long long ge_ = __ballot((x) >= a" + I(L) +
                   "), nz_ = __ballot(a" + I(R) + " != 0.0);");
            w.line(ind + "if (((ge_ & nz_) >> (b)) & 1ull) { (x) = (x) - cwc_rl(a" + I(L) + ", (b));");
        }
        emit(R, depth + 1);
        w.line(ind + "} else {");
        emit(L, depth + 1);
        w.line(ind + "} }");
    };
    emit(1, 0);
    w.line("}");
    w.end();

    // update: uniform switch over (kind, position)
    w.begin("CWC_APPLY(kind, pos, b, pb, lane, mypar, cap, ovf)");
    w.line("switch ((kind) * " + I(PL) + " + (pos)) {");
    for (size_t kd = 0; kd < kinds.size(); ++kd) {
        const int q = rep[kd];
        for (int l = 0; l < PL; ++l) {
            int si = f.leaf_slot[q * PL + l];
            if (si < 0) continue;
            const Slot &s = f.slots[si];
            w.line("case " + I((int)kd * PL + l) + ": {");
            w.line("  bool o_ = false;");
            // new values and overflow checks, owner lanes only
            for (auto &dv : s.delta) {
                const int cell = dv.first, d = dv.second;
                std::string v = var_of(q, cell);
                std::string role = (v[1] == 'p') ? "(pb)" : "(b)";
                std::string own = (v[1] == 'p') ? "nc" + v.substr(2) : v;
                if (d > 0)
                    w.line("  if ((lane) == " + role + ") o_ = o_ || ((unsigned)" + own + " + " +
                           I(d) + "u > (cap));");
            }
            w.line("  (ovf) = __any(o_);");
            w.line("  if (!(ovf)) {");
            for (auto &dv : s.delta) {
                const int cell = dv.first, d = dv.second;
                std::string v = var_of(q, cell);
                const bool wrap = v[1] == 'w';
                const std::string sp = v.substr(2);
                std::string role = (v[1] == 'p') ? "(pb)" : "(b)";
                if (wrap) {
                    w.line("    if ((lane) == " + role + ") nw" + sp + " += " + I(d) + ";");
                } else {
                    w.line("    if ((lane) == " + role + ") nc" + sp + " += " + I(d) + ";");
                    w.line("    if ((mypar) == " + role + ") np" + sp + " += " + I(d) + ";");
                }
            }
            w.line("  }");
            w.line("  break; }");
        }
    }
    w.line("default: (ovf) = false; break;");
    w.line("}");
    w.end();
    return o.str();
}

}  // namespace cwc
