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
//   draw:  Philox4x32-10, 10 rounds x (2 wide multiplies [4 each], 4 xor,
//          2 key adds) = 140; two 53-bit uniforms 14; ssa_log 45 (split,
//          fold, atanh series of 11 terms, one division); tau = -l/a0 and
//          t + tau 15; one sample-time compare 1                     = 215
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
    double fixed = 215.0 + 1.0 + 5.0 * D;
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
    // node is picked from the level-(d+1) nodes by halving them with the
    // decisions already taken (most significant first), so no value is
    // ever picked with a lane-varying index and the temporaries of one
    // level die before the next level starts.
    w.begin("CWC_DESCEND(x, j)");
    w.line("{");
    w.line("int jj_ = 0;");
    std::vector<std::string> bits;   // decision of each depth ("" = constant false)
    int tmp = 0;
    for (int d = 0; d < D; ++d) {
        std::vector<std::string> vals;
        for (int m = 0; m < (2 << d); ++m) vals.push_back(val((2 << d) + m));
        for (int q = 0; q < d; ++q) {
            const size_t half = vals.size() / 2;
            std::vector<std::string> nv(half);
            for (size_t m = 0; m < half; ++m) {
                const std::string &A = vals[m + half], &B = vals[m];
                if (bits[q].empty() || A == B) {
                    nv[m] = B;
                } else {
                    const std::string t = "t" + I(tmp++) + "_";
                    w.line("const double " + t + " = " + bits[q] + " ? " + A + " : " + B + ";");
                    nv[m] = t;
                }
            }
            vals = nv;
        }
        const std::string L = vals[0], R = vals[1];
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

    // --- net change of the chosen leaf, branch-free: for every cell and
    // every binary digit b of the |change| values it receives, a P-bit mask
    // of the leaves whose change has that digit (one mask for increases,
    // one for decreases), so d = sum_b ((M+_b >> j) & 1) << b - (...).
    // Nothing is written if any count would exceed the cap.
    std::vector<std::vector<std::pair<int, int>>> per_cell(C);   // (leaf, delta)
    for (auto &s : f.slots)
        for (auto &dv : s.delta) per_cell[dv.first].push_back({s.leaf, dv.second});
    const bool wide = P > 32;
    auto mask_lit = [&](unsigned long long m) {
        char b[40];
        std::snprintf(b, sizeof b, wide ? "0x%llxull" : "0x%llxu", m);
        return std::string(b);
    };
    w.begin("CWC_APPLY(j, cap, ovf)");
    w.line("{");
    w.line("bool o_ = false;");
    w.line(wide ? "const unsigned js_ = (unsigned)(j);" : "const unsigned js_ = (unsigned)(j);");
    for (int c = 0; c < C; ++c) {
        if (per_cell[c].empty()) continue;
        bool pos = false;
        std::string e = "(unsigned)n" + I(c);
        for (int sign = 1; sign >= -1; sign -= 2) {
            for (int b = 0; b < 21; ++b) {
                unsigned long long m = 0;
                for (auto &ld : per_cell[c]) {
                    int v = ld.second * sign;
                    if (v > 0 && ((v >> b) & 1)) m |= 1ull << ld.first;
                }
                if (!m) continue;
                if (sign > 0) pos = true;
                std::string bit = wide ? "(unsigned)((" + mask_lit(m) + " >> js_) & 1ull)"
                                       : "((" + mask_lit(m) + " >> js_) & 1u)";
                if (b) bit = "(" + bit + " << " + I(b) + ")";
                e += (sign > 0 ? " + " : " - ") + bit;
            }
        }
        w.line("const unsigned v" + I(c) + "_ = " + e + ";");
        if (pos) w.line("o_ = o_ || (v" + I(c) + "_ > (cap));");
    }
    w.line("if (!o_) {");
    for (int c = 0; c < C; ++c)
        if (!per_cell[c].empty()) w.line("    n" + I(c) + " = (int)v" + I(c) + "_;");
    w.line("}");
    w.line("(ovf) = o_;");
    w.line("}");
    w.end();

    // --- stage the counts for the on-line reduction (see CWC_EMIT)
    w.begin("CWC_STAGE(ptr, stride)");
    for (int c = 0; c < C; ++c) w.line("(ptr)[" + I(c) + " * (stride)] = n" + I(c) + ";");
    w.end();
    return o.str();
}

}  // namespace cwc
