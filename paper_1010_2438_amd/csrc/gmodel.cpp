// General CWC models (paper Sec. 2.1): validation of a cwc_gmodel_desc and
// the model header of the general engine (engine_gen.h).
//
// The term is a pool of compartment slots: the initial compartments take
// slots 0.. in preorder (slot 0 the top level), later ones the lowest free
// slot.  A rule names its context label and optionally a child and a
// grandchild compartment label; its *anchor* is the deepest compartment it
// names, so each slot holds one match per rule anchored at its label.  The
// leaf array is slot-major: the block of a slot lists the rules anchored at
// its label in ascending rule index, padded to G_PL = next power of two of
// the longest such list; slots are padded to a power of two.  Everything
// the engine needs about the model is written as compile-time tables, so
// the engine's per-rule code is specialised per model by the compiler.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "gmodel.h"

namespace cwc {

namespace {

int next_pow2(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

int log2i(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

cwc_status bad(std::string *err, cwc_status code, const std::string &msg)
{
    *err = msg;
    return code;
}

}  // namespace

cwc_status gflatten(const cwc_gmodel_desc *d, GFlat *g, std::string *err)
{
    if (!d) return bad(err, CWC_E_INVALID, "null model descriptor");
    const int NS = d->n_species, NL = d->n_labels;
    if (NS < 1 || NS > 32) return bad(err, CWC_E_INVALID, "n_species must be in [1, 32]");
    if (NL < 1 || NL > 16) return bad(err, CWC_E_INVALID, "n_labels must be in [1, 16]");
    if (d->max_comp < 1 || d->max_comp > 64)
        return bad(err, CWC_E_UNSUPPORTED, "max_comp must be in [1, 64] (one wavefront lane per slot)");
    if (d->n_comp < 1 || d->n_comp > d->max_comp)
        return bad(err, CWC_E_INVALID, "the initial term needs 1..max_comp compartments");
    if (d->n_rules < 0 || d->n_rules > 64) return bad(err, CWC_E_UNSUPPORTED, "at most 64 rules");
    if (!d->has_wrap || !d->comps || (d->n_rules > 0 && !d->rules))
        return bad(err, CWC_E_INVALID, "null array in the model descriptor");
    g->n_species = NS;
    g->n_labels = NL;
    g->max_comp = d->max_comp;
    g->has_wrap.assign(d->has_wrap, d->has_wrap + NL);
    for (int &w : g->has_wrap) w = w ? 1 : 0;
    g->n_init = d->n_comp;
    g->init_label.resize(d->n_comp);
    g->init_parent.resize(d->n_comp);
    g->init_wrap.assign((size_t)d->n_comp * NS, 0);
    g->init_content.assign((size_t)d->n_comp * NS, 0);
    for (int i = 0; i < d->n_comp; ++i) {
        const cwc_gcomp &c = d->comps[i];
        if (c.label < 0 || c.label >= NL) return bad(err, CWC_E_INVALID, "compartment label out of range");
        if (i == 0 ? c.parent != -1 : (c.parent < 0 || c.parent >= i))
            return bad(err, CWC_E_INVALID, "compartments must be in preorder, the top level first");
        g->init_label[i] = c.label;
        g->init_parent[i] = c.parent;
        for (int a = 0; a < NS; ++a) {
            const int w = c.wrap ? c.wrap[a] : 0, x = c.content ? c.content[a] : 0;
            if (w < 0 || x < 0) return bad(err, CWC_E_INVALID, "negative initial count");
            if (w && !g->has_wrap[c.label])
                return bad(err, CWC_E_INVALID, "wrap atoms on a label without a wrap");
            g->init_wrap[(size_t)i * NS + a] = w;
            g->init_content[(size_t)i * NS + a] = x;
        }
    }
    const int R = d->n_rules;
    g->n_rules = R;
    g->depth.assign(R, 0);
    g->labels.assign((size_t)R * 3, -1);
    g->lhs.assign((size_t)R * 5 * NS, 0);
    g->delta.assign((size_t)R * 5 * NS, 0);
    g->action.assign(R, CWC_ACT_NONE);
    g->level.assign(R, 0);
    g->new_label.assign(R, -1);
    g->new_wrap.assign((size_t)R * NS, 0);
    g->new_content.assign((size_t)R * NS, 0);
    g->release.assign(R, 0);
    g->k.assign(R, 0.0);
    for (int r = 0; r < R; ++r) {
        const cwc_grule &u = d->rules[r];
        char where[32];
        std::snprintf(where, sizeof where, "rule %d: ", r);
        const std::string W = where;
        const int dep = u.child < 0 ? 0 : (u.grandchild < 0 ? 1 : 2);
        const int lab[3] = {u.context, u.child, u.grandchild};
        for (int l = 0; l <= dep; ++l)
            if (lab[l] < 0 || lab[l] >= NL) return bad(err, CWC_E_INVALID, W + "label out of range");
        if (!(std::isfinite(u.k) && u.k > 0.0 && u.k <= 1e250))
            return bad(err, CWC_E_INVALID, W + "k must be finite and > 0");
        g->depth[r] = dep;
        for (int l = 0; l < 3; ++l) g->labels[(size_t)r * 3 + l] = l <= dep ? lab[l] : -1;
        g->k[r] = u.k;
        int order = 0;
        auto terms = [&](int n, const cwc_term *t, int sign) -> cwc_status {
            if (n < 0 || (n > 0 && !t)) return bad(err, CWC_E_INVALID, W + "bad term list");
            for (int i = 0; i < n; ++i) {
                const int q = t[i].region, a = t[i].species, m = t[i].mult;
                if (q < 0 || q > 2 * dep) return bad(err, CWC_E_INVALID, W + "region beyond the pattern's depth");
                if (a < 0 || a >= NS || m < 0) return bad(err, CWC_E_INVALID, W + "bad atom or multiplicity");
                if ((q == 1 || q == 3) && !g->has_wrap[lab[(q + 1) / 2]])
                    return bad(err, CWC_E_INVALID, W + "wrap region of a label without a wrap");
                g->delta[((size_t)r * 5 + q) * NS + a] += sign * m;
                if (sign < 0) {
                    g->lhs[((size_t)r * 5 + q) * NS + a] += m;
                    order += m;
                }
            }
            return CWC_OK;
        };
        cwc_status st = terms(u.n_lhs, u.lhs, -1);
        if (st != CWC_OK) return st;
        st = terms(u.n_rhs, u.rhs, +1);
        if (st != CWC_OK) return st;
        for (int i = 0; i < 5 * NS; ++i)
            if (g->lhs[(size_t)r * 5 * NS + i] > 2)
                return bad(err, CWC_E_UNSUPPORTED, W + "an atom with multiplicity above 2");
        if (order > 2) return bad(err, CWC_E_UNSUPPORTED, W + "total reactant order above 2");
        const int act = u.action, lv = u.level;
        g->action[r] = act;
        g->level[r] = lv;
        if (act == CWC_ACT_CREATE) {
            if (lv < 0 || lv > dep) return bad(err, CWC_E_INVALID, W + "creates below its pattern");
            if (u.new_label < 0 || u.new_label >= NL) return bad(err, CWC_E_INVALID, W + "new label out of range");
            g->new_label[r] = u.new_label;
            for (int a = 0; a < NS; ++a) {
                const int w = u.new_wrap ? u.new_wrap[a] : 0, x = u.new_content ? u.new_content[a] : 0;
                if (w < 0 || x < 0) return bad(err, CWC_E_INVALID, W + "negative count in the new compartment");
                if (w && !g->has_wrap[u.new_label])
                    return bad(err, CWC_E_INVALID, W + "wrap atoms on a label without a wrap");
                g->new_wrap[(size_t)r * NS + a] = w;
                g->new_content[(size_t)r * NS + a] = x;
            }
        } else if (act == CWC_ACT_DISSOLVE || act == CWC_ACT_DELETE) {
            if (lv < 1 || lv > dep)
                return bad(err, CWC_E_INVALID, W + "dissolves or deletes a compartment it does not name");
            g->release[r] = (act == CWC_ACT_DISSOLVE && u.release_wrap) ? 1 : 0;
        } else if (act != CWC_ACT_NONE) {
            return bad(err, CWC_E_INVALID, W + "unknown action");
        }
    }
    // leaf layout
    int longest = 1;
    g->rule_at.clear();
    std::vector<std::vector<int>> lists(NL);
    for (int r = 0; r < R; ++r) lists[g->labels[(size_t)r * 3 + g->depth[r]]].push_back(r);
    for (auto &l : lists) longest = std::max<int>(longest, (int)l.size());
    g->p_local = next_pow2(longest);
    g->p_slots = next_pow2(g->max_comp);
    g->rule_at.assign((size_t)NL * g->p_local, -1);
    for (int l = 0; l < NL; ++l)
        for (size_t i = 0; i < lists[l].size(); ++i) g->rule_at[(size_t)l * g->p_local + i] = lists[l][i];
    if (g->p_local > 64) return bad(err, CWC_E_UNSUPPORTED, "more than 64 rules anchored at one label");
    g->n_obs = 0;
    for (int l = 0; l < NL; ++l) g->n_obs += NS * (g->has_wrap[l] ? 2 : 1) + 1;
    return CWC_OK;
}

// Flat view for the run machinery: cells = observables, rules, k; the
// initial term lives in the generated code (init tables do not apply).
void gflat_to_flat(const GFlat &g, Flat *f)
{
    *f = Flat();
    f->n_species = g.n_species;
    f->n_types = g.n_labels;
    f->n_comp = g.n_init;
    f->n_rules = g.n_rules;
    f->n_cells = g.n_obs;
    f->k = g.k;
    f->init.assign(1, 0);
    f->p_local = g.p_local;
    f->p_comp = g.p_slots;
    f->n_leaves = g.p_local * g.p_slots;
    f->layout = 2;
}

std::string codegen_gen(const GFlat &g)
{
    std::ostringstream o;
    const int NS = g.n_species, NL = g.n_labels, R = std::max(1, g.n_rules);
    auto list = [&](const std::vector<int> &v, size_t from, size_t n) {
        std::string s = "{";
        for (size_t i = 0; i < n; ++i) s += (i ? "," : "") + std::to_string(i + from < v.size() ? v[from + i] : 0);
        return s + "}";
    };
    o << "// ---- generated model header (general CWC engine)\n";
    o << "#define G_NS " << NS << "\n#define G_NL " << NL << "\n#define G_NR " << g.n_rules
      << "\n#define G_MAXC " << g.max_comp << "\n#define G_NP " << g.p_slots << "\n#define G_LP "
      << log2i(g.p_slots) << "\n#define G_PL " << g.p_local << "\n#define G_LL "
      << log2i(g.p_local) << "\n#define G_NOBS " << g.n_obs << "\n#define G_NINIT " << g.n_init
      << "\n#define GEN_CREATE " << CWC_ACT_CREATE << "\n#define GEN_DISSOLVE "
      << CWC_ACT_DISSOLVE << "\n#define GEN_DELETE " << CWC_ACT_DELETE << "\n";
    o << "constexpr int g_rule_at[" << NL << "][" << g.p_local << "] = {";
    for (int l = 0; l < NL; ++l)
        o << (l ? "," : "") << list(g.rule_at, (size_t)l * g.p_local, g.p_local);
    o << "};\n";
    auto per_rule = [&](const char *name, const std::vector<int> &v) {
        o << "constexpr int " << name << "[" << R << "] = " << list(v, 0, R) << ";\n";
    };
    per_rule("g_depth", g.depth);
    per_rule("g_action", g.action);
    per_rule("g_level", g.level);
    per_rule("g_new_label", g.new_label);
    per_rule("g_release", g.release);
    o << "constexpr int g_lab[" << R << "][3] = {";
    for (int r = 0; r < R; ++r) o << (r ? "," : "") << list(g.labels, (size_t)r * 3, 3);
    o << "};\n";
    auto per_rule_reg = [&](const char *name, const std::vector<int> &v) {
        o << "constexpr int " << name << "[" << R << "][5][" << NS << "] = {";
        for (int r = 0; r < R; ++r) {
            o << (r ? "," : "") << "{";
            for (int q = 0; q < 5; ++q)
                o << (q ? "," : "") << list(v, ((size_t)r * 5 + q) * NS, NS);
            o << "}";
        }
        o << "};\n";
    };
    per_rule_reg("g_lhs", g.lhs);
    per_rule_reg("g_delta", g.delta);
    auto per_rule_sp = [&](const char *name, const std::vector<int> &v) {
        o << "constexpr int " << name << "[" << R << "][" << NS << "] = {";
        for (int r = 0; r < R; ++r) o << (r ? "," : "") << list(v, (size_t)r * NS, NS);
        o << "};\n";
    };
    per_rule_sp("g_new_wrap", g.new_wrap);
    per_rule_sp("g_new_content", g.new_content);
    o << "constexpr int g_has_wrap[" << NL << "] = " << list(g.has_wrap, 0, NL) << ";\n";
    // the initial term, read per lane at the start of each trajectory
    o << "__constant__ int g_init_label[" << g.n_init << "] = " << list(g.init_label, 0, g.n_init) << ";\n";
    o << "__constant__ int g_init_parent[" << g.n_init << "] = " << list(g.init_parent, 0, g.n_init) << ";\n";
    o << "__constant__ int g_init_wrap[" << g.n_init * NS << "] = "
      << list(g.init_wrap, 0, (size_t)g.n_init * NS) << ";\n";
    o << "__constant__ int g_init_content[" << g.n_init * NS << "] = "
      << list(g.init_content, 0, (size_t)g.n_init * NS) << ";\n";
    return o.str();
}

// Work of one applied event in VALU issue slots (the roofline's unit, as
// for fixed trees): the draw and time (195), selection over the slot and
// block levels, the rule's atom changes, and the re-evaluation of the
// anchored leaves whose counts changed (the product's factors) with their
// paths; structural actions touch a slot's row.
double galgorithmic_slots_per_event(const GFlat &g)
{
    const double levels = std::log2((double)g.p_local * g.p_slots);
    double upd = 0.0;
    for (int r = 0; r < g.n_rules; ++r) {
        int changed = 0;
        for (int i = 0; i < 5 * g.n_species; ++i) changed += g.delta[(size_t)r * 5 * g.n_species + i] != 0;
        upd += 2.0 * changed + (g.action[r] != CWC_ACT_NONE ? 2.0 * (3 + 2 * g.n_species) : 0.0);
    }
    if (g.n_rules) upd /= g.n_rules;
    return 195.0 + 1.0 + 5.0 * levels + upd + 4.0 + levels;
}

}  // namespace cwc
