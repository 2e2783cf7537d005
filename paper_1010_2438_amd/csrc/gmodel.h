// General CWC models (compartments created, dissolved and deleted at run
// time; patterns two levels deep): host-side validation and the model
// header of the general engine (engine_gen.h).
#ifndef CWC_GMODEL_H
#define CWC_GMODEL_H

#include <string>
#include <vector>

#include "../../include/cwcssa.h"
#include "model.h"

namespace cwc {

struct GFlat {
    int n_species = 0, n_labels = 0, max_comp = 0, n_init = 0, n_rules = 0;
    std::vector<int> has_wrap;                            // [labels]
    std::vector<int> init_label, init_parent;             // [n_init]
    std::vector<int> init_wrap, init_content;             // [n_init][NS]
    std::vector<int> depth, labels;                       // [R], [R][3]
    std::vector<int> lhs, delta;                          // [R][5][NS]
    std::vector<int> action, level, new_label, release;   // [R]
    std::vector<int> new_wrap, new_content;               // [R][NS]
    std::vector<double> k;                                // [R]
    int p_local = 1, p_slots = 1, n_obs = 0;
    std::vector<int> rule_at;                             // [labels][p_local]
};

cwc_status gflatten(const cwc_gmodel_desc *d, GFlat *out, std::string *err);
void gflat_to_flat(const GFlat &g, Flat *f);
std::string codegen_gen(const GFlat &g);
double galgorithmic_slots_per_event(const GFlat &g);

}  // namespace cwc
#endif
