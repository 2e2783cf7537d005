// Host-side model compilation: validation of a cwc_model_desc, flattening
// of the fixed compartment tree into rule/context slots and leaf layout,
// and generation of the model-specific device code.
#ifndef CWC_MODEL_H
#define CWC_MODEL_H

#include <string>
#include <utility>
#include <vector>

#include "../../include/cwcssa.h"

// LDS a lane-layout kernel may use statically for its per-leaf change
// table in the byte layout, and a pair- or quad-layout kernel for its
// per-lane table; the host keeps the largest, with the resident kernels'
// parameter copies, out of the dynamic LDS it gives a block.
constexpr size_t kLaneStaticLdsBytes = 64 * 8;
constexpr size_t kPairStaticLdsBytes = 2 * 64 * 8;
constexpr size_t kQuadStaticLdsBytes = 4 * 64 * 8;

namespace cwc {

struct Slot {
    int rule = -1;        // rule index
    int ctx = -1;         // context compartment
    int leaf = -1;        // leaf index = ctx * p_local + position
    int n_react = 0;      // reactant terms (<= 2)
    int react_cell[2] = {0, 0};
    int react_mult[2] = {0, 0};
    std::vector<std::pair<int, int>> delta;   // (cell, net change), cell-sorted
};

struct Flat {
    int n_species = 0, n_types = 0, n_comp = 0, n_rules = 0;
    int n_cells = 0;
    std::vector<int> comp_type, comp_parent, has_wrap;
    std::vector<int> content_base, wrap_base;     // per compartment, -1 = none
    std::vector<int> init;                        // [n_cells]
    std::vector<double> k;                        // [n_rules]
    int p_local = 1, p_comp = 1, n_leaves = 1;
    std::vector<Slot> slots;                      // context-major order
    std::vector<int> leaf_slot;                   // [n_leaves] slot or -1
    int layout = 0;                               // 0 lane, 1 wave
};

// Returns CWC_OK or an error code with *err set.
cwc_status flatten(const cwc_model_desc *d, Flat *out, std::string *err);

// Algorithmic VALU issue slots per applied event of the direct method on
// this model (see model.cpp); the roofline's work unit.
double algorithmic_slots_per_event(const Flat &f);

// Device source of the model section for the given layout (to be followed
// by the engine source).
std::string codegen_lane(const Flat &f);
std::string codegen_wave(const Flat &f);

// Layout the library picks for a flattened model: 0 = lane per replica
// (all state of a trajectory in one lane's registers), 1 = wavefront per
// replica (lane q owns compartment q), -1 = neither fits.
int choose_layout(const Flat &f);
bool fits_lane(const Flat &f);
bool fits_wave(const Flat &f);

}  // namespace cwc
#endif
