// codegen.hpp -- mechanism-specific device source generation.
#pragma once

#include <string>

#include "mechanism.hpp"

namespace chemmi {

// HIP source of namespace mech { NS, NR, N, rhs(), rhs_jac(), jtv_param() } for
// m: straight-line code for the one-cell-per-lane kernels.
std::string generate_mechanism_source(const MechanismData& m);

// Layout of the wave-cooperative form: G lanes per cell (a power of two >= n),
// and the per-cell LDS scratch in doubles.
struct WideLayout {
    int G = 64;
    int maxt = 1;          // most terms on one side of a reaction
    int nslot = 2;         // species partial slots per reaction (2 maxt)
    int pw = 4;            // doubles per reaction in the partials block
    int jw = 1;            // row stride of the concentration Jacobian (odd)
    int l_y = 0, l_c = 0, l_g = 0, l_h = 0, l_q = 0, l_p = 0, l_j = 0, l_t0 = 0, l_w = 0;
    int lds_cell = 0;      // doubles per cell
    int adj_lds_cell = 0;  // doubles per cell in the adjoint: the scratch for dual numbers,
                           // then the pivot row and indices (untouched by source evaluations)
    int cells_per_wave() const { return 64 / G; }
    unsigned lds_bytes() const { return (unsigned)(cells_per_wave() * lds_cell * sizeof(double)); }
    unsigned adj_lds_bytes() const { return (unsigned)(cells_per_wave() * adj_lds_cell * sizeof(double)); }
};

// The layout for m, or an empty optional-like result (G = 0) if m does not
// fit the form (n > 64, or more than 3 terms on a reaction side).
WideLayout wide_layout(const MechanismData& m);

// HIP source of namespace mech for the wave-cooperative kernels: sizes,
// layout constants and the thermo, reaction and species tables they read.
std::string generate_wide_source(const MechanismData& m, const WideLayout& w);

}  // namespace chemmi
