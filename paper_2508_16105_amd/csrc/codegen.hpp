// codegen.hpp -- mechanism-specific device source generation.
#pragma once

#include <string>

#include "mechanism.hpp"

namespace chemmi {

// HIP source of namespace mech { NS, NR, N, rhs(), rhs_jac() } for m.
std::string generate_mechanism_source(const MechanismData& m);

}  // namespace chemmi
