// mechanism.hpp -- host representation of a reaction mechanism read from a
// `chemmi-mech 1` file or a CHEMKIN-format file: species with NASA-7 thermo,
// reversible or irreversible reactions with modified-Arrhenius rates,
// third-body efficiencies, Lindemann/Troe/SRI falloff and pressure-tabulated
// (PLOG) rates (the "reactions and thermo data" of the detailed-chemistry
// model, Sec. 2.1).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace chemmi {

constexpr double kRu = 8.314462618;      // J/(mol K)
constexpr double kPatm = 101325.0;       // Pa, standard state of the equilibrium constants
constexpr size_t kMaxPlog = 16;          // pressures of one PLOG rate

enum class RxnKind { Elementary, ThirdBody, Lindemann, Troe, Sri, Plog };

inline bool is_falloff(RxnKind k) { return k == RxnKind::Lindemann || k == RxnKind::Troe || k == RxnKind::Sri; }

// One pressure of a PLOG rate: ln p (p in Pa) and the Arrhenius set there.
struct PlogEntry {
    double lnp, lnA, b, EaR;
}; 

struct SpeciesData {
    std::string name;
    std::vector<int> atoms;              // per element
    double W = 0.0;                      // kg/mol
    double tmid = 1000.0;
    double lo[7] = {0}, hi[7] = {0};     // NASA-7, T < tmid and T >= tmid
    bool has_thermo = false;
};

struct Term {
    int sp;
    int nu;
};

struct ReactionData {
    RxnKind kind = RxnKind::Elementary;
    std::vector<Term> reac, prod;
    int dnu = 0;                         // sum nu'' - sum nu'
    double lnA = 0.0, b = 0.0, EaR = 0.0; // main rate, SI, Ea/R in K
    double lnA0 = 0.0, b0 = 0.0, EaR0 = 0.0;   // low-pressure limit (falloff)
    double alpha = 0.0, T3 = 1.0, T1 = 1.0, T2 = 0.0;
    bool has_T2 = false;
    double sri[5] = {0.0, 0.0, 1.0, 1.0, 0.0};  // SRI a, b (K), c (K), d, e
    std::vector<PlogEntry> plog;         // increasing pressure; the main rate multiplies it
    bool reversible = true;
    std::vector<double> eff;             // per species (third-body and falloff)
};

struct MechanismData {
    std::string name;
    std::vector<std::string> elements;
    std::vector<double> element_w;       // g/mol
    std::vector<SpeciesData> species;
    std::vector<ReactionData> reactions;
    int ns() const { return (int)species.size(); }
    int nr() const { return (int)reactions.size(); }
};

// Parse and validate.  Returns 0, or a negative chem error code with `err` set.
int parse_mechanism(const std::string& path, MechanismData& out, std::string& err);

// Read a CHEMKIN-format mechanism (ELEMENTS, SPECIES, THERMO, REACTIONS),
// with the thermo data in the same file or in `thermo_path` (may be empty).
int parse_chemkin(const std::string& path, const std::string& thermo_path, MechanismData& out,
                  std::string& err);

// Read an OpenFOAM chemistry dictionary pair: the `reactions` file (species
// list, reactions dictionary) and the `thermo` file (molWeight, janaf NASA-7
// coefficients, element counts per species).
int parse_openfoam(const std::string& reactions_path, const std::string& thermo_path, MechanismData& out,
                   std::string& err);

// Checks shared by the readers once everything is read: species present, each
// with thermo data, and within CHEM_MAX_SPECIES.
int validate_mechanism(MechanismData& m, std::string& err);

// Arrhenius parameters in the layout the kernels read: lnA[nr], b[nr], EaR[nr].
std::vector<double> pack_params(const MechanismData& m);

}  // namespace chemmi
