// Mutation test of the host mechanism readers (native, CHEMKIN, OpenFOAM):
// every mutated file must give 0 or one of the documented error codes, never a
// crash; built with the host address and undefined-behaviour sanitizers by
// tests/test_readers_fuzz.py.  Usage: readers_fuzz <kind> <file> [<thermo>]
// <seed> <count> <tmpdir>, kind = native | chemkin | openfoam.
#include <cstdio>
#include <fstream>
#include <random>
#include <sstream>
#include <string>

#include "../include/chem.h"
#include "../paper_2508_16105_amd/csrc/mechanism.hpp"

static std::string slurp(const std::string& p)
{
    std::ifstream in(p);
    std::stringstream ss;
    ss << in.rdbuf();
    return ss.str();
}

static std::string mutate(std::string s, std::mt19937& rng)
{
    std::uniform_int_distribution<int> op(0, 6);
    const int nops = 1 + (int)(rng() % 4);
    for (int k = 0; k < nops && !s.empty(); ++k) {
        const size_t at = rng() % s.size();
        switch (op(rng)) {
        case 0: s.resize(at); break;                                           // truncate
        case 1: s.erase(at, 1 + rng() % 40); break;                            // delete a span
        case 2: s.insert(at, std::string(1, " \n/(){};=+!#-.0123456789eEDM"[rng() % 27])); break;
        case 3: s[at] = (char)(32 + rng() % 95); break;                        // overwrite a byte
        case 4: {                                                              // duplicate a line
            const size_t a = s.rfind('\n', at), b = s.find('\n', at);
            if (a != std::string::npos && b != std::string::npos) s.insert(b, s.substr(a, b - a));
            break;
        }
        case 5: s.insert(at, "1e308 -1e308 nan inf 0 "); break;                // extreme numbers
        default: {                                                             // drop a line
            const size_t a = s.rfind('\n', at), b = s.find('\n', at);
            if (a != std::string::npos && b != std::string::npos) s.erase(a, b - a);
        }
        }
    }
    return s;
}

int main(int argc, char** argv)
{
    if (argc < 6) return 2;
    const std::string kind = argv[1];
    const bool two = kind == "openfoam" || (kind == "chemkin" && argc == 7);
    const std::string file = argv[2], thermo = two ? argv[3] : "";
    const int a0 = two ? 4 : 3;
    const unsigned seed = (unsigned)std::stoul(argv[a0]);
    const int count = std::stoi(argv[a0 + 1]);
    const std::string tmp = argv[a0 + 2];
    const std::string base = slurp(file), tbase = two ? slurp(thermo) : "";
    std::mt19937 rng(seed);
    int ok = 0, errors = 0;
    for (int i = 0; i < count; ++i) {
        const bool on_thermo = two && (rng() % 3 == 0);
        const std::string mf = tmp + "/m.txt", tf = tmp + "/t.txt";
        std::ofstream(mf) << (on_thermo ? base : mutate(base, rng));
        if (two) std::ofstream(tf) << (on_thermo ? mutate(tbase, rng) : tbase);
        chemmi::MechanismData m;
        std::string err;
        int rc;
        if (kind == "native") rc = chemmi::parse_mechanism(mf, m, err);
        else if (kind == "chemkin") rc = chemmi::parse_chemkin(mf, two ? tf : "", m, err);
        else rc = chemmi::parse_openfoam(mf, tf, m, err);
        if (rc == 0) ++ok;
        else if (rc == CHEM_E_INVAL || rc == CHEM_E_PARSE || rc == CHEM_E_MECH_INVALID || rc == CHEM_E_UNSUPPORTED)
            ++errors;
        else {
            std::printf("unexpected code %d (%s) at mutation %d\n", rc, err.c_str(), i);
            return 1;
        }
        if (rc != 0 && err.empty()) {
            std::printf("error %d without a message at mutation %d\n", rc, i);
            return 1;
        }
    }
    std::printf("%d loaded, %d refused\n", ok, errors);
    return 0;
}
