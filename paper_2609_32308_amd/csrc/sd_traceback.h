// Canonical traceback interface (host replay over completed tables copied from the device).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sd_lattice.h"

namespace sd {

struct TraceTables {
    std::vector<int64_t> V, B, S1, S2, X;  // row layout (V: 6 per cell)
    std::vector<int> ccnt, cc;              // candidate segments (cc < 0: non-strict entry)
};

struct TraceResult {
    std::string mrna, structure;
    int32_t energy = 0;
    int64_t path_u = 0;
    double codon_cost = 0.0;
    bool ok = false;
};

int trace_design(const Lattice& L, const Params& P, const TraceTables& T, TraceResult& R);

}  // namespace sd
