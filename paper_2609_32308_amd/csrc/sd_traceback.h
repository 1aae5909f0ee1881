// Canonical traceback interface (host replay over completed tables copied from the device).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "sd_lattice.h"

namespace sd {

// Views of the downloaded tables (row layout, V: 6 per cell; candidate segments with cc < 0
// for non-strict entries).  The memory is either the context's pinned download buffer (valid
// until the context's next download) or owned by `own`.
struct TraceTables {
    const int64_t *V = nullptr, *B = nullptr, *S1 = nullptr, *S2 = nullptr, *X = nullptr;
    const int64_t* G = nullptr;  // gap table (generic lattices only)
    const int *ccnt = nullptr, *cc = nullptr;
    std::unique_ptr<char[]> own;
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
