// Results of the device traceback and their host-side completion.
#pragma once
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "sd_lattice.h"
#include "sd_trace_status.h"

namespace sd {

// Views of a design's tables copied to the host in the row layout (V: 6 per cell; candidate
// segments with cc < 0 for non-strict entries).  Only the dense-table test hooks download them;
// a design itself never copies its tables back.
struct TraceTables {
    const int64_t *V = nullptr, *B = nullptr, *S1 = nullptr, *S2 = nullptr, *X = nullptr;
    const int64_t* G = nullptr;  // gap table (generic lattices only)
    const int *ccnt = nullptr, *cc = nullptr;
    std::unique_ptr<char[]> own;
};

// What the device traceback leaves for the host (O(n + N) values): the base at every position
// (-1 if none was emitted), the partner of every position (-1 unpaired), the energy and path
// cost it summed, its status, X(s), and the strict candidates per right endpoint.
struct TraceOut {
    std::vector<int32_t> seq, pair, counts;
    int64_t energy = 0, path_u = 0, status = 0, xs = 0;
};

struct TraceResult {
    std::string mrna, structure;
    int32_t energy = 0;
    int64_t path_u = 0;
    double codon_cost = 0.0;
    bool ok = false;
};

// Builds the strings and checks the design exactly: the emitted bases spell a complete path
// s -> t of the automaton, its rounded costs sum to the traceback's path cost, and
// E * 2^s + path cost equals X(s).  SD_E_INTERNAL if any check fails; *why (if given) then
// names the check.
int finish_trace(const Lattice& L, const TraceOut& T, TraceResult& R, std::string* why = nullptr);

}  // namespace sd
