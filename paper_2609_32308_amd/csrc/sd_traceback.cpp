// Host completion of the device traceback (k_trace in sd_trace.hip): strings, codon cost and the
// exact self-check of Sec. 7.1 (the DP value at the source equals the design's energy in fixed
// point plus its rounded codon costs).
#include "sd_traceback.h"

#include "../../include/sparsedesign.h"

namespace sd {

int finish_trace(const Lattice& L, const TraceOut& T, TraceResult& R, std::string* why) {
    std::string reason;
    bool ok = true;
    if (T.status != kTrOk) {
        static const char* const names[] = {"failed", "ok", "no alternative matched a stored value",
                                            "a position emitted twice", "a frame-stack wait timed out",
                                            "a deferred frame outside the design", "frame stack overflow",
                                            "X(s) is infinite"};
        const int k = T.status >= 0 && T.status <= 7 ? (int)T.status : 0;
        reason = "device traceback status " + std::to_string(T.status) + " (" + names[k] + ")";
        ok = false;
    } else if ((int)T.seq.size() != L.n || (int)T.pair.size() != L.n) {
        reason = "result arrays of the wrong length";
        ok = false;
    }
    int st = 0;
    int64_t Uw = 0;
    double C = 0.0;
    for (int i = 0; i < L.n && ok; i++) {
        const int x = T.seq[i];
        if (x < 0 || x > 3) {
            reason = "no base emitted at position " + std::to_string(i);
            ok = false;
            break;
        }
        const int e = st * 4 + x;
        if (L.out_dst[e] < 0) {
            reason = "the base at position " + std::to_string(i) + " leaves the automaton";
            ok = false;
            break;
        }
        Uw += L.out_U[e];
        if (L.out_cod[e] >= 0) C += L.out_q[e];
        st = L.out_dst[e];
    }
    if (ok && L.layer[st] != L.n) {
        reason = "the path does not end in the last layer";
        ok = false;
    }
    if (ok && Uw != T.path_u) {
        reason = "path costs sum to " + std::to_string(Uw) + ", the traceback summed " + std::to_string(T.path_u);
        ok = false;
    }
    if (ok && T.energy * ((int64_t)1 << L.shift) + T.path_u != T.xs) {
        reason = "E * 2^s + path cost differs from X(s)";
        ok = false;
    }
    // pairs are mutual
    for (int i = 0; i < L.n && ok; i++) {
        const int j = T.pair[i];
        if (j >= 0 && (j >= L.n || T.pair[j] != i)) {
            reason = "the partner of position " + std::to_string(i) + " is not mutual";
            ok = false;
        }
    }
    R.mrna.assign(L.n, 'N');
    R.structure.assign(L.n, '.');
    for (int i = 0; i < L.n && i < (int)T.seq.size(); i++) {
        if (T.seq[i] >= 0 && T.seq[i] < 4) R.mrna[i] = "ACGU"[T.seq[i]];
        if (T.pair[i] >= 0) R.structure[i] = T.pair[i] > i ? '(' : ')';
    }
    R.energy = (int32_t)T.energy;
    R.path_u = T.path_u;
    R.codon_cost = C;
    R.ok = ok;
    if (why) *why = reason;
    return ok ? SD_OK : SD_E_INTERNAL;
}

}  // namespace sd
