// Host completion of the device traceback (k_trace in sd_trace.hip): strings, codon cost and the
// exact self-check of Sec. 7.1 (the DP value at the source equals the design's energy in fixed
// point plus its rounded codon costs).
#include "sd_traceback.h"

#include "../../include/sparsedesign.h"

namespace sd {

int finish_trace(const Lattice& L, const TraceOut& T, TraceResult& R) {
    bool ok = T.status == 1 && (int)T.seq.size() == L.n && (int)T.pair.size() == L.n;
    int st = 0;
    int64_t Uw = 0;
    double C = 0.0;
    for (int i = 0; i < L.n && ok; i++) {
        const int x = T.seq[i];
        if (x < 0 || x > 3) {
            ok = false;
            break;
        }
        const int e = st * 4 + x;
        if (L.out_dst[e] < 0) {
            ok = false;
            break;
        }
        Uw += L.out_U[e];
        if (L.out_cod[e] >= 0) C += L.out_q[e];
        st = L.out_dst[e];
    }
    if (ok && L.layer[st] != L.n) ok = false;
    if (ok && (Uw != T.path_u || T.energy * ((int64_t)1 << L.shift) + T.path_u != T.xs)) ok = false;
    // pairs are mutual
    for (int i = 0; i < L.n && ok; i++) {
        const int j = T.pair[i];
        if (j >= 0 && (j >= L.n || T.pair[j] != i)) ok = false;
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
    return ok ? SD_OK : SD_E_INTERNAL;
}

}  // namespace sd
