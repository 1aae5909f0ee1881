// Supported lambda envelope of one protein.
//
// For fixed designs, F_i(lambda) = E_i / 100 + lambda * C_i is a line, and F*(lambda) of eq. 1 is
// the lower envelope of the lines of all designs; the designs that are optimal on some interval
// of lambda are the supported ones (the tools of Sec. 10 report them).  The search below is the
// exact dichotomic (parametric) method: with supported designs a and b optimal at lambda_a <
// lambda_b and C_a > C_b, their lines cross at lambda* = (E_b - E_a) / (100 (C_a - C_b)); the
// optimum at lambda* either lies on both lines (a and b are adjacent on the envelope) or
// strictly below them (a new supported design between a and b).  All open intervals of one
// level are evaluated together as one batched call.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sd_host.h"

using namespace sd;

namespace {

struct Point {
    double lambda;  // a lambda at which the design is optimal
    sd_result r;
};

double line(const sd_result& r, double lam) { return r.energy_centi / 100.0 + lam * r.codon_cost; }

bool same_design(const sd_result& a, const sd_result& b) {
    return a.energy_centi == b.energy_centi && fabs(a.codon_cost - b.codon_cost) <= 1e-12 * (1.0 + fabs(a.codon_cost));
}

}  // namespace

extern "C" sd_status sd_lambda_envelope(sd_context* ctx, const char* protein, double lambda_lo,
                                        double lambda_hi, int max_designs, const sd_codon_table* table,
                                        const sd_params* params, sd_result* outs, double* breaks,
                                        int* n_out) {
    try {
        if (!ctx || !protein || !table || !params || !outs || !breaks || !n_out || max_designs < 2)
            return fail(SD_E_ARG, "null argument or max_designs < 2");
        if (!(lambda_lo >= 0.0) || !(lambda_hi > lambda_lo) || !isfinite(lambda_hi))
            return fail(SD_E_LAMBDA, "need 0 <= lambda_lo < lambda_hi, finite");
        std::vector<Point> pts;  // supported designs found so far, in increasing lambda
        auto run = [&](const std::vector<double>& lams, std::vector<sd_result>& res) -> sd_status {
            std::vector<const char*> ps(lams.size(), protein);
            res.assign(lams.size(), sd_result{});
            return sd_design_batch(ctx, (int)lams.size(), ps.data(), lams.data(), table, params, res.data());
        };
        std::vector<sd_result> res;
        sd_status s = run({lambda_lo, lambda_hi}, res);
        if (s) return s;
        pts.push_back({lambda_lo, res[0]});
        if (same_design(res[0], res[1])) {
            sd_result_free(&res[1]);
        } else {
            pts.push_back({lambda_hi, res[1]});
        }
        // intervals (i, i+1) of pts still open
        std::vector<char> open(pts.size(), 1);
        for (;;) {
            std::vector<int> which;
            std::vector<double> lams;
            for (size_t i = 0; i + 1 < pts.size(); i++) {
                if (!open[i]) continue;
                const sd_result &a = pts[i].r, &b = pts[i + 1].r;
                const double dc = a.codon_cost - b.codon_cost;
                if (!(dc > 0.0)) {  // equal costs: the cheaper line dominates; nothing between
                    open[i] = 0;
                    continue;
                }
                const double ls = (b.energy_centi - a.energy_centi) / (100.0 * dc);
                if (!(ls > pts[i].lambda && ls < pts[i + 1].lambda)) {
                    open[i] = 0;
                    continue;
                }
                which.push_back((int)i);
                lams.push_back(ls);
            }
            if (which.empty() || (int)(pts.size() + which.size()) > max_designs) break;
            s = run(lams, res);
            if (s) {
                for (auto& p : pts) sd_result_free(&p.r);
                return s;
            }
            // merge: new supported designs strictly below both lines at the crossing
            std::vector<Point> np;
            std::vector<char> nopen;
            size_t k = 0;
            for (size_t i = 0; i < pts.size(); i++) {
                np.push_back(pts[i]);
                if (k < which.size() && which[k] == (int)i) {
                    const sd_result& d = res[k];
                    const double ls = lams[k], on = line(pts[i].r, ls);
                    const double tol = 1e-9 * (1.0 + fabs(on));
                    if (line(d, ls) < on - tol) {
                        nopen.push_back(1);
                        np.push_back({ls, d});
                        nopen.push_back(1);
                    } else {
                        sd_result_free(&res[k]);
                        nopen.push_back(0);  // a and b are adjacent on the envelope
                    }
                    k++;
                } else if (i + 1 < pts.size()) {
                    nopen.push_back(open[i]);
                }
            }
            pts.swap(np);
            open.swap(nopen);
            open.resize(pts.size(), 0);
        }
        // a design optimal only at an end point (a tie there, dominated inside the range) has an
        // empty interval: drop it
        auto cross = [&](size_t i) {
            const sd_result &a = pts[i].r, &b = pts[i + 1].r;
            return (b.energy_centi - a.energy_centi) / (100.0 * (a.codon_cost - b.codon_cost));
        };
        while (pts.size() >= 2 && cross(0) <= lambda_lo) {
            sd_result_free(&pts[0].r);
            pts.erase(pts.begin());
        }
        while (pts.size() >= 2 && cross(pts.size() - 2) >= lambda_hi) {
            sd_result_free(&pts.back().r);
            pts.pop_back();
        }
        // breakpoints: lambda_lo, the crossings of consecutive supported lines, lambda_hi
        const int m = (int)pts.size();
        breaks[0] = lambda_lo;
        for (int i = 0; i + 1 < m; i++) {
            const sd_result &a = pts[i].r, &b = pts[i + 1].r;
            breaks[i + 1] = (b.energy_centi - a.energy_centi) / (100.0 * (a.codon_cost - b.codon_cost));
        }
        breaks[m] = lambda_hi;
        for (int i = 0; i < m; i++) outs[i] = pts[i].r;
        *n_out = m;
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}

// Inverse lambda: the smallest lambda in [0, lambda_hi] at which a supported design reaches a
// target CAI.  The optimal codon cost is a non-increasing step function of lambda whose steps are
// the envelope's breakpoints, so the answer is the left breakpoint of the first supported design
// (in increasing lambda) whose CAI meets the target.
extern "C" sd_status sd_inverse_lambda(sd_context* ctx, const char* protein, double target_cai,
                                       double lambda_hi, int max_designs, const sd_codon_table* table,
                                       const sd_params* params, sd_result* out, double* lambda_out) {
    try {
        if (!ctx || !protein || !table || !params || !out || !lambda_out || max_designs < 2)
            return fail(SD_E_ARG, "null argument or max_designs < 2");
        if (!(target_cai > 0.0 && target_cai <= 1.0)) return fail(SD_E_ARG, "target CAI must lie in (0, 1]");
        std::vector<sd_result> outs(max_designs);
        std::vector<double> breaks(max_designs + 1);
        int m = 0;
        sd_status s = sd_lambda_envelope(ctx, protein, 0.0, lambda_hi, max_designs, table, params, outs.data(),
                                         breaks.data(), &m);
        if (s) return s;
        int pick = -1;
        for (int i = 0; i < m && pick < 0; i++)
            if (outs[i].cai >= target_cai * (1.0 - 1e-12)) pick = i;
        for (int i = 0; i < m; i++)
            if (i != pick) sd_result_free(&outs[i]);
        if (pick < 0) return fail(SD_E_INFEASIBLE, "no supported design on [0, lambda_hi] reaches the target CAI");
        *out = outs[pick];
        *lambda_out = breaks[pick];
        return SD_OK;
    } catch (const std::bad_alloc&) {
        return fail(SD_E_NOMEM, "host allocation");
    } catch (...) {
        return fail(SD_E_INTERNAL, "unexpected exception");
    }
}
