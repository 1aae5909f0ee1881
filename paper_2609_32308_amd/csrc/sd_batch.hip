// Batched designs.
#include <hip/hip_runtime.h>
#include <string.h>

#include "sd_device.h"

namespace sd {
sd_status design_plain_entry(sd_context* c, const char* protein, const sd_codon_table* table,
                             const sd_params* params, double lambda, sd_result* out);
}

sd_status design_batch_impl(sd_context* ctx, int n, const char* const* proteins,
                            const double* lambdas, const sd_codon_table* table,
                            const sd_params* params, sd_result* outs) {
    if (!ctx || n < 0 || (n > 0 && (!proteins || !lambdas || !outs))) return SD_E_ARG;
    for (int i = 0; i < n; i++) {
        sd_status s = sd_design(ctx, proteins[i], table, params, lambdas[i], &outs[i]);
        if (s) {
            for (int j = 0; j < i; j++) sd_result_free(&outs[j]);
            return s;
        }
    }
    return SD_OK;
}
