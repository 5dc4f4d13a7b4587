// Batched mixed-precision path (n x B FP32 block).
#include "ppr_internal.h"

namespace ppr {

void run_mixed_batch(Graph& g, const int32_t* sources, int32_t B, double alpha, double lambda,
                     const ppr_options& opt, double* pi_out, double* r_out, ppr_stats* st) {
    (void)g; (void)sources; (void)B; (void)alpha; (void)lambda; (void)opt; (void)pi_out; (void)r_out; (void)st;
    fail(PPR_ERR_ARG, "PPR_MIXED is not available in this build");
}

}  // namespace ppr
