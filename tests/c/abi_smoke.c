/* A plain C99 caller of libppr: builds the 5-node graph of Figure 1 from CSR,
 * asks one FP64 and one batched mixed query, and checks the results against
 * the values the paper prints for the Figure 1 example (pi_s for s = v1,
 * alpha = 0.2) and against each other.  Exit codes: 0 pass, 2 no GPU (the
 * library reported PPR_ERR_DEVICE), 1 failure. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ppr.h"

int main(void) {
    /* Figure 1: v1 -> v2, v3; v2 -> v1, v3, v4, v5; v3 -> v2, v4; v4 -> v1, v2, v3; v5 -> v2, v3 */
    const int64_t row_ptr[6] = {0, 2, 6, 8, 11, 13};
    const int32_t col[13] = {1, 2, 0, 2, 3, 4, 1, 3, 0, 1, 2, 1, 2};
    ppr_graph* g = NULL;
    ppr_status st = ppr_graph_create(row_ptr, col, 5, 13, 0, &g);
    if (st == PPR_ERR_DEVICE) {
        printf("no device: %s\n", ppr_last_error());
        return 2;
    }
    if (st != PPR_OK) {
        printf("create failed: %d %s\n", (int)st, ppr_last_error());
        return 1;
    }
    ppr_graph_info info;
    if (ppr_graph_get_info(g, &info) != PPR_OK || info.n != 5 || info.m != 13) return 1;
    double pi[5], pib[3 * 5];
    ppr_stats s;
    if (ppr_query(g, 0, 0.2, 1e-12, PPR_FP64, pi, &s) != PPR_OK) {
        printf("query failed: %s\n", ppr_last_error());
        return 1;
    }
    const double want[5] = {0.29366106, 0.27166882, 0.23285899, 0.14747736, 0.05433376};
    double err = 0.0;
    for (int i = 0; i < 5; ++i) err += fabs(pi[i] - want[i]);
    const int32_t src[3] = {0, 0, 3};
    if (ppr_query_batch(g, src, 3, 0.2, 1e-10, PPR_MIXED, pib, NULL) != PPR_OK) {
        printf("batch failed: %s\n", ppr_last_error());
        return 1;
    }
    double diff = 0.0;
    for (int i = 0; i < 5; ++i) diff += fabs(pib[i] - pi[i]) + fabs(pib[5 + i] - pi[i]);
    /* power iteration traced: the l1 error after k sweeps is 0.8^k (Eq. 6) */
    ppr_options o;
    ppr_options_default(&o);
    o.switch_param = 1e30;
    ppr_trace_point tr[256];
    int32_t cnt = 0;
    if (ppr_query_trace(g, 0, 0.2, 1e-12, &o, pi, tr, 256, &cnt, NULL) != PPR_OK) {
        printf("trace failed: %s\n", ppr_last_error());
        return 1;
    }
    double tdev = 0.0, a = 1.0;
    for (int k = 0; k < cnt && k < 256; ++k) {
        a *= 0.8;
        tdev = fmax(tdev, fabs(tr[k].r_sum - a) / a);
        if (tr[k].phase != 1 || tr[k].index != k + 1 || tr[k].edge_pushes != 13 * (int64_t)(k + 1)) tdev = 1.0;
    }
    ppr_graph_destroy(g);
    printf("fp64 l1 vs printed %.3e, mixed vs fp64 %.3e, sweeps %d, trace points %d (rel dev %.1e)\n", err,
           diff, s.sweeps, (int)cnt, tdev);
    /* the printed values carry 8 decimals; ceil(ln 1e-12 / ln 0.8) = 124 sweeps */
    return (err <= 5 * 5e-9 + 1e-12 && diff <= 2 * (1e-10 + 1e-12) + 1e-12 && cnt == 124 && tdev <= 1e-12) ? 0 : 1;
}
