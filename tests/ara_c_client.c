/* A plain C client of libara: the hand-worked example through the C-ABI only (no
 * Python, no torch).  Host arrays in, YLT / occurrence maxima / PML / TVaR out, one
 * line per value ("name index value-in-%.17g").  Exit status: 0 on success, else the
 * first failing ara_status (negated). */
#include <math.h>
#include <stdio.h>

#include "ara.h"

#define CHECK(call)                                                                         \
    do {                                                                                    \
        ara_status st_ = (call);                                                            \
        if (st_ != ARA_OK) {                                                                \
            fprintf(stderr, "%s failed: %s (%s)\n", #call, ara_status_str(st_),             \
                    ara_last_error(ctx));                                                    \
            return -st_;                                                                    \
        }                                                                                   \
    } while (0)

int main(void) {
    ara_ctx *ctx = NULL;
    ara_status st = ara_ctx_create(0, NULL, &ctx);
    if (st != ARA_OK) {
        fprintf(stderr, "ara_ctx_create: %s (%s)\n", ara_status_str(st), ara_last_error(NULL));
        return -st;
    }
    /* catalog of 5 events; trials T0 = [3,0,2,0,4], T1 = [1], T2 = [], T3 = [2,2] */
    const int32_t ids[] = {3, 0, 2, 0, 4, 1, 2, 2};
    const int64_t offs[] = {0, 5, 6, 6, 8};
    const int32_t e1_ids[] = {0, 2, 3};
    const double e1_loss[] = {40.0, 100.0, 5.0};
    const int32_t e2_ids[] = {0, 1, 3};
    const double e2_loss[] = {15.0, 70.0, 2.0};
    const ara_layer_terms terms = {10.0, 50.0, 30.0, 100.0};
    ara_yet *yet = NULL;
    ara_elt *elts[2] = {NULL, NULL};
    ara_layer *layer = NULL;
    CHECK(ara_yet_create(ctx, ids, 8, offs, 4, 5, ARA_MEM_HOST, &yet));
    CHECK(ara_elt_create(ctx, e1_ids, e1_loss, 3, 5, NULL, ARA_F64, ARA_MEM_HOST, &elts[0]));
    CHECK(ara_elt_create(ctx, e2_ids, e2_loss, 3, 5, NULL, ARA_F64, ARA_MEM_HOST, &elts[1]));
    CHECK(ara_layer_create(ctx, elts, 2, 5, &terms, &layer));
    double ylt[4], omax[4];
    CHECK(ara_analyze(ctx, yet, layer, 0, 4, ylt, ARA_MEM_HOST));
    CHECK(ara_analyze_occ_max(ctx, yet, layer, 0, 4, omax, ARA_MEM_HOST));
    const double rps[] = {1.0, 2.0, 4.0};
    double pml[3], tvar[3];
    CHECK(ara_risk_measures(ctx, ylt, 4, ARA_MEM_HOST, rps, 3, pml, tvar, NULL, 0));
    for (int t = 0; t < 4; ++t) printf("ylt %d %.17g\n", t, ylt[t]);
    for (int t = 0; t < 4; ++t) printf("occ_max %d %.17g\n", t, omax[t]);
    for (int i = 0; i < 3; ++i) printf("pml %d %.17g\ntvar %d %.17g\n", i, pml[i], i, tvar[i]);
    CHECK(ara_sync(ctx));
    CHECK(ara_layer_release(layer));
    CHECK(ara_elt_release(elts[0]));
    CHECK(ara_elt_release(elts[1]));
    CHECK(ara_yet_release(yet));
    CHECK(ara_ctx_destroy(ctx));
    return 0;
}
