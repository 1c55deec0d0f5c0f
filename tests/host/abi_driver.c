/*
 * Host-side driver of libpsp's C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer against a host-only sanitized build of the
 * library (no device code: every path exercised here is host logic --
 * argument validation, the Gaussian-sum fit, sizes, launch shapes, the
 * tuning table, error strings, call-order and missing-device errors).
 * Exits 0 when every call returns what the header promises.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "psp.h"

static int failures = 0;
#define EXPECT(cond, what)                                                   \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "FAIL %s (line %d): %s\n", what, __LINE__,      \
                    psp_last_error());                                       \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

static int smooth_2_3(int m) {
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

int main(void) {
    psp_plan *p = NULL;
    /* every n: accepted exactly when even, in [4, 384], 2n = 2^a 3^b */
    for (int n = 1; n <= 400; ++n) {
        const int ok = n % 2 == 0 && n >= 4 && n <= 384 && smooth_2_3(2 * n);
        psp_status st = psp_plan_create(n, 2.0 / n, 40, PSP_F64, &p);
        EXPECT((st == PSP_OK) == ok, "plan_create acceptance");
        if (st != PSP_OK) {
            EXPECT(p == NULL, "plan NULL on failure");
            continue;
        }
        double om[40], al[40];
        EXPECT(psp_plan_get_gs(p, om, al) == PSP_OK, "get_gs");
        for (int s = 1; s < 40; ++s) EXPECT(al[s] > al[s - 1] && om[s] > om[s - 1], "GS terms increase");
        size_t ws = 0, sb = 0;
        EXPECT(psp_plan_workspace_bytes(p, &ws) == PSP_OK && ws > 0, "workspace bytes");
        EXPECT(psp_plan_spectrum_bytes(p, &sb) == PSP_OK && sb >= 8 * (size_t)(n + 1) * (n + 1) * (n + 1),
               "spectrum bytes");
        int plan[5], tile[5];
        EXPECT(psp_plan_get_shape(p, plan, tile) == PSP_OK, "get_shape");
        int bad[5] = {0, 0, 0, 0, 99};
        EXPECT(psp_plan_set_shape(p, plan, bad) == PSP_EINVAL, "set_shape rejects a tile");
        EXPECT(psp_plan_set_tuning(p, 2, 0) == PSP_OK && psp_plan_set_tuning(p, 0, 0) == PSP_OK, "set_tuning");
        /* call order: nothing runs before precompute */
        EXPECT(psp_solve(p, (void *)16, (void *)32, NULL) == PSP_ESTATE, "solve before precompute");
        EXPECT(psp_solve_noalloc(p, (void *)16, (void *)32, NULL) == PSP_ESTATE, "noalloc before precompute");
        EXPECT(psp_solve_padded_debug(p, (void *)16, (void *)32, NULL) == PSP_ESTATE, "debug before precompute");
        double m[8];
        EXPECT(psp_plan_get_multiplier(p, m) == PSP_ESTATE, "multiplier before precompute");
        psp_plan_destroy(p);
        p = NULL;
    }
    /* large R and explicit cutoffs */
    EXPECT(psp_plan_create_ex(32, 0.1, 2048, PSP_F32, 1e-4, 3.0, &p) == PSP_OK, "R = 2048");
    psp_plan_destroy(p);
    EXPECT(psp_plan_create_ex(32, 0.1, 40, PSP_F64, 3.0, 1.0, &p) == PSP_EINVAL, "eps >= delta");
    EXPECT(psp_plan_create(32, 0.1, 0, PSP_F64, &p) == PSP_EINVAL, "R = 0");
    EXPECT(psp_plan_create(32, -1.0, 40, PSP_F64, &p) == PSP_EINVAL, "h < 0");
    EXPECT(psp_plan_create(32, 0.1, 40, (psp_dtype)7, &p) == PSP_EINVAL, "dtype");
    EXPECT(psp_plan_create(32, 0.1, 40, PSP_F64, NULL) == PSP_EINVAL, "out NULL");
    /* boxes and grids */
    const double hs[3] = {0.1, 0.07, 0.05};
    const int ns[3] = {16, 36, 54};
    EXPECT(psp_plan_create_box(32, hs, 40, PSP_F64, -1.0, -1.0, &p) == PSP_OK, "box");
    psp_plan_destroy(p);
    EXPECT(psp_plan_create_grid(ns, hs, 40, PSP_F32, -1.0, -1.0, &p) == PSP_OK, "grid");
    EXPECT(psp_plan_set_tuning(p, 1, 0) == PSP_EUNSUPPORTED, "grid chunking");
    psp_plan_destroy(p);
    EXPECT(psp_plan_create_box(32, NULL, 40, PSP_F64, -1.0, -1.0, &p) == PSP_EINVAL, "box NULL h");
    /* tuning table */
    int pl[5] = {0, 0, 2, 0, 0}, tl[5] = {3, 2, 9, 0, 3}, pg[5], tg[5];
    EXPECT(psp_tuning_set(256, PSP_F64, pl, tl) == PSP_OK, "tuning_set");
    EXPECT(psp_tuning_get(256, PSP_F64, pg, tg) == PSP_OK && memcmp(pl, pg, sizeof pl) == 0 &&
               memcmp(tl, tg, sizeof tl) == 0,
           "tuning_get");
    EXPECT(psp_tuning_set(10, PSP_F64, pl, tl) == PSP_EUNSUPPORTED, "tuning_set size");
    /* batches and modes */
    EXPECT(psp_solve_batched(0, NULL, NULL, NULL, NULL) == PSP_OK, "empty batch");
    EXPECT(psp_solve_batched(-1, NULL, NULL, NULL, NULL) == PSP_EINVAL, "negative batch");
    EXPECT(psp_set_batch_mode(3) == PSP_EINVAL && psp_set_batch_mode(0) == PSP_OK, "batch mode");
    psp_graph *g = NULL;
    EXPECT(psp_graph_capture(NULL, NULL, NULL, NULL, &g) == PSP_EINVAL, "graph NULL");
    /* errors */
    for (int e = -7; e <= 0; ++e) EXPECT(psp_strerror((psp_status)e) != NULL, "strerror");
    EXPECT(psp_last_error() != NULL, "last_error");
    /* the device-side entry points report a missing device, they do not crash */
    EXPECT(psp_plan_create(16, 0.1, 8, PSP_F64, &p) == PSP_OK, "plan for precompute");
    psp_status st = psp_kernel_precompute(p, NULL);
    EXPECT(st == PSP_OK || st == PSP_EHIP || st == PSP_ENOMEM, "precompute status");
    psp_plan_destroy(p);
    psp_server *sv = NULL;
    st = psp_serve_create(0, 4, &sv);
    EXPECT(st == PSP_EINVAL, "serve budget 0");
    printf("abi_driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
