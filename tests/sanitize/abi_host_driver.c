/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * host side of libqbsm's C ABI (test infrastructure).  Calls only what runs
 * without a GPU -- argument validation, status strings, handle lifetimes and
 * the error paths of calls whose first device step fails -- so the
 * sanitizers see every host-side check, the exception-to-status mapping and
 * the handle cleanup.  Exit status 0 on success.
 */
#include <stdio.h>
#include <string.h>

#include "../../include/qbsm.h"

static int fails = 0;
#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            fprintf(stderr, "abi driver: line %d: %s (last error: %s)\n", __LINE__, #cond, \
                    qbsm_last_error());                                           \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

static void *fake_alloc(size_t bytes, void *stream, void *ctx)
{
    (void)bytes; (void)stream; (void)ctx;
    return NULL; /* every device allocation fails */
}
static void fake_release(void *p, void *stream, void *ctx) { (void)p; (void)stream; (void)ctx; }

int main(void)
{
    for (int s = 0; s <= 8; ++s) EXPECT(qbsm_status_string((qbsm_status)s) != NULL);
    EXPECT(strcmp(qbsm_status_string(QBSM_ERR_PATTERN), "invalid block pattern") == 0);
    EXPECT(qbsm_version() == 10000);

    qbsm_matrix a = NULL, b = NULL, m = NULL;
    EXPECT(qbsm_matrix_create(100, 100, 48, &a) == QBSM_ERR_UNSUPPORTED);
    EXPECT(qbsm_matrix_create(-1, 100, 64, &a) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_create(100, 100, 64, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_create((int64_t)64 * 65537, 64, 64, &a) == QBSM_ERR_UNSUPPORTED);
    EXPECT(qbsm_matrix_create(300, 200, 64, &a) == QBSM_OK);
    EXPECT(qbsm_matrix_create(250, 170, 64, &b) == QBSM_OK);
    EXPECT(qbsm_matrix_create(300, 170, 32, &m) == QBSM_OK);

    int64_t nr = 0, nc = 0, nb = -1;
    int32_t bs = 0;
    EXPECT(qbsm_matrix_info(a, &nr, &nc, &bs, &nb) == QBSM_OK);
    EXPECT(nr == 300 && nc == 200 && bs == 64 && nb == 0);
    EXPECT(qbsm_matrix_info(NULL, &nr, NULL, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_get_pattern(a, NULL, NULL, NULL) == QBSM_OK);  /* nothing stored */
    EXPECT(qbsm_matrix_get_values(a, NULL, NULL) == QBSM_OK);

    /* construction arguments checked before any device work */
    int32_t idx[2] = {0, 1};
    double vals[1];
    EXPECT(qbsm_matrix_set_blocks(a, -1, idx, idx, vals, 0.0, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_set_blocks(a, 2, NULL, idx, vals, 0.0, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_set_blocks(a, 2, idx, idx, vals, -1.0, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_set_blocks(NULL, 0, NULL, NULL, NULL, 0.0, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_matrix_truncate(a, -1.0, NULL, NULL) != QBSM_OK);
    EXPECT(qbsm_matrix_store_f32(a, NULL) == QBSM_ERR_STATE);
    EXPECT(qbsm_matrix_prepack(a, QBSM_F64, 3, NULL) == QBSM_ERR_STATE);
    EXPECT(qbsm_matrix_prepack(a, (qbsm_mode)9, 3, NULL) == QBSM_ERR_ARG);

    /* the multiply needs stored blocks; shapes and leaf sizes are checked */
    qbsm_plan p = NULL;
    int64_t nout = 0, nprod = 0;
    EXPECT(qbsm_multiply_symbolic(a, b, NULL, NULL, &p, &nout, &nprod) == QBSM_ERR_STATE);
    EXPECT(qbsm_multiply_symbolic(NULL, b, NULL, NULL, &p, &nout, &nprod) == QBSM_ERR_ARG);
    EXPECT(qbsm_multiply_symbolic(a, b, NULL, NULL, NULL, &nout, &nprod) == QBSM_ERR_ARG);
    qbsm_plan_opts bad = {0};
    bad.spamm_tol = -1.0;
    EXPECT(qbsm_multiply_symbolic(a, b, &bad, NULL, &p, NULL, NULL) == QBSM_ERR_ARG);
    bad.spamm_tol = 0.0;
    bad.upper = 2;
    EXPECT(qbsm_multiply_symbolic(a, b, &bad, NULL, &p, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_plan_info(NULL, &nout, NULL, NULL, NULL, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_multiply_numeric(NULL, QBSM_F64, a, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_multiply_numeric_noalloc(NULL, QBSM_F64, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_multiply_backward(a, b, NULL, QBSM_F64, NULL, NULL, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_multiply_backward(a, b, b, QBSM_F64, NULL, NULL, NULL, NULL) == QBSM_ERR_SHAPE);
    EXPECT(qbsm_batch_create(-1, NULL, QBSM_F32, NULL, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_batch_run(NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_batch_set_occupancy(NULL, 1) == QBSM_ERR_ARG);
    EXPECT(qbsm_autotune_unit(a, b, QBSM_F64, 0, NULL, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_profile_read(7, NULL, NULL) == QBSM_ERR_ARG);

    /* allocator hooks: both or neither; a hook that always fails turns the
     * first device allocation of a call into QBSM_ERR_OOM (the handle stays
     * valid and unchanged) */
    EXPECT(qbsm_set_allocator(fake_alloc, NULL, NULL) == QBSM_ERR_ARG);
    EXPECT(qbsm_set_allocator(fake_alloc, fake_release, NULL) == QBSM_OK);
    qbsm_status st = qbsm_matrix_set_blocks(a, 0, NULL, NULL, NULL, 0.0, NULL, NULL);
    EXPECT(st == QBSM_ERR_OOM || st == QBSM_ERR_HIP);
    EXPECT(qbsm_matrix_info(a, NULL, NULL, NULL, &nb) == QBSM_OK && nb == 0);
    EXPECT(qbsm_set_allocator(NULL, NULL, NULL) == QBSM_OK);

    EXPECT(qbsm_plan_destroy(NULL) == QBSM_OK);
    EXPECT(qbsm_batch_destroy(NULL) == QBSM_OK);
    EXPECT(qbsm_matrix_destroy(a) == QBSM_OK);
    EXPECT(qbsm_matrix_destroy(b) == QBSM_OK);
    EXPECT(qbsm_matrix_destroy(m) == QBSM_OK);
    EXPECT(qbsm_matrix_destroy(NULL) == QBSM_OK);
    if (fails) return 1;
    printf("abi host driver ok\n");
    return 0;
}
