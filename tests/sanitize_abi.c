/* Drives the host-side argument validation of every C-ABI entry point
 * (include/bdesc.h) with malformed arguments: null pointers, negative
 * counts, unsupported widths, bad pitches, non-finite scalars, sizes past the
 * addressing limits, and a null context where the arguments are valid.
 * Linked against the library's objects built with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host side only (the GPU code is
 * unchanged) by tests/test_host_sanitize.py; no call reaches a kernel.  Each
 * check compares the return code with the documented one; the exit status
 * is the number of mismatches (sanitizer reports abort with their own). */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../include/bdesc.h"

static int g_fail = 0;

static void expect(int got, int want, const char* what)
{
    if (got != want) {
        fprintf(stderr, "%s: returned %d, expected %d (%s)\n", what, got, want, bd_last_error());
        ++g_fail;
    }
}

#define EXPECT(call, want) expect((call), (want), #call)

int main(void)
{
    void* p = (void*)16; /* never dereferenced: validation fails before any access */
    const float nanf_ = NAN;

    bd_context* ctx = NULL;
    EXPECT(bd_context_create(NULL, 0), BD_EINVAL);
    {
        const int rc = bd_context_create(&ctx, 0); /* no device here, or device 0 */
        if (rc == BD_OK) bd_context_destroy(ctx);
        else expect(rc, BD_EDEVICE, "bd_context_create(&ctx, 0)");
    }
    EXPECT(bd_context_create(&ctx, -1) < 0, 1);
    EXPECT(bd_context_destroy(NULL), BD_OK);
    uint64_t count = 9;
    EXPECT(bd_context_poll(NULL, NULL), BD_EINVAL);
    EXPECT(bd_context_poll(NULL, &count), BD_EINVAL);
    if (count != 0) ++g_fail;
    if (strncmp(bd_version(), "bdesc", 5) != 0) ++g_fail;

    EXPECT(bd_build_integral(NULL, p, 0, 5, 5, p, 6, NULL), BD_EINVAL);
    EXPECT(bd_build_integral(NULL, p, 8, 5, 7, p, 9, NULL), BD_EINVAL);
    EXPECT(bd_build_integral(NULL, p, 8, 5, 8, p, 8, NULL), BD_EINVAL);
    EXPECT(bd_build_integral(NULL, p, 40000, 60000, 40000, p, 40001, NULL), BD_EINVAL);
    EXPECT(bd_build_integral(NULL, NULL, 8, 5, 8, p, 9, NULL), BD_EINVAL);
    EXPECT(bd_build_integral(NULL, p, 8, 5, 8, p, 9, NULL), BD_EINVAL);

    EXPECT(bd_build_integral_order(NULL, p, 0, 5, 5, p, 6, p, 3, p, NULL), BD_EINVAL);
    EXPECT(bd_build_integral_order(NULL, p, 8, 5, 8, p, 9, p, -1, p, NULL), BD_EINVAL);
    EXPECT(bd_build_integral_order(NULL, p, 8, 5, 8, p, 9, NULL, 3, p, NULL), BD_EINVAL);
    EXPECT(bd_build_integral_order(NULL, p, 8, 5, 8, p, 9, NULL, 0, NULL, NULL), BD_EINVAL);
    EXPECT(bd_prepare_view(NULL, p, 8, 5, 8, p, 9, p, 3, p, p, 32, NULL, 64, NULL), BD_EINVAL);
    EXPECT(bd_prepare_view(NULL, p, 8, 5, 8, p, 9, p, 3, p, p, 28, p, 64, NULL), BD_EINVAL);
    EXPECT(bd_prepare_view(NULL, p, 8, 5, 8, p, 9, p, 3, p, p, 32, p, 60, NULL), BD_EINVAL);
    EXPECT(bd_prepare_view(NULL, p, 8, 5, 8, p, 9, p, 3, p, p, 32, p, 64, NULL), BD_EINVAL);
    EXPECT(bd_prepare_view(NULL, p, 8, 5, 8, p, 9, p, 3, p, NULL, 0, NULL, 0, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_features(NULL, p, BD_DTYPE_F32_ROWPAIR, 10, 10, 84, p, 3, NULL, p, NULL), BD_EINVAL);
    EXPECT(bd_keypoint_order(NULL, p, 5, 0, 10, p, NULL), BD_EINVAL);
    EXPECT(bd_keypoint_order(NULL, p, -1, 10, 10, p, NULL), BD_EINVAL);
    EXPECT(bd_keypoint_order(NULL, NULL, 5, 10, 10, p, NULL), BD_EINVAL);
    EXPECT(bd_keypoint_order(NULL, p, 5, 10, 10, p, NULL), BD_EINVAL);

    EXPECT(bd_describe_bad(NULL, p, 10, 10, 11, p, 4, NULL, p, 128, p, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_describe_bad(NULL, p, 10, 10, 10, p, 4, NULL, p, 256, p, NULL), BD_EINVAL);
    EXPECT(bd_describe_bad(NULL, p, 10, 10, 11, p, -1, NULL, p, 256, p, NULL), BD_EINVAL);
    EXPECT(bd_describe_bad(NULL, p, 10, 10, 11, NULL, 4, NULL, p, 256, p, NULL), BD_EINVAL);
    EXPECT(bd_describe_bad(NULL, p, 60000, 60000, 60001, p, 4, NULL, p, 256, p, NULL), BD_EINVAL);
    EXPECT(bd_describe_bad(NULL, NULL, 10, 10, 11, NULL, 0, NULL, NULL, 256, NULL, NULL), BD_EINVAL);

    bd_bad_table* table = (bd_bad_table*)p;
    EXPECT(bd_bad_table_create(NULL, p, 256, NULL, NULL), BD_EINVAL);
    EXPECT(bd_bad_table_create(NULL, p, 100, &table, NULL), BD_EUNSUPPORTED);
    if (table != NULL) ++g_fail; /* cleared on error */
    EXPECT(bd_bad_table_create(NULL, NULL, 256, &table, NULL), BD_EINVAL);
    EXPECT(bd_bad_table_create(NULL, p, 256, &table, NULL), BD_EINVAL);
    EXPECT(bd_bad_table_destroy(NULL), BD_OK);
    EXPECT(bd_describe_bad_table(NULL, p, 10, 10, 11, p, 4, NULL, NULL, p, NULL), BD_EINVAL);

    EXPECT(bd_describe_hashsift(NULL, p, BD_DTYPE_F32, 10, 10, 40, p, 3, NULL, p, p, 384, BD_PREC_FP32, 1e-3f, p,
                                NULL, NULL, NULL, NULL),
           BD_EUNSUPPORTED);
    EXPECT(bd_describe_hashsift(NULL, p, 7, 10, 10, 40, p, 3, NULL, p, p, 256, BD_PREC_FP32, 1e-3f, p, NULL, NULL,
                                NULL, NULL),
           BD_EUNSUPPORTED);
    EXPECT(bd_describe_hashsift(NULL, p, BD_DTYPE_F32, 10, 10, 42, p, 3, NULL, p, p, 256, BD_PREC_FP32, 1e-3f, p,
                                NULL, NULL, NULL, NULL),
           BD_EINVAL);
    EXPECT(bd_describe_hashsift(NULL, p, BD_DTYPE_U8, 10, 1 << 24, 10, p, 3, NULL, p, p, 256, BD_PREC_FP32, 1e-3f,
                                p, NULL, NULL, NULL, NULL),
           BD_EINVAL);
    EXPECT(bd_describe_hashsift(NULL, p, BD_DTYPE_F32, 10, 10, 40, p, 3, NULL, p, p, 256, BD_PREC_BF16, nanf_, p,
                                NULL, NULL, NULL, NULL),
           BD_EINVAL);
    EXPECT(bd_describe_hashsift(NULL, p, BD_DTYPE_F32, 10, 10, 40, p, -3, NULL, p, p, 256, BD_PREC_FP8, 1e-3f, p,
                                NULL, NULL, NULL, NULL),
           BD_EINVAL);
    EXPECT(bd_describe_hashsift(NULL, p, BD_DTYPE_F32, 10, 10, 40, p, 3, NULL, p, p, 256, BD_PREC_FP8, 1e-3f, p,
                                NULL, NULL, NULL, NULL),
           BD_EINVAL);
    EXPECT(bd_hashsift_features(NULL, p, BD_DTYPE_U8, 0, 10, 10, p, 3, NULL, p, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_features(NULL, p, BD_DTYPE_U8, 10, 10, 10, p, 3, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_features(NULL, p, BD_DTYPE_U8, 10, 10, 10, p, 3, NULL, p, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_project(NULL, p, NULL, 3, p, p, 128, BD_PREC_FP32, 0.0f, p, NULL, NULL, NULL),
           BD_EUNSUPPORTED);
    EXPECT(bd_hashsift_project(NULL, p, NULL, 3, p, p, 256, 7, 0.0f, p, NULL, NULL, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_hashsift_project(NULL, NULL, NULL, 3, p, p, 256, BD_PREC_FP32, 0.0f, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_project(NULL, p, NULL, 3, p, p, 256, BD_PREC_FP32, 0.0f, p, NULL, NULL, NULL), BD_EINVAL);

    EXPECT(bd_match_hamming_knn(NULL, p, 4, p, 4, 9, 1, p, p, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_match_hamming_knn(NULL, p, 4, p, 4, 4, 3, p, p, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_match_hamming_knn(NULL, p, -1, p, 4, 4, 1, p, p, NULL), BD_EINVAL);
    EXPECT(bd_match_hamming_knn(NULL, p, 4, NULL, 4, 4, 1, p, p, NULL), BD_EINVAL);
    EXPECT(bd_match_hamming_knn(NULL, p, 4, p, 4, 4, 1, p, p, NULL), BD_EINVAL);
    EXPECT(bd_match_hamming_knn_noalloc(NULL, p, 4, p, 4, 0, 1, p, p, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_match_hamming_knn_noalloc(NULL, p, 4, p, -4, 4, 1, p, p, NULL), BD_EINVAL);
    EXPECT(bd_match_hamming_knn_noalloc(NULL, p, 4, p, 4, 4, 1, p, NULL, NULL), BD_EINVAL);
    EXPECT(bd_match_hamming_knn_noalloc(NULL, p, 4, p, 4, 4, 1, p, p, NULL), BD_EINVAL);
    EXPECT(bd_match_mutual(NULL, p, 4, p, 4, 9, 0.8f, p, p, NULL, NULL, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_match_mutual(NULL, p, 4, p, 4, 4, -0.5f, p, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_match_mutual(NULL, p, 4, p, 4, 4, nanf_, p, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_match_mutual(NULL, p, 4, p, 4, 4, 0.8f, NULL, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_match_mutual(NULL, p, 4, p, 4, 4, 0.8f, p, p, NULL, NULL, NULL), BD_EINVAL);

    EXPECT(bd_find_threshold(NULL, p, -1, p, p, 0.5f, p, 4, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_find_threshold(NULL, p, 10, p, p, 0.3f, p, 4, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_find_threshold(NULL, p, 10, p, p, nanf_, p, 4, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_find_threshold(NULL, p, (1 << 24) + 1, p, p, 0.5f, p, 4, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_find_threshold(NULL, p, 10, p, p, 1.5f, p, 4, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_select_features(NULL, p, 100, p, 50, p, 10, 0, 1.0f, p, NULL, NULL, NULL, NULL, NULL),
           BD_EUNSUPPORTED);
    EXPECT(bd_select_features(NULL, p, 100, p, 101, p, 10, 64, 1.0f, p, NULL, NULL, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_select_features(NULL, p, 100, p, 50, p, 10, 64, 0.7f, p, NULL, NULL, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_select_features(NULL, p, 100, p, 50, p, 10, 64, 1.0f, p, NULL, NULL, NULL, NULL, NULL), BD_EINVAL);

    EXPECT(bd_hashsift_patch_features(NULL, p, -1, p, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_patch_features(NULL, p, 4, p, NULL), BD_EINVAL);
    EXPECT(bd_relaxed_bad_fwd(NULL, p, 4, p, p, p, p, 100, 10.0f, p, NULL, NULL, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_relaxed_bad_fwd(NULL, p, 4, p, p, p, p, 256, 0.0f, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_relaxed_bad_fwd(NULL, p, 4, p, p, p, p, 256, 10.0f, p, NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_relaxed_bad_bwd(NULL, p, p, p, p, 4, 256, 10.0f, NULL, p, p, NULL), BD_EINVAL);
    EXPECT(bd_relaxed_hashsift_fwd(NULL, p, 4, p, p, 320, 10.0f, NULL, p, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_relaxed_hashsift_bwd(NULL, p, p, p, 4, 256, nanf_, p, p, NULL), BD_EINVAL);
    EXPECT(bd_trl_hnm_fwd(NULL, p, p, 0, 256, 0.5f, p, p, p, NULL), BD_EINVAL);
    EXPECT(bd_trl_hnm_fwd(NULL, p, p, 8, 256, 0.5f, p, p, p, NULL), BD_EINVAL);
    EXPECT(bd_trl_hnm_bwd(NULL, p, p, 8, 100, p, p, p, p, p, NULL), BD_EUNSUPPORTED);
    EXPECT(bd_augment_patches(NULL, p, 0, p, 4, p, p, p, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_train_step(NULL, p, 100, p, 8, p, p, p, p, 512, p, 0, 2e-4f, 0.5f, 1.0f, p, NULL), BD_EINVAL);
    EXPECT(bd_hashsift_train_step(NULL, p, 100, p, 8, p, p, p, p, 512, p, 1, 2e-4f, 0.5f, 1.0f, p, NULL), BD_EINVAL);

    bd_batch_image imgs[2];
    memset(imgs, 0, sizeof imgs);
    imgs[0].img = p;
    imgs[0].pitch = 64;
    imgs[0].W = 64;
    imgs[0].H = 48;
    imgs[0].n_kp = 10;
    imgs[1] = imgs[0];
    imgs[1].pitch = 99;
    imgs[1].W = 100;
    bd_batch_match m = {0, 1};
    bd_batch* batch = (bd_batch*)p;
    EXPECT(bd_batch_create(NULL, imgs, 2, &m, 1, 512, 256, BD_PREC_FP32, 1e-3f, 2, NULL), BD_EINVAL);
    EXPECT(bd_batch_create(NULL, imgs, 0, &m, 1, 512, 256, BD_PREC_FP32, 1e-3f, 2, &batch), BD_EINVAL);
    if (batch != NULL) ++g_fail;
    EXPECT(bd_batch_create(NULL, imgs, 2, &m, 1, 128, 256, BD_PREC_FP32, 1e-3f, 2, &batch), BD_EUNSUPPORTED);
    EXPECT(bd_batch_create(NULL, imgs, 2, &m, 1, 512, 256, BD_PREC_FP32, 1e-3f, 2, &batch), BD_EINVAL);
    imgs[1].pitch = 100;
    m.train_image = 2;
    EXPECT(bd_batch_create(NULL, imgs, 2, &m, 1, 512, 256, BD_PREC_FP32, 1e-3f, 2, &batch), BD_EINVAL);
    m.train_image = 1;
    EXPECT(bd_batch_create(NULL, imgs, 2, &m, 1, 512, 256, BD_PREC_FP32, 1e-3f, 2, &batch), BD_EINVAL);
    bd_batch_tuning tn;
    EXPECT(bd_batch_default_tuning(&tn), BD_OK);
    EXPECT(bd_batch_default_tuning(NULL), BD_EINVAL);
    EXPECT(bd_batch_set_tuning(NULL, &tn), BD_EINVAL);
    EXPECT(bd_batch_get_tuning(NULL, &tn), BD_EINVAL);
    EXPECT(bd_batch_info(NULL, NULL, NULL), BD_EINVAL);
    EXPECT(bd_batch_run(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 1, NULL), BD_EINVAL);
    EXPECT(bd_batch_autotune(NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 3, NULL), BD_EINVAL);
    EXPECT(bd_batch_destroy(NULL), BD_OK);

    if (g_fail == 0) puts("host validation under ASan/UBSan: every code as documented, no reports");
    return g_fail;
}
