/* Exercises every function of the CPU oracle (oracle/bdref.c) on small
 * seeded inputs, including the edge cases the tests pin (invalid and border
 * keypoints, huge scales, fewer train codes than k, empty sets, special
 * floating-point values).  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py; every buffer
 * is a heap block of exactly the documented size, so any read or write past
 * a documented extent is reported.  Exit status 0 means no report. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/bdref.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;

static uint64_t next_u64(void) /* splitmix64 */
{
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform(double lo, double hi) { return lo + (hi - lo) * (double)(next_u64() >> 11) * 0x1p-53; }

static void* xmalloc(size_t n)
{
    void* p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void fill_pairs(bdref_box_pair* p, int n)
{
    for (int j = 0; j < n; ++j) {
        p[j].x1 = (int8_t)(next_u64() % 29) - 14;
        p[j].y1 = (int8_t)(next_u64() % 29) - 14;
        p[j].x2 = (int8_t)(next_u64() % 29) - 14;
        p[j].y2 = (int8_t)(next_u64() % 29) - 14;
        p[j].radius = (uint8_t)(1 + next_u64() % 5);
        memset(p[j].pad, 0, sizeof p[j].pad);
        p[j].threshold = (float)((int)(next_u64() % 41) - 20);
    }
}

static void fill_keypoints(bdref_keypoint* k, int n, int W, int H)
{
    for (int i = 0; i < n; ++i) {
        k[i].x = (float)uniform(0.0, W - 1);
        k[i].y = (float)uniform(0.0, H - 1);
        k[i].scale = (float)uniform(0.5, 4.0);
        k[i].angle = (float)uniform(0.0, 6.283185307179586);
    }
    /* invalid, far outside, huge scale, image corners */
    k[0].x = NAN;
    k[1].scale = 0.0f;
    k[2].angle = INFINITY;
    k[3].x = -1e9f;
    k[3].y = 1e9f;
    k[4].scale = 1e30f;
    k[5].x = 0.0f;
    k[5].y = 0.0f;
    k[6].x = (float)(W - 1);
    k[6].y = (float)(H - 1);
}

static void integral_and_bad(void)
{
    const int W = 37, H = 29, n_kp = 24, n_bits = 256;
    const int64_t pitch = 40, ii_pitch = 39;
    uint8_t* img = xmalloc((size_t)pitch * H);
    for (int64_t i = 0; i < pitch * H; ++i) img[i] = (uint8_t)next_u64();
    uint32_t* ii = xmalloc(sizeof(uint32_t) * (size_t)ii_pitch * (H + 1));
    bdref_build_integral(img, W, H, pitch, ii, ii_pitch);
    bdref_keypoint* kps = xmalloc(sizeof(bdref_keypoint) * n_kp);
    fill_keypoints(kps, n_kp, W, H);
    bdref_box_pair* pairs = xmalloc(sizeof(bdref_box_pair) * n_bits);
    fill_pairs(pairs, n_bits);
    uint64_t* codes = xmalloc(sizeof(uint64_t) * n_kp * (n_bits / 64));
    (void)bdref_describe_bad(ii, W, H, ii_pitch, kps, n_kp, pairs, n_bits, codes);
    for (int i = 0; i < n_kp; ++i) (void)bdref_keypoint_valid(&kps[i]);
    /* 1x1 image: every box is capped at radius 0 */
    uint8_t* one = xmalloc(1);
    one[0] = 200;
    uint32_t* ii1 = xmalloc(sizeof(uint32_t) * 4);
    bdref_build_integral(one, 1, 1, 1, ii1, 2);
    uint64_t* code1 = xmalloc(sizeof(uint64_t) * 4);
    bdref_describe_bad(ii1, 1, 1, 2, kps + 5, 1, pairs, 256, code1);
    free(code1);
    free(ii1);
    free(one);
    free(codes);
    free(pairs);
    free(kps);
    free(ii);
    free(img);
}

static void hashsift(void)
{
    const int W = 45, H = 33, n_kp = 12, n_bits = 256;
    const int64_t pitch_u8 = 47, pitch_f = 46 * 4;
    uint8_t* img8 = xmalloc((size_t)pitch_u8 * H);
    for (int64_t i = 0; i < pitch_u8 * H; ++i) img8[i] = (uint8_t)next_u64();
    float* imgf = xmalloc((size_t)pitch_f * H);
    for (int64_t i = 0; i < (pitch_f / 4) * H; ++i) imgf[i] = (float)uniform(0.0, 1.0);
    bdref_keypoint* kps = xmalloc(sizeof(bdref_keypoint) * n_kp);
    fill_keypoints(kps, n_kp, W, H);
    double* hist = xmalloc(sizeof(double) * n_kp * 128);
    bdref_hashsift_hist(img8, 0, W, H, pitch_u8, kps, n_kp, hist);
    bdref_hashsift_hist(imgf, 1, W, H, pitch_f, kps, n_kp, hist);
    float* B = xmalloc(sizeof(float) * n_bits * 128);
    float* t = xmalloc(sizeof(float) * n_bits);
    for (int i = 0; i < n_bits * 128; ++i) B[i] = (float)uniform(-0.2, 0.2);
    for (int i = 0; i < n_bits; ++i) t[i] = (float)uniform(-0.1, 0.1);
    uint8_t* valid = xmalloc(n_kp);
    for (int i = 0; i < n_kp; ++i) valid[i] = (uint8_t)bdref_keypoint_valid(&kps[i]);
    double* resp = xmalloc(sizeof(double) * n_kp * n_bits);
    uint64_t* codes = xmalloc(sizeof(uint64_t) * n_kp * (n_bits / 64));
    bdref_hashsift_project(hist, n_kp, B, t, n_bits, valid, resp, codes);
    bdref_hashsift_project(hist, n_kp, B, t, n_bits, NULL, NULL, codes);
    float* histf = xmalloc(sizeof(float) * n_kp * 128);
    for (int i = 0; i < n_kp * 128; ++i) histf[i] = (float)hist[i];
    bdref_project_lowp(histf, n_kp, B, t, n_bits, 1, resp);
    bdref_project_lowp(histf, n_kp, B, t, n_bits, 2, resp);
    const float special[] = {0.0f, -0.0f, 1.0f, 448.0f, 465.0f, 1e-10f, -3.3e38f, INFINITY, 0x1p-9f, 0x1p-10f};
    for (unsigned i = 0; i < sizeof special / sizeof special[0]; ++i) {
        (void)bdref_round_bf16(special[i]);
        (void)bdref_round_e4m3(special[i]);
    }
    free(histf);
    free(codes);
    free(resp);
    free(valid);
    free(t);
    free(B);
    free(hist);
    free(kps);
    free(imgf);
    free(img8);
}

static void matching(void)
{
    const int n_q = 50, n_t = 33, n_words = 3;
    uint64_t* q = xmalloc(sizeof(uint64_t) * n_q * n_words);
    uint64_t* tr = xmalloc(sizeof(uint64_t) * n_t * n_words);
    for (int i = 0; i < n_q * n_words; ++i) q[i] = next_u64();
    for (int i = 0; i < n_t * n_words; ++i) tr[i] = next_u64();
    memcpy(tr, q, sizeof(uint64_t) * n_words);  /* an exact match */
    memcpy(tr + n_words, q, sizeof(uint64_t) * n_words);  /* and a tie */
    int32_t* idx = xmalloc(sizeof(int32_t) * n_q * 2);
    uint32_t* dist = xmalloc(sizeof(uint32_t) * n_q * 2);
    bdref_match_knn(q, n_q, tr, n_t, n_words, 2, idx, dist);
    bdref_match_knn(q, n_q, tr, 1, n_words, 2, idx, dist);  /* fewer train codes than k */
    bdref_match_knn(q, n_q, tr, 0, n_words, 1, idx, dist);
    int32_t* match = xmalloc(sizeof(int32_t) * n_q);
    double* ratio = xmalloc(sizeof(double) * n_q);
    (void)bdref_match_mutual(q, n_q, tr, n_t, n_words, 0.8, match, dist, ratio);
    (void)bdref_match_mutual(q, n_q, tr, 1, n_words, 0.0, match, dist, NULL);
    (void)bdref_match_mutual(q, n_q, tr, 0, n_words, 0.5, match, dist, ratio);
    free(ratio);
    free(match);
    free(dist);
    free(idx);
    free(tr);
    free(q);
}

static void differentiation(void)
{
    const int n = 6, K = 128;
    float* patches = xmalloc(sizeof(float) * n * 1024);
    for (int i = 0; i < n * 1024; ++i) patches[i] = (float)uniform(0.0, 1.0);
    bdref_box_pair* pairs = xmalloc(sizeof(bdref_box_pair) * K);
    fill_pairs(pairs, K);
    double* w1 = xmalloc(sizeof(double) * K);
    double* w2 = xmalloc(sizeof(double) * K);
    double* theta = xmalloc(sizeof(double) * K);
    for (int j = 0; j < K; ++j) {
        w1[j] = 1.0;
        w2[j] = uniform(0.5, 1.5);
        theta[j] = uniform(-0.1, 0.1);
    }
    double* rho = xmalloc(sizeof(double) * n * K);
    double* dt = xmalloc(sizeof(double) * n * K);
    double* m1 = xmalloc(sizeof(double) * n * K);
    double* m2 = xmalloc(sizeof(double) * n * K);
    bdref_relaxed_bad(patches, n, pairs, w1, w2, theta, K, 10.0, rho, dt, m1, m2);
    bdref_relaxed_bad(patches, n, pairs, w1, w2, theta, K, 10.0, NULL, dt, NULL, NULL);
    double* f = xmalloc(sizeof(double) * n * 128);
    bdref_hashsift_patch_features(patches, n, f);
    double* Bd = xmalloc(sizeof(double) * K * 128);
    double* td = xmalloc(sizeof(double) * K);
    for (int i = 0; i < K * 128; ++i) Bd[i] = uniform(-0.3, 0.3);
    for (int i = 0; i < K; ++i) td[i] = uniform(-0.1, 0.1);
    bdref_relaxed_hashsift(f, n, Bd, td, K, 10.0, rho, dt);
    /* half the batch as anchors, half as positives */
    int32_t* neg = xmalloc(sizeof(int32_t) * (n / 2));
    double* gA = xmalloc(sizeof(double) * (n / 2) * K);
    double* gP = xmalloc(sizeof(double) * (n / 2) * K);
    (void)bdref_trl_hnm(dt, dt + (n / 2) * K, n / 2, K, 0.5, neg, gA, gP);
    (void)bdref_trl_hnm(dt, dt + (n / 2) * K, n / 2, K, 0.5, NULL, NULL, NULL);
    double* gD = xmalloc(sizeof(double) * n * K);
    for (int i = 0; i < n * K; ++i) gD[i] = uniform(-1.0, 1.0);
    double* g1 = xmalloc(sizeof(double) * K);
    double* g2 = xmalloc(sizeof(double) * K);
    double* g3 = xmalloc(sizeof(double) * K);
    bdref_relaxed_bad_grad(gD, dt, m1, m2, n, K, 10.0, g1, g2, g3);
    double* gB = xmalloc(sizeof(double) * K * 128);
    bdref_relaxed_hashsift_grad(gD, dt, f, n, K, 10.0, gB, g3);
    free(gB);
    free(g3);
    free(g2);
    free(g1);
    free(gD);
    free(gP);
    free(gA);
    free(neg);
    free(td);
    free(Bd);
    free(f);
    free(m2);
    free(m1);
    free(dt);
    free(rho);
    free(theta);
    free(w2);
    free(w1);
    free(pairs);
    free(patches);
}

static void selection_and_training(void)
{
    const int n_tr = 5, n_c = 3;
    uint8_t* patches = xmalloc((size_t)3 * n_tr * 1024);
    for (int i = 0; i < 3 * n_tr * 1024; ++i) patches[i] = (uint8_t)next_u64();
    memset(patches, 128, 1024); /* a flat patch: every feature is 0 */
    int32_t* s_ap = xmalloc(sizeof(int32_t) * n_tr);
    int32_t* s_an = xmalloc(sizeof(int32_t) * n_tr);
    for (int i = 0; i < n_tr; ++i) {
        s_ap[i] = (int32_t)(next_u64() % 9) - 4;
        s_an[i] = (int32_t)(next_u64() % 9) - 4;
    }
    bdref_box_pair* cands = xmalloc(sizeof(bdref_box_pair) * 70 * n_c);
    fill_pairs(cands, 70 * n_c);
    cands[0].radius = 15; /* the largest box a 32x32 patch allows */
    (void)bdref_threshold_bin(patches, &cands[0]);
    int32_t* best_bin = xmalloc(sizeof(int32_t) * n_c);
    double* best_loss = xmalloc(sizeof(double) * n_c);
    bdref_find_threshold(patches, n_tr, s_ap, s_an, 1.0, cands, n_c, best_bin, best_loss);
    bdref_find_threshold(patches, 0, s_ap, s_an, 0.5, cands, n_c, best_bin, best_loss);

    const int n_pairs = 8, n_sample = 4, n_bits = 70, n_words = 2;
    uint64_t* ac = xmalloc(sizeof(uint64_t) * n_pairs * n_words);
    uint64_t* pc = xmalloc(sizeof(uint64_t) * n_pairs * n_words);
    for (int i = 0; i < n_pairs * n_words; ++i) {
        ac[i] = next_u64() & 0xF;
        pc[i] = next_u64() & 0xF;
    }
    int32_t* neg = xmalloc(sizeof(int32_t) * n_pairs);
    int32_t* dn = xmalloc(sizeof(int32_t) * n_pairs);
    int32_t* dp = xmalloc(sizeof(int32_t) * n_pairs);
    bdref_hnm_codes(ac, pc, n_pairs, n_words, neg, dn, dp);
    uint8_t* pool = xmalloc((size_t)2 * n_pairs * 1024);
    for (int i = 0; i < 2 * n_pairs * 1024; ++i) pool[i] = (uint8_t)next_u64();
    int32_t* samples = xmalloc(sizeof(int32_t) * n_bits * n_sample);
    for (int i = 0; i < n_bits * n_sample; ++i) samples[i] = (int32_t)(next_u64() % n_pairs);
    bdref_box_pair* table = xmalloc(sizeof(bdref_box_pair) * n_bits);
    int32_t* chosen = xmalloc(sizeof(int32_t) * n_bits);
    int32_t* chosen_bin = xmalloc(sizeof(int32_t) * n_bits);
    double* round_loss = xmalloc(sizeof(double) * n_bits);
    uint64_t* pool_codes = xmalloc(sizeof(uint64_t) * 2 * n_pairs * n_words);
    bdref_select_features(pool, n_pairs, samples, n_sample, cands, n_c, n_bits, 1.0, table, chosen, chosen_bin,
                          round_loss, pool_codes);
    bdref_select_features(pool, n_pairs, samples, n_sample, cands, n_c, 3, 0.5, table, NULL, NULL, NULL, NULL);

    const int n = 4;
    float* src = xmalloc(sizeof(float) * n * 1024);
    for (int i = 0; i < n * 1024; ++i) src[i] = (float)uniform(0.0, 1.0);
    double* params = xmalloc(sizeof(double) * n * 5);
    const double p[4][5] = {{0.0, 1.0, 1.0, 0.0, 0.0}, {0.17, 0.9, 1.2, -0.1, 1.0}, {-0.17, 1.1, 0.8, 0.1, 4.0},
                            {3.14159, 2.0, 1.0, 0.0, 0.3}};
    memcpy(params, p, sizeof p);
    float* noise = xmalloc(sizeof(float) * n * 1024);
    for (int i = 0; i < n * 1024; ++i) noise[i] = (float)uniform(-0.05, 0.05);
    float* dst = xmalloc(sizeof(float) * n * 1024);
    bdref_augment_patches(src, n, params, noise, dst);
    free(dst);
    free(noise);
    free(params);
    free(src);
    free(pool_codes);
    free(round_loss);
    free(chosen_bin);
    free(chosen);
    free(table);
    free(samples);
    free(pool);
    free(dp);
    free(dn);
    free(neg);
    free(pc);
    free(ac);
    free(best_loss);
    free(best_bin);
    free(cands);
    free(s_an);
    free(s_ap);
    free(patches);
}

int main(void)
{
    integral_and_bad();
    hashsift();
    matching();
    differentiation();
    selection_and_training();
    puts("oracle under ASan/UBSan: no reports");
    return 0;
}
