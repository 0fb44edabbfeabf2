/*
 * bdref.h -- plain CPU oracle for the describe-and-match path of
 * "Revisiting Binary Local Image Description for Resource Limited Devices"
 * (Suarez, Buenaposada, Baumela; RA-L 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with the
 * GPU library: its own types, its own loops, FP64 for every floating-point
 * step, no blocking and no reordering beyond the definitions it follows.
 * All pointers are host pointers.  Nothing is allocated for the caller.
 */
#ifndef BDREF_H
#define BDREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Keypoint: centre (x right, y down, pixel centres on integer coordinates),
 * scale = image pixels per normalized-patch pixel, angle in radians. */
typedef struct { float x, y, scale, angle; } bdref_keypoint;

/* BAD weak descriptor: box centres u1 = (x1, y1), u2 = (x2, y2) as offsets
 * from the keypoint in normalized-patch pixels, box radius r (side 2r+1 before
 * scaling) and threshold theta in grey levels.  12 bytes. */
typedef struct {
    int8_t x1, y1, x2, y2;
    uint8_t radius;
    uint8_t pad[3];
    float threshold;
} bdref_box_pair;

/* Integral image (Sec. III-A: box averages in constant time): ii is
 * (H+1) x (W+1) with row stride ii_pitch elements, ii[0][*] = ii[*][0] = 0 and
 * ii[y+1][x+1] = sum of img[y'][x'] over y' <= y, x' <= x, modulo 2^32. */
void bdref_build_integral(const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch,
                          uint32_t* ii, int64_t ii_pitch);

/* BAD codes (Sec. III-A, weak descriptor h(x; f, theta) and the binary vector
 * h(x)).  codes is n_kp x (n_bits/64) words, bit j of a keypoint in word j/64
 * at position j%64, set when f <= theta.  Returns the number of box centres
 * whose rounding lies within 1e-9 of a half-integer tie (near-tie audit). */
int64_t bdref_describe_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch,
                           const bdref_keypoint* kps, int32_t n_kp,
                           const bdref_box_pair* pairs, int32_t n_bits, uint64_t* codes);

/* HashSIFT features (Sec. III-B: SIFT features of the normalized 32x32
 * patch): hist is n_kp x 128, L2-normalized 4x4x8 gradient-orientation
 * histograms in FP64.  dtype 0 = u8 image (read as v/255), 1 = f32 image.
 * img_pitch is in bytes. */
void bdref_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                         const bdref_keypoint* kps, int32_t n_kp, double* hist);

/* HashSIFT binarization (Sec. III-B, D(x) = sgn(B [f; 1])): resp[i][j] =
 * sum_k B[j][k] f_i[k] - t[j] in FP64, bit j set when resp > 0.  B is
 * n_bits x 128 (f32, row major), t has n_bits entries.  resp may be NULL.
 * valid (may be NULL) marks keypoints whose code is forced to zero when 0. */
void bdref_hashsift_project(const double* hist, int32_t n_kp, const float* B, const float* t,
                            int32_t n_bits, const uint8_t* valid, double* resp, uint64_t* codes);

/* Reduced-precision operand rounding (not in the paper; the precision
 * extension of the projection).  Round-to-nearest-even to bfloat16, and to
 * OCP float8 e4m3 (4 exponent bits, bias 7, 3 mantissa bits, largest finite
 * 448), saturating at +-448. */
float bdref_round_bf16(float x);
float bdref_round_e4m3(float x);

/* Responses of the projection with rounded operands, accumulated exactly in
 * FP64: precision 1 = BF16 (both operands rounded to bfloat16), 2 = FP8
 * (per-row scale s = the smallest power of two >= 2^-126 with
 * max|row| <= 448 s, for every feature row and every B row, so that x / s is
 * exact; operands x / s rounded to e4m3; response = s_f * s_B * sum q_B q_f
 * - t).  hist is n_kp x 128 float32. */
void bdref_project_lowp(const float* hist, int32_t n_kp, const float* B, const float* t, int32_t n_bits,
                        int32_t precision, double* resp);

/* ---- Relaxed descriptors and the triplet ranking loss (Sec. III-A Eq. 1,
 * Sec. III-B Eq. 3; the differentiation extension).  Patches are n 32x32
 * float32 images (row-major, 1024 values each).
 *
 * Relaxed BAD on a patch: the patch is an image with keypoint (15.5, 15.5),
 * scale 1, angle 0, so pair j's box of radius R = r_j is centred at
 * (16 + u_x, 16 + u_y) clamped to [R, 31 - R]; m1, m2 are the two box means
 * (FP64 pixel sums / (2R+1)^2) and
 *   rho_j = theta_j - (w1_j m1_j - w2_j m2_j),   D_j = tanh(beta rho_j).
 * With w1 = w2 = 1 the bit [rho_j >= 0] is the BAD stump [f <= theta].
 * rho, dt, m1, m2 are n x K (any may be NULL). */
void bdref_relaxed_bad(const float* patches, int32_t n, const bdref_box_pair* pairs, const double* w1,
                       const double* w2, const double* theta, int32_t n_bits, double beta, double* rho,
                       double* dt, double* m1, double* m2);

/* Relaxed HashSIFT: rho = B f - t for features f (n x 128, FP64),
 * D = tanh(beta rho).  B is K x 128, t has K entries (FP64). */
void bdref_relaxed_hashsift(const double* f, int32_t n, const double* B, const double* t, int32_t n_bits,
                            double beta, double* rho, double* dt);

/* Triplet ranking loss with in-batch hardest negatives and anchor swap:
 * s(x, y) = D(x) . D(y) / K for anchors A (n x K) and positives P (n x K);
 * s_neg(i) = max(max_{j != i} s(a_i, p_j), max_{j != i} s(a_j, p_i)) (ties:
 * the row candidate first, then the lowest j); loss = mean_i
 * [tau - s(a_i, p_i) + s_neg(i)]_+.  Outputs: the loss; for each i the
 * chosen negative neg[i] = j for a row candidate s(a_i, p_j) or -1 - j for a
 * column candidate s(a_j, p_i); and the analytic gradients dL/dA, dL/dP
 * (n x K, may be NULL) with a zero subgradient at the hinge kink. */
double bdref_trl_hnm(const double* A, const double* P, int32_t n, int32_t n_bits, double tau, int32_t* neg,
                     double* gA, double* gP);

/* Chain rule through the relaxed descriptors: from dL/dD (n x K) and D,
 *   BAD:      dL/dtheta_j = sum_x g_j, dL/dw1_j = -sum_x g_j m1_j, dL/dw2_j = sum_x g_j m2_j
 *   HashSIFT: dL/dB = sum_x g f^T (K x 128), dL/dt = -sum_x g
 * with g = dL/dD * beta * (1 - D^2).  Outputs are accumulated (+=). */
void bdref_relaxed_bad_grad(const double* gD, const double* dt, const double* m1, const double* m2, int32_t n,
                            int32_t n_bits, double beta, double* g_w1, double* g_w2, double* g_theta);
void bdref_relaxed_hashsift_grad(const double* gD, const double* dt, const double* f, int32_t n, int32_t n_bits,
                                 double beta, double* gB, double* gt);

/* HashSIFT features of 32x32 patches (keypoint (15.5, 15.5), scale 1,
 * angle 0, so every sample is a patch pixel, clamp-to-edge in the apron). */
void bdref_hashsift_patch_features(const float* patches, int32_t n, double* f);

/* 1 when the keypoint has finite fields and a positive scale. */
int32_t bdref_keypoint_valid(const bdref_keypoint* kp);

/* Brute-force Hamming k-NN (Sec. III-A similarity S = h(x)^T h(y), i.e. K
 * minus twice the Hamming distance): for each query the k smallest
 * (distance, train index) pairs in lexicographic order.  Slots beyond n_t
 * get idx = -1, dist = 0xFFFFFFFF. */
void bdref_match_knn(const uint64_t* query, int32_t n_q, const uint64_t* train, int32_t n_t,
                     int32_t n_words, int32_t k, int32_t* idx, uint32_t* dist);

/* Mutual nearest neighbours with a distance-ratio filter (the Hamming MNN
 * matcher of the Sec. IV pipeline timing, Table of pipeline steps).  For
 * query i let j = the train index of the smallest distance d1 (ties: lowest
 * index) and d2 the second smallest distance over the other train codes.
 * i and j match when i is also the nearest query of train j (ties: lowest
 * index) and, if max_ratio > 0, d1 < max_ratio * d2 in double precision
 * (always true when n_t < 2).  match[i] = j or -1; dist[i] = d1
 * (0xFFFFFFFF when n_t = 0); ratio[i] = d1 / d2 (1 when d2 = 0, 0 when
 * n_t < 2), may be NULL.  Returns the number of matches. */
int32_t bdref_match_mutual(const uint64_t* query, int32_t n_q, const uint64_t* train, int32_t n_t,
                           int32_t n_words, double max_ratio, int32_t* match, uint32_t* dist, double* ratio);

/* ------------------------------------------------------------------ feature selection */

/* Threshold search of a candidate BAD feature over a triplet set (Sec. III-A,
 * Alg. 2 with the integer-sorting speed-up).  patches: 3 n_triplets u8
 * 32x32 patches, triplet i = (anchor 3i, positive 3i+1, negative 3i+2).  The
 * candidate's feature on a patch is f = mean(box 1) - mean(box 2), boxes of
 * side 2r+1 (r <= 15) centred at 16 + (x, y) clamped to [r, 31 - r]; its
 * bin is q = floor((f + 255) * 10) in [0, 5100] of BDREF_THRESHOLD_BINS =
 * 5110 (precision 0.1 over [-255, 255]).  A threshold after bin b gives the
 * stump h(x) = +1 if q(x) <= b, else -1, and the loss of Eq. 2,
 *   L(b) = sum_i [tau - s_ap[i] - h(a_i) h(p_i) + s_an[i] + h(a_i) h(n_i)]_+,
 * with s_ap, s_an the similarities of the previously selected bits.  Per
 * candidate: best_bin = the lowest b with the smallest L(b), best_loss =
 * L(best_bin).  Per-triplet loss changes are attributed to the triplet's
 * three patches in the order of (bin, position in the triplet), so tied
 * values flip together exactly. */
#define BDREF_THRESHOLD_BINS 5110
int32_t bdref_threshold_bin(const uint8_t* patch, const bdref_box_pair* cand);
void bdref_find_threshold(const uint8_t* patches, int32_t n_triplets, const int32_t* s_ap, const int32_t* s_an,
                          double tau, const bdref_box_pair* cands, int32_t n_cands, int32_t* best_bin,
                          double* best_loss);

/* In-batch hardest negatives with anchor swap for n (anchor, positive) code
 * pairs of n_words words: for pair s the row candidate is the positive p_j
 * (j != s) nearest to a_s and the column candidate the anchor a_j (j != s)
 * nearest to p_s (Hamming distance; among equal distances the first j in the
 * cyclic order s+1, s+2, ..., s-1 mod n).  The row candidate wins ties
 * between the two.  neg[s] = j for a row candidate, -1 - j for a column
 * candidate; dist_neg[s] = its distance, dist_pos[s] = d(a_s, p_s).  n >= 2. */
void bdref_hnm_codes(const uint64_t* a_codes, const uint64_t* p_codes, int32_t n, int32_t n_words, int32_t* neg,
                     int32_t* dist_neg, int32_t* dist_pos);

/* Greedy BAD feature selection (Sec. III-A, Alg. 1).  pool: 2 n_pairs u8
 * 32x32 patches, pair i = (anchor 2i, positive 2i+1), each pair its own 3D
 * point.  Round k (0 <= k < n_bits) samples the pairs samples[k * n_sample ..]
 * (n_sample >= 2), forms triplets with bdref_hnm_codes on the codes of the k
 * bits selected so far (a column candidate swaps anchor and positive: the
 * triplet is (p_s, a_s, a_j)), sets s_ap = k - 2 d(anchor, positive) and
 * s_an = k - 2 d(anchor, negative), runs bdref_find_threshold for the
 * candidates cands[k * n_cands ..] and keeps the first candidate of lowest
 * loss.  Its stump (+1 iff bin <= best bin) becomes bit k of every pool
 * patch.  Outputs: table[k] = the chosen pair with threshold
 * (bin + 1 - 2550) / 10 - 1 / (20 area) (so that f <= threshold iff
 * bin <= best bin), chosen[k], chosen_bin[k], round_loss[k] (each optional
 * except table), pool_codes (2 n_pairs x ceil(n_bits / 64) words, optional;
 * bit j of a patch in word j / 64 at position j % 64). */
void bdref_select_features(const uint8_t* pool, int32_t n_pairs, const int32_t* samples, int32_t n_sample,
                           const bdref_box_pair* cands, int32_t n_cands, int32_t n_bits, double tau,
                           bdref_box_pair* table, int32_t* chosen, int32_t* chosen_bin, double* round_loss,
                           uint64_t* pool_codes);

/* Data augmentation of 32x32 float patches for HashSIFT training (Sec.
 * III-B lists the kinds of perturbation; here each patch is rotated and
 * rescaled about its centre, blurred, given a gain and a bias, and has
 * Gaussian noise added; the random draws are inputs).  params: n x 5
 * (angle, scale, gain, bias, sigma) per patch.  Output pixel (i, j) takes
 *   1. the bilinear sample (clamp-to-edge) of the source at
 *      (15.5, 15.5) + scale * Rot(angle) (j - 15.5, i - 15.5),
 *   2. a separable Gaussian blur of standard deviation sigma (at most 4; weights
 *      exp(-d^2 / (2 sigma^2)) for |d| <= ceil(3 sigma), normalised,
 *      clamp-to-edge; none when sigma <= 0),
 *   3. gain * v + bias, 4. + noise[i][j], 5. clipped to [0, 1].
 * FP64 throughout, result rounded to float. */
void bdref_augment_patches(const float* src, int32_t n, const double* params, const float* noise, float* dst);

#ifdef __cplusplus
}
#endif
#endif
