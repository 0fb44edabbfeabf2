/*
 * bdesc.h -- C ABI of the describe-and-match library for AMD Instinct MI355X
 * (gfx950): BAD and HashSIFT binary local descriptors and brute-force
 * Hamming k-NN, after Suarez, Buenaposada and Baumela, "Revisiting Binary
 * Local Image Description for Resource Limited Devices" (RA-L 2021).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Every array argument is a DEVICE pointer allocated and owned by the
 *    caller.  The library never frees caller memory and keeps no reference
 *    to it after the call returns.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    the call returns without synchronizing.  A device fault surfaces at the
 *    caller's next synchronization.
 *  - Arguments are validated on the host before anything is enqueued.  The
 *    return value is BD_OK (0) or a negative BD_E* code; bd_last_error()
 *    then returns a message for the calling thread.  Nothing is thrown and
 *    nothing aborts across this boundary.
 *  - A bd_context owns the library's device workspace (grown on demand;
 *    growing it synchronizes the stream) and is bound to one device.  A
 *    context is not thread-safe: use one per host thread, and do not let
 *    calls on different streams overlap on one context.
 *  - Keypoints: pixel centres lie on integer coordinates, x to the right, y
 *    down.  `scale` is image pixels per normalized-patch pixel, `angle` in
 *    radians rotates the patch x axis onto (cos a, sin a).  A keypoint with a
 *    non-finite field or scale <= 0 is invalid and gets an all-zero code.
 *  - Codes: n_bits/64 uint64 words per keypoint, bit j in word j/64 at
 *    position j%64 (LSB first).
 */
#ifndef BDESC_H
#define BDESC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BD_OK 0
#define BD_EINVAL (-1)        /* null pointer, bad size, pitch or count */
#define BD_EUNSUPPORTED (-2)  /* n_bits, k, dtype or precision not provided */
#define BD_ENOMEM (-3)        /* workspace allocation failed */
#define BD_EDEVICE (-4)       /* HIP runtime error (launch, device query) */

#define BD_DTYPE_U8 0  /* grey levels 0..255; HashSIFT reads v / 255 */
#define BD_DTYPE_F32 1 /* float32 grey levels */
/* float32 grey levels stored as row pairs (HashSIFT only): element (y, x)
 * is the float2 (I[y][x], I[min(y + 1, H - 1)][x]), W float2 per row, row
 * stride a multiple of 8 bytes; bd_prepare_view writes it.  Same features as
 * BD_DTYPE_F32 on I, bit for bit; the sampler reads a sample's four corner
 * pixels with one 16-byte load instead of two 8-byte ones. */
#define BD_DTYPE_F32_ROWPAIR 2

#define BD_PREC_FP32 0 /* FP32 operands, FP32 MFMA */
#define BD_PREC_BF16 1 /* bfloat16 operands (round to nearest even), FP32 accumulation */
#define BD_PREC_FP8 2  /* OCP float8 e4m3 operands, each row scaled by a power of two, FP32 accumulation */

typedef struct bd_keypoint {
    float x, y, scale, angle;
} bd_keypoint; /* 16 bytes */

/* One BAD weak descriptor (Sec. III-A, h(x; f, theta) on f(x; u1, u2, s)):
 * box centres u1 = (x1, y1), u2 = (x2, y2) as offsets from the keypoint in
 * normalized-patch pixels, box radius (side 2*radius+1 before scaling) and
 * threshold theta in grey levels. */
typedef struct bd_box_pair {
    int8_t x1, y1, x2, y2;
    uint8_t radius;
    uint8_t pad[3];
    float threshold;
} bd_box_pair; /* 12 bytes */

typedef struct bd_context bd_context;

/* Create a context bound to HIP device `device`.  *out receives the context.
 * The first context on a device also resolves that device's address of the
 * fixed scratch array of bd_match_hamming_knn_noalloc. */
int bd_context_create(bd_context** out, int device);

/* Free the context's workspace (synchronizes the device).  NULL is a no-op. */
int bd_context_destroy(bd_context* ctx);

/* Invalid keypoints (Sec. III-A, III-B: one code per keypoint; a keypoint
 * with a non-finite field or scale <= 0 has no patch and gets an all-zero
 * code, or a zero feature row).  Every describe call made with this context
 * adds one to a device counter per invalid keypoint it meets:
 * bd_describe_bad, bd_describe_bad_table, bd_describe_hashsift (once per
 * keypoint, although it also projects), bd_hashsift_features, and the BAD
 * and HashSIFT stages of bd_batch_run.  bd_hashsift_project does not count
 * (its kps argument only masks codes).  bd_context_poll synchronizes the
 * context's device, stores the count accumulated since the context was
 * created or last polled in *invalid_count, and resets the counter to zero.
 * Errors: BD_EINVAL (null pointer), BD_EDEVICE. */
int bd_context_poll(bd_context* ctx, uint64_t* invalid_count);

/* Message describing the last non-zero return on the calling thread. */
const char* bd_last_error(void);

/* Library version string. */
const char* bd_version(void);

/*
 * Integral image of a u8 grey image (Sec. III-A: box averages in constant
 * time from an integral image).
 *   img      H rows of W bytes, row stride img_pitch bytes (>= W)
 *   ii       (H+1) rows of (W+1) uint32, row stride ii_pitch elements
 *            (>= W+1); ii[0][*] = ii[*][0] = 0 and ii[y+1][x+1] is the sum of
 *            img over rows <= y and columns <= x, modulo 2^32.
 * W, H >= 1 and (H+1) * ii_pitch < 2^31.  Two kernels for images of up to
 * 2048 rows (tile and group sums, tile prefixes with their carries summed
 * from the sums), three above (tile sums, carry scans, tile prefixes); about
 * (W*H/16 * 1.25 + 1024) * 4 bytes of workspace.
 */
int bd_build_integral(bd_context* ctx, const uint8_t* img, int32_t W, int32_t H,
                      int64_t img_pitch, uint32_t* ii, int64_t ii_pitch, void* stream);

/*
 * Spatial processing order for a keypoint set: order receives a permutation
 * of 0..n_kp-1 that groups keypoints by cell of a 64 x 64 grid over the W x H
 * image, cells in Morton order (keypoints within a cell in no fixed order).
 * Passing it to the describe calls makes each XCD of the GPU work on one
 * image region, which keeps its gathers in that XCD's L2.  It never changes
 * the codes: every code is still written at its keypoint's own index.  One
 * order serves BAD and HashSIFT of the same keypoints.  n_kp <= 2^31 - 1.
 */
int bd_keypoint_order(bd_context* ctx, const bd_keypoint* kps, int32_t n_kp, int32_t W, int32_t H,
                      int32_t* order, void* stream);

/*
 * bd_build_integral and bd_keypoint_order of one view in one call: the
 * integral image of img and the processing order of kps over the same
 * W x H image, with the sort running in one extra workgroup of the integral
 * image's first pass instead of in a launch of its own (the two results
 * share nothing, so a chain integral -> describe waits for one launch
 * fewer).  Arguments, layouts and errors as in the two calls; ii is written
 * exactly as bd_build_integral writes it and order is a permutation with
 * the same cell grouping as bd_keypoint_order's (keypoints within a cell
 * in no fixed order).  n_kp = 0 builds the integral image only.
 */
int bd_build_integral_order(bd_context* ctx, const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch,
                            uint32_t* ii, int64_t ii_pitch, const bd_keypoint* kps, int32_t n_kp,
                            int32_t* order, void* stream);

/*
 * Everything the describe calls of one view read, from one call:
 * bd_build_integral_order plus, when hs_img is given, the row-pair copy of
 * the view's float32 HashSIFT image (BD_DTYPE_F32_ROWPAIR) written to
 * pairs, all in the same launches.
 *   hs_img   H rows of W float32 (the HashSIFT source), row stride hs_pitch
 *            bytes (a multiple of 4, >= 4 W); NULL with pairs NULL for none
 *   pairs    H rows of W float2, row stride pairs_pitch bytes (a multiple of
 *            8, >= 8 W): element (y, x) = (hs[y][x], hs[min(y+1, H-1)][x])
 * Pass pairs to bd_hashsift_features / bd_describe_hashsift with dtype
 * BD_DTYPE_F32_ROWPAIR and img_pitch = pairs_pitch: the features are those
 * of hs_img, bit for bit.  Errors as in bd_build_integral_order, and
 * BD_EINVAL for a missing half of the HashSIFT pair or bad pitches.
 */
int bd_prepare_view(bd_context* ctx, const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch, uint32_t* ii,
                    int64_t ii_pitch, const bd_keypoint* kps, int32_t n_kp, int32_t* order, const float* hs_img,
                    int64_t hs_pitch, float* pairs, int64_t pairs_pitch, void* stream);

/*
 * BAD codes (Sec. III-A: weak descriptor h(x; f, theta) = +1 when
 * f(x; u1, u2, s) <= theta, f the difference of the mean grey levels of two
 * boxes of side s; the bits of h(x) = [h_1 .. h_K]).
 *   ii       integral image of a W x H u8 image as written by
 *            bd_build_integral, row stride ii_pitch elements
 *   kps      n_kp keypoints;  pairs  n_bits box pairs
 *   order    optional (NULL): processing order from bd_keypoint_order (any
 *            permutation of 0..n_kp-1; entries outside that range are skipped)
 *   codes    n_kp x n_bits/64 words; bit j set when h_j = +1
 * n_bits is 256 or 512.  Per keypoint and pair: box radius
 * R = floor(radius * scale + 0.5) capped at (min(W,H)-1)/2, centre = patch
 * point kp + scale * Rot(angle) * u rounded half up (FP64) and clamped so the
 * box lies inside the image, bit = [S1 - S2 <= theta * (2R+1)^2] exactly.
 */
int bd_describe_bad(bd_context* ctx, const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch,
                    const bd_keypoint* kps, int32_t n_kp, const int32_t* order,
                    const bd_box_pair* pairs, int32_t n_bits, uint64_t* codes, void* stream);

/* Compiled BAD table: the distinct boxes of the pairs, each pair referring
 * to its two boxes, and for each of 32 bins of the keypoint angle an order
 * of all box corners sorted by their image position at the bin's central
 * angle.  bd_describe_bad_table gathers a keypoint's corners in its bin's
 * order (so the lanes of a load instruction and the next loads fall on few
 * cache lines), forms the box sums and the bits from them; the codes are
 * identical to bd_describe_bad's.  Create enqueues the compilation on
 * `stream` (use the table on that stream, or after synchronizing it); the
 * table holds its own device memory (16 + 16 n_bits + 512 n_bits bytes)
 * until destroyed (destroy synchronizes the device).  n_bits 256 or 512. */
typedef struct bd_bad_table bd_bad_table;
int bd_bad_table_create(bd_context* ctx, const bd_box_pair* pairs, int32_t n_bits, bd_bad_table** out, void* stream);
int bd_bad_table_destroy(bd_bad_table* table);
int bd_describe_bad_table(bd_context* ctx, const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch,
                          const bd_keypoint* kps, int32_t n_kp, const int32_t* order, const bd_bad_table* table,
                          uint64_t* codes, void* stream);

/*
 * HashSIFT codes (Sec. III-B: D(x) = sgn(B [f(x); 1]) with f the SIFT
 * feature vector of the normalized 32x32 patch).
 *   img      H rows of W pixels (dtype BD_DTYPE_U8, BD_DTYPE_F32 or
 *            BD_DTYPE_F32_ROWPAIR), row stride img_pitch bytes (a multiple
 *            of 4 for f32, of 8 for row pairs)
 *   order    optional (NULL) processing order, as for bd_describe_bad
 *   B        n_bits x 128 float32, row major;  t  n_bits thresholds
 *            (the paper's last column of B is -t)
 *   codes    n_kp x n_bits/64 words; bit j set when r_j = B_j . f - t_j > 0
 *   hist_out optional (NULL) n_kp x 128 float32 features f
 *   resp_out optional (NULL) n_kp x n_bits float32 responses r
 *   precision BD_PREC_FP32, BD_PREC_BF16 or BD_PREC_FP8 (the reduced-precision
 *            forms are an extension: the paper fixes no precision).  With
 *            BF16/FP8 every response with |r| < margin is recomputed from the
 *            unrounded FP32 operands and decides the bit: four partial sums
 *            over the float4 groups k/4 = j mod 4, each in four running sums
 *            over the components (added as (s0 + s1) + (s2 + s3)), the four
 *            partials added in pairs; in FP64 when that FP32 value is within
 *            1e-6 of the threshold.  A NaN response gives bit 0.  FP8 scales
 *            every row of f and of B by the smallest power of two
 *            s >= 2^-126 with max|row| <= 448 s before rounding to e4m3;
 *            recheck_count (optional device u32, caller-zeroed) is increased
 *            by the number of such responses.  margin is ignored for FP32.
 * n_bits is 256 or 512.  f: 34x34 bilinear
 * samples (clamp-to-edge) at patch offsets (j - 15.5, i - 15.5), central
 * differences, Gaussian window sigma 16, trilinear votes into 4x4 cells x 8
 * orientations (index (cy*4 + cx)*8 + o), L2-normalized (zero stays zero).
 * The projection runs on FP32 MFMA.
 */
int bd_describe_hashsift(bd_context* ctx, const void* img, int32_t dtype, int32_t W, int32_t H,
                         int64_t img_pitch, const bd_keypoint* kps, int32_t n_kp, const int32_t* order,
                         const float* B, const float* t, int32_t n_bits, int32_t precision, float margin,
                         uint64_t* codes, float* hist_out, float* resp_out, uint32_t* recheck_count,
                         void* stream);

/*
 * HashSIFT features only (the f(x) of Sec. III-B, exactly as computed inside
 * bd_describe_hashsift): hist receives n_kp x 128 float32, L2-normalized;
 * invalid keypoints give zero rows.  Arguments as bd_describe_hashsift.
 */
int bd_hashsift_features(bd_context* ctx, const void* img, int32_t dtype, int32_t W, int32_t H,
                         int64_t img_pitch, const bd_keypoint* kps, int32_t n_kp, const int32_t* order,
                         float* hist, void* stream);

/*
 * HashSIFT binarization of given features (Sec. III-B, D = sgn(B [f; 1])):
 * r = B f - t on MFMA in the given precision (as bd_describe_hashsift, with
 * the same margin re-check), bit j set when r_j > 0.
 *   hist     n_kp x 128 float32 features (row stride 128)
 *   kps      optional (NULL = all valid): keypoints whose codes are forced
 *            to zero when invalid, as in bd_describe_hashsift
 *   resp_out optional (NULL) n_kp x n_bits float32 responses
 */
int bd_hashsift_project(bd_context* ctx, const float* hist, const bd_keypoint* kps, int32_t n_kp,
                        const float* B, const float* t, int32_t n_bits, int32_t precision, float margin,
                        uint64_t* codes, float* resp_out, uint32_t* recheck_count, void* stream);

/*
 * Brute-force Hamming k-NN (Sec. III-A: S(x, y) = h(x)^T h(y) = K - 2 d_H,
 * so the most similar code has the smallest Hamming distance).
 *   query    n_q x n_words words;  train  n_t x n_words words
 *   idx      n_q x k int32 train indices;  dist  n_q x k uint32 distances
 * For each query the k smallest (distance, train index) pairs in
 * lexicographic order (equal distances: lower index first).  Slots beyond
 * n_t get idx = -1 and dist = 0xFFFFFFFF.  n_words in 1..8, k in 1..2.
 * Codes of 4 and 8 words (256 and 512 bits) run on the int8 MFMA units as
 * the inner product of {0, -64} query bytes with +-1 train bytes (exact);
 * other widths on a lane-per-query XOR/popcount kernel.  Codes must be
 * 8-byte aligned.
 */
int bd_match_hamming_knn(bd_context* ctx, const uint64_t* query, int32_t n_q,
                         const uint64_t* train, int32_t n_t, int32_t n_words, int32_t k,
                         int32_t* idx, uint32_t* dist, void* stream);

/* bd_match_hamming_knn without any allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops
 * and harnesses that forbid hipMalloc.  Same arguments, kernels, launch
 * shapes and results as bd_match_hamming_knn; the per-split partial keys go
 * to a fixed scratch array of BD_NOALLOC_SCRATCH_BYTES in device memory
 * instead of the context workspace (its address on each device is resolved
 * once, by bd_context_create; each device keeps its copy until the process
 * ends).  A problem whose partial keys, 4 * k * n_q * splits bytes with
 * splits = ceil(n_t / rows per split) (the planner's choice, up to 2048 rows
 * for 256/512-bit codes), exceed that size is rejected with BD_EINVAL
 * before anything is enqueued.  The call never allocates, frees or
 * synchronizes.  Every call on one device shares that device's array and
 * leaves its last contents there (nothing needs to start at zero: each slot
 * is written before it is read), so calls that overlap in time on one
 * device, on any stream or context, race and must be serialized by the
 * caller. */
#define BD_NOALLOC_SCRATCH_BYTES (16 * 1024 * 1024)
int bd_match_hamming_knn_noalloc(bd_context* ctx, const uint64_t* query, int32_t n_q,
                                 const uint64_t* train, int32_t n_t, int32_t n_words, int32_t k,
                                 int32_t* idx, uint32_t* dist, void* stream);

/* Mutual nearest neighbours with a distance-ratio filter: the Hamming MNN
 * matcher of the paper's pipeline timing (Sec. IV, Table of the pipeline
 * steps).  For query i, j is its nearest train code (smallest distance d1,
 * ties: lowest index) and d2 the smallest distance to any other train code.
 * i and j match when query i is also train j's nearest query (ties: lowest
 * index) and, if max_ratio > 0, d1 < max_ratio * d2 (evaluated in double;
 * always true when n_t < 2).  Outputs (device, n_q each): match[i] = j or
 * -1, dist[i] = d1 (0xFFFFFFFF when n_t = 0), ratio[i] = d1 / d2 (1 when
 * d2 = 0, 0 when n_t < 2; optional), *count = number of matches (optional
 * device int32).  n_words 1..8; max_ratio finite, >= 0 (0: no filter).
 * Uses the context workspace for both k-NN passes. */
int bd_match_mutual(bd_context* ctx, const uint64_t* query, int32_t n_q, const uint64_t* train, int32_t n_t,
                    int32_t n_words, float max_ratio, int32_t* match, uint32_t* dist, float* ratio, int32_t* count,
                    void* stream);

/* Threshold search for candidate BAD features (Sec. III-A, Alg. 2 with the
 * integer sorting the paper proposes for it).  patches: 3 n_triplets u8
 * 32x32 patches (1024 bytes each, row-major), triplet i = (anchor 3i,
 * positive 3i+1, negative 3i+2); s_ap, s_an (n_triplets int32): the
 * similarities h^T h of each triplet's (anchor, positive) and (anchor,
 * negative) under the features selected so far; cands: n_cands box pairs
 * (threshold field ignored).  A candidate's feature on a patch is
 * f = mean(box 1) - mean(box 2), boxes of side 2r+1 (r <= 15) centred at
 * 16 + (x, y) clamped to [r, 31 - r]; its bin is q = floor((f + 255) * 10),
 * one of m = 5110 bins (precision 0.1 over [-255, 255]).  The stump after
 * bin b is h(x) = +1 if q(x) <= b, else -1, with the loss of Eq. 2
 *   L(b) = sum_i [tau - s_ap - h(a)h(p) + s_an + h(a)h(n)]_+.
 * Outputs per candidate (device): best_bin = the lowest b of smallest L(b),
 * best_theta = (best_bin + 1 - 2550) / 10 (so h = +1 iff f < best_theta;
 * optional), best_loss = L(best_bin) (optional).  tau must be a multiple of
 * 1/2 (all loss values are then exact).  Workspace: 5110 x n_cands int32. */
int bd_find_threshold(bd_context* ctx, const uint8_t* patches, int32_t n_triplets, const int32_t* s_ap,
                      const int32_t* s_an, float tau, const bd_box_pair* cands, int32_t n_cands, int32_t* best_bin,
                      float* best_theta, double* best_loss, void* stream);

/* Greedy BAD feature selection (Sec. III-A, Alg. 1), all rounds on the
 * device.  pool: 2 n_pairs u8 32x32 patches (16-byte aligned), pair i =
 * (anchor 2i, positive 2i+1), each pair its own 3D point.  Round k
 * (0 <= k < n_bits) takes the n_sample pairs samples[k n_sample ..] (indices
 * in [0, n_pairs); out-of-range values are clamped), forms triplets by
 * in-batch hardest negatives on the codes of the k bits selected so far,
 * with anchor swap (for pair s the nearest positive p_j of a_s, j != s, and
 * the nearest anchor a_j of p_s; equal distances go to the first j in
 * cyclic order s+1, s+2, ..., and a positive beats an anchor; an
 * anchor winner makes the triplet (p_s, a_s, a_j)), runs the threshold
 * search of bd_find_threshold with s_ap = k - 2 d(anchor, positive),
 * s_an = k - 2 d(anchor, negative) over the n_cands candidates
 * cands[k n_cands ..], and keeps the first candidate of lowest loss; its
 * stump becomes bit k of every pool patch.  Outputs (device): table[k] =
 * the chosen pair, threshold (bin + 1 - 2550) / 10 - 1 / (20 area) so that
 * the BAD stump f <= threshold equals bin <= chosen bin; chosen[k],
 * chosen_bin[k], round_loss[k] and pool_codes (2 n_pairs x ceil(n_bits/64)
 * u64) are optional.  n_bits 1..512, 2 <= n_sample <= n_pairs, tau a
 * multiple of 1/2.  Uses the context workspace. */
int bd_select_features(bd_context* ctx, const uint8_t* pool, int32_t n_pairs, const int32_t* samples,
                       int32_t n_sample, const bd_box_pair* cands, int32_t n_cands, int32_t n_bits, float tau,
                       bd_box_pair* table, int32_t* chosen, int32_t* chosen_bin, double* round_loss,
                       uint64_t* pool_codes, void* stream);

/* ------------------------------------------------------------------------
 * Differentiation extension (not proposed by the paper): relaxed descriptors
 * D = tanh(beta * rho) and the triplet ranking loss with in-batch hardest
 * negatives (Sec. III-A Eq. 1, Sec. III-B Eq. 3; HNM and anchor swap as in
 * the training of Sec. III), with hand-written backward passes.  Patches are
 * n 32x32 float32 images (1024 values each, row-major); per-sample arrays
 * are n x n_bits float32, row-major.  All reductions have a fixed order.
 * ---------------------------------------------------------------------- */

/* HashSIFT features of 32x32 patches: each patch is an image with its
 * keypoint at the centre (15.5, 15.5), scale 1, angle 0.  hist: n x 128. */
int bd_hashsift_patch_features(bd_context* ctx, const float* patches, int32_t n, float* hist, void* stream);

/* Relaxed BAD: with box means m1, m2 of pair j on the patch (boxes centred at
 * 16 + u, radius r, clamped to [r, 31 - r]),
 *   rho_j = theta_j - (w1_j m1_j - w2_j m2_j),  D_j = tanh(beta rho_j).
 * With w1 = w2 = 1 the sign of rho_j is the BAD stump of Sec. III-A.
 * m1, m2 (n x n_bits, optional) keep the box means for the backward pass.
 * n_bits: a multiple of 64 (<= 4096); beta > 0. */
int bd_relaxed_bad_fwd(bd_context* ctx, const float* patches, int32_t n, const bd_box_pair* pairs, const float* w1,
                       const float* w2, const float* theta, int32_t n_bits, float beta, float* D, float* m1,
                       float* m2, void* stream);

/* Gradients of the relaxed BAD parameters from dL/dD (gD): with
 * g = gD * beta * (1 - D^2): dL/dtheta_j = sum g_j, dL/dw1_j = -sum g_j m1_j,
 * dL/dw2_j = sum g_j m2_j over the n patches (outputs overwritten). */
int bd_relaxed_bad_bwd(bd_context* ctx, const float* gD, const float* D, const float* m1, const float* m2, int32_t n,
                       int32_t n_bits, float beta, float* g_w1, float* g_w2, float* g_theta, void* stream);

/* Relaxed HashSIFT: rho = B f - t (FP32 MFMA), D = tanh(beta rho); f is
 * n x 128, B n_bits x 128, t n_bits; rho (optional) receives rho. */
int bd_relaxed_hashsift_fwd(bd_context* ctx, const float* f, int32_t n, const float* B, const float* t, int32_t n_bits,
                            float beta, float* rho, float* D, void* stream);

/* dL/dB = sum_x g f^T (n_bits x 128), dL/dt = -sum_x g, g = gD beta (1 - D^2). */
int bd_relaxed_hashsift_bwd(bd_context* ctx, const float* gD, const float* D, const float* f, int32_t n,
                            int32_t n_bits, float beta, float* gB, float* gt, void* stream);

/* Triplet ranking loss with in-batch hardest negatives and anchor swap:
 * s(x, y) = D(x) . D(y) / n_bits for anchors A and positives P (n x n_bits),
 * s_neg(i) = max(max_{j != i} s(a_i, p_j), max_{j != i} s(a_j, p_i)) (ties:
 * the row candidate, then the lowest j), loss = mean_i [tau - s(a_i, p_i) +
 * s_neg(i)]_+ (one float at *loss).  neg[i] = j for a row candidate, -1 - j
 * for a column candidate; hinge[i] = tau - s(a_i, p_i) + s_neg(i).  The
 * n x n similarity is formed in 128 x 128 MFMA tiles and never stored. */
int bd_trl_hnm_fwd(bd_context* ctx, const float* A, const float* P, int32_t n, int32_t n_bits, float tau, float* loss,
                   int32_t* neg, float* hinge, void* stream);

/* dL/dA, dL/dP (n x n_bits) for upstream gradient *grad_loss (device), from
 * the neg and hinge arrays of the forward pass; zero subgradient at the kink. */
int bd_trl_hnm_bwd(bd_context* ctx, const float* A, const float* P, int32_t n, int32_t n_bits, const int32_t* neg,
                   const float* hinge, const float* grad_loss, float* gA, float* gP, void* stream);

/* ------------------------------------------------------------------------
 * Batching extension (not proposed by the paper): many images of uneven
 * sizes and keypoint counts described and matched together.  Every stage of
 * the single-image path above (spatial order, integral image, BAD, HashSIFT
 * histogram and projection, Hamming k-NN) runs as one persistent, XCD-aware
 * launch over the whole batch, and bd_batch_run can replay the sequence as
 * one captured HIP graph.  Codes and matches are identical, bit for bit, to
 * the single-image calls on each image, under every tuning.
 * ---------------------------------------------------------------------- */

/* One image of a batch.  img is a device u8 grey image (H rows, `pitch`
 * bytes apart) that feeds the integral image and BAD, and HashSIFT unless
 * hs_img is set: then HashSIFT reads hs_img (BD_DTYPE_U8 or BD_DTYPE_F32,
 * hs_pitch bytes between rows; row-pair images are BD_EUNSUPPORTED here)
 * instead.  The image's n_kp keypoints follow
 * those of the previous images in the flat keypoint array. */
typedef struct bd_batch_image {
    const uint8_t* img;
    int64_t pitch;
    const void* hs_img;
    int64_t hs_pitch;
    int32_t hs_dtype;
    int32_t W, H;
    int32_t n_kp;
} bd_batch_image;

/* One k-NN problem: the codes of query_image's keypoints against those of
 * train_image (indices into the image array).  Its n_kp(query_image) x k
 * results follow those of the previous problems; idx counts keypoints of
 * train_image from 0. */
typedef struct bd_batch_match {
    int32_t query_image, train_image;
} bd_batch_match;

/* Schedule knobs.  Grids are blocks_per_cu x CUs (capped by the stage's
 * work units, rounded to a multiple of the 8 XCDs).  knn_*[0] set the BAD
 * matcher, knn_*[1] the HashSIFT matcher: the engine, knn_qpl = 0 for the
 * int8 MFMA engine (blocks of 256 queries) or 1, 2, 4 queries per lane of
 * the lane-per-query kernel, and train rows per work unit
 * (BD_BATCH_MIN_ROWS .. BD_BATCH_MAX_ROWS; for the MFMA engine a multiple of
 * 16 and at most BD_BATCH_MFMA_MAX_ROWS).  Results do not depend on the
 * knobs. */
typedef struct bd_batch_tuning {
    int32_t order_blocks_per_cu;
    int32_t integral_blocks_per_cu;
    int32_t bad_blocks_per_cu;
    int32_t hist_blocks_per_cu;
    int32_t knn_qpl[2];
    int32_t knn_rows[2];
    int32_t knn_blocks_per_cu[2];
} bd_batch_tuning;

#define BD_BATCH_MIN_ROWS 256
#define BD_BATCH_MAX_ROWS (1 << 22)
#define BD_BATCH_MFMA_MAX_ROWS 2048

typedef struct bd_batch bd_batch;

/* Plans a batch: validates the host arrays `images` (n_images >= 1) and
 * `matches` (n_matches >= 0), allocates the batch's own device memory
 * (integral images with their tile tables, keypoint order, 128-float
 * features per keypoint, partial k-NN results, unit prefixes) and uploads
 * the plan; synchronous.  bad_bits and hs_bits are 0 (stage off), 256 or
 * 512, not both 0; hs_precision and hs_margin as in bd_describe_hashsift;
 * k is 1 or 2.  At most 2^22 keypoints in total.  The image memory must stay
 * valid until bd_batch_destroy.  Errors: BD_EINVAL, BD_EUNSUPPORTED,
 * BD_ENOMEM, BD_EDEVICE; *out is NULL on error. */
int bd_batch_create(bd_context* ctx, const bd_batch_image* images, int32_t n_images, const bd_batch_match* matches,
                    int32_t n_matches, int32_t bad_bits, int32_t hs_bits, int32_t hs_precision, float hs_margin,
                    int32_t k, bd_batch** out);

/* Synchronizes the device, then frees the batch and its graph. */
int bd_batch_destroy(bd_batch* b);

/* Describes and matches the whole batch on `stream`.  Device arrays:
 * kps (total keypoints), pairs (bad_bits entries), B (hs_bits x 128), t
 * (hs_bits); outputs bad_codes (total x bad_bits/64 u64), hs_codes (total x
 * hs_bits/64 u64), bad_idx/bad_dist and hs_idx/hs_dist (match rows x k).
 * Arrays of a disabled stage may be NULL.  With use_graph != 0 the launch
 * sequence is captured once per distinct argument set (on the batch's own
 * stream) and replayed with one hipGraphLaunch; otherwise the kernels are
 * enqueued directly.  Runs on one batch must not overlap. */
int bd_batch_run(bd_batch* b, const bd_keypoint* kps, const bd_box_pair* pairs, const float* B, const float* t,
                 uint64_t* bad_codes, uint64_t* hs_codes, int32_t* bad_idx, uint32_t* bad_dist, int32_t* hs_idx,
                 uint32_t* hs_dist, int32_t use_graph, void* stream);

/* Autotuner: with the arguments of bd_batch_run, times every stage alone
 * (reps launches per candidate, HIP events on `stream`) over the candidate
 * grids, queries per lane and rows per unit, keeps the fastest and leaves
 * that tuning's outputs in place.  Synchronizes `stream`. */
int bd_batch_autotune(bd_batch* b, const bd_keypoint* kps, const bd_box_pair* pairs, const float* B, const float* t,
                      uint64_t* bad_codes, uint64_t* hs_codes, int32_t* bad_idx, uint32_t* bad_dist,
                      int32_t* hs_idx, uint32_t* hs_dist, int32_t reps, void* stream);

/* The tuning a new batch starts with (no device needed). */
int bd_batch_default_tuning(bd_batch_tuning* out);
int bd_batch_get_tuning(const bd_batch* b, bd_batch_tuning* out);
/* Validates and applies a tuning; synchronizes the device. */
int bd_batch_set_tuning(bd_batch* b, const bd_batch_tuning* t);
/* Total keypoints and total match rows of the batch (either pointer may be NULL). */
int bd_batch_info(const bd_batch* b, int64_t* total_kp, int32_t* match_rows);

/* ------------------------------------------------------------------------
 * HashSIFT training (Sec. III-B, Eq. 3): Adam on B and t for the relaxed
 * descriptors tanh(beta (B f - t)) under the triplet ranking loss with
 * in-batch hardest negatives and anchor swap (bd_trl_hnm_fwd), every patch
 * augmented.  pool: 2 n_pairs float32 32x32 patches, pair i = (anchor 2i,
 * positive 2i+1); batch: n pair indices (clamped into range).
 * ---------------------------------------------------------------------- */

/* Augmentation of the batch's 2n patches into out (2n x 1024 floats: the n
 * anchors, then the n positives).  params and noise rows 2s (anchor of pair
 * s) and 2s+1 (its positive): params = (angle, scale, gain, bias, sigma),
 * noise = 1024 floats.  Output pixel (i, j): the bilinear sample
 * (clamp-to-edge) at (15.5, 15.5) + scale Rot(angle) (j - 15.5, i - 15.5),
 * blurred by a separable Gaussian of standard deviation sigma (clamped to
 * 4; weights exp(-d^2 / 2 sigma^2), |d| <= ceil(3 sigma), clamp-to-edge;
 * none for sigma <= 0), then gain v + bias + noise, clipped to [0, 1]. */
int bd_augment_patches(bd_context* ctx, const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n,
                       const float* params, const float* noise, float* out, void* stream);

/* One training iteration: augment (as bd_augment_patches), HashSIFT
 * features of the 2n patches, relaxed descriptors, hardest-negative triplet
 * loss (*loss, device) with margin tau, its gradient with respect to B
 * (n_bits x 128) and t (n_bits), and one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, learning rate lr, bias correction for `step`, counted from 1)
 * applied to B and t in place.  adam_state: 2 n_bits 128 + 2 n_bits floats
 * (first and second moments of B, then of t), zero before step 1.  n_bits 256
 * or 512; n >= 2.  Uses the context workspace. */
int bd_hashsift_train_step(bd_context* ctx, const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n,
                           const float* params, const float* noise, float* B, float* t, int32_t n_bits,
                           float* adam_state, int32_t step, float lr, float tau, float beta, float* loss,
                           void* stream);

#ifdef __cplusplus
}
#endif
#endif
