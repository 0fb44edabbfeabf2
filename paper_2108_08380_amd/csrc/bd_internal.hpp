// Internal declarations shared by the library's translation units: the
// context, error reporting and the kernel launchers.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/bdesc.h"

struct bd_context {
    int device = 0;
    void* workspace = nullptr;  // device memory, grown on demand
    size_t workspace_bytes = 0;
    int num_cus = 0;
    unsigned long long* invalid = nullptr;  // device counter of invalid keypoints met by describe calls
};

namespace bd {

// Thread-local error message; returns `code` for tail calls.
int fail(int code, const char* fmt, ...);

// Ensure the context owns at least `bytes` of device workspace.  Growing
// synchronizes `stream` first so no enqueued kernel still uses the old block.
int reserve_workspace(bd_context* ctx, size_t bytes, hipStream_t stream, void** out);

int check_launch(const char* what);

constexpr int kWave = 64;
constexpr int kXcds = 8;

// XCD-aware block mapping.  Workgroups of one dispatch go to the 8 XCDs in
// round-robin order of their block index, so block b runs on XCD b % 8.
// Logical block (b % 8) * ceil(nb / 8) + b / 8 gives XCD x the contiguous
// logical range [x * ceil(nb/8), (x+1) * ceil(nb/8)); with keypoints in
// spatial order that range is one region of the image, which then fits the
// XCD's own L2.  The grid is padded to a multiple of 8 and blocks whose
// logical index reaches nb exit.
inline int xcd_grid(int nb) { return (nb + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_logical_block(int b, int nb)
{
    const int per = (nb + kXcds - 1) / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

// Persistent kernels: work units [0, total) are cut into 8 contiguous ranges,
// one per XCD, and the blocks of an XCD (b % 8 == x) take its range in a
// grid-stride loop.  gridDim.x must be a multiple of 8.
struct UnitRange {
    int first, end, stride;
};
__device__ __forceinline__ UnitRange xcd_units(int total)
{
    const int x = (int)blockIdx.x % kXcds, r = (int)blockIdx.x / kXcds;
    const int begin = (int)((int64_t)total * x / kXcds);
    const int end = (int)((int64_t)total * (x + 1) / kXcds);
    return UnitRange{begin + r, end, (int)gridDim.x / kXcds};
}

// Index i of the segment holding unit u for an inclusive-exclusive prefix
// array pre[0..n] (pre[0] = 0, nondecreasing): pre[i] <= u < pre[i+1].
__device__ __forceinline__ int segment_of(const int32_t* __restrict__ pre, int n, int u)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Device-side record of one image of a batch.
struct BatchImage {
    const uint8_t* img_u8;  // pixels for the integral image and BAD
    int64_t pitch_u8;
    const uint8_t* img_hs;  // pixels for HashSIFT (u8 or f32)
    int64_t pitch_hs;
    int32_t hs_dtype;
    int32_t W, H;
    int32_t kp_offset, n_kp;  // range of the flat keypoint array
    uint32_t* ii;             // integral image, (H+1) x ii_pitch
    int64_t ii_pitch;
    uint32_t* colsum;  // integral tile tables
    uint32_t* rowsum;
    int32_t strips, slabs;
    int64_t col_pitch;
    int32_t aligned;
    float inv_cell;  // 1 / cell size of the spatial order grid
};

// Device-side record of one k-NN problem of a batch.  Offsets are rows of
// the flat code array (q_off, t_off), rows of the flat result arrays
// (out_off) and u32 elements of the partial-result buffer (part_off).
struct BatchMatch {
    int32_t q_off, n_q;
    int32_t t_off, n_t;
    int32_t out_off;
    int32_t splits;   // ceil(n_t / rows_per_split), at least 1
    int32_t qgroups;  // ceil(n_q / (64 * queries per lane))
    int32_t pad;
    int64_t part_off;  // splits x n_q x k keys when splits > 1
};

// ---- integral image (integral.hip)
struct IntegralPlan {
    int32_t W, H;
    int32_t strips, slabs;  // 16-row strips, 256-column slabs
    int64_t col_pitch;      // elements per strip row of the column-sum table
    size_t workspace_bytes() const;
};
IntegralPlan plan_integral(int32_t W, int32_t H);
void launch_integral(const IntegralPlan& p, const uint8_t* img, int64_t img_pitch, uint32_t* ii,
                     int64_t ii_pitch, void* workspace, hipStream_t stream);
// launch_integral with, in the blocks of its first pass, the keypoint order
// of the same view (as launch_keypoint_order writes it; n_kp > 0) and the
// row-pair copy of its float HashSIFT image (hs non-null; pitches of hs and
// pairs in elements: floats and float2).
void launch_prepare_view(const IntegralPlan& p, const uint8_t* img, int64_t img_pitch, uint32_t* ii,
                         int64_t ii_pitch, void* workspace, const bd_keypoint* kps, int32_t n_kp, int32_t* order,
                         const float* hs, int64_t hs_pitch, float* pairs, int64_t pairs_pitch, hipStream_t stream);
int integral_tile_blocks(const IntegralPlan& p);   // units of the tile passes
int integral_carry_blocks(const IntegralPlan& p);  // units of the carry pass
void launch_integral_batch(const BatchImage* imgs, int32_t n_img, const int32_t* tile_pre, const int32_t* carry_pre,
                           int grid, hipStream_t stream);

// ---- BAD (bad.hip)
void launch_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                int32_t n_kp, const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes,
                unsigned long long* invalid, hipStream_t stream);

size_t bad_table_bytes(int32_t n_bits);
void launch_bad_compile(const bd_box_pair* pairs, int32_t n_bits, uint8_t* table, hipStream_t stream);
void launch_bad_compiled(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                         int32_t n_kp, const int32_t* order, const uint8_t* table, int32_t n_words, uint64_t* codes,
                         unsigned long long* invalid, hipStream_t stream);
void launch_bad_compiled_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                               const int32_t* order, const uint8_t* table, int32_t n_words, uint64_t* codes, int grid,
                               unsigned long long* invalid, hipStream_t stream);
void launch_bad_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                      const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes, int grid,
                      unsigned long long* invalid, hipStream_t stream);

// ---- spatial keypoint order (order.hip)
float order_inv_cell(int32_t W, int32_t H);
void launch_keypoint_order(const bd_keypoint* kps, int32_t n_kp, int32_t W, int32_t H, int32_t* order,
                           hipStream_t stream);
void launch_keypoint_order_batch(const BatchImage* imgs, int32_t n_img, const bd_keypoint* kps, int32_t* order,
                                 int grid, hipStream_t stream);

// ---- HashSIFT (hashsift.hip)
// Images the HashSIFT sampler addresses with 32-bit offsets and 24-bit row
// multiplies: pitch < 2^24 bytes, H < 2^24 and pitch * H <= 2^32.
inline bool hashsift_image_fits(int64_t pitch, int32_t H)
{
    return pitch < ((int64_t)1 << 24) && H < (1 << 24) && pitch * (int64_t)H <= ((int64_t)1 << 32);
}
void launch_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                          const bd_keypoint* kps, int32_t n_kp, const int32_t* order, float* hist,
                          unsigned long long* invalid, hipStream_t stream);
void launch_hashsift_patch_features(const float* patches, int32_t n, float* hist, hipStream_t stream);
// dtypes: bit (1 << dtype) set for every dtype among the images.
void launch_hashsift_hist_batch(const BatchImage* imgs, int32_t n_img, int32_t dtypes, const int32_t* pre,
                                const bd_keypoint* kps, const int32_t* order, float* hist, int grid,
                                unsigned long long* invalid, hipStream_t stream);
void launch_hashsift_project(int32_t precision, const float* hist, const bd_keypoint* kps, int32_t n_kp,
                             const float* B, const float* t, int32_t n_words, float margin, uint64_t* codes,
                             float* resp, uint32_t* recheck_count, hipStream_t stream);

// ---- differentiation (relaxed.hip)
void launch_relaxed_bad_fwd(const float* patches, int32_t n, const bd_box_pair* pairs, const float* w1,
                            const float* w2, const float* theta, int32_t n_bits, float beta, float* D, float* m1,
                            float* m2, hipStream_t stream);
size_t relaxed_bad_bwd_workspace(int32_t n, int32_t n_bits);
void launch_relaxed_bad_bwd(const float* gD, const float* D, const float* m1, const float* m2, int32_t n,
                            int32_t n_bits, float beta, float* g_w1, float* g_w2, float* g_theta, void* workspace,
                            hipStream_t stream);
void launch_tanh_scale(const float* rho, int64_t count, float beta, float* D, hipStream_t stream);
size_t relaxed_hs_bwd_workspace(int32_t n, int32_t n_bits);
void launch_relaxed_hs_bwd(const float* gD, const float* D, const float* f, int32_t n, int32_t n_bits, float beta,
                           float* gB, float* gt, void* workspace, hipStream_t stream);
size_t trl_workspace(int32_t n);
void launch_trl_fwd(const float* A, const float* P, int32_t n, int32_t K, float tau, float* loss, int32_t* neg,
                    float* hinge, void* workspace, hipStream_t stream);
void launch_trl_bwd(const float* A, const float* P, int32_t n, int32_t K, const int32_t* neg, const float* hinge,
                    const float* grad_loss, float* gA, float* gP, void* workspace, hipStream_t stream);

// ---- Hamming k-NN (hamming.hip)
struct KnnPlan {
    int32_t n_q, n_t, n_words, k;
    int32_t mfma;            // 1: int8 MFMA engine (4 or 8 words), 0: lane-per-query kernel
    int32_t qpl;             // queries per lane (lane-per-query kernel)
    int32_t splits;          // train-set splits (grid.y)
    int32_t rows_per_split;  // <= 2^22 so a (distance, local row) key fits 32 bits
    size_t workspace_bytes() const;
};
KnnPlan plan_knn(int32_t n_q, int32_t n_t, int32_t n_words, int32_t k, int num_cus);
void launch_knn(const KnnPlan& p, const uint64_t* query, const uint64_t* train, int32_t* idx,
                uint32_t* dist, void* workspace, hipStream_t stream);

// ---- mutual nearest neighbours + ratio filter (mutual.hip)
struct MutualPlan {
    int32_t n_q, n_t;
    KnnPlan qt, tq;  // query -> train (k = 2), train -> query (k = 1)
    size_t workspace_bytes() const;
};
MutualPlan plan_mutual(int32_t n_q, int32_t n_t, int32_t n_words, int num_cus);
void launch_mutual(const MutualPlan& p, const uint64_t* query, const uint64_t* train, float max_ratio,
                   int32_t* match, uint32_t* dist, float* ratio, int32_t* count, void* workspace,
                   hipStream_t stream);

// ---- BAD feature selection: threshold search (select.hip)
size_t select_workspace(int32_t n_cands);
void launch_find_threshold(const uint8_t* patches, const int32_t* patch_index, int32_t n, const int32_t* s_ap,
                           const int32_t* s_an, int tau2, const bd_box_pair* cands, int32_t n_cands,
                           int32_t* best_bin, float* best_theta, double* best_loss, void* workspace, int num_cus,
                           hipStream_t stream);
size_t select_features_workspace(int32_t n_pairs, int32_t n_sample, int32_t n_cands, int32_t n_bits, int num_cus);
void launch_select_features(const uint8_t* pool, int32_t n_pairs, const int32_t* samples, int32_t n_sample,
                            const bd_box_pair* cands, int32_t n_cands, int32_t n_bits, int tau2,
                            bd_box_pair* table, int32_t* chosen, int32_t* chosen_bin, double* round_loss,
                            uint64_t* pool_codes_out, void* workspace, int num_cus, hipStream_t stream);

// ---- HashSIFT training (train.hip)
size_t train_step_workspace(int32_t n, int32_t n_bits);
void launch_train_step(const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n, const float* params,
                       const float* noise, float* B, float* t, int32_t n_bits, float* adam_state, int32_t step,
                       float lr, float tau, float beta, float* loss, void* workspace, hipStream_t stream);
void launch_augment(const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n, const float* params,
                    const float* noise, float* out, hipStream_t stream);

// Batched k-NN over BatchMatch problems sharing n_words (4 or 8) and k.
struct KnnBatchPlan {
    int32_t n_words, k;
    int32_t qpl;             // 0: int8 MFMA engine; 1, 2, 4: queries per lane of the lane-per-query kernel
    int32_t rows_per_split;  // train rows per unit, <= 2^22
    int32_t grid;            // blocks of the k-NN kernel (multiple of 8)
    int32_t merge_units, merge_grid;
};
// Queries per unit of the k-NN: a wavefront of the lane-per-query kernel
// (qpl 1, 2, 4) or a block of the MFMA engine (qpl 0).
int knn_queries_per_unit(int qpl, int n_words);
void launch_knn_batch(const KnnBatchPlan& p, const BatchMatch* m, int32_t n_m, const int32_t* pre,
                      const int32_t* merge_pre, const uint64_t* codes, uint32_t* partial, int32_t* idx,
                      uint32_t* dist, hipStream_t stream);

}  // namespace bd
