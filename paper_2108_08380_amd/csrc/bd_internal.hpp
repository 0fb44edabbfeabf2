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

// ---- BAD (bad.hip)
void launch_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                int32_t n_kp, const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes,
                hipStream_t stream);

// ---- spatial keypoint order (order.hip)
void launch_keypoint_order(const bd_keypoint* kps, int32_t n_kp, int32_t W, int32_t H, int32_t* order,
                           hipStream_t stream);

// ---- HashSIFT (hashsift.hip)
void launch_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                          const bd_keypoint* kps, int32_t n_kp, const int32_t* order, float* hist,
                          hipStream_t stream);
void launch_hashsift_patch_features(const float* patches, int32_t n, float* hist, hipStream_t stream);
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
    int32_t qpl;             // queries per lane
    int32_t splits;          // train-set splits (grid.y)
    int32_t rows_per_split;  // <= 2^22 so a (distance, local row) key fits 32 bits
    size_t workspace_bytes() const;
};
KnnPlan plan_knn(int32_t n_q, int32_t n_t, int32_t n_words, int32_t k, int num_cus);
void launch_knn(const KnnPlan& p, const uint64_t* query, const uint64_t* train, int32_t* idx,
                uint32_t* dist, void* workspace, hipStream_t stream);

}  // namespace bd
