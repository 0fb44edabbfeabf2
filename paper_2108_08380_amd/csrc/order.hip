// Spatial processing order of keypoints.
//
// Describing keypoints in a spatially coherent order lets every XCD's L2
// hold the part of the image its workgroups touch: with the XCD-aware block
// mapping of the describe kernels, XCD x processes the x-th eighth of the
// ordered list, i.e. one compact region of the image.  The order is a
// counting sort of keypoints by the Morton index of their cell in a 64 x 64
// grid laid over the image.  It only changes which workgroup describes a
// keypoint, never the code written for it.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kGridBits = 6;                 // 64 x 64 cells
constexpr int kBins = 1 << (2 * kGridBits);  // 4096
constexpr int kThreads = 1024;

__device__ __forceinline__ uint32_t spread_bits(uint32_t v)  // 6 bits -> even positions
{
    v &= 0x3fu;
    v = (v | (v << 4)) & 0x30fu;
    v = (v | (v << 2)) & 0x333u;
    v = (v | (v << 1)) & 0x555u;
    return v;
}

__device__ __forceinline__ uint32_t cell_key(const bd_keypoint& k, float inv_cell)
{
    // non-finite coordinates land in cell 0; the describe kernels handle them
    const float fx = k.x * inv_cell, fy = k.y * inv_cell;
    const int cx = (fx >= 0.0f && fx < 64.0f) ? (int)fx : (fx >= 64.0f ? 63 : 0);
    const int cy = (fy >= 0.0f && fy < 64.0f) ? (int)fy : (fy >= 64.0f ? 63 : 0);
    return spread_bits((uint32_t)cx) | (spread_bits((uint32_t)cy) << 1);
}

// One workgroup: histogram of cell keys in LDS, exclusive scan, scatter.
// Keypoints sharing a cell are placed in arbitrary order.  The first 8192
// keypoints keep their cell keys in registers between the histogram and the
// scatter; the scan is four bins per thread, a wavefront scan by shuffles
// and a scan of the 16 wavefront totals.
__device__ __forceinline__ void order_body(const bd_keypoint* __restrict__ kps, int32_t n, float inv_cell,
                                           int32_t* __restrict__ order, uint32_t* bins, uint32_t* part)
{
    constexpr int kKeep = 8;
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    for (int b = t; b < kBins; b += kThreads) bins[b] = 0;
    __syncthreads();
    uint32_t keys[kKeep];
#pragma unroll
    for (int r = 0; r < kKeep; ++r) {
        const int i = t + r * kThreads;
        keys[r] = i < n ? cell_key(kps[i], inv_cell) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kKeep; ++r)
        if (t + r * kThreads < n) atomicAdd(&bins[keys[r]], 1u);
    for (int i = t + kKeep * kThreads; i < n; i += kThreads) atomicAdd(&bins[cell_key(kps[i], inv_cell)], 1u);
    __syncthreads();
    // exclusive scan of the 4096 bins
    constexpr int kPer = kBins / kThreads;
    uint32_t local[kPer], sum = 0u;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        local[k] = sum;
        sum += bins[t * kPer + k];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += v;
    }
    if (lane == kWave - 1) part[wave] = incl;
    __syncthreads();
    if (t < kWave) {
        constexpr int kWaves = kThreads / kWave;  // 16
        uint32_t w = t < kWaves ? part[t] : 0u;
#pragma unroll
        for (int d = 1; d < kWaves; d <<= 1) {
            const uint32_t v = __shfl_up(w, d, kWave);
            if (t >= d) w += v;
        }
        if (t < kWaves) part[kWaves + t] = w;  // inclusive totals
    }
    __syncthreads();
    const uint32_t base = (wave > 0 ? part[kThreads / kWave + wave - 1] : 0u) + incl - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) bins[t * kPer + k] = base + local[k];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKeep; ++r) {
        const int i = t + r * kThreads;
        if (i < n) order[atomicAdd(&bins[keys[r]], 1u)] = i;
    }
    for (int i = t + kKeep * kThreads; i < n; i += kThreads) order[atomicAdd(&bins[cell_key(kps[i], inv_cell)], 1u)] = i;
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void keypoint_order_kernel(const bd_keypoint* __restrict__ kps, int32_t n,
                                                                 float inv_cell, int32_t* __restrict__ order)
{
    __shared__ uint32_t bins[kBins];
    __shared__ uint32_t part[kThreads];
    order_body(kps, n, inv_cell, order, bins, part);
}

// Batch: one image per unit; order entries are indices local to the image.
__global__ __launch_bounds__(kThreads) void keypoint_order_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                                const bd_keypoint* __restrict__ kps,
                                                                int32_t* __restrict__ order)
{
    __shared__ uint32_t bins[kBins];
    __shared__ uint32_t part[kThreads];
    const UnitRange ur = xcd_units(n_img);
    for (int i = ur.first; i < ur.end; i += ur.stride) {
        const BatchImage& im = imgs[i];
        order_body(kps + im.kp_offset, im.n_kp, im.inv_cell, order + im.kp_offset, bins, part);
    }
}

}  // namespace

float order_inv_cell(int32_t W, int32_t H)
{
    const int side = W > H ? W : H;
    return 1.0f / (float)((side + 63) / 64 > 0 ? (side + 63) / 64 : 1);
}

void launch_keypoint_order(const bd_keypoint* kps, int32_t n_kp, int32_t W, int32_t H, int32_t* order,
                           hipStream_t stream)
{
    hipLaunchKernelGGL(keypoint_order_kernel, dim3(1), dim3(kThreads), 0, stream, kps, n_kp, order_inv_cell(W, H),
                       order);
}

void launch_keypoint_order_batch(const BatchImage* imgs, int32_t n_img, const bd_keypoint* kps, int32_t* order,
                                 int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(keypoint_order_batch, dim3(grid), dim3(kThreads), 0, stream, imgs, n_img, kps, order);
}

}  // namespace bd
