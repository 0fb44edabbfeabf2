// Spatial processing order of keypoints: the sort itself, shared by the
// order kernels and by the first pass of the integral image, which can run
// it in one of its blocks (bd_build_integral_order).
//
// A counting sort of keypoints by the Morton index of their cell in a
// 64 x 64 grid laid over the image (one workgroup of kOrderThreads).
#pragma once
#include "bd_internal.hpp"

namespace bd {
namespace order_impl {

constexpr int kGridBits = 6;                      // 64 x 64 cells
constexpr int kOrderBins = 1 << (2 * kGridBits);  // 4096
constexpr int kOrderThreads = 1024;

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
    for (int b = t; b < kOrderBins; b += kOrderThreads) bins[b] = 0;
    __syncthreads();
    uint32_t keys[kKeep];
#pragma unroll
    for (int r = 0; r < kKeep; ++r) {
        const int i = t + r * kOrderThreads;
        keys[r] = i < n ? cell_key(kps[i], inv_cell) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kKeep; ++r)
        if (t + r * kOrderThreads < n) atomicAdd(&bins[keys[r]], 1u);
    for (int i = t + kKeep * kOrderThreads; i < n; i += kOrderThreads) atomicAdd(&bins[cell_key(kps[i], inv_cell)], 1u);
    __syncthreads();
    // exclusive scan of the 4096 bins
    constexpr int kPer = kOrderBins / kOrderThreads;
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
        constexpr int kWaves = kOrderThreads / kWave;  // 16
        uint32_t w = t < kWaves ? part[t] : 0u;
#pragma unroll
        for (int d = 1; d < kWaves; d <<= 1) {
            const uint32_t v = __shfl_up(w, d, kWave);
            if (t >= d) w += v;
        }
        if (t < kWaves) part[kWaves + t] = w;  // inclusive totals
    }
    __syncthreads();
    const uint32_t base = (wave > 0 ? part[kOrderThreads / kWave + wave - 1] : 0u) + incl - sum;
#pragma unroll
    for (int k = 0; k < kPer; ++k) bins[t * kPer + k] = base + local[k];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kKeep; ++r) {
        const int i = t + r * kOrderThreads;
        if (i < n) order[atomicAdd(&bins[keys[r]], 1u)] = i;
    }
    for (int i = t + kKeep * kOrderThreads; i < n; i += kOrderThreads) order[atomicAdd(&bins[cell_key(kps[i], inv_cell)], 1u)] = i;
    __syncthreads();
}

}  // namespace order_impl
}  // namespace bd
