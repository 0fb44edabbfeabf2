// Threshold search for candidate BAD features (Sec. III-A, Alg. 2 with the
// integer-sorting speed-up): for every candidate box pair, the feature
// f = mean(box 1) - mean(box 2) of all 3N triplet patches is binned at a
// precision of 0.1 over [-255, 255] (m = 5110 bins), each triplet's loss
// change (Eq. 3) as the threshold passes each of its patches is added to the
// patch's bin, and a prefix sum over the bins gives the loss of every
// threshold; the first minimum is the candidate's threshold.
//
// select_hist_kernel: the candidates are split into eight ranges, one per
// XCD (block b works on range b % 8), so the histograms a block updates live
// in its own XCD's L2.  A block loads a tile of four triplets, builds their
// twelve 33 x 33 integral images in LDS, and for 64 candidates at a time a
// thread computes the three features of one (candidate, triplet), the three
// loss changes in (bin, position) order, and adds the non-zero ones to the
// candidate's histogram with integer atomics.  Loss values are multiples of
// 1/2 (2 tau is an integer), so twice the loss changes are exact integers
// and the result does not depend on the order of the atomics.
// select_scan_kernel: one block per candidate, prefix sum over the bins and
// the first minimum.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kBins = 5110;
constexpr int kTileTriplets = 4;
constexpr int kTilePatches = 3 * kTileTriplets;
constexpr int kIIPitch = 33;
constexpr int kIISize = 33 * 33;
constexpr int kThreads = 256;
constexpr int kCandsPerPass = kThreads / kTileTriplets;  // 64

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Twice the hinge of Eq. 3 for one triplet, from twice tau (an integer).
__device__ __forceinline__ int trl2(int tau2, int s_ap, int s_an, int ha, int hp, int hn)
{
    const int v = tau2 + 2 * (-s_ap - ha * hp + s_an + ha * hn);
    return v > 0 ? v : 0;
}

// Sum of the box of radius r centred at (cx, cy) from a 33 x 33 integral image.
__device__ __forceinline__ int box_sum(const uint32_t* ii, int cx, int cy, int r)
{
    const int y0 = cy - r, y1 = cy + r + 1, x0 = cx - r, x1 = cx + r + 1;
    return (int)(ii[y1 * kIIPitch + x1] - ii[y0 * kIIPitch + x1] - ii[y1 * kIIPitch + x0] + ii[y0 * kIIPitch + x0]);
}

struct CandGeom {
    int cx1, cy1, cx2, cy2, r, area;
};

__device__ __forceinline__ CandGeom geometry(const bd_box_pair& c)
{
    CandGeom g;
    g.r = c.radius > 15 ? 15 : c.radius;
    g.area = (2 * g.r + 1) * (2 * g.r + 1);
    g.cx1 = clampi(16 + c.x1, g.r, 31 - g.r);
    g.cy1 = clampi(16 + c.y1, g.r, 31 - g.r);
    g.cx2 = clampi(16 + c.x2, g.r, 31 - g.r);
    g.cy2 = clampi(16 + c.y2, g.r, 31 - g.r);
    return g;
}

// floor((f + 255) * 10) for f = (s1 - s2) / area: the numerator is below
// 5101 * 961 < 2^24, so a float quotient is within one of the result and one
// integer correction makes it exact.
__device__ __forceinline__ int feature_bin(const uint32_t* ii, const CandGeom& g)
{
    const int d = box_sum(ii, g.cx1, g.cy1, g.r) - box_sum(ii, g.cx2, g.cy2, g.r);
    const int num = 10 * d + 2550 * g.area;
    int q = (int)((float)num * __builtin_amdgcn_rcpf((float)g.area));
    if (q * g.area > num) --q;
    if ((q + 1) * g.area <= num) ++q;
    return q;
}

__global__ __launch_bounds__(kThreads) void select_zero_kernel(int32_t* __restrict__ hist, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        hist[i] = 0;
}

// Twice the loss with every stump at -1 (threshold below all values), in a
// fixed order: per-thread partial sums, then a tree.
__global__ __launch_bounds__(1024) void select_base_kernel(const int32_t* __restrict__ s_ap,
                                                           const int32_t* __restrict__ s_an, int32_t n, int tau2,
                                                           int64_t* __restrict__ base2)
{
    __shared__ int64_t part[1024];
    int64_t s = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += trl2(tau2, s_ap[i], s_an[i], -1, -1, -1);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) part[threadIdx.x] += part[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *base2 = part[0];
}

__global__ __launch_bounds__(kThreads) void select_hist_kernel(const uint8_t* __restrict__ patches, int32_t n,
                                                               const int32_t* __restrict__ s_ap,
                                                               const int32_t* __restrict__ s_an, int tau2,
                                                               const bd_box_pair* __restrict__ cands,
                                                               int32_t n_cands, int32_t* __restrict__ hist)
{
    __shared__ uint32_t ii[kTilePatches][kIISize];
    const int x = (int)blockIdx.x % kXcds;
    const int c_begin = (int)((int64_t)n_cands * x / kXcds), c_end = (int)((int64_t)n_cands * (x + 1) / kXcds);
    if (c_begin >= c_end) return;
    const int n_tiles = (n + kTileTriplets - 1) / kTileTriplets;
    const int t = threadIdx.x;

    for (int tile = (int)blockIdx.x / kXcds; tile < n_tiles; tile += (int)gridDim.x / kXcds) {
        const int tri0 = tile * kTileTriplets;
        const int n_here = min(kTileTriplets, n - tri0);
        // row prefix sums: task = (patch, row), 12 x 32 tasks; zero first row and column
        for (int task = t; task < kTilePatches * 32; task += kThreads) {
            const int p = task / 32, y = task % 32;
            uint32_t* dst = ii[p] + (y + 1) * kIIPitch;
            dst[0] = 0u;
            if (p < 3 * n_here) {
                const uint8_t* src = patches + ((int64_t)(3 * tri0 + p) * 32 + y) * 32;
                uint32_t acc = 0;
#pragma unroll 8
                for (int xx = 0; xx < 32; ++xx) {
                    acc += src[xx];
                    dst[xx + 1] = acc;
                }
            } else {
                for (int xx = 0; xx < 32; ++xx) dst[xx + 1] = 0u;
            }
        }
        for (int task = t; task < kTilePatches * 33; task += kThreads) ii[task / 33][task % 33] = 0u;
        __syncthreads();
        // column prefix sums: task = (patch, column)
        for (int task = t; task < kTilePatches * 32; task += kThreads) {
            uint32_t* col = ii[task / 32] + (task % 32) + 1;
            uint32_t acc = 0;
            for (int y = 1; y <= 32; ++y) {
                acc += col[y * kIIPitch];
                col[y * kIIPitch] = acc;
            }
        }
        __syncthreads();

        const int lt = t % kTileTriplets;
        const int tri = tri0 + lt;
        const bool active = lt < n_here;
        const int sap = active ? s_ap[tri] : 0, san = active ? s_an[tri] : 0;
        for (int c0 = c_begin; c0 < c_end; c0 += kCandsPerPass) {
            const int c = c0 + t / kTileTriplets;
            if (!active || c >= c_end) continue;
            const CandGeom g = geometry(cands[c]);
            int q[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) q[m] = feature_bin(ii[3 * lt + m], g);
            // flip the stumps in the order of (bin, position in the triplet)
            int h[3] = {-1, -1, -1};
            int done = 0;
            int32_t* hc = hist + (int64_t)c * kBins;
            int prev = trl2(tau2, sap, san, -1, -1, -1);
#pragma unroll
            for (int step = 0; step < 3; ++step) {
                int nx = -1;
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    if (!(done & (1 << m)) && (nx < 0 || q[m] < q[nx])) nx = m;
                done |= 1 << nx;
                h[nx] = 1;
                const int cur = trl2(tau2, sap, san, h[0], h[1], h[2]);
                if (cur != prev) atomicAdd(hc + q[nx], cur - prev);
                prev = cur;
            }
        }
        __syncthreads();  // the integral images are rebuilt for the next tile
    }
}

// One block per candidate: inclusive prefix over the bins (five per thread),
// then the lowest bin with the smallest cumulative loss.
__global__ __launch_bounds__(1024) void select_scan_kernel(const int32_t* __restrict__ hist,
                                                           const int64_t* __restrict__ base2,
                                                           int32_t* __restrict__ best_bin,
                                                           float* __restrict__ best_theta,
                                                           double* __restrict__ best_loss)
{
    constexpr int kPer = (kBins + 1023) / 1024;  // 5
    __shared__ int64_t part[1024];
    __shared__ int64_t best_v[1024];
    __shared__ int32_t best_b[1024];
    const int c = blockIdx.x, t = threadIdx.x;
    const int32_t* h = hist + (int64_t)c * kBins;
    int64_t local[kPer];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int b = t * kPer + k;
        s += b < kBins ? h[b] : 0;
        local[k] = s;
    }
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const int64_t offset = *base2 + part[t] - s;
    int64_t bv = INT64_MAX;
    int32_t bb = INT32_MAX;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int b = t * kPer + k;
        if (b < kBins && offset + local[k] < bv) {
            bv = offset + local[k];
            bb = b;
        }
    }
    best_v[t] = bv;
    best_b[t] = bb;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if (t < d) {
            const int64_t ov = best_v[t + d];
            const int32_t ob = best_b[t + d];
            if (ov < best_v[t] || (ov == best_v[t] && ob < best_b[t])) {
                best_v[t] = ov;
                best_b[t] = ob;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        best_bin[c] = best_b[0];
        // -255 + (b + 1) / 10 as one correctly rounded quotient of integers
        if (best_theta) best_theta[c] = (float)((double)(best_b[0] + 1 - 2550) / 10.0);
        if (best_loss) best_loss[c] = 0.5 * (double)best_v[0];
    }
}

}  // namespace

size_t select_workspace(int32_t n_cands) { return 256 + sizeof(int32_t) * (size_t)kBins * (size_t)n_cands; }

void launch_find_threshold(const uint8_t* patches, int32_t n, const int32_t* s_ap, const int32_t* s_an, int tau2,
                           const bd_box_pair* cands, int32_t n_cands, int32_t* best_bin, float* best_theta,
                           double* best_loss, void* workspace, int num_cus, hipStream_t stream)
{
    int64_t* base2 = static_cast<int64_t*>(workspace);
    int32_t* hist = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + 256);
    const int64_t count = (int64_t)kBins * n_cands;
    const int zb = (int)((count + kThreads - 1) / kThreads < 4096 ? (count + kThreads - 1) / kThreads : 4096);
    hipLaunchKernelGGL(select_zero_kernel, dim3(zb > 0 ? zb : 1), dim3(kThreads), 0, stream, hist, count);
    hipLaunchKernelGGL(select_base_kernel, dim3(1), dim3(1024), 0, stream, s_ap, s_an, n, tau2, base2);
    const int n_tiles = (n + kTileTriplets - 1) / kTileTriplets;
    if (n_tiles > 0) {
        // three blocks per CU of an XCD's 32 CUs, at most one per tile
        const int per_xcd_cap = 3 * (num_cus > 0 ? num_cus : 256) / kXcds;
        const int per_xcd = n_tiles < per_xcd_cap ? n_tiles : per_xcd_cap;
        hipLaunchKernelGGL(select_hist_kernel, dim3(kXcds * per_xcd), dim3(kThreads), 0, stream, patches, n, s_ap,
                           s_an, tau2, cands, n_cands, hist);
    }
    hipLaunchKernelGGL(select_scan_kernel, dim3(n_cands), dim3(1024), 0, stream, hist, base2, best_bin, best_theta,
                       best_loss);
}

}  // namespace bd
