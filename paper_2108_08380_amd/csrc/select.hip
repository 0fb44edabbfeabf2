// Threshold search for candidate BAD features (Sec. III-A, Alg. 2 with the
// integer-sorting speed-up): for every candidate box pair, the feature
// f = mean(box 1) - mean(box 2) of all 3N triplet patches is binned at a
// precision of 0.1 over [-255, 255] (m = 5110 bins), each triplet's loss
// change (Eq. 2) as the threshold passes each of its patches is added to the
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

// Twice the hinge of Eq. 2 for one triplet, from twice tau (an integer).
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

__global__ __launch_bounds__(kThreads) void select_hist_kernel(const uint8_t* __restrict__ patches,
                                                               const int32_t* __restrict__ patch_index, int32_t n,
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
                const int64_t pid = patch_index ? patch_index[3 * tri0 + p] : 3 * tri0 + p;
                const uint8_t* src = patches + (pid * 32 + y) * 32;
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

// ---- Alg. 1 (greedy selection) steps

__global__ __launch_bounds__(kThreads) void sel_zero_u64_kernel(uint64_t* __restrict__ p, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__device__ __forceinline__ int sample_pair(const int32_t* samples, int s, int32_t n_pairs)
{
    return clampi(samples[s], 0, n_pairs - 1);  // out-of-range indices are clamped, never dereferenced
}

// Codes of the sampled anchors and positives (pair i: pool patches 2i, 2i+1).
__global__ __launch_bounds__(kThreads) void sel_gather_codes_kernel(const uint64_t* __restrict__ pool_codes,
                                                                    int32_t W, const int32_t* __restrict__ samples,
                                                                    int32_t n, int32_t n_pairs,
                                                                    uint64_t* __restrict__ ac,
                                                                    uint64_t* __restrict__ pc)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * W) return;
    const int s = e / W, w = e - s * W;
    const int i = sample_pair(samples, s, n_pairs);
    ac[e] = pool_codes[(int64_t)(2 * i) * W + w];
    pc[e] = pool_codes[(int64_t)(2 * i + 1) * W + w];
}

__global__ __launch_bounds__(kThreads) void sel_fill_keys_kernel(uint32_t* __restrict__ keys, int32_t count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) keys[i] = 0xffffffffu;
}

// In-batch nearest other code with a cyclic tie-break.  Lane = query s
// (codes in VGPRs), train rows j of this split wave-uniform (scalar loads);
// the key (d << 22) | ((j - s - 1) mod n) orders candidates by distance, then
// cyclically from s + 1, and j = s (rank n - 1) is skipped.  Per-split
// minima meet through atomicMin, whose result does not depend on the order.
// grid = (ceil(n / 256), splits), direction y: 0 = anchors vs positives,
// 1 = positives vs anchors.
template <int W>
__global__ __launch_bounds__(kThreads) void sel_hnm_dist_kernel(const uint64_t* __restrict__ ac,
                                                                const uint64_t* __restrict__ pc, int32_t n,
                                                                int32_t rows_per_split, uint32_t* __restrict__ keys)
{
    const int dir = blockIdx.z;
    const uint64_t* query = dir == 0 ? ac : pc;
    const uint64_t* train = dir == 0 ? pc : ac;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y * rows_per_split;
    const int j1 = min(n, j0 + rows_per_split);
    if (blockIdx.x * blockDim.x >= (unsigned)n) return;
    uint64_t q[W];
#pragma unroll
    for (int w = 0; w < W; ++w) q[w] = s < n ? query[(int64_t)s * W + w] : 0ull;
    uint32_t best = 0xffffffffu;
    for (int j = j0; j < j1; ++j) {
        uint32_t d = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) d += __popcll(q[w] ^ train[(int64_t)j * W + w]);
        int c = j - s - 1;
        c += c < 0 ? n : 0;
        const uint32_t key = (d << 22) | (uint32_t)c;
        if (j != s) best = min(best, key);
    }
    if (s < n) atomicMin(&keys[dir * n + s], best);
}

// Hardest in-batch negative with anchor swap from the two nearest-other
// keys: the row candidate (a positive) wins ties.  Writes the triplet's pool
// patch indices and the similarities k - 2 d of (anchor, positive) and
// (anchor, negative) under the k bits selected so far.
__global__ __launch_bounds__(kThreads) void sel_hnm_kernel(const uint32_t* __restrict__ keys,
                                                           const uint64_t* __restrict__ ac,
                                                           const uint64_t* __restrict__ pc, int32_t n, int32_t W,
                                                           int32_t k, const int32_t* __restrict__ samples,
                                                           int32_t n_pairs, int32_t* __restrict__ patch_index,
                                                           int32_t* __restrict__ s_ap, int32_t* __restrict__ s_an)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t kr = keys[s], kc = keys[n + s];
    const uint32_t dr = kr >> 22, dc = kc >> 22;
    int jr = s + 1 + (int)(kr & 0x3fffffu), jc = s + 1 + (int)(kc & 0x3fffffu);
    jr -= jr >= n ? n : 0;
    jc -= jc >= n ? n : 0;
    uint32_t dp = 0;
    for (int w = 0; w < W; ++w) dp += __popcll(ac[(int64_t)s * W + w] ^ pc[(int64_t)s * W + w]);
    const int i = sample_pair(samples, s, n_pairs);
    const bool row = dr <= dc;
    const int j = sample_pair(samples, clampi(row ? jr : jc, 0, n - 1), n_pairs);
    patch_index[3 * s] = row ? 2 * i : 2 * i + 1;
    patch_index[3 * s + 1] = row ? 2 * i + 1 : 2 * i;
    patch_index[3 * s + 2] = row ? 2 * j + 1 : 2 * j;
    s_ap[s] = k - 2 * (int)dp;
    s_an[s] = k - 2 * (int)(row ? dr : dc);
}

// First candidate of lowest loss; writes the table entry and the round's
// outputs, and keeps (candidate, bin) for the bit update.
__global__ __launch_bounds__(1024) void sel_best_kernel(const int32_t* __restrict__ best_bin,
                                                        const double* __restrict__ best_loss, int32_t n_cands,
                                                        const bd_box_pair* __restrict__ cands, int32_t k,
                                                        bd_box_pair* __restrict__ table, int32_t* __restrict__ chosen,
                                                        int32_t* __restrict__ chosen_bin,
                                                        double* __restrict__ round_loss, int2* __restrict__ state)
{
    __shared__ double lv[1024];
    __shared__ int32_t li[1024];
    const int t = threadIdx.x;
    double bv = INFINITY;
    int bi = INT32_MAX;
    for (int c = t; c < n_cands; c += blockDim.x)
        if (best_loss[c] < bv) {  // ascending c per thread: the first minimum
            bv = best_loss[c];
            bi = c;
        }
    lv[t] = bv;
    li[t] = bi;
    __syncthreads();
    for (int d = 512; d >= 1; d >>= 1) {
        if (t < d && (lv[t + d] < lv[t] || (lv[t + d] == lv[t] && li[t + d] < li[t]))) {
            lv[t] = lv[t + d];
            li[t] = li[t + d];
        }
        __syncthreads();
    }
    if (t == 0) {
        const int c = li[0];
        const int b = best_bin[c];
        bd_box_pair e = cands[c];
        const int r = e.radius > 15 ? 15 : e.radius;
        const double area = (double)((2 * r + 1) * (2 * r + 1));
        e.threshold = (float)((double)(b + 1 - 2550) / 10.0 - 1.0 / (20.0 * area));
        table[k] = e;
        if (chosen) chosen[k] = c;
        if (chosen_bin) chosen_bin[k] = b;
        if (round_loss) round_loss[k] = lv[0];
        *state = int2{c, b};
    }
}

// Bit k of every pool patch from the chosen stump: one wavefront per patch
// (16 bytes per lane cover the 32 x 32 patch), box sums by a wavefront sum.
__global__ __launch_bounds__(kThreads) void sel_update_kernel(const uint8_t* __restrict__ pool, int32_t n_patches,
                                                              const bd_box_pair* __restrict__ cands,
                                                              const int2* __restrict__ state,
                                                              uint64_t* __restrict__ pool_codes, int32_t W,
                                                              int32_t k)
{
    const int lane = threadIdx.x % kWave;
    const int x = blockIdx.x * (kThreads / kWave) + threadIdx.x / kWave;
    if (x >= n_patches) return;
    const int2 st = *state;
    const CandGeom g = geometry(cands[st.x]);
    const uint4 v = reinterpret_cast<const uint4*>(pool + (int64_t)x * 1024)[lane];
    const int y = lane >> 1, x0 = (lane & 1) * 16;  // this lane: row y, columns x0 .. x0+15
    const uint32_t words[4] = {v.x, v.y, v.z, v.w};
    int d = 0;
    const bool row1 = y >= g.cy1 - g.r && y <= g.cy1 + g.r;
    const bool row2 = y >= g.cy2 - g.r && y <= g.cy2 + g.r;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int px = (int)((words[e >> 2] >> (8 * (e & 3))) & 0xffu);
        const int xx = x0 + e;
        if (row1 && xx >= g.cx1 - g.r && xx <= g.cx1 + g.r) d += px;
        if (row2 && xx >= g.cx2 - g.r && xx <= g.cx2 + g.r) d -= px;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, kWave);
    if (lane == 0) {
        const int num = 10 * d + 2550 * g.area;
        const int q = num / g.area;  // num >= 0
        if (q <= st.y) pool_codes[(int64_t)x * W + k / 64] |= 1ull << (k % 64);
    }
}

size_t align_up256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

template <int W>
void launch_hnm_dist_w(const uint64_t* ac, const uint64_t* pc, int32_t n, int32_t rows, int32_t splits,
                       uint32_t* keys, hipStream_t stream)
{
    hipLaunchKernelGGL((sel_hnm_dist_kernel<W>), dim3((n + kThreads - 1) / kThreads, splits, 2), dim3(kThreads), 0,
                       stream, ac, pc, n, rows, keys);
}

void launch_hnm_dist(const uint64_t* ac, const uint64_t* pc, int32_t n, int32_t W, uint32_t* keys, int num_cus,
                     hipStream_t stream)
{
    // splits of the train rows so that about 8 wavefronts per CU are busy
    const int qblocks = (n + kThreads - 1) / kThreads;
    const int want = 2 * (num_cus > 0 ? num_cus : 256);
    int splits = (want + 2 * qblocks - 1) / (2 * qblocks);
    const int max_splits = (n + 63) / 64;
    splits = splits < 1 ? 1 : (splits > max_splits ? max_splits : splits);
    const int rows = (n + splits - 1) / splits;
    splits = (n + rows - 1) / rows;
    hipLaunchKernelGGL(sel_fill_keys_kernel, dim3((2 * n + kThreads - 1) / kThreads), dim3(kThreads), 0, stream, keys,
                       2 * n);
    switch (W) {
        case 1: launch_hnm_dist_w<1>(ac, pc, n, rows, splits, keys, stream); break;
        case 2: launch_hnm_dist_w<2>(ac, pc, n, rows, splits, keys, stream); break;
        case 3: launch_hnm_dist_w<3>(ac, pc, n, rows, splits, keys, stream); break;
        case 4: launch_hnm_dist_w<4>(ac, pc, n, rows, splits, keys, stream); break;
        case 5: launch_hnm_dist_w<5>(ac, pc, n, rows, splits, keys, stream); break;
        case 6: launch_hnm_dist_w<6>(ac, pc, n, rows, splits, keys, stream); break;
        case 7: launch_hnm_dist_w<7>(ac, pc, n, rows, splits, keys, stream); break;
        default: launch_hnm_dist_w<8>(ac, pc, n, rows, splits, keys, stream); break;
    }
}

size_t select_features_workspace(int32_t n_pairs, int32_t n_sample, int32_t n_cands, int32_t n_bits, int num_cus)
{
    (void)num_cus;
    const size_t W = (size_t)(n_bits + 63) / 64, N = (size_t)n_sample;
    return align_up256(sizeof(uint64_t) * 2 * (size_t)n_pairs * W) + 2 * align_up256(sizeof(uint64_t) * N * W) +
           align_up256(sizeof(uint32_t) * 2 * N) + 2 * align_up256(sizeof(int32_t) * N) +
           align_up256(sizeof(int32_t) * 3 * N) +
           align_up256(select_workspace(n_cands)) + align_up256(sizeof(int32_t) * n_cands) +
           align_up256(sizeof(double) * n_cands) + 256;
}

void launch_select_features(const uint8_t* pool, int32_t n_pairs, const int32_t* samples, int32_t n_sample,
                            const bd_box_pair* cands, int32_t n_cands, int32_t n_bits, int tau2,
                            bd_box_pair* table, int32_t* chosen, int32_t* chosen_bin, double* round_loss,
                            uint64_t* pool_codes_out, void* workspace, int num_cus, hipStream_t stream)
{
    const int32_t W = (n_bits + 63) / 64, N = n_sample;
    char* ws = static_cast<char*>(workspace);
    auto take = [&](size_t bytes) {
        void* p = ws;
        ws += align_up256(bytes);
        return p;
    };
    uint64_t* codes = static_cast<uint64_t*>(take(sizeof(uint64_t) * 2 * (size_t)n_pairs * W));
    uint64_t* ac = static_cast<uint64_t*>(take(sizeof(uint64_t) * (size_t)N * W));
    uint64_t* pc = static_cast<uint64_t*>(take(sizeof(uint64_t) * (size_t)N * W));
    uint32_t* keys = static_cast<uint32_t*>(take(sizeof(uint32_t) * 2 * (size_t)N));
    int32_t* s_ap = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)N));
    int32_t* s_an = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)N));
    int32_t* patch_index = static_cast<int32_t*>(take(sizeof(int32_t) * 3 * (size_t)N));
    void* thr_ws = take(select_workspace(n_cands));
    int32_t* bins = static_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n_cands));
    double* losses = static_cast<double*>(take(sizeof(double) * (size_t)n_cands));
    int2* state = static_cast<int2*>(take(sizeof(int2)));

    const int64_t n_codes = 2 * (int64_t)n_pairs * W;
    hipLaunchKernelGGL(sel_zero_u64_kernel, dim3((int)((n_codes + kThreads - 1) / kThreads < 4096 ? (n_codes + kThreads - 1) / kThreads : 4096)),
                       dim3(kThreads), 0, stream, codes, n_codes);
    const int nb = (N + kThreads - 1) / kThreads;
    const int nbw = (N * W + kThreads - 1) / kThreads;
    const int n_patches = 2 * n_pairs;
    const int ub = (n_patches + kThreads / kWave - 1) / (kThreads / kWave);
    for (int32_t k = 0; k < n_bits; ++k) {
        const int32_t* smp = samples + (int64_t)k * N;
        const bd_box_pair* ck = cands + (int64_t)k * n_cands;
        hipLaunchKernelGGL(sel_gather_codes_kernel, dim3(nbw), dim3(kThreads), 0, stream, codes, W, smp, N, n_pairs,
                           ac, pc);
        launch_hnm_dist(ac, pc, N, W, keys, num_cus, stream);
        hipLaunchKernelGGL(sel_hnm_kernel, dim3(nb), dim3(kThreads), 0, stream, keys, ac, pc, N, W, k, smp, n_pairs,
                           patch_index, s_ap, s_an);
        launch_find_threshold(pool, patch_index, N, s_ap, s_an, tau2, ck, n_cands, bins, nullptr, losses, thr_ws,
                              num_cus, stream);
        hipLaunchKernelGGL(sel_best_kernel, dim3(1), dim3(1024), 0, stream, bins, losses, n_cands, ck, k, table,
                           chosen, chosen_bin, round_loss, state);
        hipLaunchKernelGGL(sel_update_kernel, dim3(ub), dim3(kThreads), 0, stream, pool, n_patches, ck, state, codes,
                           W, k);
    }
    if (pool_codes_out)
        (void)hipMemcpyAsync(pool_codes_out, codes, sizeof(uint64_t) * (size_t)n_codes, hipMemcpyDeviceToDevice,
                             stream);
}

size_t select_workspace(int32_t n_cands) { return 256 + sizeof(int32_t) * (size_t)kBins * (size_t)n_cands; }

void launch_find_threshold(const uint8_t* patches, const int32_t* patch_index, int32_t n, const int32_t* s_ap,
                           const int32_t* s_an, int tau2, const bd_box_pair* cands, int32_t n_cands,
                           int32_t* best_bin, float* best_theta, double* best_loss, void* workspace, int num_cus,
                           hipStream_t stream)
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
        hipLaunchKernelGGL(select_hist_kernel, dim3(kXcds * per_xcd), dim3(kThreads), 0, stream, patches,
                           patch_index, n, s_ap, s_an, tau2, cands, n_cands, hist);
    }
    hipLaunchKernelGGL(select_scan_kernel, dim3(n_cands), dim3(1024), 0, stream, hist, base2, best_bin, best_theta,
                       best_loss);
}

}  // namespace bd
