// Brute-force Hamming k-NN (Sec. III-A: S(x, y) = h(x)^T h(y) = K - 2 d_H,
// so the best match is the train code at the smallest Hamming distance).
//
// Lane = query: each lane keeps QPL query codes in VGPRs and walks a range
// of train rows.  The train row index is wave-uniform, so its words arrive
// through scalar loads and every XOR takes an SGPR operand: per (query,
// train) pair the work is n_words * (2 XOR + 2 popcount-accumulate) plus the
// top-k update, with no LDS traffic.  Distances and rows are packed into one
// u32 key (distance << 22 | row within the split), so the lexicographic
// (distance, index) order is plain unsigned order and the top-2 update is
// three v_min/v_max.
//
// The train set is split over grid.y so that small query sets still fill
// the GPU; per-split results go to the workspace and a second kernel merges
// them.  The top-k of a strict total order does not depend on the merge
// order, so results are deterministic.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr uint32_t kRowBits = 22;
constexpr uint32_t kRowMask = (1u << kRowBits) - 1u;
constexpr uint32_t kEmpty = 0xffffffffu;

template <int KK>
__device__ __forceinline__ void topk_insert(uint32_t (&best)[KK], uint32_t key)
{
    if constexpr (KK == 1) {
        best[0] = min(best[0], key);
    } else {
        const uint32_t hi = max(best[0], key);
        best[0] = min(best[0], key);
        best[1] = min(best[1], hi);
    }
}

// One wavefront: queries q0 + p * 64 + lane (p < QPL) against train rows
// [t0, t1).  Results go straight to (idx, dist) when `direct`, else as
// packed keys to partial[split][query][k].
template <int NW, int KK, int QPL>
__device__ __forceinline__ void knn_wave_body(const uint64_t* __restrict__ query, int32_t n_q, int q0,
                                              const uint64_t* __restrict__ train, int t0, int t1, int split,
                                              uint32_t* __restrict__ partial, int32_t* __restrict__ out_idx,
                                              uint32_t* __restrict__ out_dist, bool direct, int lane)
{
    uint32_t ql[QPL][NW], qh[QPL][NW];
    uint32_t best[QPL][KK];
#pragma unroll
    for (int p = 0; p < QPL; ++p) {
        const int qi = q0 + p * kWave + lane;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint64_t v = qi < n_q ? query[(int64_t)qi * NW + w] : 0ull;
            ql[p][w] = (uint32_t)v;
            qh[p][w] = (uint32_t)(v >> 32);
        }
#pragma unroll
        for (int s = 0; s < KK; ++s) best[p][s] = kEmpty;
    }

    const uint32_t* rows = reinterpret_cast<const uint32_t*>(train);
#pragma unroll 2
    for (int r = t0; r < t1; ++r) {
        const uint32_t* row = rows + (int64_t)r * (2 * NW);
        uint32_t tl[NW], th[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            tl[w] = row[2 * w];
            th[w] = row[2 * w + 1];
        }
        const uint32_t local = (uint32_t)(r - t0);
#pragma unroll
        for (int p = 0; p < QPL; ++p) {
            uint32_t d = 0u;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                d = __popc(ql[p][w] ^ tl[w]) + d;
                d = __popc(qh[p][w] ^ th[w]) + d;
            }
            topk_insert<KK>(best[p], (d << kRowBits) | local);
        }
    }

#pragma unroll
    for (int p = 0; p < QPL; ++p) {
        const int qi = q0 + p * kWave + lane;
        if (qi >= n_q) continue;
        if (direct) {
#pragma unroll
            for (int s = 0; s < KK; ++s) {
                const uint32_t key = best[p][s];
                const bool empty = key == kEmpty;
                out_idx[(int64_t)qi * KK + s] = empty ? -1 : (int32_t)(t0 + (key & kRowMask));
                out_dist[(int64_t)qi * KK + s] = empty ? kEmpty : key >> kRowBits;
            }
        } else {
#pragma unroll
            for (int s = 0; s < KK; ++s) partial[((int64_t)split * n_q + qi) * KK + s] = best[p][s];
        }
    }
}

template <int NW, int KK, int QPL>
__global__ __launch_bounds__(256) void hamming_knn_kernel(const uint64_t* __restrict__ query, int32_t n_q,
                                                          const uint64_t* __restrict__ train, int32_t n_t,
                                                          int32_t rows_per_split,
                                                          uint32_t* __restrict__ partial,
                                                          int32_t* __restrict__ out_idx,
                                                          uint32_t* __restrict__ out_dist, int direct)
{
    const int lane = threadIdx.x % kWave;
    const int qgroup = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int q0 = qgroup * kWave * QPL;
    if (q0 >= n_q) return;
    const int split = blockIdx.y;
    const int t0 = split * rows_per_split;
    const int t1 = min(n_t, t0 + rows_per_split);
    knn_wave_body<NW, KK, QPL>(query, n_q, q0, train, t0, t1, split, partial, out_idx, out_dist, direct != 0, lane);
}

// Batch: units are (problem, split, query group) triples, one per wavefront,
// problem-major and query group fastest, so consecutive units share a train
// split.  The XCD ranges of xcd_units are cut at wavefront granularity.
template <int NW, int KK, int QPL>
__global__ __launch_bounds__(256) void hamming_knn_batch(const BatchMatch* __restrict__ m, int32_t n_m,
                                                         const int32_t* __restrict__ pre,
                                                         const uint64_t* __restrict__ codes,
                                                         int32_t rows_per_split, uint32_t* __restrict__ partial,
                                                         int32_t* __restrict__ out_idx,
                                                         uint32_t* __restrict__ out_dist)
{
    const int lane = threadIdx.x % kWave;
    const int total = pre[n_m];
    const int x = (int)blockIdx.x % kXcds;
    const int stride = (int)gridDim.x / kXcds * kWavesPerBlock;
    // the wavefront index is uniform; readfirstlane lets the compiler keep
    // the unit, its record and the train row pointer in SGPRs
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int first = (int)((int64_t)total * x / kXcds) + (int)blockIdx.x / kXcds * kWavesPerBlock + wave;
    const int end = (int)((int64_t)total * (x + 1) / kXcds);
    for (int u = first; u < end; u += stride) {
        const int i = segment_of(pre, n_m, u);
        const BatchMatch& b = m[i];
        const int local = u - pre[i];
        const int split = local / b.qgroups;
        const int q0 = (local - split * b.qgroups) * kWave * QPL;
        const int t0 = split * rows_per_split;
        const int t1 = min(b.n_t, t0 + rows_per_split);
        knn_wave_body<NW, KK, QPL>(codes + (int64_t)b.q_off * NW, b.n_q, q0, codes + (int64_t)b.t_off * NW, t0, t1,
                                   split, partial + b.part_off, out_idx + (int64_t)b.out_off * KK,
                                   out_dist + (int64_t)b.out_off * KK, b.splits == 1, lane);
    }
}

// Merge of the per-split top-k: a block covers 64 queries, its four
// wavefronts take every fourth split each (eight loads in flight per lane),
// and the four partial results meet in LDS.  Keys become 64-bit (distance in
// the high word, global row in the low word) so the order stays
// lexicographic in (distance, index).
template <int KK>
__device__ __forceinline__ void topk_insert64(uint64_t (&best)[KK], uint64_t k64)
{
    if constexpr (KK == 1) {
        best[0] = k64 < best[0] ? k64 : best[0];
    } else {
        const uint64_t hi = k64 > best[0] ? k64 : best[0];
        best[0] = k64 < best[0] ? k64 : best[0];
        best[1] = hi < best[1] ? hi : best[1];
    }
}

// Block of four wavefronts: queries 64 * qb + lane of one problem.  Ends
// with a barrier so a persistent block can reuse `part`.
template <int KK>
__device__ __forceinline__ void merge_block_body(const uint32_t* __restrict__ partial, int32_t n_q, int32_t splits,
                                                 int32_t rows_per_split, int qb, int32_t* __restrict__ out_idx,
                                                 uint32_t* __restrict__ out_dist, uint64_t (*part)[kWave][KK])
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int qi = qb * kWave + lane;
    uint64_t best[KK];
#pragma unroll
    for (int s = 0; s < KK; ++s) best[s] = ~0ull;
    if (qi < n_q) {
        constexpr int kBatch = 8;
        for (int sp0 = wave; sp0 < splits; sp0 += 4 * kBatch) {
            uint32_t key[kBatch][KK];
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const int sp = sp0 + 4 * b;
#pragma unroll
                for (int s = 0; s < KK; ++s) key[b][s] = sp < splits ? partial[((int64_t)sp * n_q + qi) * KK + s] : kEmpty;
            }
#pragma unroll
            for (int b = 0; b < kBatch; ++b) {
                const int sp = sp0 + 4 * b;
#pragma unroll
                for (int s = 0; s < KK; ++s) {
                    if (key[b][s] == kEmpty) continue;
                    const uint32_t row = (uint32_t)(sp * rows_per_split) + (key[b][s] & kRowMask);
                    topk_insert64<KK>(best, ((uint64_t)(key[b][s] >> kRowBits) << 32) | row);
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < KK; ++s) part[wave][lane][s] = best[s];
    __syncthreads();
    if (wave == 0 && qi < n_q) {
#pragma unroll
        for (int w = 1; w < 4; ++w)
#pragma unroll
            for (int s = 0; s < KK; ++s) topk_insert64<KK>(best, part[w][lane][s]);
#pragma unroll
        for (int s = 0; s < KK; ++s) {
            const bool empty = best[s] == ~0ull;
            out_idx[(int64_t)qi * KK + s] = empty ? -1 : (int32_t)(uint32_t)best[s];
            out_dist[(int64_t)qi * KK + s] = empty ? kEmpty : (uint32_t)(best[s] >> 32);
        }
    }
    __syncthreads();
}

template <int KK>
__global__ __launch_bounds__(256) void hamming_merge_kernel(const uint32_t* __restrict__ partial, int32_t n_q,
                                                            int32_t splits, int32_t rows_per_split,
                                                            int32_t* __restrict__ out_idx,
                                                            uint32_t* __restrict__ out_dist)
{
    __shared__ uint64_t part[4][kWave][KK];
    merge_block_body<KK>(partial, n_q, splits, rows_per_split, blockIdx.x, out_idx, out_dist, part);
}

// Batch merge: units are blocks of 64 queries of the problems with more
// than one split (pre counts zero units for the others).
template <int KK>
__global__ __launch_bounds__(256) void hamming_merge_batch(const BatchMatch* __restrict__ m, int32_t n_m,
                                                           const int32_t* __restrict__ pre, int32_t rows_per_split,
                                                           const uint32_t* __restrict__ partial,
                                                           int32_t* __restrict__ out_idx,
                                                           uint32_t* __restrict__ out_dist)
{
    __shared__ uint64_t part[4][kWave][KK];
    const UnitRange ur = xcd_units(pre[n_m]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_m, u);
        const BatchMatch& b = m[i];
        merge_block_body<KK>(partial + b.part_off, b.n_q, b.splits, rows_per_split, u - pre[i],
                             out_idx + (int64_t)b.out_off * KK, out_dist + (int64_t)b.out_off * KK, part);
    }
}

template <int NW, int KK>
void launch_nw_k(const KnnPlan& p, const uint64_t* query, const uint64_t* train, uint32_t* partial,
                 int32_t* idx, uint32_t* dist, hipStream_t stream)
{
    const int direct = p.splits == 1;
    const int per_block = kWavesPerBlock * kWave * p.qpl;
    const dim3 grid((p.n_q + per_block - 1) / per_block, p.splits);
    const dim3 block(kWavesPerBlock * kWave);
    switch (p.qpl) {
        case 1:
            hipLaunchKernelGGL((hamming_knn_kernel<NW, KK, 1>), grid, block, 0, stream, query, p.n_q, train, p.n_t,
                               p.rows_per_split, partial, idx, dist, direct);
            break;
        case 2:
            hipLaunchKernelGGL((hamming_knn_kernel<NW, KK, 2>), grid, block, 0, stream, query, p.n_q, train, p.n_t,
                               p.rows_per_split, partial, idx, dist, direct);
            break;
        default:
            hipLaunchKernelGGL((hamming_knn_kernel<NW, KK, 4>), grid, block, 0, stream, query, p.n_q, train, p.n_t,
                               p.rows_per_split, partial, idx, dist, direct);
            break;
    }
    if (!direct) {
        hipLaunchKernelGGL((hamming_merge_kernel<KK>), dim3((p.n_q + kWave - 1) / kWave), dim3(4 * kWave), 0, stream,
                           partial, p.n_q, p.splits, p.rows_per_split, idx, dist);
    }
}

template <int NW>
void launch_nw(const KnnPlan& p, const uint64_t* query, const uint64_t* train, uint32_t* partial, int32_t* idx,
               uint32_t* dist, hipStream_t stream)
{
    if (p.k == 1)
        launch_nw_k<NW, 1>(p, query, train, partial, idx, dist, stream);
    else
        launch_nw_k<NW, 2>(p, query, train, partial, idx, dist, stream);
}

template <int NW, int KK>
void launch_batch_nw_k(const KnnBatchPlan& p, const BatchMatch* m, int32_t n_m, const int32_t* pre,
                       const int32_t* merge_pre, const uint64_t* codes, uint32_t* partial, int32_t* idx,
                       uint32_t* dist, hipStream_t stream)
{
    const dim3 block(kWavesPerBlock * kWave);
    switch (p.qpl) {
        case 1:
            hipLaunchKernelGGL((hamming_knn_batch<NW, KK, 1>), dim3(p.grid), block, 0, stream, m, n_m, pre, codes,
                               p.rows_per_split, partial, idx, dist);
            break;
        case 2:
            hipLaunchKernelGGL((hamming_knn_batch<NW, KK, 2>), dim3(p.grid), block, 0, stream, m, n_m, pre, codes,
                               p.rows_per_split, partial, idx, dist);
            break;
        default:
            hipLaunchKernelGGL((hamming_knn_batch<NW, KK, 4>), dim3(p.grid), block, 0, stream, m, n_m, pre, codes,
                               p.rows_per_split, partial, idx, dist);
            break;
    }
    if (p.merge_units > 0)
        hipLaunchKernelGGL((hamming_merge_batch<KK>), dim3(p.merge_grid), block, 0, stream, m, n_m, merge_pre,
                           p.rows_per_split, partial, idx, dist);
}

template <int NW>
void launch_batch_nw(const KnnBatchPlan& p, const BatchMatch* m, int32_t n_m, const int32_t* pre,
                     const int32_t* merge_pre, const uint64_t* codes, uint32_t* partial, int32_t* idx,
                     uint32_t* dist, hipStream_t stream)
{
    if (p.k == 1)
        launch_batch_nw_k<NW, 1>(p, m, n_m, pre, merge_pre, codes, partial, idx, dist, stream);
    else
        launch_batch_nw_k<NW, 2>(p, m, n_m, pre, merge_pre, codes, partial, idx, dist, stream);
}

}  // namespace

int knn_queries_per_wave(int qpl) { return kWave * qpl; }

void launch_knn_batch(const KnnBatchPlan& p, const BatchMatch* m, int32_t n_m, const int32_t* pre,
                      const int32_t* merge_pre, const uint64_t* codes, uint32_t* partial, int32_t* idx,
                      uint32_t* dist, hipStream_t stream)
{
    if (p.n_words == 4)
        launch_batch_nw<4>(p, m, n_m, pre, merge_pre, codes, partial, idx, dist, stream);
    else
        launch_batch_nw<8>(p, m, n_m, pre, merge_pre, codes, partial, idx, dist, stream);
}

size_t KnnPlan::workspace_bytes() const
{
    return splits > 1 ? sizeof(uint32_t) * (size_t)splits * (size_t)n_q * (size_t)k : 0;
}

KnnPlan plan_knn(int32_t n_q, int32_t n_t, int32_t n_words, int32_t k, int num_cus)
{
    KnnPlan p{};
    p.n_q = n_q;
    p.n_t = n_t;
    p.n_words = n_words;
    p.k = k;
    // Aim for ~16 wavefronts per CU while keeping every split at >= 64 rows.
    const int64_t target_waves = 16ll * (num_cus > 0 ? num_cus : 256);
    p.qpl = n_q >= 64 * 2 * target_waves ? 4 : (n_q >= 64 * target_waves ? 2 : 1);
    int64_t qgroups = ((int64_t)n_q + 64 * p.qpl - 1) / (64 * p.qpl);
    if (qgroups < 1) qgroups = 1;  // an empty query set still gets a valid plan
    int64_t splits = (target_waves + qgroups - 1) / qgroups;
    const int64_t max_splits = (n_t + 63) / 64;
    if (splits > max_splits) splits = max_splits;
    const int64_t min_splits = ((int64_t)n_t + kRowMask) / (kRowMask + 1);
    if (splits < min_splits) splits = min_splits;
    if (splits < 1) splits = 1;
    p.rows_per_split = (int32_t)((n_t + splits - 1) / splits);
    if (p.rows_per_split < 1) p.rows_per_split = 1;
    p.splits = (int32_t)((n_t + p.rows_per_split - 1) / p.rows_per_split);
    if (p.splits < 1) p.splits = 1;
    return p;
}

void launch_knn(const KnnPlan& p, const uint64_t* query, const uint64_t* train, int32_t* idx, uint32_t* dist,
                void* workspace, hipStream_t stream)
{
    uint32_t* partial = static_cast<uint32_t*>(workspace);
    switch (p.n_words) {
        case 1: launch_nw<1>(p, query, train, partial, idx, dist, stream); break;
        case 2: launch_nw<2>(p, query, train, partial, idx, dist, stream); break;
        case 3: launch_nw<3>(p, query, train, partial, idx, dist, stream); break;
        case 4: launch_nw<4>(p, query, train, partial, idx, dist, stream); break;
        case 5: launch_nw<5>(p, query, train, partial, idx, dist, stream); break;
        case 6: launch_nw<6>(p, query, train, partial, idx, dist, stream); break;
        case 7: launch_nw<7>(p, query, train, partial, idx, dist, stream); break;
        default: launch_nw<8>(p, query, train, partial, idx, dist, stream); break;
    }
}

}  // namespace bd
