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

// ---- MFMA engine (codes of 4 or 8 words)
//
// The Hamming distance as a dense contraction.  With the query bits
// expanded to bytes q' = 1 - 2q (the negated +-1 form of Sec. III-A's inner
// product) and the train bits to bytes t in {0, 1},
//   sum_k q'_k t_k = |t| - 2 |q AND t|,   so   d_H(q, t) = |q| + q'.t,
// exactly, in int32: the MFMA chain starts from |q| and ends on the
// distance.  One v_mfma_i32_16x16x64_i8 takes one 64-bit word of 16 queries
// x 16 train codes: lane (g, m) supplies bits 16g..16g+15 of the word of
// query row m (A) and of train row m (B), the same byte order on both
// sides, and receives the distances of query rows 4g..4g+3 to train row m
// (D).
//
// A block of four wavefronts holds 16 QM queries per wavefront as operands
// in registers and streams its train split through LDS in chunks of four
// 16-row tiles.  Codes stay packed in memory (expanding them there would
// multiply the operand traffic by eight); they are expanded on chip through
// two 256-entry LDS tables (a byte to its eight bit-bytes, in {0, 1} and in
// {+1, -1}).  Each thread loads 16 bytes of the next chunk while the
// current one is multiplied, and expands them into the other LDS buffer;
// one barrier per chunk.  Keys and the top-k update are those of the
// lane-per-query kernel (d << 22 | row within the split; top-2 by min and
// med3); the 16 lanes sharing a query row merge their lists by a butterfly
// at the end.
typedef int int32x4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 4;
constexpr int kMfmaChunk = 64;  // train rows per LDS stage: four 16-row tiles
// query tiles of 16 per wavefront: every B operand read from LDS feeds QM
// MFMAs; the A operands take 4 QM NW VGPRs
template <int NW>
constexpr int mfma_qm() { return 4; }

__device__ __forceinline__ uint32_t med3u(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Insert into a sorted top-k list (best[0] <= best[1]).
template <int KK>
__device__ __forceinline__ void topk_insert_med3(uint32_t (&best)[KK], uint32_t key)
{
    if constexpr (KK == 2) best[1] = med3u(best[0], best[1], key);
    best[0] = min(best[0], key);
}

// Merge the top-k list of the lane CTRL (a DPP row rotation) away inside
// the lane's row of 16: after rotations by 8, 4, 2 and 1 every lane of the
// row has merged the 16 disjoint lists of the row.
template <int KK, int CTRL>
__device__ __forceinline__ void topk_merge_ror(uint32_t (&best)[KK])
{
    const uint32_t p0 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)best[0], CTRL, 0xf, 0xf, false);
    if constexpr (KK == 2) {
        const uint32_t p1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)best[1], CTRL, 0xf, 0xf, false);
        best[1] = min(max(best[0], p0), min(best[1], p1));
    }
    best[0] = min(best[0], p0);
}

// Eight bytes of a 16-byte operand from two table entries: bytes lo and hi
// of a 16-bit piece.
__device__ __forceinline__ int32x4 expand16(const uint2* table, uint32_t piece)
{
    const uint2 a = table[piece & 0xffu], b = table[piece >> 8];
    return int32x4{(int)a.x, (int)a.y, (int)b.x, (int)b.y};
}

// LDS of a block: the two chunk buffers and the two expansion tables.
template <int NW>
struct MfmaShared {
    int32x4 tiles[2][4 * NW * kWave];
    uint2 bits01[256], bits_pm[256];
};

// The expansion tables: byte v -> bit j of v as byte j, in {0, 1} and in
// {+1, -1} (0x01 / 0xff).  Followed by a barrier in the block body.
template <int NW>
__device__ __forceinline__ void mfma_tables(MfmaShared<NW>& sh)
{
    const uint32_t v = threadIdx.x;
    uint32_t lo = 0u, hi = 0u, plo = 0u, phi = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t b0 = (v >> j) & 1u, b1 = (v >> (j + 4)) & 1u;
        lo |= b0 << (8 * j);
        hi |= b1 << (8 * j);
        plo |= (b0 ? 0xffu : 0x01u) << (8 * j);
        phi |= (b1 ? 0xffu : 0x01u) << (8 * j);
    }
    sh.bits01[v] = make_uint2(lo, hi);
    sh.bits_pm[v] = make_uint2(plo, phi);
}

// Distances of the wavefront's 16 QM queries to the 16 rows of tile tau of
// an LDS chunk: D[qm] = |q| + sum over the NW words of the MFMA products.
template <int NW, int QM>
__device__ __forceinline__ void mfma_tile(const int32x4* chunk, int tau, int lane, const int32x4 (&A)[QM][NW],
                                          const int32x4 (&pa)[QM], int32x4 (&D)[QM])
{
    {
        const int32x4 b = chunk[(tau * NW) * kWave + lane];
#pragma unroll
        for (int qm = 0; qm < QM; ++qm) D[qm] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[qm][0], b, pa[qm], 0, 0, 0);
    }
#pragma unroll
    for (int kc = 1; kc < NW; ++kc) {
        const int32x4 b = chunk[(tau * NW + kc) * kWave + lane];
#pragma unroll
        for (int qm = 0; qm < QM; ++qm) D[qm] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[qm][kc], b, D[qm], 0, 0, 0);
    }
}

// One block (256 threads): queries 64 QM qb .. of one problem against train
// split `split` (splits start on 16-row tiles: rows_per_split is a multiple
// of 16).  Every thread of the block calls it with the same arguments.
template <int NW, int KK>
__device__ __forceinline__ void mfma_block_body(const uint64_t* __restrict__ query, int32_t n_q,
                                                const uint64_t* __restrict__ train, int32_t n_t,
                                                int32_t rows_per_split, int qb, int split,
                                                uint32_t* __restrict__ partial, int32_t* __restrict__ out_idx,
                                                uint32_t* __restrict__ out_dist, bool direct, MfmaShared<NW>& sh)
{
    constexpr int QM = mfma_qm<NW>();
    auto& tiles = sh.tiles;
    const uint2* bits01 = sh.bits01;
    const uint2* bits_pm = sh.bits_pm;
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int g = lane >> 4, m = lane & 15;
    const int qt0 = (qb * kMfmaWaves + wave) * QM;
    const int t0 = split * rows_per_split;
    const int t1 = min(n_t, t0 + rows_per_split);

    // chunk staging: 64 rows x NW words, 16 bytes (two words) per thread;
    // thread t < 32 NW holds words 2 (t % (NW / 2)), +1 of chunk row
    // t / (NW / 2)
    constexpr int kLoaders = 32 * NW;
    const bool loader = (int)threadIdx.x < kLoaders;
    const int s_row = (int)threadIdx.x / (NW / 2), s_word = ((int)threadIdx.x % (NW / 2)) * 2;
    uint4 pre = make_uint4(0u, 0u, 0u, 0u);
    auto load_chunk = [&](int c0) {
        const int r = c0 + s_row;
        if (loader) {
            // two 8-byte loads: codes are only guaranteed 8-byte aligned
            const uint2* src = reinterpret_cast<const uint2*>(train + (int64_t)r * NW + s_word);
            const uint2 a = r < t1 ? src[0] : make_uint2(0u, 0u), b = r < t1 ? src[1] : make_uint2(0u, 0u);
            pre = make_uint4(a.x, a.y, b.x, b.y);
        }
    };
    auto store_chunk = [&](int b) {
        if (!loader) return;
        const int tau = s_row >> 4, n = s_row & 15;
        const uint32_t w[4] = {pre.x, pre.y, pre.z, pre.w};  // words s_word, s_word + 1 (low, high halves)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int32x4* dst = &tiles[b][(tau * NW + s_word + h) * kWave + n];
#pragma unroll
            for (int gg = 0; gg < 4; ++gg)
                dst[16 * gg] = expand16(bits01, (w[2 * h + (gg >> 1)] >> (16 * (gg & 1))) & 0xffffu);
        }
    };

    // the wavefront's query codes (rows past n_q read as zero codes; a zero
    // code yields zero operands below), loaded before the table barrier
    uint32_t qcode[QM][NW];  // bits 16g..16g+15 of each word
    uint32_t pc[QM];         // |q| of query row m
    {
        const bool all_in = (qt0 + QM) * 16 <= n_q;
#pragma unroll
        for (int qm = 0; qm < QM; ++qm) {
            const int qi = (qt0 + qm) * 16 + m;
            const bool in = all_in || qi < n_q;
            pc[qm] = 0u;
#pragma unroll
            for (int kc = 0; kc < NW; ++kc) {
                const uint64_t v = in ? query[(int64_t)qi * NW + kc] : 0ull;
                pc[qm] += (uint32_t)__popcll(v);
                qcode[qm][kc] = (uint32_t)(v >> (16 * g)) & 0xffffu;
            }
        }
    }
    load_chunk(t0);
    __syncthreads();  // tables; the previous unit's reads of the buffers

    // queries as -+1 operands (zero for rows past n_q); |q| of the rows this
    // lane receives in D
    int32x4 A[QM][NW], pa[QM];
#pragma unroll
    for (int qm = 0; qm < QM; ++qm) {
        const bool in = (qt0 + qm) * 16 + m < n_q;
#pragma unroll
        for (int kc = 0; kc < NW; ++kc)
            A[qm][kc] = in ? expand16(bits_pm, qcode[qm][kc]) : int32x4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < 4; ++i) pa[qm][i] = __shfl((int)pc[qm], 4 * g + i, kWave);
    }
    uint32_t best[QM][4][KK];
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int s = 0; s < KK; ++s) best[qm][i][s] = kEmpty;

    store_chunk(0);
    __syncthreads();
    int buf = 0;
    for (int c0 = t0; c0 < t1; c0 += kMfmaChunk) {
        const bool more = c0 + kMfmaChunk < t1;
        if (more) load_chunk(c0 + kMfmaChunk);
        const bool full = c0 + kMfmaChunk <= t1;
        const uint32_t row0 = (uint32_t)(c0 - t0 + m);
        if (NW == 4 && full) {
            // software pipeline over the four tiles: the MFMAs of tile tau + 1
            // run while tile tau's distances are inserted (8-word operands
            // leave no registers for the second accumulator set)
            int32x4 D[2][QM];
            mfma_tile<NW, QM>(tiles[buf], 0, lane, A, pa, D[0]);
#pragma unroll
            for (int tau = 0; tau < 4; ++tau) {
                if (tau < 3) mfma_tile<NW, QM>(tiles[buf], tau + 1, lane, A, pa, D[(tau + 1) & 1]);
#pragma unroll
                for (int qm = 0; qm < QM; ++qm)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        topk_insert_med3<KK>(best[qm][i], ((uint32_t)D[tau & 1][qm][i] << kRowBits) | (row0 + 16 * tau));
            }
        } else {
            // 8-word codes, and partial chunks: one tile at a time
#pragma unroll
            for (int tau = 0; tau < 4; ++tau) {
                if (!full && c0 + 16 * tau >= t1) break;  // tiles past the split end
                int32x4 D[QM];
                mfma_tile<NW, QM>(tiles[buf], tau, lane, A, pa, D);
                const bool valid = full || c0 + 16 * tau + m < t1;
#pragma unroll
                for (int qm = 0; qm < QM; ++qm)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        topk_insert_med3<KK>(best[qm][i],
                                             valid ? ((uint32_t)D[qm][i] << kRowBits) | (row0 + 16 * tau) : kEmpty);
            }
        }
        if (more) store_chunk(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // merge over the 16 lanes of each query row (DPP row_ror:8, 4, 2, 1),
    // then lane m == 0 writes
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            topk_merge_ror<KK, 0x128>(best[qm][i]);
            topk_merge_ror<KK, 0x124>(best[qm][i]);
            topk_merge_ror<KK, 0x122>(best[qm][i]);
            topk_merge_ror<KK, 0x121>(best[qm][i]);
        }
    if (m != 0) return;
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int qi = (qt0 + qm) * 16 + 4 * g + i;
            if (qi >= n_q) continue;
#pragma unroll
            for (int s = 0; s < KK; ++s) {
                const uint32_t key = best[qm][i][s];
                if (direct) {
                    const bool empty = key == kEmpty;
                    out_idx[(int64_t)qi * KK + s] = empty ? -1 : (int32_t)(t0 + (key & kRowMask));
                    out_dist[(int64_t)qi * KK + s] = empty ? kEmpty : key >> kRowBits;
                } else {
                    partial[((int64_t)split * n_q + qi) * KK + s] = key;
                }
            }
        }
}

template <int NW, int KK>
__global__ __launch_bounds__(256, 2) void hamming_mfma_kernel(const uint64_t* __restrict__ query, int32_t n_q,
                                                              const uint64_t* __restrict__ train, int32_t n_t,
                                                              int32_t rows_per_split, uint32_t* __restrict__ partial,
                                                              int32_t* __restrict__ out_idx,
                                                              uint32_t* __restrict__ out_dist, int direct)
{
    __shared__ MfmaShared<NW> sh;
    mfma_tables<NW>(sh);
    mfma_block_body<NW, KK>(query, n_q, train, n_t, rows_per_split, blockIdx.x, blockIdx.y, partial, out_idx, out_dist,
                            direct != 0, sh);
}

// Batch: units are (problem, split, block of 256 queries), problem-major and
// query block fastest, so consecutive units share a train split.
template <int NW, int KK>
__global__ __launch_bounds__(256, 2) void hamming_mfma_batch(const BatchMatch* __restrict__ mt, int32_t n_m,
                                                             const int32_t* __restrict__ pre,
                                                             const uint64_t* __restrict__ codes,
                                                             int32_t rows_per_split, uint32_t* __restrict__ partial,
                                                             int32_t* __restrict__ out_idx,
                                                             uint32_t* __restrict__ out_dist)
{
    __shared__ MfmaShared<NW> sh;
    mfma_tables<NW>(sh);
    const UnitRange ur = xcd_units(pre[n_m]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_m, u);
        const BatchMatch& b = mt[i];
        const int local = u - pre[i];
        const int split = local / b.qgroups;
        const int qb = local - split * b.qgroups;
        mfma_block_body<NW, KK>(codes + (int64_t)b.q_off * NW, b.n_q, codes + (int64_t)b.t_off * NW, b.n_t,
                                rows_per_split, qb, split, partial + b.part_off, out_idx + (int64_t)b.out_off * KK,
                                out_dist + (int64_t)b.out_off * KK, b.splits == 1, sh);
    }
}

template <int NW, int KK>
void launch_mfma_nw_k(const KnnPlan& p, const uint64_t* query, const uint64_t* train, uint32_t* partial, int32_t* idx,
                      uint32_t* dist, hipStream_t stream)
{
    const int direct = p.splits == 1;
    const int per_block = kMfmaWaves * 16 * mfma_qm<NW>();
    const dim3 grid((p.n_q + per_block - 1) / per_block, p.splits);
    hipLaunchKernelGGL((hamming_mfma_kernel<NW, KK>), grid, dim3(kMfmaWaves * kWave), 0, stream, query, p.n_q, train,
                       p.n_t, p.rows_per_split, partial, idx, dist, direct);
    if (!direct)
        hipLaunchKernelGGL((hamming_merge_kernel<KK>), dim3((p.n_q + kWave - 1) / kWave), dim3(4 * kWave), 0, stream,
                           partial, p.n_q, p.splits, p.rows_per_split, idx, dist);
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
    if constexpr (NW == 4 || NW == 8) {
        if (p.mfma) {
            if (p.k == 1)
                launch_mfma_nw_k<NW, 1>(p, query, train, partial, idx, dist, stream);
            else
                launch_mfma_nw_k<NW, 2>(p, query, train, partial, idx, dist, stream);
            return;
        }
    }
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
        case 0:
            hipLaunchKernelGGL((hamming_mfma_batch<NW, KK>), dim3(p.grid), block, 0, stream, m, n_m, pre, codes,
                               p.rows_per_split, partial, idx, dist);
            break;
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

int knn_queries_per_unit(int qpl, int n_words)
{
    return qpl == 0 ? kMfmaWaves * 16 * (n_words == 4 ? mfma_qm<4>() : mfma_qm<8>()) : kWave * qpl;
}

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
    if (n_words == 4 || n_words == 8) {
        // MFMA engine: blocks of 64 QM queries; as many splits as fill one
        // round of one block per CU (a small problem then leaves room for a
        // concurrent one on another stream), or of two blocks per CU when
        // splits would exceed 1024 rows (a wavefront alone on its SIMD does
        // not keep the matrix pipe busy); splits of at least one 64-row chunk
        p.mfma = 1;
        p.qpl = 0;
        const int64_t per_block = knn_queries_per_unit(0, n_words);
        const int64_t qblocks = n_q > 0 ? ((int64_t)n_q + per_block - 1) / per_block : 1;
        const int64_t cus = num_cus > 0 ? num_cus : 256;
        int64_t splits = cus / qblocks;
        if (splits >= 1 && ((int64_t)n_t + splits - 1) / splits > 1024) splits = 2 * cus / qblocks;
        const int64_t max_splits = (n_t + 63) / 64;
        if (splits > max_splits) splits = max_splits;
        const int64_t min_splits = ((int64_t)n_t + kRowMask) / (kRowMask + 1);
        if (splits < min_splits) splits = min_splits;
        if (splits < 1) splits = 1;
        // splits start on 16-row tiles; at most 2^22 - 16 rows keep keys in 32 bits
        int64_t rows = ((n_t + splits - 1) / splits + 15) / 16 * 16;
        if (rows > (int64_t)kRowMask + 1 - 16) rows = (int64_t)kRowMask + 1 - 16;
        if (rows < 16) rows = 16;
        p.rows_per_split = (int32_t)rows;
        p.splits = (int32_t)((n_t + rows - 1) / rows);
        if (p.splits < 1) p.splits = 1;
        return p;
    }
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
