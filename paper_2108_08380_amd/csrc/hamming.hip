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
// The Hamming distance as a dense contraction that ends on the sort key.
// With the query bits as bytes -64 q (q in {0, 1}) and the train bits as
// bytes t' = 2t - 1 in {-1, +1} (the +-1 form of Sec. III-A's inner
// product),
//   sum_k (-64 q_k) t'_k = 64 (|q| - 2 |q AND t|) = 64 (d_H(q, t) - |t|),
// exactly, in int32.  One v_mfma_i32_32x32x32_i8 takes 32 bits of 32
// queries x 32 train codes: lane (g, m) supplies bits 16g..16g+15 of the
// 32-bit slice of query row m (A) and of train row m (B), the same byte
// order on both sides, and receives the products of query rows
// 8j + 4g + i (j, i < 4) with train row m (D).  Each chain starts with one
// more slice whose bytes add 64 |t| + tag (A: four columns of -64 and one of
// -1; B: -|t| cut into four parts of at most 128, and -tag), so the MFMA
// delivers key = 64 d_H + tag < 2^16, where tag < 64 numbers the 32-row tile
// inside the split (so splits hold at most 2048 rows) and the lane numbers
// the row inside the tile.  Two keys of neighbouring query rows share a
// register as 16-bit halves, and the top-2 update is three packed 16-bit
// min/max per pair, after one byte permute.  After the split the lists are
// rewritten as (d << 22 | row within the split) and merged over the 32 lanes
// that share a query row by a transposing butterfly.
//
// A block of four wavefronts holds 32 QM queries per wavefront as operands
// in registers and streams its train split through LDS in chunks of two
// 32-row tiles.  Codes stay packed in memory (expanding them there would
// multiply the operand traffic by eight) and are expanded on chip: the
// queries once per block through a 256-entry LDS table (a byte to its eight
// bit-bytes), the train rows on the VALU (a nibble spread to four bytes by a
// multiply and a mask, then a byte permute).  Each thread loads a quarter
// row of the next chunk at the start of a chunk and expands it into the
// other LDS buffer in steps between the MFMAs of the chunk's second tile;
// one barrier per chunk.  The 32x32 form is used because it leaves issue
// cycles for VALU work between matrix instructions, where the 16x16x64 form
// does not; for 4-word codes the keys of one tile are also inserted between
// the MFMAs of the next.
typedef int int32x4 __attribute__((ext_vector_type(4)));
typedef int int32x16 __attribute__((ext_vector_type(16)));

constexpr int kMfmaWaves = 4;
constexpr int kMfmaTile = 32;                            // train rows per MFMA tile
constexpr int kMfmaChunk = 2 * kMfmaTile;                // train rows per LDS stage
// 32-query tiles per wavefront (four for 8-word codes was tried: the
// operands then exceed even the accumulation registers and spill)
constexpr int kMfmaQM = 2;
constexpr int kMfmaQueries = kMfmaWaves * 32 * kMfmaQM;  // queries per block
constexpr uint32_t kTagBits = 6;
constexpr uint32_t kTagMask = (1u << kTagBits) - 1u;
constexpr int kMfmaMaxRows = (1 << kTagBits) * kMfmaTile;  // train rows per split
constexpr uint32_t kEmpty16 = 0xffffu;
// Resident blocks per CU the kernels are compiled for: two, so that a
// wavefront's MFMAs overlap the other block's expansion and barrier, and a
// small problem shares the CUs with a concurrent matcher.
constexpr int kMfmaMinBlocks = 2;
static_assert(kMfmaMaxRows == BD_BATCH_MFMA_MAX_ROWS, "the batch limit is the key tag's range");

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Insert a pair of 16-bit keys (two query rows, one per half) into the
// pair's sorted top-k lists (best[0] <= best[1] in each half).
template <int KK>
__device__ __forceinline__ void topk_insert_pair(uint32_t (&best)[KK], uint32_t keys)
{
    const u16x2 k = __builtin_bit_cast(u16x2, keys);
    const u16x2 b0 = __builtin_bit_cast(u16x2, best[0]);
    if constexpr (KK == 2) {
        const u16x2 b1 = __builtin_bit_cast(u16x2, best[1]);
        best[1] = __builtin_bit_cast(uint32_t, __builtin_elementwise_min(b1, __builtin_elementwise_max(b0, k)));
    }
    best[0] = __builtin_bit_cast(uint32_t, __builtin_elementwise_min(b0, k));
}

// The 16-bit keys of query rows 2p and 2p + 1 of a product tile as one
// register (the keys are below 2^16).
__device__ __forceinline__ uint32_t key_pair(const int32x16& D, int p)
{
    return __builtin_amdgcn_perm((uint32_t)D[2 * p + 1], (uint32_t)D[2 * p], 0x05040100u);
}

// Merge two disjoint sorted top-k lists into `best`.
template <int KK>
__device__ __forceinline__ void topk_merge(uint32_t (&best)[KK], const uint32_t (&other)[KK])
{
    if constexpr (KK == 2) best[1] = min(max(best[0], other[0]), min(best[1], other[1]));
    best[0] = min(best[0], other[0]);
}

// Eight bytes of a 16-byte operand from two table entries: bytes lo and hi
// of a 16-bit piece.
__device__ __forceinline__ int32x4 expand16(const uint2* table, uint32_t piece)
{
    const uint2 a = table[piece & 0xffu], b = table[piece >> 8];
    return int32x4{(int)a.x, (int)a.y, (int)b.x, (int)b.y};
}

// The same sixteen bytes from VALU alone: a nibble spread to the low bits of
// four bytes by one 24-bit multiply and a mask, then a byte permute that
// maps 0 / 1 to bytes 0 / 1 of `lut`.  Four instructions per dword, no LDS
// traffic.
__device__ __forceinline__ int32x4 expand16_valu(uint32_t piece, uint32_t lut)
{
    int32x4 r;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        r[j] = (int)__builtin_amdgcn_perm(0u, lut, (((piece >> (4 * j)) & 15u) * 0x00204081u) & 0x01010101u);
    return r;
}

// LDS of a block: the two chunk buffers of B operands ([tile][slice][lane],
// slice 0 the key slice) and the query expansion table.
template <int NW>
struct MfmaShared {
    int32x4 tiles[2][2 * (2 * NW + 1) * kWave];
    uint2 bits_q[256];
};

// The query expansion table: byte v -> bit j of v as byte j in {0, -64}.
// Followed by a barrier in the block body.
template <int NW>
__device__ __forceinline__ void mfma_tables(MfmaShared<NW>& sh)
{
    const uint32_t v = threadIdx.x;
    uint32_t qlo = 0u, qhi = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        qlo |= (((v >> j) & 1u) ? 0xc0u : 0x00u) << (8 * j);
        qhi |= (((v >> (j + 4)) & 1u) ? 0xc0u : 0x00u) << (8 * j);
    }
    sh.bits_q[v] = make_uint2(qlo, qhi);
}

// Keys of the wavefront's QM query tiles against train tile tau of an LDS
// chunk: D[qm] = the key slice's product plus the 2 NW code slices'.  The
// operand reads run kAhead slices ahead of their MFMAs (the LDS latency
// would otherwise stall every slice).  With PIPE, the keys Dp of the previous
// tile are inserted between the MFMAs, a share after each, so that the
// selection issues in the matrix pipe's shadow; side(step) adds other work
// after MFMA step s QM + qm; scheduling barriers keep that order.
template <int NW, int KK, int QM, bool PIPE, typename Side>
__device__ __forceinline__ void mfma_tile(const int32x4* chunk, int tau, int lane, const int32x4& Ak,
                                          const int32x4 (&A)[QM][2 * NW], int32x16 (&D)[QM],
                                          const int32x16 (&Dp)[QM], uint32_t (&best)[QM][8][KK], Side&& side)
{
    constexpr int S = 2 * NW + 1;
    constexpr int kAhead = NW == 4 ? 3 : 2;
    constexpr int kPairs = QM * 8;
    int32x4 b[S];
#pragma unroll
    for (int s = 0; s < kAhead; ++s) b[s] = chunk[(tau * S + s) * kWave + lane];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (s + kAhead < S) b[s + kAhead] = chunk[(tau * S + s + kAhead) * kWave + lane];
#pragma unroll
        for (int qm = 0; qm < QM; ++qm) {
            if (s == 0) {
                const int32x16 zero = {};
                D[qm] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Ak, b[0], zero, 0, 0, 0);
            } else {
                D[qm] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[qm][s - 1], b[s], D[qm], 0, 0, 0);
            }
            if constexpr (PIPE) {
                // key pairs j0 .. j1 - 1 of the previous tile after MFMA (s, qm)
                constexpr int kSteps = S * QM;
                const int step = s * QM + qm;
                const int j0 = step * kPairs / kSteps, j1 = (step + 1) * kPairs / kSteps;
#pragma unroll
                for (int j = j0; j < j1; ++j) {
                    topk_insert_pair<KK>(best[j / 8][j % 8], key_pair(Dp[j / 8], j % 8));
                    // a use of the lists here keeps the compiler from sinking
                    // the updates out of the MFMA sequence
#pragma unroll
                    for (int k = 0; k < KK; ++k) asm volatile("" ::"v"(best[j / 8][j % 8][k]));
                }
            }
            side(s * QM + qm);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Insert the keys of each query tile (invalid train rows give none).
template <int KK, int QM>
__device__ __forceinline__ void mfma_select(const int32x16 (&D)[QM], bool valid, uint32_t (&best)[QM][8][KK])
{
    const uint32_t mask = valid ? 0u : 0xffffffffu;
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int p = 0; p < 8; ++p) topk_insert_pair<KK>(best[qm][p], key_pair(D[qm], p) | mask);
}

// One round of the transposing butterfly over H-slot halves: `lo` and `hi`
// are the lane's slots, `upper` selects the half it keeps; CTRL is the DPP
// control that reaches the partner (0: the lane 16 away, through the LDS
// crossbar).
template <int H, int KK, int CTRL>
__device__ __forceinline__ void bfly_round(const uint32_t (*lo)[KK], const uint32_t (*hi)[KK], uint32_t (&out)[H][KK],
                                           int upper)
{
#pragma unroll
    for (int j = 0; j < H; ++j) {
        uint32_t recv[KK];
#pragma unroll
        for (int s = 0; s < KK; ++s) {
            const uint32_t keep = upper ? hi[j][s] : lo[j][s];
            const uint32_t send = upper ? lo[j][s] : hi[j][s];
            out[j][s] = keep;
            if constexpr (CTRL == 0)
                recv[s] = (uint32_t)__shfl_xor((int)send, 16, kWave);
            else
                recv[s] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)send, CTRL, 0xf, 0xf, false);
        }
        topk_merge<KK>(out[j], recv);
    }
}
template <int H, int KK, int CTRL>
__device__ __forceinline__ void bfly_round(const uint32_t (&in)[2 * H][KK], uint32_t (&out)[H][KK], int upper)
{
    bfly_round<H, KK, CTRL>(&in[0], &in[H], out, upper);
}

// After the split: widen the lane's 16-bit keys to (key << 16 | tag << 5 |
// lane row), which order as (d, row within the split) across lanes, merge
// the 32 lanes of each half-wave by a transposing butterfly (in each round a
// lane keeps one half of its slots and merges into it the partner's lists
// of that half; after five rounds lane (g, n) holds the lists of slots
// QM / 2 n + i, i < QM / 2, slot 16 qm + v) and rewrite those as
// (d << 22 | row within the split).
template <int KK, int QM>
__device__ __forceinline__ void mfma_merge(const uint32_t (&best)[QM][8][KK], int n, uint32_t (&out)[QM / 2][KK])
{
    uint32_t w[16 * QM][KK];
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int p = 0; p < 8; ++p)
#pragma unroll
            for (int s = 0; s < KK; ++s) {
                const uint32_t k2 = best[qm][p][s];  // keys of slots 2p (low half) and 2p + 1
                w[16 * qm + 2 * p][s] = (k2 << 16) | ((k2 & kTagMask) << 5) | (uint32_t)n;
                w[16 * qm + 2 * p + 1][s] = (k2 & 0xffff0000u) | (((k2 >> 16) & kTagMask) << 5) | (uint32_t)n;
            }
    uint32_t c16[8 * QM][KK], c8[4 * QM][KK], c4[2 * QM][KK], c2[QM][KK], c1[QM / 2][KK];
    bfly_round<8 * QM, KK, 0>(w, c16, (n >> 4) & 1);
    bfly_round<4 * QM, KK, 0x128>(c16, c8, (n >> 3) & 1);  // row_ror:8 (lane ^ 8)
    bfly_round<2 * QM, KK, 0x141>(c8, c4, (n >> 2) & 1);   // row_half_mirror (lane ^ 7)
    bfly_round<QM, KK, 0x4E>(c4, c2, (n >> 1) & 1);        // quad_perm 2,3,0,1 (lane ^ 2)
    bfly_round<QM / 2, KK, 0xB1>(c2, c1, n & 1);           // quad_perm 1,0,3,2 (lane ^ 1)
#pragma unroll
    for (int i = 0; i < QM / 2; ++i)
#pragma unroll
        for (int s = 0; s < KK; ++s) {
            const uint32_t k = c1[i][s] >> 16;
            out[i][s] = k == kEmpty16 ? kEmpty : ((k >> kTagBits) << kRowBits) | (c1[i][s] & (kTagMask << 5 | 31u));
        }
}

// One block (256 threads): queries 128 QM qb .. of one problem against
// train split `split` (splits start on 16-row boundaries: rows_per_split is
// a multiple of 16, at most kMfmaMaxRows).  Every thread of the block calls
// it with the same arguments.
template <int NW, int KK, int QM>
__device__ __forceinline__ void mfma_block_body(const uint64_t* __restrict__ query, int32_t n_q,
                                                const uint64_t* __restrict__ train, int32_t n_t,
                                                int32_t rows_per_split, int qb, int split,
                                                uint32_t* __restrict__ partial, int32_t* __restrict__ out_idx,
                                                uint32_t* __restrict__ out_dist, bool direct, MfmaShared<NW>& sh)
{
    constexpr int S = 2 * NW + 1;   // slices of a tile: the key slice, then 32-bit code slices
    constexpr int WPT = NW / 4;     // words per loader thread
    auto& tiles = sh.tiles;
    const uint2* bits_q = sh.bits_q;
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int g = lane >> 5, m = lane & 31;
    const int qt0 = (qb * kMfmaWaves + wave) * QM;
    const int t0 = split * rows_per_split;
    const int t1 = min(n_t, t0 + rows_per_split);

    // chunk staging: thread t holds words WPT (t % 4) .. of chunk row t / 4
    const int s_row = (int)threadIdx.x >> 2, s_q = (int)threadIdx.x & 3;
    uint2 pre[WPT];
    auto load_chunk = [&](int c0) {
        const int r = c0 + s_row;
        const uint2* src = reinterpret_cast<const uint2*>(train + (int64_t)r * NW + WPT * s_q);
#pragma unroll
        for (int w = 0; w < WPT; ++w) pre[w] = r < t1 ? src[w] : make_uint2(0u, 0u);
    };
    // expansion of the staged chunk into LDS buffer b, in 4 WPT + 1 steps
    // that can be spread over the MFMAs of the current chunk: step k < 4 WPT
    // expands piece k of the thread's words on the VALU (piece p = bits
    // 16p..16p+15 of the row goes to code slice p / 2, half-wave p % 2 of
    // the row's tile) and stores it; the last step writes the row's key
    // slice
    constexpr int kExpandSteps = 4 * WPT + 1;
    uint32_t pc = 0u;
    auto expand_step = [&](int k, int b, int c0) {
        const int tau = s_row >> 5, n = s_row & 31;
        int32x4* tile = &tiles[b][tau * S * kWave];
        if (k < 4 * WPT) {
            const int w = k >> 2, h = k & 3;
            uint2 v = pre[w];
            // pin the step here: without it the compiler hoists the VALU
            // work above the MFMAs, where it also waits for the load
            asm volatile("" : "+v"(v.x), "+v"(v.y));
            if (h == 0) pc = (w == 0 ? 0u : pc) + (uint32_t)__popc(v.x) + (uint32_t)__popc(v.y);
            const int p = 4 * (WPT * s_q + w) + h;
            tile[(1 + (p >> 1)) * kWave + (p & 1) * 32 + n] =
                expand16_valu(((h < 2 ? v.x : v.y) >> (16 * (h & 1))) & 0xffffu, 0x01ffu);
        } else {
            // |t| of the row (its four threads are adjacent lanes); key slice:
            // bytes -x1..-x4 (x1 + .. + x4 = |t|, each at most 128) and -tag in
            // half-wave 0, zeros in half-wave 1 (threads 0, 2 and 1, 3 of the
            // row store the same values)
            uint32_t t = pc;
            asm volatile("" : "+v"(t));
            t += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0xB1, 0xf, 0xf, false);  // quad_perm 1,0,3,2
            t += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0x4E, 0xf, 0xf, false);  // quad_perm 2,3,0,1
            const uint32_t tag = (uint32_t)((c0 - t0) / kMfmaTile + tau);
            uint32_t x = 0u;
#pragma unroll
            for (int i = 0; i < 4; ++i) x |= ((0u - ((t + 3u - (uint32_t)i) >> 2)) & 0xffu) << (8 * i);
            const bool hi = (s_q & 1) != 0;
            tile[(hi ? 32 : 0) + n] = hi ? int32x4{0, 0, 0, 0} : int32x4{(int)x, (int)((0u - tag) & 0xffu), 0, 0};
        }
    };

    // the wavefront's query codes, loaded coalesced (lane l: word l % NW of
    // tile row l / NW, 64 / NW rows per load) and staged in the second chunk
    // buffer, which is free until the first chunk has been multiplied;
    // rows past n_q read as zero codes, which give zero operands
    constexpr int kQWords = QM * 32 * NW;  // words of the wavefront's queries
    uint2* qstage = reinterpret_cast<uint2*>(&tiles[1][0]) + wave * kQWords;
    {
        const int64_t w0 = (int64_t)qt0 * 32 * NW;
        const int64_t w_end = (int64_t)n_q * NW;
        uint2 v[kQWords / kWave];
#pragma unroll
        for (int k = 0; k < kQWords / kWave; ++k) {
            const int64_t w = w0 + k * kWave + lane;
            v[k] = w < w_end ? reinterpret_cast<const uint2*>(query)[w] : make_uint2(0u, 0u);
        }
        load_chunk(t0);
#pragma unroll
        for (int k = 0; k < kQWords / kWave; ++k) qstage[k * kWave + lane] = v[k];
    }
    __syncthreads();  // tables, staged queries; the previous unit's reads of the buffers

    // query operands: code slice s of query row m of tile qm is word s / 2,
    // bits 32 (s % 2) + 16 g ..; the key slice's A is four columns of -64 and
    // one of -1 in half-wave 0
    int32x4 A[QM][S - 1];
#pragma unroll
    for (int qm = 0; qm < QM; ++qm) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint2 q = qstage[(qm * 32 + m) * NW + w];
            A[qm][2 * w] = expand16(bits_q, (q.x >> (16 * g)) & 0xffffu);
            A[qm][2 * w + 1] = expand16(bits_q, (q.y >> (16 * g)) & 0xffffu);
        }
    }
    const int32x4 Ak = g == 0 ? int32x4{(int)0xc0c0c0c0u, 0xff, 0, 0} : int32x4{0, 0, 0, 0};
    uint32_t best[QM][8][KK];  // key pairs of query rows 2p, 2p + 1
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int p = 0; p < 8; ++p)
#pragma unroll
            for (int s = 0; s < KK; ++s) best[qm][p][s] = kEmpty;

#pragma unroll
    for (int k = 0; k < kExpandSteps; ++k) expand_step(k, 0, t0);
    __syncthreads();  // chunk 0; the staged queries have been read

    // full chunks; for 4-word codes software-pipelined over tiles: the keys
    // of one tile are inserted while those of the next are computed (the
    // first insertion takes kEmpty keys, a no-op); 8-word operands leave no
    // registers for the second key set
    constexpr bool kPipe = NW == 4;
    int32x16 Dp[QM];
#pragma unroll
    for (int qm = 0; qm < QM; ++qm)
#pragma unroll
        for (int v = 0; v < 16; ++v) Dp[qm][v] = (int)kEmpty;
    const int t_full = t0 + (t1 - t0) / kMfmaChunk * kMfmaChunk;
    int buf = 0;
    int c0 = t0;
    for (; c0 < t_full; c0 += kMfmaChunk) {
        // the next chunk (rows past t1 load as zeros) is loaded here and
        // expanded into the other buffer between the MFMAs of tile 1, one
        // step after every kEvery MFMAs
        load_chunk(c0 + kMfmaChunk);
#pragma unroll
        for (int tau = 0; tau < 2; ++tau) {
            int32x16 D[QM];
            mfma_tile<NW, KK, QM, kPipe>(tiles[buf], tau, lane, Ak, A, D, Dp, best, [&](int step) {
                constexpr int kEvery = S * QM / kExpandSteps;
                if (tau == 1 && step % kEvery == kEvery - 1 && step / kEvery < kExpandSteps)
                    expand_step(step / kEvery, buf ^ 1, c0 + kMfmaChunk);
            });
            if constexpr (kPipe) {
#pragma unroll
                for (int qm = 0; qm < QM; ++qm) Dp[qm] = D[qm];
            } else {
                mfma_select<KK, QM>(D, true, best);
            }
        }
        __syncthreads();
        buf ^= 1;
    }
    if constexpr (kPipe) mfma_select<KK, QM>(Dp, true, best);
    // the partial last chunk, one tile at a time
    if (c0 < t1) {
#pragma unroll
        for (int tau = 0; tau < 2; ++tau) {
            if (c0 + kMfmaTile * tau >= t1) break;
            int32x16 D[QM];
            mfma_tile<NW, KK, QM, false>(tiles[buf], tau, lane, Ak, A, D, Dp, best, [](int) {});
            mfma_select<KK, QM>(D, c0 + kMfmaTile * tau + m < t1, best);
        }
        __syncthreads();  // a persistent block reuses the buffers
    }
    uint32_t glob[QM / 2][KK];
    mfma_merge<KK, QM>(best, m, glob);

    // slot j = QM / 2 m + i of lane (g, m) is query row 8 (v / 4) + 4 g + v % 4
    // of tile qm, j = 16 qm + v
#pragma unroll
    for (int i = 0; i < QM / 2; ++i) {
        const int j = QM / 2 * m + i;
        const int qi = (qt0 + (j >> 4)) * 32 + 8 * ((j >> 2) & 3) + 4 * g + (j & 3);
        if (qi >= n_q) continue;
#pragma unroll
        for (int s = 0; s < KK; ++s) {
            const uint32_t key = glob[i][s];
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
__global__ __launch_bounds__(256, kMfmaMinBlocks) void hamming_mfma_kernel(const uint64_t* __restrict__ query, int32_t n_q,
                                                              const uint64_t* __restrict__ train, int32_t n_t,
                                                              int32_t rows_per_split, uint32_t* __restrict__ partial,
                                                              int32_t* __restrict__ out_idx,
                                                              uint32_t* __restrict__ out_dist, int direct)
{
    __shared__ MfmaShared<NW> sh;
    mfma_tables<NW>(sh);
    mfma_block_body<NW, KK, kMfmaQM>(query, n_q, train, n_t, rows_per_split, blockIdx.x, blockIdx.y, partial, out_idx, out_dist,
                            direct != 0, sh);
}

// Batch: units are (problem, split, block of kMfmaQueries queries), problem-major and
// query block fastest, so consecutive units share a train split.
template <int NW, int KK>
__global__ __launch_bounds__(256, kMfmaMinBlocks) void hamming_mfma_batch(const BatchMatch* __restrict__ mt, int32_t n_m,
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
        mfma_block_body<NW, KK, kMfmaQM>(codes + (int64_t)b.q_off * NW, b.n_q, codes + (int64_t)b.t_off * NW, b.n_t,
                                rows_per_split, qb, split, partial + b.part_off, out_idx + (int64_t)b.out_off * KK,
                                out_dist + (int64_t)b.out_off * KK, b.splits == 1, sh);
    }
}

template <int NW, int KK>
void launch_mfma_nw_k(const KnnPlan& p, const uint64_t* query, const uint64_t* train, uint32_t* partial, int32_t* idx,
                      uint32_t* dist, hipStream_t stream)
{
    const int direct = p.splits == 1;
    const int per_block = kMfmaQueries;
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
    return qpl == 0 ? kMfmaQueries : kWave * qpl;
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
        // MFMA engine: blocks of kMfmaQueries queries; as many splits as
        // fill one round of one block per CU (a small problem then leaves
        // room for a concurrent one on another stream), or of two blocks per
        // CU when splits would exceed 1024 rows; splits of at least one
        // 64-row chunk and at most kMfmaMaxRows rows
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
        // splits start on 16-row tiles and hold at most 128 tiles (the key's tag)
        int64_t rows = ((n_t + splits - 1) / splits + 15) / 16 * 16;
        if (rows > kMfmaMaxRows) rows = kMfmaMaxRows;
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
