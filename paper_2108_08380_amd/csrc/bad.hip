// BAD codes (Sec. III-A): bit j of a keypoint is the decision stump
// [f(x; u1_j, u2_j, s_j) <= theta_j] on the difference of two box means,
// each box sum taken from four integral-image corners.
//
// One wavefront per keypoint; lane l evaluates pair 64*w + l for word w and
// the 64 comparison results are packed by a single ballot.  Keypoints are
// taken in the caller's spatial order (optional) with an XCD-aware block
// mapping, so the corner gathers of an XCD stay within one image region.  The keypoint's
// rotation (scale*cos, scale*sin, FP64) is computed once per block by one
// lane per keypoint and shared through LDS.  Box centres are computed in
// FP64 with contraction disabled, in the same operation order as the
// definition (p = c + (a ux - b uy), then floor(p + 0.5)), so the rounding
// to pixels is reproducible; the comparison S1 - S2 <= theta * A is exact.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kKpPerBlock = 4;  // one wavefront each

struct KpFrame {
    double x, y, sa, sb, scale;
    int valid;
};

__device__ __forceinline__ bool finite_f(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }

__device__ __forceinline__ int box_centre(double p, int R, int n)
{
    double c = floor(p + 0.5);
    c = fmax(c, (double)R);
    c = fmin(c, (double)(n - 1 - R));
    return (int)c;
}

// One block of four wavefronts: the keypoints at positions 4*lb .. 4*lb+3 of
// the (optional) order, one per wavefront.  frames/index are block-shared.
__device__ __forceinline__ void bad_block_body(const uint32_t* __restrict__ ii, int32_t W, int32_t H,
                                               int64_t ii_pitch, const bd_keypoint* __restrict__ kps, int32_t n_kp,
                                               const int32_t* __restrict__ order,
                                               const bd_box_pair* __restrict__ pairs, int32_t n_words,
                                               uint64_t* __restrict__ codes, int lb, KpFrame* frames, int* index,
                                               unsigned long long* __restrict__ invalid)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x < kKpPerBlock) {
        const int pos = lb * kKpPerBlock + threadIdx.x;
        int i = pos < n_kp ? (order ? order[pos] : pos) : -1;
        if (i >= n_kp) i = -1;  // malformed order entries are skipped
        index[threadIdx.x] = i;
        KpFrame f{};
        if (i >= 0) {
            const bd_keypoint k = kps[i];
            f.valid = finite_f(k.x) && finite_f(k.y) && finite_f(k.scale) && finite_f(k.angle) && k.scale > 0.0f;
            if (f.valid) {
                double sn, cs;
                sincos((double)k.angle, &sn, &cs);
                f.x = k.x;
                f.y = k.y;
                f.scale = k.scale;
                f.sa = (double)k.scale * cs;
                f.sb = (double)k.scale * sn;
            }
        }
        frames[threadIdx.x] = f;
    }
    __syncthreads();

    const int i = index[wave];
    if (i >= 0) {
        const KpFrame f = frames[wave];
        uint64_t* out = codes + (int64_t)i * n_words;
        if (!f.valid) {
            if (lane < n_words) out[lane] = 0ull;
            if (invalid && lane == 0) atomicAdd(invalid, 1ull);
        } else {
            const int r_cap = ((W < H ? W : H) - 1) / 2;
            const uint32_t pitch = (uint32_t)ii_pitch;
            uint64_t my_word = 0ull;
            // Words are processed in groups of four: the 32 corner gathers of a
            // group are all issued before the first comparison waits on them.
            constexpr int kGroup = 4;
            for (int w0 = 0; w0 < n_words; w0 += kGroup) {
                uint32_t off[kGroup][8];
                double limit[kGroup];
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    const int w = w0 + g < n_words ? w0 + g : n_words - 1;
                    const bd_box_pair pr = pairs[w * kWave + lane];
                    const double rr = floor((double)pr.radius * f.scale + 0.5);
                    const int R = rr > (double)r_cap ? r_cap : (int)rr;
                    const double ux1 = pr.x1, uy1 = pr.y1, ux2 = pr.x2, uy2 = pr.y2;
                    const double p1x = f.x + (f.sa * ux1 - f.sb * uy1);
                    const double p1y = f.y + (f.sb * ux1 + f.sa * uy1);
                    const double p2x = f.x + (f.sa * ux2 - f.sb * uy2);
                    const double p2y = f.y + (f.sb * ux2 + f.sa * uy2);
                    const int c1x = box_centre(p1x, R, W), c1y = box_centre(p1y, R, H);
                    const int c2x = box_centre(p2x, R, W), c2y = box_centre(p2y, R, H);
                    // four corners per box: rows cy-R and cy+R+1, columns cx-R and cx+R+1
                    const uint32_t t1 = (uint32_t)(c1y - R) * pitch, b1 = (uint32_t)(c1y + R + 1) * pitch;
                    const uint32_t t2 = (uint32_t)(c2y - R) * pitch, b2 = (uint32_t)(c2y + R + 1) * pitch;
                    off[g][0] = b1 + c1x + R + 1;
                    off[g][1] = t1 + c1x + R + 1;
                    off[g][2] = b1 + c1x - R;
                    off[g][3] = t1 + c1x - R;
                    off[g][4] = b2 + c2x + R + 1;
                    off[g][5] = t2 + c2x + R + 1;
                    off[g][6] = b2 + c2x - R;
                    off[g][7] = t2 + c2x - R;
                    const int side = 2 * R + 1;
                    limit[g] = (double)pr.threshold * (double)(side * side);
                }
                uint32_t v[kGroup][8];
#pragma unroll
                for (int g = 0; g < kGroup; ++g)
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[g][k] = ii[off[g][k]];
#pragma unroll
                for (int g = 0; g < kGroup; ++g) {
                    if (w0 + g >= n_words) break;
                    const uint32_t s1 = v[g][0] - v[g][1] - v[g][2] + v[g][3];
                    const uint32_t s2 = v[g][4] - v[g][5] - v[g][6] + v[g][7];
                    const double lhs = (double)((int64_t)s1 - (int64_t)s2);
                    const uint64_t word = __ballot(lhs <= limit[g]);
                    if (lane == w0 + g) my_word = word;
                }
            }
            if (lane < n_words) out[lane] = my_word;
        }
    }
    __syncthreads();  // frames and index are reused by the next unit of a persistent block
}

__global__ __launch_bounds__(256) void bad_describe_kernel(const uint32_t* __restrict__ ii, int32_t W, int32_t H,
                                                           int64_t ii_pitch, const bd_keypoint* __restrict__ kps,
                                                           int32_t n_kp, const int32_t* __restrict__ order,
                                                           const bd_box_pair* __restrict__ pairs, int32_t n_words,
                                                           uint64_t* __restrict__ codes,
                                                           unsigned long long* __restrict__ invalid)
{
    __shared__ KpFrame frames[kKpPerBlock];
    __shared__ int index[kKpPerBlock];
    const int nb = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    const int lb = xcd_logical_block(blockIdx.x, nb);
    if (lb >= nb) return;
    bad_block_body(ii, W, H, ii_pitch, kps, n_kp, order, pairs, n_words, codes, lb, frames, index, invalid);
}

// Batch: units are blocks of four keypoints of every image in turn (pre is
// the prefix of ceil(n_kp / 4) over images); order entries are image-local.
__global__ __launch_bounds__(256) void bad_describe_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                          const int32_t* __restrict__ pre,
                                                          const bd_keypoint* __restrict__ kps,
                                                          const int32_t* __restrict__ order,
                                                          const bd_box_pair* __restrict__ pairs, int32_t n_words,
                                                          uint64_t* __restrict__ codes,
                                                          unsigned long long* __restrict__ invalid)
{
    __shared__ KpFrame frames[kKpPerBlock];
    __shared__ int index[kKpPerBlock];
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        bad_block_body(im.ii, im.W, im.H, im.ii_pitch, kps + im.kp_offset, im.n_kp, order + im.kp_offset, pairs,
                       n_words, codes + (int64_t)im.kp_offset * n_words, u - pre[i], frames, index, invalid);
    }
}

// ---------------------------------------------------------------- compiled tables
//
// A compiled table lists the distinct boxes of the pairs in Morton order of
// their centre offsets, so that the 64 boxes a wavefront sums with one load
// instruction lie close together in the patch and hence in the image: fewer
// cache lines per instruction and more L1 reuse between instructions.  Each
// pair refers to its two boxes by index.  Layout (device bytes):
//   int32 n_boxes, int32 n_bits, int32 pad[2]
//   uint32 box[2 n_bits]    (ux & 255) | (uy & 255) << 8 | r << 16
//   uint32 pair[n_bits]     b1 | b2 << 10 | r << 20
//   float  theta[n_bits]

constexpr int kMaxBoxes = 1024;

__device__ __forceinline__ uint32_t spread8(uint32_t v)  // 8 bits -> even positions of 16
{
    v &= 0xffu;
    v = (v | (v << 4)) & 0x0f0fu;
    v = (v | (v << 2)) & 0x3333u;
    v = (v | (v << 1)) & 0x5555u;
    return v;
}

__global__ __launch_bounds__(1024) void bad_compile_kernel(const bd_box_pair* __restrict__ pairs, int32_t K,
                                                           uint8_t* __restrict__ table)
{
    __shared__ uint64_t key[kMaxBoxes];
    __shared__ uint32_t uid[kMaxBoxes];
    const int t = threadIdx.x;
    const int n = 2 * K;
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    // key: Morton code of the centre offset, radius, then slot (2 j + side)
    if (t < n2) {
        uint64_t k = ~0ull;
        if (t < n) {
            const bd_box_pair& p = pairs[t >> 1];
            const int ux = (t & 1) ? p.x2 : p.x1, uy = (t & 1) ? p.y2 : p.y1;
            const uint32_t m = spread8((uint32_t)(ux + 128)) | (spread8((uint32_t)(uy + 128)) << 1);
            k = ((uint64_t)m << 32) | ((uint64_t)p.radius << 24) | (uint64_t)t;
        }
        key[t] = k;
    }
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (t < n2) {
                const int o = t ^ stride;
                if (o > t) {
                    const bool up = (t & size) == 0;
                    const uint64_t a = key[t], b = key[o];
                    if ((a > b) == up) {
                        key[t] = b;
                        key[o] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // distinct boxes: a new box starts where (offset, radius) changes
    const bool first = t < n && (t == 0 || (key[t] >> 24) != (key[t - 1] >> 24));
    uid[t] = first ? 1u : 0u;
    __syncthreads();
    for (int d = 1; d < kMaxBoxes; d <<= 1) {
        const uint32_t v = t >= d ? uid[t - d] : 0u;
        __syncthreads();
        uid[t] += v;
        __syncthreads();
    }
    int32_t* head = reinterpret_cast<int32_t*>(table);
    uint32_t* box = reinterpret_cast<uint32_t*>(table + 16);
    uint32_t* pair = box + n;
    float* theta = reinterpret_cast<float*>(pair + K);
    const uint32_t my_uid = uid[t] - 1u;  // index of the distinct box of sorted position t
    __syncthreads();
    // reuse key[] as slot -> distinct box index
    uint32_t slot = 0;
    if (t < n) {
        slot = (uint32_t)(key[t] & 0xffffffu);
        if (first) {
            const bd_box_pair& p = pairs[slot >> 1];
            const int ux = (slot & 1) ? p.x2 : p.x1, uy = (slot & 1) ? p.y2 : p.y1;
            box[my_uid] = ((uint32_t)ux & 0xffu) | (((uint32_t)uy & 0xffu) << 8) | ((uint32_t)p.radius << 16);
        }
    }
    __syncthreads();
    if (t < n) key[slot] = my_uid;
    if (t == 0) {
        head[0] = (int32_t)uid[n - 1];
        head[1] = K;
        head[2] = 0;
        head[3] = 0;
    }
    __syncthreads();
    if (t < K) {
        pair[t] = (uint32_t)key[2 * t] | ((uint32_t)key[2 * t + 1] << 10) | ((uint32_t)pairs[t].radius << 20);
        theta[t] = pairs[t].threshold;
    }
}

// One block of four wavefronts, one keypoint each: first the sums of all
// distinct boxes in table order (lane = box, 16 corner gathers in flight per
// lane) into the wavefront's LDS row, then per 64-bit word the pairs'
// comparisons from LDS and one ballot.  Same arithmetic as bad_block_body.
__device__ __forceinline__ void bad_compiled_body(const uint32_t* __restrict__ ii, int32_t W, int32_t H,
                                                  int64_t ii_pitch, const bd_keypoint* __restrict__ kps,
                                                  int32_t n_kp, const int32_t* __restrict__ order,
                                                  const uint8_t* __restrict__ table, int32_t n_words,
                                                  uint64_t* __restrict__ codes, int lb, KpFrame* frames,
                                                  int* index, uint32_t (*sums)[kMaxBoxes],
                                                  unsigned long long* __restrict__ invalid)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x < kKpPerBlock) {
        const int pos = lb * kKpPerBlock + threadIdx.x;
        int i = pos < n_kp ? (order ? order[pos] : pos) : -1;
        if (i >= n_kp) i = -1;
        index[threadIdx.x] = i;
        KpFrame f{};
        if (i >= 0) {
            const bd_keypoint k = kps[i];
            f.valid = finite_f(k.x) && finite_f(k.y) && finite_f(k.scale) && finite_f(k.angle) && k.scale > 0.0f;
            if (f.valid) {
                double sn, cs;
                sincos((double)k.angle, &sn, &cs);
                f.x = k.x;
                f.y = k.y;
                f.scale = k.scale;
                f.sa = (double)k.scale * cs;
                f.sb = (double)k.scale * sn;
            }
        }
        frames[threadIdx.x] = f;
    }
    __syncthreads();

    const int i = index[wave];
    if (i >= 0) {
        const KpFrame f = frames[wave];
        uint64_t* out = codes + (int64_t)i * n_words;
        if (!f.valid) {
            if (lane < n_words) out[lane] = 0ull;
            if (invalid && lane == 0) atomicAdd(invalid, 1ull);
        } else {
            const int n_bits = n_words * 64;
            const int32_t nb_raw = *reinterpret_cast<const int32_t*>(table);
            const int n_boxes = nb_raw < 1 ? 1 : (nb_raw > 2 * n_bits ? 2 * n_bits : nb_raw);
            const uint32_t* box = reinterpret_cast<const uint32_t*>(table + 16);
            const uint32_t* pair = box + 2 * n_bits;
            const float* theta = reinterpret_cast<const float*>(pair + n_bits);
            const int r_cap = ((W < H ? W : H) - 1) / 2;
            const uint32_t pitch = (uint32_t)ii_pitch;
            uint32_t* S = sums[wave];
            // 1. box sums, four chunks of 64 boxes per batch of gathers
            constexpr int kChunks = 4;
            for (int c0 = 0; c0 < n_boxes; c0 += kChunks * kWave) {
                uint32_t off[kChunks][4];
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    int b = c0 + c * kWave + lane;
                    b = b < n_boxes ? b : n_boxes - 1;
                    const uint32_t code = box[b];
                    const double ux = (double)(int8_t)(code & 0xffu), uy = (double)(int8_t)((code >> 8) & 0xffu);
                    const double rr = floor((double)(code >> 16) * f.scale + 0.5);
                    const int R = rr > (double)r_cap ? r_cap : (int)rr;
                    const double px = f.x + (f.sa * ux - f.sb * uy);
                    const double py = f.y + (f.sb * ux + f.sa * uy);
                    const int cx = box_centre(px, R, W), cy = box_centre(py, R, H);
                    const uint32_t top = (uint32_t)(cy - R) * pitch, bot = (uint32_t)(cy + R + 1) * pitch;
                    off[c][0] = bot + cx + R + 1;
                    off[c][1] = top + cx + R + 1;
                    off[c][2] = bot + cx - R;
                    off[c][3] = top + cx - R;
                }
                uint32_t v[kChunks][4];
#pragma unroll
                for (int c = 0; c < kChunks; ++c)
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[c][q] = ii[off[c][q]];
#pragma unroll
                for (int c = 0; c < kChunks; ++c) {
                    const int b = c0 + c * kWave + lane;
                    if (b < n_boxes) S[b] = v[c][0] - v[c][1] - v[c][2] + v[c][3];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            // 2. comparisons, one ballot per word
            uint64_t my_word = 0ull;
            for (int w = 0; w < n_words; ++w) {
                const int j = w * kWave + lane;
                const uint32_t pc = pair[j];
                const uint32_t b1 = (pc & 0x3ffu) < (uint32_t)n_boxes ? (pc & 0x3ffu) : 0u;
                const uint32_t b2 = ((pc >> 10) & 0x3ffu) < (uint32_t)n_boxes ? ((pc >> 10) & 0x3ffu) : 0u;
                const double rr = floor((double)(pc >> 20) * f.scale + 0.5);
                const int R = rr > (double)r_cap ? r_cap : (int)rr;
                const int side = 2 * R + 1;
                const double limit = (double)theta[j] * (double)(side * side);
                const double lhs = (double)((int64_t)S[b1] - (int64_t)S[b2]);
                const uint64_t word = __ballot(lhs <= limit);
                if (lane == w) my_word = word;
            }
            if (lane < n_words) out[lane] = my_word;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void bad_compiled_kernel(const uint32_t* __restrict__ ii, int32_t W, int32_t H,
                                                           int64_t ii_pitch, const bd_keypoint* __restrict__ kps,
                                                           int32_t n_kp, const int32_t* __restrict__ order,
                                                           const uint8_t* __restrict__ table, int32_t n_words,
                                                           uint64_t* __restrict__ codes,
                                                           unsigned long long* __restrict__ invalid)
{
    __shared__ KpFrame frames[kKpPerBlock];
    __shared__ int index[kKpPerBlock];
    __shared__ uint32_t sums[kKpPerBlock][kMaxBoxes];
    const int nb = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    const int lb = xcd_logical_block(blockIdx.x, nb);
    if (lb >= nb) return;
    bad_compiled_body(ii, W, H, ii_pitch, kps, n_kp, order, table, n_words, codes, lb, frames, index, sums, invalid);
}

__global__ __launch_bounds__(256) void bad_compiled_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                          const int32_t* __restrict__ pre,
                                                          const bd_keypoint* __restrict__ kps,
                                                          const int32_t* __restrict__ order,
                                                          const uint8_t* __restrict__ table, int32_t n_words,
                                                          uint64_t* __restrict__ codes,
                                                          unsigned long long* __restrict__ invalid)
{
    __shared__ KpFrame frames[kKpPerBlock];
    __shared__ int index[kKpPerBlock];
    __shared__ uint32_t sums[kKpPerBlock][kMaxBoxes];
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        bad_compiled_body(im.ii, im.W, im.H, im.ii_pitch, kps + im.kp_offset, im.n_kp, order + im.kp_offset, table,
                          n_words, codes + (int64_t)im.kp_offset * n_words, u - pre[i], frames, index, sums,
                          invalid);
    }
}

}  // namespace

size_t bad_table_bytes(int32_t n_bits) { return 16 + 16 * (size_t)n_bits; }

void launch_bad_compile(const bd_box_pair* pairs, int32_t n_bits, uint8_t* table, hipStream_t stream)
{
    hipLaunchKernelGGL(bad_compile_kernel, dim3(1), dim3(1024), 0, stream, pairs, n_bits, table);
}

void launch_bad_compiled(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                         int32_t n_kp, const int32_t* order, const uint8_t* table, int32_t n_words, uint64_t* codes,
                         unsigned long long* invalid, hipStream_t stream)
{
    const int nb = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    hipLaunchKernelGGL(bad_compiled_kernel, dim3(xcd_grid(nb)), dim3(kKpPerBlock * kWave), 0, stream, ii, W, H,
                       ii_pitch, kps, n_kp, order, table, n_words, codes, invalid);
}

void launch_bad_compiled_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                               const int32_t* order, const uint8_t* table, int32_t n_words, uint64_t* codes, int grid,
                               unsigned long long* invalid, hipStream_t stream)
{
    hipLaunchKernelGGL(bad_compiled_batch, dim3(grid), dim3(kKpPerBlock * kWave), 0, stream, imgs, n_img, pre, kps,
                       order, table, n_words, codes, invalid);
}

void launch_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                int32_t n_kp, const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes,
                unsigned long long* invalid, hipStream_t stream)
{
    const int blocks = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    hipLaunchKernelGGL(bad_describe_kernel, dim3(xcd_grid(blocks)), dim3(kKpPerBlock * kWave), 0, stream, ii, W, H,
                       ii_pitch, kps, n_kp, order, pairs, n_words, codes, invalid);
}

void launch_bad_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                      const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes, int grid,
                      unsigned long long* invalid, hipStream_t stream)
{
    hipLaunchKernelGGL(bad_describe_batch, dim3(grid), dim3(kKpPerBlock * kWave), 0, stream, imgs, n_img, pre, kps,
                       order, pairs, n_words, codes, invalid);
}

}  // namespace bd
