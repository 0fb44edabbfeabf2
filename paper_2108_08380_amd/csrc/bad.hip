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
// A compiled table lists the distinct boxes of the pairs (in Morton order of
// their centre offsets), each pair referring to its two boxes by index, and
// for each of kAngleBins angle bins the order in which the corners of all
// boxes are gathered: sorted by image position, so that the lanes of one
// load and the next loads of a block fall on few cache lines (fewer L1-to-L2
// requests than gathering box by box).  Layout (device bytes):
//   int32 n_boxes, int32 n_bits, int32 pad[2]
//   uint32 box[2 n_bits]    (ux & 255) | (uy & 255) << 8 | r << 16
//   uint32 pair[n_bits]     b1 | b2 << 10 | r << 20
//   float  theta[n_bits]
//   uint16 corner[kAngleBins][8 n_bits]
// corner[a] lists the corners 4 b + q of the n_boxes distinct boxes (q: 0
// bottom-right, 1 top-right, 2 bottom-left, 3 top-left) sorted by image row,
// then column, for a keypoint at angle (a + 1/2) 2 pi / kAngleBins and scale
// 4: the order in which bad_sorted_kernel gathers them for keypoints whose
// angle falls in bin a.  Rotation and scaling about the keypoint keep that
// order nearly sorted for the whole bin and every scale.

constexpr int kMaxBoxes = 1024;
constexpr int kAngleBins = 32;
constexpr double kSortScale = 4.0;

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

// Corner orders of a compiled table, one block per angle bin: the 4 n_boxes
// corners at the bin's central angle and scale kSortScale (keypoint at the
// origin, no clamping), keyed by (row, column, corner), bitonic sort in LDS.
__global__ __launch_bounds__(1024) void bad_sort_corners_kernel(int32_t K, uint8_t* __restrict__ table)
{
#pragma clang fp contract(off)
    __shared__ uint64_t key[4 * kMaxBoxes];
    const int32_t nb_raw = *reinterpret_cast<const int32_t*>(table);
    const int n_boxes = nb_raw < 1 ? 1 : (nb_raw > 2 * K ? 2 * K : nb_raw);
    const uint32_t* box = reinterpret_cast<const uint32_t*>(table + 16);
    uint16_t* corner = reinterpret_cast<uint16_t*>(table + 16 + 16 * (size_t)K) + (size_t)blockIdx.x * 8 * K;
    const int n = 4 * n_boxes;
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    double sn, cs;
    sincos(((double)blockIdx.x + 0.5) * (2.0 * 3.141592653589793) / kAngleBins, &sn, &cs);
    for (int t = threadIdx.x; t < n2; t += blockDim.x) {
        uint64_t k = ~0ull;
        if (t < n) {
            const uint32_t code = box[t >> 2];
            const int q = t & 3;
            const double ux = (double)(int8_t)(code & 0xffu), uy = (double)(int8_t)((code >> 8) & 0xffu);
            const int R = (int)floor((double)(code >> 16) * kSortScale + 0.5);
            const int cx = (int)floor(kSortScale * (cs * ux - sn * uy) + 0.5);
            const int cy = (int)floor(kSortScale * (sn * ux + cs * uy) + 0.5);
            const int row = (q & 1) ? cy - R : cy + R + 1, col = (q & 2) ? cx - R : cx + R + 1;
            k = ((uint64_t)(uint32_t)(row + 32768) << 48) | ((uint64_t)(uint32_t)(col + 32768) << 32) | (uint64_t)t;
        }
        key[t] = k;
    }
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < n2; t += blockDim.x) {
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
    for (int t = threadIdx.x; t < n; t += blockDim.x) corner[t] = (uint16_t)(key[t] & 0xffffu);
}

// One block of four wavefronts per keypoint (position `pos` of the optional
// order): the geometry of every distinct box into LDS (lane = box), then the
// corner gathers in the order of the keypoint's angle bin, so that the 64
// lanes of a load and the next loads of the block fall on few cache lines,
// each value stored by corner; then the box sums and, one 64-bit word per
// wavefront at a time, the comparisons and a ballot.  Same arithmetic as
// bad_block_body, so the codes are bd_describe_bad's.
template <int NW>
__device__ __forceinline__ void bad_sorted_body(const uint32_t* __restrict__ ii, int32_t W, int32_t H,
                                                int64_t ii_pitch, const bd_keypoint* __restrict__ kps,
                                                int32_t n_kp, const int32_t* __restrict__ order,
                                                const uint8_t* __restrict__ table, uint64_t* __restrict__ codes,
                                                int pos, uint4* geo, uint32_t* val, KpFrame* frame, int* bin_index,
                                                unsigned long long* __restrict__ invalid)
{
#pragma clang fp contract(off)
    constexpr int n_bits = 64 * NW;
    constexpr int kThreads = kKpPerBlock * kWave;
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    if (t == 0) {
        int i = pos < n_kp ? (order ? order[pos] : pos) : -1;
        if (i >= n_kp) i = -1;
        KpFrame f{};
        int bin = 0;
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
                double a = fmod((double)k.angle, 2.0 * 3.141592653589793);
                if (a < 0.0) a += 2.0 * 3.141592653589793;
                bin = (int)(a * (kAngleBins / (2.0 * 3.141592653589793)));
                bin = bin < 0 ? 0 : (bin >= kAngleBins ? kAngleBins - 1 : bin);
            }
        }
        *frame = f;
        bin_index[0] = bin;
        bin_index[1] = i;
    }
    __syncthreads();
    const int i = bin_index[1];
    if (i < 0) return;  // uniform per block
    const KpFrame f = *frame;
    uint64_t* out = codes + (int64_t)i * NW;
    if (!f.valid) {
        if (t < NW) out[t] = 0ull;
        if (invalid && t == 0) atomicAdd(invalid, 1ull);
        return;
    }
    const int32_t nb_raw = *reinterpret_cast<const int32_t*>(table);
    const int n_boxes = nb_raw < 1 ? 1 : (nb_raw > 2 * n_bits ? 2 * n_bits : nb_raw);
    const uint32_t* box = reinterpret_cast<const uint32_t*>(table + 16);
    const uint32_t* pair = box + 2 * n_bits;
    const float* theta = reinterpret_cast<const float*>(pair + n_bits);
    const uint16_t* corner = reinterpret_cast<const uint16_t*>(theta + n_bits) + (size_t)bin_index[0] * 8 * n_bits;
    const int r_cap = ((W < H ? W : H) - 1) / 2;
    const uint32_t pitch = (uint32_t)ii_pitch;

    // 1. box geometry: row offsets of the top and bottom corners, left and right columns
    for (int b = t; b < n_boxes; b += kThreads) {
        const uint32_t code = box[b];
        const double ux = (double)(int8_t)(code & 0xffu), uy = (double)(int8_t)((code >> 8) & 0xffu);
        const double rr = floor((double)(code >> 16) * f.scale + 0.5);
        const int R = rr > (double)r_cap ? r_cap : (int)rr;
        const double px = f.x + (f.sa * ux - f.sb * uy);
        const double py = f.y + (f.sb * ux + f.sa * uy);
        const int cx = box_centre(px, R, W), cy = box_centre(py, R, H);
        geo[b] = make_uint4((uint32_t)(cy - R) * pitch, (uint32_t)(cy + R + 1) * pitch, (uint32_t)(cx - R),
                            (uint32_t)(cx + R + 1));
    }
    __syncthreads();

    // 2. corner gathers in the bin's order, all of a thread's in flight
    constexpr int kPer = 8 * n_bits / kThreads;
    const int n_corners = 4 * n_boxes;
    uint32_t cid[kPer], v[kPer];
#pragma unroll
    for (int g = 0; g < kPer; ++g) {
        const int p = t + g * kThreads;
        cid[g] = p < n_corners ? (uint32_t)corner[p] : 0u;
    }
#pragma unroll
    for (int g = 0; g < kPer; ++g) {
        const uint4 gb = geo[cid[g] >> 2];
        const uint32_t off = ((cid[g] & 1u) ? gb.x : gb.y) + ((cid[g] & 2u) ? gb.z : gb.w);
        v[g] = t + g * kThreads < n_corners ? ii[off] : 0u;
    }
#pragma unroll
    for (int g = 0; g < kPer; ++g)
        if (t + g * kThreads < n_corners) val[cid[g]] = v[g];
    __syncthreads();

    // 3. box sums S = v(bottom-right) - v(top-right) - v(bottom-left) + v(top-left)
    uint32_t* S = reinterpret_cast<uint32_t*>(geo);
    for (int b = t; b < n_boxes; b += kThreads) {
        const uint4 cv = reinterpret_cast<const uint4*>(val)[b];
        S[4 * b] = cv.x - cv.y - cv.z + cv.w;
    }
    __syncthreads();

    // 4. comparisons, one ballot per word
    for (int w = wave; w < NW; w += kKpPerBlock) {
        const int j = w * kWave + lane;
        const uint32_t pc = pair[j];
        const uint32_t b1 = (pc & 0x3ffu) < (uint32_t)n_boxes ? (pc & 0x3ffu) : 0u;
        const uint32_t b2 = ((pc >> 10) & 0x3ffu) < (uint32_t)n_boxes ? ((pc >> 10) & 0x3ffu) : 0u;
        const double rr = floor((double)(pc >> 20) * f.scale + 0.5);
        const int R = rr > (double)r_cap ? r_cap : (int)rr;
        const int side = 2 * R + 1;
        const double limit = (double)theta[j] * (double)(side * side);
        const double lhs = (double)((int64_t)S[4 * b1] - (int64_t)S[4 * b2]);
        const uint64_t word = __ballot(lhs <= limit);
        if (lane == 0) out[w] = word;
    }
}

template <int NW>
__global__ __launch_bounds__(kKpPerBlock * kWave) void bad_sorted_kernel(
    const uint32_t* __restrict__ ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* __restrict__ kps,
    int32_t n_kp, const int32_t* __restrict__ order, const uint8_t* __restrict__ table,
    uint64_t* __restrict__ codes, unsigned long long* __restrict__ invalid)
{
    __shared__ uint4 geo[2 * 64 * NW];
    __shared__ __align__(16) uint32_t val[8 * 64 * NW];
    __shared__ KpFrame frame;
    __shared__ int bin_index[2];
    bad_sorted_body<NW>(ii, W, H, ii_pitch, kps, n_kp, order, table, codes, xcd_logical_block(blockIdx.x, n_kp),
                        geo, val, &frame, bin_index, invalid);
}

// Batch: units are blocks of four keypoints of every image in turn (pre is
// the prefix of ceil(n_kp / 4)); the block describes the unit's keypoints
// one after the other.
template <int NW>
__global__ __launch_bounds__(kKpPerBlock * kWave) void bad_sorted_batch(
    const BatchImage* __restrict__ imgs, int32_t n_img, const int32_t* __restrict__ pre,
    const bd_keypoint* __restrict__ kps, const int32_t* __restrict__ order, const uint8_t* __restrict__ table,
    uint64_t* __restrict__ codes, unsigned long long* __restrict__ invalid)
{
    __shared__ uint4 geo[2 * 64 * NW];
    __shared__ __align__(16) uint32_t val[8 * 64 * NW];
    __shared__ KpFrame frame;
    __shared__ int bin_index[2];
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        for (int k = 0; k < kKpPerBlock; ++k)
            bad_sorted_body<NW>(im.ii, im.W, im.H, im.ii_pitch, kps + im.kp_offset, im.n_kp, order + im.kp_offset,
                                table, codes + (int64_t)im.kp_offset * NW, (u - pre[i]) * kKpPerBlock + k, geo, val,
                                &frame, bin_index, invalid);
    }
}

}  // namespace

size_t bad_table_bytes(int32_t n_bits)
{
    return 16 + 16 * (size_t)n_bits + sizeof(uint16_t) * (size_t)kAngleBins * 8 * (size_t)n_bits;
}

void launch_bad_compile(const bd_box_pair* pairs, int32_t n_bits, uint8_t* table, hipStream_t stream)
{
    hipLaunchKernelGGL(bad_compile_kernel, dim3(1), dim3(1024), 0, stream, pairs, n_bits, table);
    hipLaunchKernelGGL(bad_sort_corners_kernel, dim3(kAngleBins), dim3(1024), 0, stream, n_bits, table);
}

void launch_bad_compiled(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                         int32_t n_kp, const int32_t* order, const uint8_t* table, int32_t n_words, uint64_t* codes,
                         unsigned long long* invalid, hipStream_t stream)
{
    if (n_words == 8)
        hipLaunchKernelGGL(bad_sorted_kernel<8>, dim3(xcd_grid(n_kp)), dim3(kKpPerBlock * kWave), 0, stream, ii, W, H,
                           ii_pitch, kps, n_kp, order, table, codes, invalid);
    else
        hipLaunchKernelGGL(bad_sorted_kernel<4>, dim3(xcd_grid(n_kp)), dim3(kKpPerBlock * kWave), 0, stream, ii, W, H,
                           ii_pitch, kps, n_kp, order, table, codes, invalid);
}

void launch_bad_compiled_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                               const int32_t* order, const uint8_t* table, int32_t n_words, uint64_t* codes, int grid,
                               unsigned long long* invalid, hipStream_t stream)
{
    if (n_words == 8)
        hipLaunchKernelGGL(bad_sorted_batch<8>, dim3(grid), dim3(kKpPerBlock * kWave), 0, stream, imgs, n_img, pre,
                           kps, order, table, codes, invalid);
    else
        hipLaunchKernelGGL(bad_sorted_batch<4>, dim3(grid), dim3(kKpPerBlock * kWave), 0, stream, imgs, n_img, pre,
                           kps, order, table, codes, invalid);
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
