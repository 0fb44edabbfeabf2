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
                                               uint64_t* __restrict__ codes, int lb, KpFrame* frames, int* index)
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
                                                           uint64_t* __restrict__ codes)
{
    __shared__ KpFrame frames[kKpPerBlock];
    __shared__ int index[kKpPerBlock];
    const int nb = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    const int lb = xcd_logical_block(blockIdx.x, nb);
    if (lb >= nb) return;
    bad_block_body(ii, W, H, ii_pitch, kps, n_kp, order, pairs, n_words, codes, lb, frames, index);
}

// Batch: units are blocks of four keypoints of every image in turn (pre is
// the prefix of ceil(n_kp / 4) over images); order entries are image-local.
__global__ __launch_bounds__(256) void bad_describe_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                          const int32_t* __restrict__ pre,
                                                          const bd_keypoint* __restrict__ kps,
                                                          const int32_t* __restrict__ order,
                                                          const bd_box_pair* __restrict__ pairs, int32_t n_words,
                                                          uint64_t* __restrict__ codes)
{
    __shared__ KpFrame frames[kKpPerBlock];
    __shared__ int index[kKpPerBlock];
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[i];
        bad_block_body(im.ii, im.W, im.H, im.ii_pitch, kps + im.kp_offset, im.n_kp, order + im.kp_offset, pairs,
                       n_words, codes + (int64_t)im.kp_offset * n_words, u - pre[i], frames, index);
    }
}

}  // namespace

void launch_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                int32_t n_kp, const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes,
                hipStream_t stream)
{
    const int blocks = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    hipLaunchKernelGGL(bad_describe_kernel, dim3(xcd_grid(blocks)), dim3(kKpPerBlock * kWave), 0, stream, ii, W, H,
                       ii_pitch, kps, n_kp, order, pairs, n_words, codes);
}

void launch_bad_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                      const int32_t* order, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes, int grid,
                      hipStream_t stream)
{
    hipLaunchKernelGGL(bad_describe_batch, dim3(grid), dim3(kKpPerBlock * kWave), 0, stream, imgs, n_img, pre, kps,
                       order, pairs, n_words, codes);
}

}  // namespace bd
