// BAD codes (Sec. III-A): bit j of a keypoint is the decision stump
// [f(x; u1_j, u2_j, s_j) <= theta_j] on the difference of two box means,
// each box sum taken from four integral-image corners.
//
// One wavefront per keypoint; lane l evaluates pair 64*w + l for word w and
// the 64 comparison results are packed by a single ballot.  The keypoint's
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

__global__ __launch_bounds__(256) void bad_describe_kernel(const uint32_t* __restrict__ ii, int32_t W,
                                                           int32_t H, int64_t ii_pitch,
                                                           const bd_keypoint* __restrict__ kps,
                                                           int32_t n_kp,
                                                           const bd_box_pair* __restrict__ pairs,
                                                           int32_t n_words, uint64_t* __restrict__ codes)
{
#pragma clang fp contract(off)
    __shared__ KpFrame frames[kKpPerBlock];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int kp_base = blockIdx.x * kKpPerBlock;

    if (threadIdx.x < kKpPerBlock) {
        const int i = kp_base + threadIdx.x;
        KpFrame f{};
        if (i < n_kp) {
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

    const int i = kp_base + wave;
    if (i >= n_kp) return;
    const KpFrame f = frames[wave];
    uint64_t* out = codes + (int64_t)i * n_words;
    if (!f.valid) {
        if (lane < n_words) out[lane] = 0ull;
        return;
    }
    const int r_cap = ((W < H ? W : H) - 1) / 2;
    const uint32_t pitch = (uint32_t)ii_pitch;
    uint64_t my_word = 0ull;
    for (int w = 0; w < n_words; ++w) {
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
        const uint32_t s1 = ii[b1 + c1x + R + 1] - ii[t1 + c1x + R + 1] - ii[b1 + c1x - R] + ii[t1 + c1x - R];
        const uint32_t s2 = ii[b2 + c2x + R + 1] - ii[t2 + c2x + R + 1] - ii[b2 + c2x - R] + ii[t2 + c2x - R];
        const int side = 2 * R + 1;
        const double lhs = (double)((int64_t)s1 - (int64_t)s2);
        const bool bit = lhs <= (double)pr.threshold * (double)(side * side);
        const uint64_t word = __ballot(bit);
        if (lane == w) my_word = word;
    }
    if (lane < n_words) out[lane] = my_word;
}

}  // namespace

void launch_bad(const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch, const bd_keypoint* kps,
                int32_t n_kp, const bd_box_pair* pairs, int32_t n_words, uint64_t* codes,
                hipStream_t stream)
{
    const int blocks = (n_kp + kKpPerBlock - 1) / kKpPerBlock;
    hipLaunchKernelGGL(bad_describe_kernel, dim3(blocks), dim3(kKpPerBlock * kWave), 0, stream, ii, W, H,
                       ii_pitch, kps, n_kp, pairs, n_words, codes);
}

}  // namespace bd
