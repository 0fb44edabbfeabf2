// HashSIFT (Sec. III-B): SIFT features f of the normalized 32x32 patch,
// then D = sgn(B [f; 1]) with the last column of B written as -t.
//
// hashsift_hist: one wavefront per keypoint, in the caller's spatial order
// (optional) with an XCD-aware block mapping so an XCD's samples stay within
// one image region.
//   1. 34x34 bilinear samples of the rotated, scaled patch (clamp-to-edge,
//      nested linear interpolation so flat regions give exactly zero
//      gradients) go to LDS, stored relative to the pixel under the keypoint
//      so small gradients in near-flat patches keep their relative precision
//      in FP32.  Positions are 32.32 fixed point: the wavefront walks the
//      interior in 8x8 blocks of samples (lane = position in the block), and
//      every lane moves by the same 64-bit step from one block to the next,
//      so a sample costs two 64-bit adds instead of FP64 arithmetic; two more
//      steps take the apron rows and columns (the four apron corners are
//      never read).  Keypoints whose patch may reach beyond 2^30 pixels take
//      the FP64 position path.
//   2. Lane (h, j) owns patch column j and 16 rows (rows 0..15 top-down for
//      h = 0, rows 31..16 bottom-up for h = 1).  With the bottom-up order the
//      vertical cell weights and Gaussian row weights of step k are the same
//      compile-time constants for both halves, so each pixel's vote is 9
//      triangular orientation weights and 8 or 16 FMAs into 3 cell rows x 8
//      orientations held in registers.  No atomics: the order of every sum is
//      fixed, so the result is deterministic.
//   3. The per-lane partial histograms (times the column's Gaussian weight)
//      go to LDS with four zero columns padding each side, and each lane
//      forms two of the 128 bins by a fixed-order sum over the 16 columns of
//      its cell's support with compile-time horizontal weights, no bounds
//      checks needed.
//   4. L2 normalization by a wavefront reduction.
//
// hashsift_project: persistent and B-stationary: a block keeps one 64-bit
// chunk of B (FP32 in LDS for the re-check, the MFMA operand in registers)
// and streams 16-keypoint tiles per wavefront; responses r = B f - t on
// MFMA (FP32, or BF16 / FP8 with FP32 accumulation and an FP32 re-check of
// responses near the threshold); the signs are packed with 16 ballots.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kApron = 34;                 // 32 + one-pixel apron on each side
constexpr int kSamples = kApron * kApron;  // 1156
// Per-lane partial histograms: entry e = slot * 8 + o (24 entries) of lane
// (half, column j) at e * kHistStride + half * 40 + 4 + j; four zero columns
// pad each side of a half so the cell-column sums need no bounds checks.
constexpr int kHistStride = 80;
constexpr int kWaveLds = 24 * kHistStride;  // floats per wavefront
static_assert(kWaveLds >= kSamples, "patch must fit the per-wave LDS slice");
constexpr int kHistWaves = 4;

// exp(x) for |x| < 1 by its power series, evaluated at compile time.
constexpr double cexp(double x)
{
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        term *= x / n;
        sum += term;
    }
    return sum;
}
// Gaussian window with sigma 16 on patch coordinate i (centre 15.5).
constexpr double gauss_w(int i) { return cexp(-((i - 15.5) * (i - 15.5)) / (2.0 * 16.0 * 16.0)); }

struct GaussTable {
    float v[32];
    constexpr GaussTable() : v{}
    {
        for (int i = 0; i < 32; ++i) v[i] = (float)gauss_w(i);
    }
};
__constant__ GaussTable kGauss = GaussTable();

// Vertical cell weight times row Gaussian for step k of a lane, slot 0..2
// (slot = cell row for the top half, 3 - cell row for the bottom half).
// Steps 0..3 vote into slot 0 only, 4..11 into slots 0 and 1, 12..15 into
// slots 1 and 2.
constexpr double row_weight(int k, int slot)
{
    double wy = 0.0;
    if (k < 4) {
        wy = slot == 0 ? (k + 4.5) / 8.0 : 0.0;
    } else if (k < 12) {
        wy = slot == 0 ? (11.5 - k) / 8.0 : (slot == 1 ? (k - 3.5) / 8.0 : 0.0);
    } else {
        wy = slot == 1 ? (19.5 - k) / 8.0 : (slot == 2 ? (k - 11.5) / 8.0 : 0.0);
    }
    return wy * gauss_w(k);
}
__host__ __device__ constexpr bool slot_active(int k, int slot)
{
    return k < 4 ? slot == 0 : (k < 12 ? slot <= 1 : slot >= 1);
}
struct RowTable {
    float v[16][3];
    constexpr RowTable() : v{}
    {
        for (int k = 0; k < 16; ++k)
            for (int s = 0; s < 3; ++s) v[k][s] = (float)row_weight(k, s);
    }
};
__constant__ RowTable kRow = RowTable();

// Horizontal cell weight of column 8 cx - 4 + t for cell column cx:
// max(0, 1 - |(t + 0.5) / 8 - 1|), the same for every cx.
struct ColTable {
    float v[16];
    constexpr ColTable() : v{}
    {
        for (int t = 0; t < 16; ++t) {
            const double d = (t + 0.5) / 8.0 - 1.0;
            const double w = 1.0 - (d < 0 ? -d : d);
            v[t] = (float)(w > 0.0 ? w : 0.0);
        }
    }
};
constexpr ColTable kCol = ColTable();

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bool finite_f(float v) { return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u; }

template <int DT>
__device__ __forceinline__ float pixel(const uint8_t* __restrict__ img, int64_t pitch, int x, int y)
{
    const uint8_t* row = img + (int64_t)y * pitch;
    if constexpr (DT == BD_DTYPE_U8) {
        return (float)row[x];  // grey levels; the 1/255 scale cancels in the L2 normalization
    } else if constexpr (DT == BD_DTYPE_F32_ROWPAIR) {
        return reinterpret_cast<const float*>(row)[2 * x];  // first of the pair: row y
    } else {
        return reinterpret_cast<const float*>(row)[x];
    }
}

// Orientation-bin coordinate of the gradient (gx, gy): atan2(gy, gx) * 8/(2 pi)
// in [0, 8].  Octant reduction to t = min/max in [0, 1], then
// atan(t) * 4/pi = t * P(t^2) with P of degree 7, whose coefficients are a
// weighted least-squares (Lawson-iterated, near-minimax) fit on Chebyshev
// nodes of u = t^2 in [0, 1] rounded to float32 (fit_orientation.py).  P is
// within 1.2e-7 bins of the octant angle, its float32 evaluation within
// 2.4e-7, and the returned coordinate within 5.5e-7 bins of the exact one
// (values near 8 are stored to half an ulp of 8).  A zero gradient gives 0.
__device__ __forceinline__ float orientation_bin(float gx, float gy)
{
    const float ax = fabsf(gx), ay = fabsf(gy);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(fmaxf(mx, 1e-30f));
    const float u = t * t;
    float p = -0.005162429064512253f;
    p = fmaf(p, u, 0.027836760506033897f);
    p = fmaf(p, u, -0.0711897537112236f);
    p = fmaf(p, u, 0.12276824563741684f);
    p = fmaf(p, u, -0.17709016799926758f);
    p = fmaf(p, u, 0.2539675533771515f);
    p = fmaf(p, u, -0.4243689775466919f);
    p = fmaf(p, u, 1.2732386589050293f);
    float b = t * p;                 // [0, 1]: angle of the reduced octant in bins
    b = ay > ax ? 2.0f - b : b;      // [0, 2]: first quadrant
    b = gx < 0.0f ? 4.0f - b : b;    // [0, 4]: upper half plane
    b = gy < 0.0f ? 8.0f - b : b;    // [0, 8]
    return b;
}

template <int DT>
__device__ __forceinline__ float pixel_at(const uint8_t* __restrict__ img, uint32_t row_off, int x)
{
    if constexpr (DT == BD_DTYPE_U8) {
        return (float)img[row_off + (uint32_t)x];
    } else if constexpr (DT == BD_DTYPE_F32_ROWPAIR) {
        return *reinterpret_cast<const float*>(img + row_off + 8u * (uint32_t)x);
    } else {
        return *reinterpret_cast<const float*>(img + row_off + 4u * (uint32_t)x);
    }
}

__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Bilinear value at a sample from its four corner pixels, relative to the
// reference level.  For u8 the corner differences are exact integers, so
// (v01 - base) - (v00 - base) is formed directly as v01 - v00.
template <int DT>
__device__ __forceinline__ float bilinear(const float (&v)[4], float fx, float fy, float base)
{
    float top, bot;
    if constexpr (DT == BD_DTYPE_U8) {
        top = fmaf(fx, v[1] - v[0], v[0] - base);
        bot = fmaf(fx, v[3] - v[2], v[2] - base);
    } else {
        const float v00 = v[0] - base, v01 = v[1] - base, v10 = v[2] - base, v11 = v[3] - base;
        top = v00 + fx * (v01 - v00);
        bot = v10 + fx * (v11 - v10);
    }
    return top + fy * (bot - top);
}

// v clamped to [0, hi] (hi >= 0) in one instruction (the compiler forms
// v_med3_i32 only for constant bounds).
__device__ __forceinline__ int clampi(int v, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(v), "v"(hi));
    return r;
}

// 32.32 fixed point of v (|v| < 2^31).
__device__ __forceinline__ int64_t to_fixed(double v) { return (int64_t)rint(v * 4294967296.0); }

typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));
typedef uint16_t u16_a1 __attribute__((aligned(1)));

// The four corner pixels and weights of the sample at fixed-point image
// position (X, Y).  Row offsets use 24-bit multiplies: the host admits only
// images with pitch < 2^24, H < 2^24 and pitch * H <= 2^32, so a pixel's
// byte offset is one 32-bit sum, which the loads take as a lane offset from
// the image's scalar base (added to the pointer term by term, the offsets
// would make 64-bit lane addresses).  PAIR (images at least 2 pixels wide):
// each row's two pixels come from one load of the pair starting at the
// column clamped to [0, W - 2] (8 bytes for float images, 2 for u8, at any
// byte offset), which halves the lane accesses; left of column 0 or right of
// column W - 1 (clamp to edge) the first or second pixel of the pair stands
// for both (float) or the weight selects it (u8).
template <int DT, bool PAIR>
__device__ __forceinline__ void fetch_fixed(const uint8_t* __restrict__ img, int wm1, int hm1, uint32_t upitch,
                                            int64_t X, int64_t Y, float (&v)[4], float& fx, float& fy)
{
    const int xi = (int)(X >> 32), yi = (int)(Y >> 32);
    fx = (float)(uint32_t)X * 0x1p-32f;
    fy = (float)(uint32_t)Y * 0x1p-32f;
    const uint32_t ra = __umul24((uint32_t)clampi(yi, hm1), upitch);
    const uint32_t rb = __umul24((uint32_t)clampi(yi + 1, hm1), upitch);
    if constexpr (PAIR && DT == BD_DTYPE_F32_ROWPAIR) {
        // one 16-byte load: (I[y][x], I[y+1][x], I[y][x+1], I[y+1][x+1]) at the
        // column clamped to [0, W - 2]; rows as the pair stores them, so above
        // row 0 (both rows clamp to 0) the weight of the second row is set to
        // 0 (top + 0 * (bot - top) is top exactly), and from row H - 1 down the
        // last row's pair holds that row twice
        typedef float float4_a8 __attribute__((ext_vector_type(4), aligned(8)));
        const uint32_t xo = 8u * (uint32_t)clampi(xi, wm1 - 1);
        const float4_a8 qd = *reinterpret_cast<const float4_a8*>(img + (ra + xo));
        const bool left = xi < 0, right = xi >= wm1;
        if (yi < 0) fy = 0.0f;
        v[0] = right ? qd.z : qd.x;
        v[1] = left ? qd.x : qd.z;
        v[2] = right ? qd.w : qd.y;
        v[3] = left ? qd.y : qd.w;
        (void)rb;
    } else if constexpr (PAIR && DT == BD_DTYPE_F32) {
        const uint32_t xo = 4u * (uint32_t)clampi(xi, wm1 - 1);
        const float2_a4 pa = *reinterpret_cast<const float2_a4*>(img + (ra + xo));
        const float2_a4 pb = *reinterpret_cast<const float2_a4*>(img + (rb + xo));
        const bool left = xi < 0, right = xi >= wm1;
        v[0] = right ? pa.y : pa.x;
        v[1] = left ? pa.x : pa.y;
        v[2] = right ? pb.y : pb.x;
        v[3] = left ? pb.x : pb.y;
    } else if constexpr (PAIR) {
        // u8: both bytes of the pair as they are, and the edge cases through
        // the weight instead: left of column 0 the pair (0, 1) with weight 0,
        // right of column W - 1 the pair (W - 2, W - 1) with weight 1.  The
        // differences are small integers, so bilinear<u8> then forms exactly
        // the value of the clamped corners (fma(1, b - a, a - base) = b - base)
        static_assert(DT == BD_DTYPE_U8, "pairs of u8 or float pixels");
        const uint32_t xo = (uint32_t)clampi(xi, wm1 - 1);
        const uint32_t pa = *reinterpret_cast<const u16_a1*>(img + (ra + xo));  // byte 0: column xo
        const uint32_t pb = *reinterpret_cast<const u16_a1*>(img + (rb + xo));
        fx = xi < 0 ? 0.0f : xi >= wm1 ? 1.0f : fx;
        v[0] = (float)(pa & 0xffu);
        v[1] = (float)(pa >> 8);
        v[2] = (float)(pb & 0xffu);
        v[3] = (float)(pb >> 8);
    } else {
        const int xa = clampi(xi, wm1), xb = clampi(xi + 1, wm1);
        v[0] = pixel_at<DT>(img, ra, xa);
        v[1] = pixel_at<DT>(img, ra, xb);
        v[2] = pixel_at<DT>(img, rb, xa);
        v[3] = pixel_at<DT>(img, rb, xb);
    }
}

// Resampling with fixed-point positions (every sample within 2^30 pixels of
// the origin).  Core: 16 steps over the 32x32 interior in 8x8 blocks of
// samples, lane (a, b) at sample (1 + 8 bi + a, 1 + 8 bj + b) in step
// 4 bi + bj.  A block's 64 samples are neighbours in the image at any
// rotation, so one gather instruction touches few cache lines (a row or a
// column of lanes along the patch axes touches up to one line per lane when
// that axis runs vertically).  Apron: rows 0 and 33 (columns 1..32) and
// columns 0 and 33 (rows 1..32), lane (h, c) with h = lane / 32 choosing
// the side, fetched with the last round.  Every load of a round of R steps
// is in flight before any is used: R = 8 (two round trips) where a launch
// holds about one keypoint per wavefront and so is bound by these round
// trips, R = 4 (fewer registers) for persistent loops.
template <int DT, int R, bool PAIR>
__device__ __forceinline__ void resample_fixed(const uint8_t* __restrict__ img, int32_t W, int32_t H,
                                               uint32_t upitch, double kx, double ky, double sa, double sb,
                                               float base, float* P, int lane)
{
    static_assert(16 % R == 0 && R % 4 == 0, "rounds must tile the 16 core steps by whole block rows");
    const int wm1 = W - 1, hm1 = H - 1;
    const int a = lane >> 3, b = lane & 7;
    const double ux = (double)b - 15.5, uy = (double)a - 15.5;
    int64_t X = to_fixed(fma(sa, ux, fma(-sb, uy, kx)));
    int64_t Y = to_fixed(fma(sb, ux, fma(sa, uy, ky)));
    // next block along the row (8 columns on), and from the last block of a
    // row to the first of the next (8 rows down, 24 columns back)
    const int64_t cX = to_fixed(8.0 * sa), cY = to_fixed(8.0 * sb);
    const int64_t nX = to_fixed(-8.0 * sb) - 3 * cX, nY = to_fixed(8.0 * sa) - 3 * cY;
    float* dst = P + (1 + a) * kApron + 1 + b;
    auto advance = [&](int t) {
        if ((t & 3) == 3) {
            X += nX;
            Y += nY;
        } else {
            X += cX;
            Y += cY;
        }
    };
    auto offset = [](int t) { return (t >> 2) * 8 * kApron + (t & 3) * 8; };
#pragma unroll 1
    for (int t0 = 0; t0 < 16 - R; t0 += R) {
        float v[R][4], fx[R], fy[R];
#pragma unroll
        for (int g = 0; g < R; ++g) {
            fetch_fixed<DT, PAIR>(img, wm1, hm1, upitch, X, Y, v[g], fx[g], fy[g]);
            advance(g);  // t0 is a multiple of 4
        }
#pragma unroll
        for (int g = 0; g < R; ++g) dst[offset(t0 + g)] = bilinear<DT>(v[g], fx[g], fy[g], base);
    }
    // last round: core steps 16 - R .. 15, then rows 0 / 33 at column 1 + c
    // and columns 0 / 33 at row 1 + c
    const int h = lane >> 5, c = lane & 31;
    float v[R + 2][4], fx[R + 2], fy[R + 2];
#pragma unroll
    for (int g = 0; g < R; ++g) {
        fetch_fixed<DT, PAIR>(img, wm1, hm1, upitch, X, Y, v[g], fx[g], fy[g]);
        advance(g);
    }
    const double ar = h ? 16.5 : -16.5, ac = (double)c - 15.5;
    fetch_fixed<DT, PAIR>(img, wm1, hm1, upitch, to_fixed(fma(sa, ac, fma(-sb, ar, kx))),
                    to_fixed(fma(sb, ac, fma(sa, ar, ky))), v[R], fx[R], fy[R]);
    fetch_fixed<DT, PAIR>(img, wm1, hm1, upitch, to_fixed(fma(sa, ar, fma(-sb, ac, kx))),
                    to_fixed(fma(sb, ar, fma(sa, ac, ky))), v[R + 1], fx[R + 1], fy[R + 1]);
#pragma unroll
    for (int g = 0; g < R; ++g) dst[offset(16 - R + g)] = bilinear<DT>(v[g], fx[g], fy[g], base);
    P[(h ? 33 : 0) * kApron + 1 + c] = bilinear<DT>(v[R], fx[R], fy[R], base);
    P[(1 + c) * kApron + (h ? 33 : 0)] = bilinear<DT>(v[R + 1], fx[R + 1], fy[R + 1], base);
}

// Resampling with FP64 positions, for keypoints far outside any image (or
// with huge scales): sample s = lane + 64 it of the 1156, three per lane in
// flight at a time.
template <int DT>
__device__ __forceinline__ void resample_f64(const uint8_t* __restrict__ img, int32_t W, int32_t H, uint32_t upitch,
                                             double kx, double ky, double sa, double sb, float base, float* P,
                                             int lane)
{
    const int wm1 = W - 1, hm1 = H - 1;
    constexpr int kIters = (kSamples + kWave - 1) / kWave;  // 19
    constexpr int kGroup = 3;
#pragma unroll 1
    for (int it0 = 0; it0 < kIters; it0 += kGroup) {
        float v[kGroup][4], fxs[kGroup], fys[kGroup];
        int sidx[kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            const int s = lane + (it0 + g) * kWave;
            sidx[g] = s;
            const int sc = s < kSamples ? s : kSamples - 1;
            const int i = sc / kApron, j = sc - i * kApron;
            const double uy = (double)((float)i - 16.5f), ux = (double)((float)j - 16.5f);
            const double px = fma(sa, ux, fma(-sb, uy, kx));
            const double py = fma(sb, ux, fma(sa, uy, ky));
            const double x0 = floor(px), y0 = floor(py);
            fxs[g] = (float)(px - x0);
            fys[g] = (float)(py - y0);
            // keep the conversion in range for far-off keypoints; clamping follows
            const int xi = (int)fmin(fmax(x0, -1.0e9), 1.0e9), yi = (int)fmin(fmax(y0, -1.0e9), 1.0e9);
            const int xa = clampi(xi, wm1), xb = clampi(xi + 1, wm1);
            const uint32_t ra = __umul24((uint32_t)clampi(yi, hm1), upitch);
            const uint32_t rb = __umul24((uint32_t)clampi(yi + 1, hm1), upitch);
            v[g][0] = pixel_at<DT>(img, ra, xa);
            v[g][1] = pixel_at<DT>(img, ra, xb);
            v[g][2] = pixel_at<DT>(img, rb, xa);
            v[g][3] = pixel_at<DT>(img, rb, xb);
        }
#pragma unroll
        for (int g = 0; g < kGroup; ++g)
            if (sidx[g] < kSamples) P[sidx[g]] = bilinear<DT>(v[g], fxs[g], fys[g], base);
    }
}

// The histogram of one keypoint, computed by one wavefront with a
// kWaveLds-float LDS slice P; writes the 128 features to out.
template <int DT, int R>
__device__ __forceinline__ void hist_one(const uint8_t* __restrict__ img, int32_t W, int32_t H, int64_t pitch,
                                         const bd_keypoint kp, float* __restrict__ out, float* P, int lane,
                                         unsigned long long* __restrict__ invalid)
{
    if (!(finite_f(kp.x) && finite_f(kp.y) && finite_f(kp.scale) && finite_f(kp.angle) && kp.scale > 0.0f)) {
        out[lane] = 0.0f;
        out[lane + kWave] = 0.0f;
        if (invalid && lane == 0) atomicAdd(invalid, 1ull);
        return;
    }
    double sn, cs;
    sincos((double)kp.angle, &sn, &cs);
    const double sa = (double)kp.scale * cs, sb = (double)kp.scale * sn;
    const double kx = kp.x, ky = kp.y;

    // reference level: the pixel under the keypoint (clamped)
    const int bx = (int)fmin(fmax(rint(kx), 0.0), (double)(W - 1));
    const int by = (int)fmin(fmax(rint(ky), 0.0), (double)(H - 1));
    const float base = pixel<DT>(img, pitch, bx, by);

    // 1. resample the 34x34 patch.  Sample (i, j) sits at patch offset
    // (j - 16.5, i - 16.5); its image position is (kx, ky) plus that offset
    // rotated and scaled by (sa, sb).
    if (fabs((double)kp.x) + 24.0 * kp.scale < 1073741824.0 && fabs((double)kp.y) + 24.0 * kp.scale < 1073741824.0)
    {
        if (W >= 2)
            resample_fixed<DT, R, true>(img, W, H, (uint32_t)pitch, kx, ky, sa, sb, base, P, lane);
        else
            resample_fixed<DT, R, false>(img, W, H, (uint32_t)pitch, kx, ky, sa, sb, base, P, lane);
    }
    else
        resample_f64<DT>(img, W, H, (uint32_t)pitch, kx, ky, sa, sb, base, P, lane);
    wave_sync();

    // 2. gradients and votes.  Pixel k of lane (half, j) is patch row
    // i = k (half 0) or 31 - k (half 1), column j.
    const int j = lane & 31, half = lane >> 5;
    float acc[3][8];
#pragma unroll
    for (int sl = 0; sl < 3; ++sl)
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[sl][o] = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = half ? 31 - k : k;
        const int c = (i + 1) * kApron + (j + 1);
        const float gx = P[c + 1] - P[c - 1];
        const float gy = P[c + kApron] - P[c - kApron];
        const float m = __builtin_amdgcn_sqrtf(gx * gx + gy * gy);
        const float bo = orientation_bin(gx, gy);
        // triangular weights max(0, 1 - |bo - o|), bin 0 also taking bo near 8:
        // for bo in [0, 8] that sum is max(0, |bo - 4| - 3).  Both forms are
        // at most 1, so a clamp to [0, 1] gives the max.
        float tri[8];
        tri[0] = __builtin_amdgcn_fmed3f(fabsf(bo - 4.0f) - 3.0f, 0.0f, 1.0f);
#pragma unroll
        for (int o = 1; o < 8; ++o) tri[o] = __builtin_amdgcn_fmed3f(1.0f - fabsf(bo - (float)o), 0.0f, 1.0f);
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
            if (slot_active(k, sl)) {
                const float w = m * kRow.v[k][sl];
#pragma unroll
                for (int o = 0; o < 8; ++o) acc[sl][o] += w * tri[o];
            }
        }
    }
    wave_sync();  // the patch is dead; its LDS now holds the lane histograms

    // lane histograms (times the column's Gaussian weight) into the padded
    // layout; lanes 0..23 of each half also zero the four pad columns on
    // each side of entry `lane`
    const float gxj = kGauss.v[j];
    float* Hl = P + half * 40 + 4 + j;
#pragma unroll
    for (int sl = 0; sl < 3; ++sl)
#pragma unroll
        for (int o = 0; o < 8; ++o) Hl[(sl * 8 + o) * kHistStride] = acc[sl][o] * gxj;
    if (j < 24) {
        float* pad = P + j * kHistStride + half * 40;
        *reinterpret_cast<float4*>(pad) = float4{0.0f, 0.0f, 0.0f, 0.0f};
        *reinterpret_cast<float4*>(pad + 36) = float4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    wave_sync();

    // 3. bin b = (cy, cx, o) of the 4x4x8 histogram: cell row cy is slot cy
    // of the top half and slot 3 - cy of the bottom half; cell column cx sums
    // columns 8 cx - 4 .. 8 cx + 11 (padding where outside) with kCol
    float h[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int b = lane + q * kWave;
        const int cy = b >> 5, cx = (b >> 3) & 3, o = b & 7;
        float sum = 0.0f;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int slot = hh ? 3 - cy : cy;
            const float* src = P + ((slot > 2 ? 2 : slot) * 8 + o) * kHistStride + hh * 40 + 8 * cx;
            float part = 0.0f;
#pragma unroll
            for (int t = 0; t < 16; ++t) part = fmaf(kCol.v[t], src[t], part);
            sum += slot > 2 ? 0.0f : part;
        }
        h[q] = sum;
    }

    // 4. L2 normalization
    const float ss = wave_sum_f(h[0] * h[0] + h[1] * h[1]);
    if (ss > 0.0f) {
        const float nrm = sqrtf(ss);
        h[0] = h[0] / nrm;
        h[1] = h[1] / nrm;
    }
    out[lane] = h[0];
    out[lane + kWave] = h[1];
}

template <int DT>
__global__ __launch_bounds__(256) void hashsift_hist_kernel(const uint8_t* __restrict__ img, int32_t W,
                                                            int32_t H, int64_t pitch,
                                                            const bd_keypoint* __restrict__ kps,
                                                            int32_t n_kp, const int32_t* __restrict__ order,
                                                            float* __restrict__ hist,
                                                            unsigned long long* __restrict__ invalid)
{
    __shared__ float smem[kHistWaves][kWaveLds];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int nb = (n_kp + kHistWaves - 1) / kHistWaves;
    const int lb = xcd_logical_block(blockIdx.x, nb);
    if (lb >= nb) return;
    const int pos = lb * kHistWaves + wave;
    if (pos >= n_kp) return;
    const int n = order ? order[pos] : pos;
    if (n < 0 || n >= n_kp) return;  // malformed order entries are skipped
    hist_one<DT, 8>(img, W, H, pitch, kps[n], hist + (int64_t)n * 128, smem[wave], lane, invalid);
}

// Batch: units are blocks of four keypoints of every image in turn (pre is
// the prefix of ceil(n_kp / 4)); order entries are image-local; features are
// written to the flat array at the keypoint's global index.  DT is the
// dtype of every image's HashSIFT source, or kMixedDtypes.  Four waves per
// SIMD: LDS would allow five, but the 96 registers of five spill.
constexpr int kMixedDtypes = -1;

template <int DT>
__global__ __launch_bounds__(256, 4) void hashsift_hist_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                              const int32_t* __restrict__ pre,
                                                              const bd_keypoint* __restrict__ kps,
                                                              const int32_t* __restrict__ order,
                                                              float* __restrict__ hist,
                                                              unsigned long long* __restrict__ invalid)
{
    __shared__ float smem[kHistWaves][kWaveLds];
    const int wave = threadIdx.x / kWave;
    const UnitRange ur = xcd_units(pre[n_img]);
    for (int u = ur.first; u < ur.end; u += ur.stride) {
        const int im_i = segment_of(pre, n_img, u);
        const BatchImage& im = imgs[im_i];
        const int pos = (u - pre[im_i]) * kHistWaves + wave;
        if (pos >= im.n_kp) continue;
        const int n = order[im.kp_offset + pos];
        if (n < 0 || n >= im.n_kp) continue;
        const int g = im.kp_offset + n;
        // lane is opaque to the compiler inside each unit, so per-lane
        // addresses are not hoisted out of the loop and kept live throughout
        int lane = threadIdx.x % kWave;
        asm volatile("" : "+v"(lane));
        if constexpr (DT != kMixedDtypes) {
            hist_one<DT, 4>(im.img_hs, im.W, im.H, im.pitch_hs, kps[g], hist + (int64_t)g * 128, smem[wave], lane,
                            invalid);
        } else if (im.hs_dtype == BD_DTYPE_U8) {
            hist_one<BD_DTYPE_U8, 4>(im.img_hs, im.W, im.H, im.pitch_hs, kps[g], hist + (int64_t)g * 128, smem[wave],
                                     lane, invalid);
        } else {
            hist_one<BD_DTYPE_F32, 4>(im.img_hs, im.W, im.H, im.pitch_hs, kps[g], hist + (int64_t)g * 128, smem[wave],
                                      lane, invalid);
        }
    }
}

// Features of 32x32 float32 patches: each patch is an image whose keypoint
// sits at its centre (15.5, 15.5) with scale 1 and angle 0, so every sample
// falls on a patch pixel (the apron clamps to the edge).
__global__ __launch_bounds__(256) void hashsift_patch_kernel(const float* __restrict__ patches, int32_t n,
                                                             float* __restrict__ hist)
{
    __shared__ float smem[kHistWaves][kWaveLds];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int i = blockIdx.x * kHistWaves + wave;
    if (i >= n) return;
    const bd_keypoint kp{15.5f, 15.5f, 1.0f, 0.0f};
    hist_one<BD_DTYPE_F32, 4>(reinterpret_cast<const uint8_t*>(patches + (int64_t)i * 1024), 32, 32, 128, kp,
                           hist + (int64_t)i * 128, smem[wave], lane, nullptr);
}

// ---------------------------------------------------------------- projection

constexpr int kProjRows = 16;                 // keypoints per wavefront tile (one MFMA row tile)
constexpr int kProjWaves = 4;                 // wavefronts per block
constexpr int kProjTile = kProjRows * kProjWaves;  // keypoints per block tile
constexpr int kProjStride = 132;              // LDS row stride in floats (128 + 4)
constexpr int kProjBlocksPerCu = 2;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 32 consecutive floats of an LDS row.
__device__ __forceinline__ void lds_row32(const float* src, float (&v)[32])
{
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float4 f = reinterpret_cast<const float4*>(src)[q];
        v[4 * q] = f.x;
        v[4 * q + 1] = f.y;
        v[4 * q + 2] = f.z;
        v[4 * q + 3] = f.w;
    }
}

// FP32 projection: persistent and B-stationary.  Block b works on XCD b % 8
// for the chunk of 64 bits (b / 8) % n_words over that XCD's contiguous
// range of 64-keypoint tiles, so the n_words blocks that need one tile run on
// the same XCD and share its rows through L2.  The block keeps its chunk of
// B in registers as the MFMA operand; each wavefront streams 16-keypoint
// tiles through its own LDS slice, the next tile's rows in flight
// (registers) while the current one is multiplied with
// v_mfma_f32_16x16x4_f32, 32 steps per subtile.  Lane (g, m) holds elements
// 32g..32g+31 of keypoint row m and of B row m of each 16-bit subtile, so the
// k order of the MFMA chain is one permutation applied to both operands.
__global__ __launch_bounds__(256, 2) void hashsift_project_kernel(const float* __restrict__ hist,
                                                                 const bd_keypoint* __restrict__ kps, int32_t n_kp,
                                                                 const float* __restrict__ B,
                                                                 const float* __restrict__ t, int32_t n_words,
                                                                 uint64_t* __restrict__ codes,
                                                                 float* __restrict__ resp)
{
    __shared__ __align__(16) float Bs[64 * kProjStride];
    __shared__ __align__(16) float As[kProjWaves][kProjRows * kProjStride];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int g = lane >> 4, m = lane & 15;
    const int x = (int)blockIdx.x % kXcds, r = (int)blockIdx.x / kXcds;
    const int chunk = r % n_words, grp = r / n_words;
    const int n_groups = (int)gridDim.x / kXcds / n_words;
    const int n_tiles = (n_kp + kProjTile - 1) / kProjTile;
    const int tile_end = (int)((int64_t)n_tiles * (x + 1) / kXcds);
    const int tile_first = (int)((int64_t)n_tiles * x / kXcds) + grp;
    if (tile_first >= tile_end) return;  // uniform per block
    const int n_bits = n_words * 64;

    // B chunk to LDS: 64 rows x 128 floats, 8 float4 per thread
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int e = (q * 256 + (int)threadIdx.x) * 4;  // float index in the chunk
        const int row = e >> 7, col = e & 127;
        *reinterpret_cast<float4*>(&Bs[row * kProjStride + col]) =
            *reinterpret_cast<const float4*>(B + (int64_t)(chunk * 64 + row) * 128 + col);
    }
    __syncthreads();

    // the MFMA operand of B in registers
    float bf[4][32];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) lds_row32(&Bs[(16 * nt + m) * kProjStride + 32 * g], bf[nt]);
    float tv[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) tv[nt] = t[chunk * 64 + 16 * nt + m];

    float* A = As[wave];
    // tile rows for this wavefront: 16 rows x 128 floats, lane l loads row l / 4, floats 32 (l % 4) ..
    const int lrow = lane >> 2, lcol = (lane & 3) * 32;
    float4 pre[8];
    auto load_tile = [&](int tile) {
        const int row = tile * kProjTile + wave * kProjRows + lrow;
        if (row < n_kp) {
            const float4* src = reinterpret_cast<const float4*>(hist + (int64_t)row * 128 + lcol);
#pragma unroll
            for (int q = 0; q < 8; ++q) pre[q] = src[q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) pre[q] = float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    load_tile(tile_first);

    for (int tile = tile_first; tile < tile_end; tile += n_groups) {
        wave_sync();  // the previous tile's LDS reads are done
#pragma unroll
        for (int q = 0; q < 8; ++q) *reinterpret_cast<float4*>(&A[lrow * kProjStride + lcol + 4 * q]) = pre[q];
        wave_sync();
        if (tile + n_groups < tile_end) load_tile(tile + n_groups);
        const int kp0 = tile * kProjTile + wave * kProjRows;

        float a[32];
        lds_row32(&A[m * kProjStride + 32 * g], a);
        floatx4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < 32; ++k)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], bf[nt][k], acc[nt], 0, 0, 0);

        // lane holds D[kp = 4g + i][bit = 16nt + m]
        float rv[4][4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) rv[nt][i] = acc[nt][i] - tv[nt];

        uint64_t mask[4][4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int bit = chunk * 64 + 16 * nt + m;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int kp = kp0 + 4 * g + i;
                if (resp && kp < n_kp) resp[(int64_t)kp * n_bits + bit] = rv[nt][i];
                mask[nt][i] = __ballot(rv[nt][i] > 0.0f);
            }
        }
        if (lane < 16) {
            const int kp = kp0 + lane;
            if (kp < n_kp) {
                bool valid = true;
                if (kps) {
                    const bd_keypoint k = kps[kp];
                    valid = finite_f(k.x) && finite_f(k.y) && finite_f(k.scale) && finite_f(k.angle) &&
                            k.scale > 0.0f;
                }
                const int gq = lane >> 2, iq = lane & 3;
                uint64_t word = 0ull;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const uint64_t mk =
                        iq == 0 ? mask[nt][0] : iq == 1 ? mask[nt][1] : iq == 2 ? mask[nt][2] : mask[nt][3];
                    word |= ((mk >> (16 * gq)) & 0xffffull) << (16 * nt);
                }
                codes[(int64_t)kp * n_words + chunk] = valid ? word : 0ull;
            }
        }
    }
}


// ---------------------------------------------------------------- reduced-precision projection, tile-shared
//
// BF16 / FP8 projection: one 512-thread block per CU walks 64-keypoint tiles
// (grid stride).  A tile is read from HBM once and kept in LDS twice, as
// FP32 (for the re-check) and rounded to the MFMA operand type, in one of two
// buffers: the next tile is staged while the current one is multiplied, with
// one block barrier per tile.  All eight wavefronts share the tile:
// wavefront w owns the 64-bit chunk w % NW of B and the tile rows
// (w / NW) * 16 * kRowSubs onwards.  The chunk's operands stay in registers
// for the whole kernel, rounded and negated once.
//
// The product is taken transposed, D = (-B) f^T + C (v_mfma_f32_16x16x32_bf16
// / _fp8_fp8, FP32 accumulation), so after a 16-keypoint subtile lane (g, n)
// holds z = t - r for keypoint n and 16 bits of its chunk: MFMA row 4 g + i
// of column tile nt is chunk bit lp_bit(nt, g, i), an assignment made when
// the rows of B are loaded so that the packing below lands every bit in
// place.  BF16 starts the accumulation at C = t; FP8 scales every row of the
// tile and of B by a power of two s (the smallest with max|row| <= 448 s, at
// least 2^-126; exact) and forms z = t + (s_row s_b) acc.
//
// Bit j is set when r_j > 0, i.e. when z_j < 0.  Thresholds are made +0
// when they are -0, so z is never -0, and while every operand is finite and
// at most 2^59 in magnitude z is finite: the sign bit of z is the code bit.
// (Other rows take min(z, 0) first, which gives +0, bit 0, for a NaN.)  Byte
// permutes spread the sign bits of four responses over four bytes, masks
// place them (bit 8 i + 7 - nt, or 8 i + 3 - nt in the odd g lanes), lanes
// g and g ^ 1 merge their halves of each byte, and the even g lanes store
// the two 32-bit halves of the keypoint's code word in LDS.  No ballots.
//
// Margin re-check: the sign bits of |z| - margin, packed like the code bits,
// are a lane's pending flags; a lane with any appends them (one 32-bit word
// and its subtile and lane) to a per-wavefront LDS list with room for every
// lane of the tile.  When the tile is done the entries are expanded into
// (row, bit) items, and four lanes re-check each
// item from the unrounded FP32 operands (the feature row from the FP32 tile,
// the row of B from memory, L2-resident): lane j of the four takes the
// float4 groups j, j + 4, ..., j + 28, accumulates the four components in
// four chains over its groups, adds them as (c0 + c1) + (c2 + c3), and the
// four lane sums are added in pairs, then the two pair sums; the same in
// FP64 when that FP32 value is within 1e-6 of the threshold.  The result
// sets or clears the bit in LDS, and each wavefront writes its own code words.
constexpr int kLpRows = 64;        // keypoints per tile
constexpr int kLpThreads = 512;    // eight wavefronts
constexpr int kLpWaves = kLpThreads / kWave;
constexpr int kLpS16 = 136;        // BF16 tile row stride (elements, 272 bytes)
constexpr int kLpS8 = 144;         // FP8 tile row stride (bytes)
constexpr int kLpEntries = 256;    // pending lanes listed per wavefront: every lane of four subtiles
constexpr int kLpS32 = 132;        // FP32 tile row stride (floats)
constexpr float kLpSafe = 0x1p59f; // operands up to this magnitude cannot overflow a response

// state of a tile row, one byte each
constexpr uint8_t kRowExists = 1, kRowValid = 2, kRowSafe = 4;

template <int PREC>
struct LpOperand;
template <>
struct LpOperand<BD_PREC_BF16> {
    typedef bf16x8 type;
    static constexpr int row_bytes = kLpS16 * 2;
};
template <>
struct LpOperand<BD_PREC_FP8> {
    typedef long type;
    static constexpr int row_bytes = kLpS8;
};

// chunk bit of MFMA row 4 g + i of column tile nt (a bijection onto 0..63)
__device__ __forceinline__ int lp_bit(int nt, int g, int i) { return 32 * (g >> 1) + 8 * i + 7 - nt - 4 * (g & 1); }

__device__ __forceinline__ uint32_t pk_bf16(float a, float b)
{
    const __bf16 x = (__bf16)a, y = (__bf16)b;
    return (uint32_t)__builtin_bit_cast(uint16_t, x) | ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
}

// Exponent e of the FP8 row scale 2^e: the smallest with m <= 448 * 2^e
// (448 = 0.875 * 2^9), at least -126; 0 for m = 0.
__device__ __forceinline__ int e4m3_pow2_exp(float m)
{
    if (!(m > 0.0f)) return 0;
    const int E = __builtin_amdgcn_frexp_expf(m);
    const float f = __builtin_amdgcn_frexp_mantf(m);  // m = f * 2^E, f in [0.5, 1)
    const int e = f <= 0.875f ? E - 9 : E - 8;
    return e < -126 ? -126 : e;
}

// v times 2^-e.  With e the row's exponent every finite element of the row
// lands within [-448, 448] exactly (max|row| <= 448 * 2^e), so no clamp is
// needed before the conversion; a NaN stays NaN, and a row holding an
// infinity is outside the safe range anyway.
__device__ __forceinline__ float e4m3_scaled(float v, int e) { return __builtin_amdgcn_ldexpf(v, -e); }

// four values times 2^-e (exact), rounded to e4m3, packed into 32 bits
__device__ __forceinline__ uint32_t pack4_e4m3_pow2(float a, float b, float c, float d, int e)
{
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_scaled(a, e), e4m3_scaled(b, e), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_scaled(c, e), e4m3_scaled(d, e), w, true);
    return (uint32_t)w;
}

// max over the 8-lane groups 8j .. 8j + 7 (lane-local DPP moves, no LDS)
__device__ __forceinline__ float max8_dpp(float v)
{
    int x = __float_as_int(v);
    // quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false)));
    return v;
}

// Sum over the 4-lane groups 4j .. 4j + 3 (pairs, then pairs of pairs);
// every lane of a group ends with the same value.
__device__ __forceinline__ float sum4_dpp(float v)
{
    int x = __float_as_int(v);
    v = v + __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
    x = __float_as_int(v);
    v = v + __int_as_float(__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));  // quad_perm [2,3,0,1]
    return v;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const uint32_t l2 = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const uint32_t h2 = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((uint64_t)h2 << 32) | l2));
}

__device__ __forceinline__ double sum4_dpp_f64(double v)
{
    v = v + dpp_f64<0xB1>(v);
    v = v + dpp_f64<0x4E>(v);
    return v;
}

template <int PREC, int NW>
__global__ __launch_bounds__(kLpThreads, 1) void hashsift_project_lowp_kernel(
    const float* __restrict__ hist, const bd_keypoint* __restrict__ kps, int32_t n_kp, const float* __restrict__ B,
    const float* __restrict__ t, float margin, uint64_t* __restrict__ codes, float* __restrict__ resp,
    uint32_t* __restrict__ recheck_count)
{
    constexpr int kRowSubs = NW == 8 ? 4 : 2;  // 16-row subtiles per wavefront
    constexpr int kWaveRows = 16 * kRowSubs;   // tile rows of a wavefront
    constexpr int kRowBytes = LpOperand<PREC>::row_bytes;
    constexpr int n_bits = NW * 64;
    typedef typename LpOperand<PREC>::type op_t;
    __shared__ __align__(16) uint8_t Alp[2][kLpRows * kRowBytes];
    __shared__ __align__(16) float A32[2][kLpRows * kLpS32];
    __shared__ float Asc[2][kLpRows];
    __shared__ uint8_t Ast[2][kLpRows];
    __shared__ uint64_t Wd[kLpWaves][kWaveRows];
    __shared__ uint32_t Ef[kLpWaves][kLpEntries];  // pending flags of a lane: response (nt, i) at bit 8 i + nt
    __shared__ uint8_t Eh[kLpWaves][kLpEntries];   // its subtile and lane
    __shared__ uint16_t Qi[kLpWaves][kWave * 16];  // items of up to 64 entries
    __shared__ uint32_t Qn[kLpWaves];

    const int tid = (int)threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    const int g = lane >> 4, n = lane & 15;
    const int chunk = wave % NW;
    const int rbase = (wave / NW) * kWaveRows;
    uint64_t* Ww = Wd[wave];
    uint32_t* Ww32 = reinterpret_cast<uint32_t*>(Ww);

    // B operands of this lane: MFMA row n of column tile nt is chunk bit
    // lp_bit(nt, n >> 2, n & 3); elements 32 s + 8 g .. + 7 of k-step s; negated
    op_t bop[4][4];
    float sbrow[4];
    bool safe = true;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float* brow = B + (int64_t)(chunk * 64 + lp_bit(nt, n >> 2, n & 3)) * 128;
        float v[4][8];
        float mx = 0.0f;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float4 lo = *reinterpret_cast<const float4*>(brow + 32 * s + 8 * g);
            const float4 hi = *reinterpret_cast<const float4*>(brow + 32 * s + 8 * g + 4);
            v[s][0] = -lo.x, v[s][1] = -lo.y, v[s][2] = -lo.z, v[s][3] = -lo.w;
            v[s][4] = -hi.x, v[s][5] = -hi.y, v[s][6] = -hi.z, v[s][7] = -hi.w;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                mx = fmaxf(mx, fabsf(v[s][e]));
                safe = safe && fabsf(v[s][e]) <= kLpSafe;  // false for NaN
            }
        }
        sbrow[nt] = 1.0f;
        if constexpr (PREC == BD_PREC_BF16) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int e = 0; e < 8; ++e) bop[nt][s][e] = (__bf16)v[s][e];
        } else {
            // the row's four lanes (g = 0..3) share its maximum
            mx = fmaxf(mx, __shfl_xor(mx, 16, kWave));
            mx = fmaxf(mx, __shfl_xor(mx, 32, kWave));
            const int e = e4m3_pow2_exp(mx);
            sbrow[nt] = __builtin_amdgcn_ldexpf(1.0f, e);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const uint32_t lo = pack4_e4m3_pow2(v[s][0], v[s][1], v[s][2], v[s][3], e);
                const uint32_t hi = pack4_e4m3_pow2(v[s][4], v[s][5], v[s][6], v[s][7], e);
                bop[nt][s] = (long)(((uint64_t)hi << 32) | lo);
            }
        }
    }
    // thresholds (and FP8 row scales of B) of this lane's responses: bit lp_bit(nt, g, i)
    floatx4 tz[4];
    float sbz[4][4];
    uint32_t msk[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float tv = t[chunk * 64 + lp_bit(nt, g, i)];
            safe = safe && fabsf(tv) <= kLpSafe;
            tz[nt][i] = tv == 0.0f ? 0.0f : tv;  // -0 becomes +0
            sbz[nt][i] = 1.0f;
            if constexpr (PREC == BD_PREC_FP8) sbz[nt][i] = __shfl(sbrow[nt], 4 * g + i, kWave);
        }
        msk[nt] = (0x80808080u >> nt) >> (4 * (g & 1));
    }
    const bool chunk_safe = __all(safe);

    // staging: thread tid moves row tid / 8, float4 groups j, j + 8, j + 16, j + 24 (j = tid % 8)
    const int prow = tid >> 3, pj = tid & 7;
    const int n_tiles = (n_kp + kLpRows - 1) / kLpRows;
    float4 pf[4];
    bool pvalid = true;
    auto load_tile = [&](int tile) {
        const int kp = tile * kLpRows + prow;
        if (kp < n_kp) {
            const float4* src = reinterpret_cast<const float4*>(hist + (int64_t)kp * 128);
#pragma unroll
            for (int q = 0; q < 4; ++q) pf[q] = src[pj + 8 * q];
            if (kps && pj == 0) {
                const bd_keypoint k = kps[kp];
                pvalid = finite_f(k.x) && finite_f(k.y) && finite_f(k.scale) && finite_f(k.angle) && k.scale > 0.0f;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) pf[q] = float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    auto store_tile = [&](int buf, int tile) {
        const int kp = tile * kLpRows + prow;
        bool ok = true;
        float mx = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float m4 = fmaxf(fmaxf(fabsf(pf[q].x), fabsf(pf[q].y)), fmaxf(fabsf(pf[q].z), fabsf(pf[q].w)));
            mx = fmaxf(mx, m4);
            ok = ok && fabsf(pf[q].x) <= kLpSafe && fabsf(pf[q].y) <= kLpSafe && fabsf(pf[q].z) <= kLpSafe &&
                 fabsf(pf[q].w) <= kLpSafe;
        }
        float4* d32 = reinterpret_cast<float4*>(&A32[buf][prow * kLpS32]);
#pragma unroll
        for (int q = 0; q < 4; ++q) d32[pj + 8 * q] = pf[q];
        uint8_t* dlp = &Alp[buf][prow * kRowBytes];
        if constexpr (PREC == BD_PREC_BF16) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<uint2*>(dlp + 8 * (pj + 8 * q)) =
                    uint2{pk_bf16(pf[q].x, pf[q].y), pk_bf16(pf[q].z, pf[q].w)};
        } else {
            mx = max8_dpp(mx);
            const int e = e4m3_pow2_exp(mx);
            if (pj == 0) Asc[buf][prow] = __builtin_amdgcn_ldexpf(1.0f, e);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                *reinterpret_cast<uint32_t*>(dlp + 4 * (pj + 8 * q)) = pack4_e4m3_pow2(pf[q].x, pf[q].y, pf[q].z, pf[q].w, e);
        }
        // the row is safe when all eight of its threads are
        const uint64_t unsafe = __ballot(!ok);
        const bool row_safe = ((unsafe >> (lane & 56)) & 0xffull) == 0ull;
        if (pj == 0)
            Ast[buf][prow] = (uint8_t)((kp < n_kp ? kRowExists : 0) | (pvalid ? kRowValid : 0) | (row_safe ? kRowSafe : 0));
    };

    int tile = (int)blockIdx.x;
    const int stride = (int)gridDim.x;
    if (tile < n_tiles) {
        load_tile(tile);
        store_tile(0, tile);
        if (tile + stride < n_tiles) load_tile(tile + stride);
    }
    uint32_t rechecked = 0;  // per lane; summed over the wavefront at the end
    uint16_t* Qw = Qi[wave];
    const int gi = lane >> 2, j = lane & 3;

    // Re-check items (row << 6 | bit) of the tile at row r0: four lanes per
    // item, two sets of sixteen items, the rows of B of one set loaded while
    // the other set is summed (the feature rows come from the FP32 tile in LDS).
    float4 bv[2][8];
    float tc[2];
    int itm[2];
    auto fetch = [&](int set, int base, int total) {
        const int it = base + gi;
        if (it < total) {
            const int item = Qw[it];
            itm[set] = item;
            const int col = item & 63;
            const float4* brow = reinterpret_cast<const float4*>(B + (int64_t)(chunk * 64 + col) * 128);
#pragma unroll
            for (int q = 0; q < 8; ++q) bv[set][q] = brow[j + 4 * q];
            tc[set] = t[chunk * 64 + col];
        } else {
            // defined either way, so the sets are not live between uses
            itm[set] = 0;
            tc[set] = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) bv[set][q] = float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    auto check = [&](int set, int base, int total, int r0, const float* a32) {
        if (base + gi < total) {
            const int wr = itm[set] >> 6, col = itm[set] & 63;
            const float4* arow = reinterpret_cast<const float4*>(a32 + (rbase + wr) * kLpS32);
            float c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 a = arow[j + 4 * q];
                c0 = fmaf(a.x, bv[set][q].x, c0);
                c1 = fmaf(a.y, bv[set][q].y, c1);
                c2 = fmaf(a.z, bv[set][q].z, c2);
                c3 = fmaf(a.w, bv[set][q].w, c3);
            }
            float res = sum4_dpp((c0 + c1) + (c2 + c3)) - tc[set];
            if (fabsf(res) < 1e-6f) {  // the same in all four lanes
                double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float4 a = arow[j + 4 * q];
                    d0 = fma((double)a.x, (double)bv[set][q].x, d0);
                    d1 = fma((double)a.y, (double)bv[set][q].y, d1);
                    d2 = fma((double)a.z, (double)bv[set][q].z, d2);
                    d3 = fma((double)a.w, (double)bv[set][q].w, d3);
                }
                res = (float)(sum4_dpp_f64((d0 + d1) + (d2 + d3)) - (double)tc[set]);
            }
            if (j == 0) {
                const uint64_t bit = 1ull << col;
                if (res > 0.0f)
                    __hip_atomic_fetch_or(&Ww[wr], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                else
                    __hip_atomic_fetch_and(&Ww[wr], ~bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                if (resp) resp[(int64_t)(r0 + rbase + wr) * n_bits + chunk * 64 + col] = res;
            }
        }
    };
    // items of the tile at row r0, its FP32 rows in a32
    auto drain = [&](int total, int r0, const float* a32) {
        fetch(0, 0, total);
        for (int b0 = 0; b0 < total; b0 += 32) {
            fetch(1, b0 + 16, total);
            check(0, b0, total, r0, a32);
            fetch(0, b0 + 32, total);
            check(1, b0 + 16, total, r0, a32);
        }
        wave_sync();
    };
    // entries e0 .. min(ne, e0 + 64) - 1 into items (in any order); returns their number
    auto expand = [&](int e0, int ne) -> int {
        if (lane == 0) Qn[wave] = 0;
        wave_sync();
        const int e = e0 + lane;
        if (e < ne) {
            const int hdr = Eh[wave][e];
            uint32_t flags = Ef[wave][e];
            const int cnt = __popc(flags);
            rechecked += (uint32_t)cnt;
            int o = (int)__hip_atomic_fetch_add(&Qn[wave], (uint32_t)cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            const int wr = 16 * (hdr >> 6) + (hdr & 15), eg = (hdr >> 4) & 3;
            while (flags) {
                const int b = __builtin_ctz(flags);  // 8 i + nt
                flags &= flags - 1u;
                Qw[o++] = (uint16_t)((wr << 6) | lp_bit(b & 7, eg, b >> 3));
            }
        }
        wave_sync();
        return __builtin_amdgcn_readfirstlane((int)Qn[wave]);
    };
    auto flush_now = [&](int ne, int r0, const float* a32) {
        for (int e0 = 0; e0 < ne; e0 += kWave) drain(expand(e0, ne), r0, a32);
    };
    // this wavefront's code words of the tile at row r0 out (rows of invalid keypoints are zero)
    auto write_words = [&](int r0, uint32_t st) {
        wave_sync();
        if (lane < kWaveRows && (st & kRowExists))
            codes[(int64_t)(r0 + rbase + lane) * NW + chunk] = (st & kRowValid) ? Ww[lane] : 0ull;
        wave_sync();
    };

    for (int buf = 0; tile < n_tiles; tile += stride, buf ^= 1) {
        // buffer buf is complete, and every read of buffer buf ^ 1 (the previous tile) is done
        __syncthreads();
        if (tile + stride < n_tiles) {
            store_tile(buf ^ 1, tile + stride);
            if (tile + 2 * stride < n_tiles) load_tile(tile + 2 * stride);
        }
        const int row0 = tile * kLpRows;
        const bool full = row0 + kLpRows <= n_kp;  // every row of the tile exists
        const uint8_t* Ab = Alp[buf];
        const float* A32b = A32[buf];

        int n_ent = 0;  // wavefront-uniform
#pragma unroll 1
        for (int pp = 0; pp < kRowSubs; pp += 2) {

            // 1. D = (-B) f^T + C for two subtiles: lane (g, n) ends with the
            //    responses of keypoint rbase + 16 p + n to bits lp_bit(nt, g, i)
            floatx4 acc[2][4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                op_t av[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int row = rbase + 16 * (pp + r) + n;
                    if constexpr (PREC == BD_PREC_BF16)
                        av[r] = *reinterpret_cast<const bf16x8*>(&Ab[row * kRowBytes + 2 * (32 * s + 8 * g)]);
                    else
                        av[r] = *reinterpret_cast<const long*>(&Ab[row * kRowBytes + 32 * s + 8 * g]);
                }
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        if constexpr (PREC == BD_PREC_BF16)
                            acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bop[nt][s], av[r],
                                                                                  s == 0 ? tz[nt] : acc[r][nt], 0, 0, 0);
                        else
                            acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(
                                bop[nt][s], av[r], s == 0 ? floatx4{0.0f, 0.0f, 0.0f, 0.0f} : acc[r][nt], 0, 0, 0);
                    }
            }

            // 2. per subtile: pending lanes listed, responses out, sign bits packed
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int wr = 16 * (pp + r) + n;  // this lane's row within the wavefront's rows
                const uint8_t st = Ast[buf][rbase + wr];
                float z[4][4];
                if constexpr (PREC == BD_PREC_BF16) {
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) z[nt][i] = acc[r][nt][i];
                } else {
                    const float sk = Asc[buf][rbase + wr];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) z[nt][i] = fmaf(acc[r][nt][i], sk * sbz[nt][i], tz[nt][i]);
                }
                if (margin > 0.0f) {
                    // pending flags: the sign bit of |z| - margin is set exactly when |z| < margin
                    // (|NaN| is a positive NaN and |inf| - margin is +inf: neither is pending)
                    uint32_t F = 0;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        float d[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) d[i] = fabsf(z[nt][i]) - margin;
                        const uint32_t pa = __builtin_amdgcn_perm(__float_as_uint(d[1]), __float_as_uint(d[0]), 0x0c0c0b09u);
                        const uint32_t pb = __builtin_amdgcn_perm(__float_as_uint(d[3]), __float_as_uint(d[2]), 0x0b090c0cu);
                        F |= (pa | pb) & (0x01010101u << nt);
                    }
                    if (!(full || (st & kRowExists))) F = 0u;
                    const uint64_t L = __ballot(F != 0u);
                    if (L) {
                        if (F) {
                            const int e = n_ent + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(L >> 32),
                                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)L, 0u));
                            Ef[wave][e] = F;
                            Eh[wave][e] = (uint8_t)(((pp + r) << 6) | lane);
                        }
                        n_ent += __popcll(L);
                    }
                }
                if (resp && (st & kRowExists)) {
                    const int64_t kp = row0 + rbase + wr;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) resp[kp * n_bits + chunk * 64 + lp_bit(nt, g, i)] = -z[nt][i];
                }
                if (!chunk_safe || !(st & kRowSafe)) {
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) z[nt][i] = fminf(z[nt][i], 0.0f);
                }
                uint32_t X = 0;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    // byte i = sign of z[nt][i] spread over the byte (selectors 9 and 11)
                    const uint32_t pa = __builtin_amdgcn_perm(__float_as_uint(z[nt][1]), __float_as_uint(z[nt][0]), 0x0c0c0b09u);
                    const uint32_t pb = __builtin_amdgcn_perm(__float_as_uint(z[nt][3]), __float_as_uint(z[nt][2]), 0x0b090c0cu);
                    X |= (pa | pb) & msk[nt];
                }
                const uint32_t half = X | (uint32_t)__shfl_xor((int)X, 16, kWave);
                if (!(g & 1)) Ww32[2 * wr + (g >> 1)] = half;
            }
        }

        // 3. re-check the listed entries, then the code words out
        if (n_ent > 0) flush_now(n_ent, row0, A32b);
        write_words(row0, lane < kWaveRows ? Ast[buf][rbase + lane] : 0u);
    }
    // each lane counted the responses of the entries it expanded
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) rechecked += (uint32_t)__shfl_xor((int)rechecked, off, kWave);
    if (recheck_count && lane == 0 && rechecked) atomicAdd(recheck_count, rechecked);
}

}  // namespace

void launch_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                          const bd_keypoint* kps, int32_t n_kp, const int32_t* order, float* hist,
                          unsigned long long* invalid, hipStream_t stream)
{
    const int blocks = xcd_grid((n_kp + kHistWaves - 1) / kHistWaves);
    const uint8_t* p = static_cast<const uint8_t*>(img);
    if (dtype == BD_DTYPE_U8)
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_U8>, dim3(blocks), dim3(kHistWaves * kWave), 0, stream,
                           p, W, H, img_pitch, kps, n_kp, order, hist, invalid);
    else if (dtype == BD_DTYPE_F32_ROWPAIR)
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_F32_ROWPAIR>, dim3(blocks), dim3(kHistWaves * kWave), 0,
                           stream, p, W, H, img_pitch, kps, n_kp, order, hist, invalid);
    else
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_F32>, dim3(blocks), dim3(kHistWaves * kWave), 0,
                           stream, p, W, H, img_pitch, kps, n_kp, order, hist, invalid);
}

void launch_hashsift_hist_batch(const BatchImage* imgs, int32_t n_img, int32_t dtypes, const int32_t* pre,
                                const bd_keypoint* kps, const int32_t* order, float* hist, int grid,
                                unsigned long long* invalid, hipStream_t stream)
{
    const dim3 block(kHistWaves * kWave);
    if (dtypes == (1 << BD_DTYPE_U8))
        hipLaunchKernelGGL(hashsift_hist_batch<BD_DTYPE_U8>, dim3(grid), block, 0, stream, imgs, n_img, pre, kps,
                           order, hist, invalid);
    else if (dtypes == (1 << BD_DTYPE_F32))
        hipLaunchKernelGGL(hashsift_hist_batch<BD_DTYPE_F32>, dim3(grid), block, 0, stream, imgs, n_img, pre, kps,
                           order, hist, invalid);
    else
        hipLaunchKernelGGL(hashsift_hist_batch<kMixedDtypes>, dim3(grid), block, 0, stream, imgs, n_img, pre, kps,
                           order, hist, invalid);
}

void launch_hashsift_patch_features(const float* patches, int32_t n, float* hist, hipStream_t stream)
{
    hipLaunchKernelGGL(hashsift_patch_kernel, dim3((n + kHistWaves - 1) / kHistWaves), dim3(kHistWaves * kWave), 0,
                       stream, patches, n, hist);
}

void launch_hashsift_project(int32_t precision, const float* hist, const bd_keypoint* kps, int32_t n_kp,
                             const float* B, const float* t, int32_t n_words, float margin, uint64_t* codes,
                             float* resp, uint32_t* recheck_count, hipStream_t stream)
{
    // groups of n_words blocks per XCD: enough to cover the XCD's tiles, at
    // most what two resident blocks per CU allow
    const int n_tiles = (n_kp + kProjTile - 1) / kProjTile;
    const int tiles_per_xcd = (n_tiles + kXcds - 1) / kXcds;
    int groups = (kProjBlocksPerCu * 256 / kXcds) / n_words;
    if (groups > tiles_per_xcd) groups = tiles_per_xcd;
    if (groups < 1) groups = 1;
    const dim3 grid(kXcds * n_words * groups);
    const dim3 block(kProjWaves * kWave);
    if (precision == BD_PREC_BF16 || precision == BD_PREC_FP8) {
        // tile-shared kernel: one block per CU at most, grid stride over the tiles
        const int lp_grid = n_tiles < 256 ? n_tiles : 256;
        const dim3 lp_block(kLpThreads);
        if (precision == BD_PREC_BF16 && n_words == 8)
            hipLaunchKernelGGL((hashsift_project_lowp_kernel<BD_PREC_BF16, 8>), dim3(lp_grid), lp_block, 0, stream,
                               hist, kps, n_kp, B, t, margin, codes, resp, recheck_count);
        else if (precision == BD_PREC_BF16)
            hipLaunchKernelGGL((hashsift_project_lowp_kernel<BD_PREC_BF16, 4>), dim3(lp_grid), lp_block, 0, stream,
                               hist, kps, n_kp, B, t, margin, codes, resp, recheck_count);
        else if (n_words == 8)
            hipLaunchKernelGGL((hashsift_project_lowp_kernel<BD_PREC_FP8, 8>), dim3(lp_grid), lp_block, 0, stream,
                               hist, kps, n_kp, B, t, margin, codes, resp, recheck_count);
        else
            hipLaunchKernelGGL((hashsift_project_lowp_kernel<BD_PREC_FP8, 4>), dim3(lp_grid), lp_block, 0, stream,
                               hist, kps, n_kp, B, t, margin, codes, resp, recheck_count);
        return;
    }
    hipLaunchKernelGGL(hashsift_project_kernel, grid, block, 0, stream, hist, kps, n_kp, B, t, n_words, codes, resp);
}

}  // namespace bd
