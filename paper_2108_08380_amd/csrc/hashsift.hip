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

// The four corner pixels and weights of the sample at fixed-point image
// position (X, Y).  Row offsets use 24-bit multiplies: the host admits only
// images with pitch < 2^24, H < 2^24 and pitch * H <= 2^32.
template <int DT>
__device__ __forceinline__ void fetch_fixed(const uint8_t* __restrict__ img, int wm1, int hm1, uint32_t upitch,
                                            int64_t X, int64_t Y, float (&v)[4], float& fx, float& fy)
{
    const int xi = (int)(X >> 32), yi = (int)(Y >> 32);
    fx = (float)(uint32_t)X * 0x1p-32f;
    fy = (float)(uint32_t)Y * 0x1p-32f;
    const int xa = clampi(xi, wm1), xb = clampi(xi + 1, wm1);
    const uint32_t ra = __umul24((uint32_t)clampi(yi, hm1), upitch);
    const uint32_t rb = __umul24((uint32_t)clampi(yi + 1, hm1), upitch);
    v[0] = pixel_at<DT>(img, ra, xa);
    v[1] = pixel_at<DT>(img, ra, xb);
    v[2] = pixel_at<DT>(img, rb, xa);
    v[3] = pixel_at<DT>(img, rb, xb);
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
template <int DT, int R>
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
            fetch_fixed<DT>(img, wm1, hm1, upitch, X, Y, v[g], fx[g], fy[g]);
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
        fetch_fixed<DT>(img, wm1, hm1, upitch, X, Y, v[g], fx[g], fy[g]);
        advance(g);
    }
    const double ar = h ? 16.5 : -16.5, ac = (double)c - 15.5;
    fetch_fixed<DT>(img, wm1, hm1, upitch, to_fixed(fma(sa, ac, fma(-sb, ar, kx))),
                    to_fixed(fma(sb, ac, fma(sa, ar, ky))), v[R], fx[R], fy[R]);
    fetch_fixed<DT>(img, wm1, hm1, upitch, to_fixed(fma(sa, ar, fma(-sb, ac, kx))),
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
        resample_fixed<DT, R>(img, W, H, (uint32_t)pitch, kx, ky, sa, sb, base, P, lane);
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
// dtype of every image's HashSIFT source, or kMixedDtypes.  The u8 form runs
// at 5 waves per SIMD, as LDS allows; the others need more registers (4).
constexpr int kMixedDtypes = -1;

template <int DT>
__global__ __launch_bounds__(256, DT == BD_DTYPE_U8 ? 5 : 4) void hashsift_hist_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
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
// (grid stride).  A tile is read from HBM once, kept in LDS as FP32 (for the
// re-check) and as the MFMA operand type, and shared by all eight
// wavefronts: wavefront w owns the 64-bit chunk w % NW of B and the tile rows
// (w / NW) * 16 * kRowSubs onwards.  The chunk's B operands stay in
// registers for the whole kernel (lane (g, n) holds row 16 nt + n, elements
// 32 s + 8 g .. + 7 of k-step s), rounded once; the next tile's rows are in
// flight while the current one is multiplied (v_mfma_f32_16x16x32_bf16 /
// _fp8_fp8, FP32 accumulation).  With FP8 every row of the tile and of B is
// scaled by a power of two s (the smallest with max|row| <= 448 s, at least
// 2^-126), so the rescaling is exact; the response is acc * s_row * s_b - t.
//
// The sign bits are gathered by ballots into the tile's code words in LDS.
// Responses within `margin` of the threshold are then queued per wavefront
// in LDS (row, column) and re-checked one per lane from the unrounded FP32
// operands (the tile row from LDS, the row of B from memory): four chains
// over the elements k mod 4, summed as (c0 + c1) + (c2 + c3), then FP64 when
// that result is within 1e-6 of the threshold.  The re-checking lane sets or
// clears its code bit in LDS and overwrites the response; the words are
// written out last.
constexpr int kLpRows = 64;       // keypoints per tile
constexpr int kLpThreads = 512;   // eight wavefronts
constexpr int kLpS32 = 132;       // FP32 tile row stride (floats)
constexpr int kLpS16 = 136;       // BF16 tile row stride (elements, 272 bytes)
constexpr int kLpS8 = 144;        // FP8 tile row stride (bytes)

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

// Eight values times 2^-e (exact), rounded to e4m3, packed into 64 bits.
__device__ __forceinline__ long pack_e4m3_pow2(const float (&v)[8], int e)
{
    float q[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = fminf(fmaxf(__builtin_amdgcn_ldexpf(v[i], -e), -448.0f), 448.0f);
    int lo = 0, hi = 0;
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(q[4], q[5], hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(q[6], q[7], hi, true);
    return (long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
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

template <int PREC, int NW>
__global__ __launch_bounds__(kLpThreads, 1) void hashsift_project_lowp_kernel(
    const float* __restrict__ hist, const bd_keypoint* __restrict__ kps, int32_t n_kp, const float* __restrict__ B,
    const float* __restrict__ t, float margin, uint64_t* __restrict__ codes, float* __restrict__ resp,
    uint32_t* __restrict__ recheck_count)
{
    constexpr int kRowSubs = NW == 8 ? 4 : 2;   // 16-row subtiles per wavefront
    constexpr int kWaveRows = 16 * kRowSubs;    // tile rows of a wavefront
    constexpr int kQueue = kWaveRows * 64;      // every response of a wavefront can be queued
    constexpr int kRowBytes = LpOperand<PREC>::row_bytes;
    typedef typename LpOperand<PREC>::type op_t;
    __shared__ __align__(16) float A32[kLpRows * kLpS32];
    __shared__ __align__(16) uint8_t Alp[kLpRows * kRowBytes];
    __shared__ float Asc[kLpRows];
    __shared__ uint64_t W[2][kLpThreads / kWave][kWaveRows];  // by tile parity
    __shared__ uint16_t Q[kLpThreads / kWave][kQueue + kWave];  // + a slot per lane for writes that drop

    const int tid = (int)threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    const int g = lane >> 4, n = lane & 15;
    const int chunk = wave % NW;
    const int rbase = (wave / NW) * kWaveRows;
    constexpr int n_bits = NW * 64;
    uint16_t* Qw = Q[wave];

    // B operands of this lane: rows 64 chunk + 16 nt + n, elements 32 s + 8 g .. + 7
    op_t bop[4][4];
    float tv[4], sb[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float* brow = B + (int64_t)(chunk * 64 + 16 * nt + n) * 128;
        float v[4][8];
        float mx = 0.0f;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float4 lo = *reinterpret_cast<const float4*>(brow + 32 * s + 8 * g);
            const float4 hi = *reinterpret_cast<const float4*>(brow + 32 * s + 8 * g + 4);
            v[s][0] = lo.x, v[s][1] = lo.y, v[s][2] = lo.z, v[s][3] = lo.w;
            v[s][4] = hi.x, v[s][5] = hi.y, v[s][6] = hi.z, v[s][7] = hi.w;
#pragma unroll
            for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(v[s][e]));
        }
        tv[nt] = t[chunk * 64 + 16 * nt + n];
        sb[nt] = 1.0f;
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
            sb[nt] = __builtin_amdgcn_ldexpf(1.0f, e);
#pragma unroll
            for (int s = 0; s < 4; ++s) bop[nt][s] = pack_e4m3_pow2(v[s], e);
        }
    }

    // staging: thread tid moves row tid / 8, elements 16 (tid % 8) .. + 15
    const int prow = tid >> 3, pcol = (tid & 7) * 16;
    const int n_tiles = (n_kp + kLpRows - 1) / kLpRows;
    float4 pf[4];
    auto load_tile = [&](int tile) {
        const int row = tile * kLpRows + prow;
        if (row < n_kp) {
            const float4* src = reinterpret_cast<const float4*>(hist + (int64_t)row * 128 + pcol);
#pragma unroll
            for (int q = 0; q < 4; ++q) pf[q] = src[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) pf[q] = float4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    if ((int)blockIdx.x < n_tiles) load_tile((int)blockIdx.x);
    uint32_t rechecked = 0;

    int parity = 0;
    for (int tile = (int)blockIdx.x; tile < n_tiles; tile += (int)gridDim.x, parity ^= 1) {
        // the barrier before the previous tile's code words went out also
        // ended every read of its rows; its words are in the other W buffer
        uint64_t* Ww = W[parity][wave];
        {
            float4* d32 = reinterpret_cast<float4*>(&A32[prow * kLpS32 + pcol]);
#pragma unroll
            for (int q = 0; q < 4; ++q) d32[q] = pf[q];
            uint8_t* dlp = &Alp[prow * kRowBytes];
            if constexpr (PREC == BD_PREC_BF16) {
                uint4 w0, w1;
                w0.x = pk_bf16(pf[0].x, pf[0].y);
                w0.y = pk_bf16(pf[0].z, pf[0].w);
                w0.z = pk_bf16(pf[1].x, pf[1].y);
                w0.w = pk_bf16(pf[1].z, pf[1].w);
                w1.x = pk_bf16(pf[2].x, pf[2].y);
                w1.y = pk_bf16(pf[2].z, pf[2].w);
                w1.z = pk_bf16(pf[3].x, pf[3].y);
                w1.w = pk_bf16(pf[3].z, pf[3].w);
                reinterpret_cast<uint4*>(dlp + 2 * pcol)[0] = w0;
                reinterpret_cast<uint4*>(dlp + 2 * pcol)[1] = w1;
            } else {
                float mx = 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    mx = fmaxf(mx, fmaxf(fmaxf(fabsf(pf[q].x), fabsf(pf[q].y)), fmaxf(fabsf(pf[q].z), fabsf(pf[q].w))));
                mx = max8_dpp(mx);
                const int e = e4m3_pow2_exp(mx);
                if ((tid & 7) == 0) Asc[prow] = __builtin_amdgcn_ldexpf(1.0f, e);
                const float v0[8] = {pf[0].x, pf[0].y, pf[0].z, pf[0].w, pf[1].x, pf[1].y, pf[1].z, pf[1].w};
                const float v1[8] = {pf[2].x, pf[2].y, pf[2].z, pf[2].w, pf[3].x, pf[3].y, pf[3].z, pf[3].w};
                const long q0 = pack_e4m3_pow2(v0, e), q1 = pack_e4m3_pow2(v1, e);
                *reinterpret_cast<uint4*>(dlp + pcol) =
                    uint4{(uint32_t)q0, (uint32_t)((uint64_t)q0 >> 32), (uint32_t)q1, (uint32_t)((uint64_t)q1 >> 32)};
            }
        }
        if (tile + (int)gridDim.x < n_tiles) load_tile(tile + (int)gridDim.x);
        __syncthreads();
        const int row0 = tile * kLpRows;
        const int limit = n_kp - (row0 + rbase);  // wavefront rows below this exist

        // two 16-row subtiles at a time: 1. responses (lane (g, n) holds the
        // response of wavefront row 16 p + 4 g + i to column 16 nt + n);
        // 2. responses out, sign bits into the code words, pending responses queued
        int queued = 0;
#pragma unroll
        for (int pp = 0; pp < kRowSubs; pp += 2) {
            floatx4 acc[2][4];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[r][nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                op_t av[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int row = rbase + 16 * (pp + r) + n;  // A operand: lane (g, m = n) holds row m
                    if constexpr (PREC == BD_PREC_BF16)
                        av[r] = *reinterpret_cast<const bf16x8*>(&Alp[row * kRowBytes + 2 * (32 * s + 8 * g)]);
                    else
                        av[r] = *reinterpret_cast<const long*>(&Alp[row * kRowBytes + 32 * s + 8 * g]);
                }
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        if constexpr (PREC == BD_PREC_BF16)
                            acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bop[nt][s], acc[r][nt], 0, 0, 0);
                        else
                            acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[r], bop[nt][s], acc[r][nt], 0, 0, 0);
                    }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int p = pp + r;
                float sk[4] = {1.0f, 1.0f, 1.0f, 1.0f};
                if constexpr (PREC == BD_PREC_FP8) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) sk[i] = Asc[rbase + 16 * p + 4 * g + i];
                }
                float rv[4][4];
                uint64_t mask[4][4];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        rv[nt][i] = acc[r][nt][i] * (sk[i] * sb[nt]) - tv[nt];
                        mask[nt][i] = __ballot(rv[nt][i] > 0.0f);
                    }
                if (margin > 0.0f) {
                    // all sixteen ballots first, then the (scalar) walk over the non-empty ones
                    uint64_t pend[4][4];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            pend[nt][i] = __ballot(16 * p + 4 * g + i < limit && fabsf(rv[nt][i]) < margin);
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const uint64_t pm = pend[nt][i];
                            if (pm) {
                                // queue position, or this lane's spare slot when it has nothing to queue
                                const bool hit = (pm >> lane) & 1ull;
                                const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(pm >> 32),
                                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)pm, 0u));
                                Qw[hit ? queued + rank : kQueue + lane] = (uint16_t)((16 * p + 4 * g + i) << 6 | (16 * nt + n));
                                queued += __popcll(pm);
                            }
                        }
                }
                if (resp) {
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int wr = 16 * p + 4 * g + i;
                            if (wr < limit) resp[(int64_t)(row0 + rbase + wr) * n_bits + chunk * 64 + 16 * nt + n] = rv[nt][i];
                        }
                }
                if (lane < 16) {
                    const int gq = lane >> 2, iq = lane & 3;
                    uint64_t word = 0ull;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const uint64_t mk =
                            iq == 0 ? mask[nt][0] : iq == 1 ? mask[nt][1] : iq == 2 ? mask[nt][2] : mask[nt][3];
                        word |= ((mk >> (16 * gq)) & 0xffffull) << (16 * nt);
                    }
                    Ww[16 * p + lane] = word;
                }
            }
        }
        rechecked += (uint32_t)queued;

        // 3. re-check the queued responses, one per lane
        wave_sync();
        for (int b0 = 0; b0 < queued; b0 += kWave) {
            if (b0 + lane < queued) {
                const int item = Qw[b0 + lane];
                const int wr = item >> 6, col = item & 63;
                const float* arow = &A32[(rbase + wr) * kLpS32];
                const float* brow = B + (int64_t)(chunk * 64 + col) * 128;
                const float tcol = t[chunk * 64 + col];
                // the row of B in quarters, each in flight at once
                float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f, d3 = 0.0f;
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    float4 bv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) bv[q] = reinterpret_cast<const float4*>(brow)[8 * h + q];
                    // the loads above stay ahead of the arithmetic below
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const float4 av = reinterpret_cast<const float4*>(arow)[8 * h + q];
                        d0 = fmaf(av.x, bv[q].x, d0);
                        d1 = fmaf(av.y, bv[q].y, d1);
                        d2 = fmaf(av.z, bv[q].z, d2);
                        d3 = fmaf(av.w, bv[q].w, d3);
                    }
                }
                float res = ((d0 + d1) + (d2 + d3)) - tcol;
                if (fabsf(res) < 1e-6f) {
                    double d = 0.0;
                    for (int k = 0; k < 128; ++k) d = fma((double)arow[k], (double)brow[k], d);
                    res = (float)(d - (double)tcol);
                }
                const uint64_t bit = 1ull << col;
                if (res > 0.0f)
                    __hip_atomic_fetch_or(&Ww[wr], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                else
                    __hip_atomic_fetch_and(&Ww[wr], ~bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                const int kp = row0 + rbase + wr;
                if (resp) resp[(int64_t)kp * n_bits + chunk * 64 + col] = res;
            }
        }
        __syncthreads();

        // 4. the tile's code rows out, coalesced: thread tid writes word tid % NW of row tid / NW
        if (tid < kLpRows * NW) {
            const int row = tid / NW, c = tid % NW;
            const int kp = row0 + row;
            if (kp < n_kp) {
                bool valid = true;
                if (kps) {
                    const bd_keypoint k = kps[kp];
                    valid = finite_f(k.x) && finite_f(k.y) && finite_f(k.scale) && finite_f(k.angle) && k.scale > 0.0f;
                }
                // chunk c of row `row` belongs to wavefront c + NW * (row / kWaveRows)
                codes[(int64_t)kp * NW + c] = valid ? W[parity][c + NW * (row / kWaveRows)][row % kWaveRows] : 0ull;
            }
        }
    }
    // rechecked is the wavefront's count (the same in every lane)
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
