// HashSIFT (Sec. III-B): SIFT features f of the normalized 32x32 patch,
// then D = sgn(B [f; 1]) with the last column of B written as -t.
//
// hashsift_hist: one wavefront per keypoint, in the caller's spatial order
// (optional) with an XCD-aware block mapping so an XCD's samples stay within
// one image region.
//   1. 34x34 bilinear samples of the rotated, scaled patch (positions in
//      FP64, clamp-to-edge, nested linear interpolation so flat regions give
//      exactly zero gradients) go to LDS, stored relative to the pixel under
//      the keypoint so small gradients in near-flat patches keep their
//      relative precision in FP32.
//   2. Lane (h, j) owns patch column j and 16 rows (rows 0..15 top-down for
//      h = 0, rows 31..16 bottom-up for h = 1).  With the bottom-up order the
//      vertical cell weights and Gaussian row weights of step k are the same
//      compile-time constants for both halves, so each pixel's vote is 18
//      triangular orientation weights and 16 FMAs into 3 cell rows x 8
//      orientations held in registers.  No atomics: the order of every sum is
//      fixed, so the result is deterministic.
//   3. The per-lane partial histograms go through LDS and each lane forms
//      two of the 128 bins by a fixed-order weighted sum over the columns of
//      its cell (horizontal cell weight times the column's Gaussian weight).
//   4. L2 normalization by a wavefront reduction.
//
// hashsift_project: responses r = B f - t on MFMA (FP32, or BF16 / FP8 with
// FP32 accumulation and an FP32 re-check near the threshold), 16 keypoints x
// 64 bits per wavefront, operands read from L2; the signs are packed into
// code words with 16 ballots.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kApron = 34;                 // 32 + one-pixel apron on each side
constexpr int kSamples = kApron * kApron;  // 1156
constexpr int kWaveLds = 24 * kWave;       // floats per wavefront (reduction needs 24 x 64)
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
// nodes of u = t^2 in [0, 1]; the float32 evaluation is within 2.4e-7 bins
// (1.9e-7 rad) of the exact angle.  A zero gradient gives 0.
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

// The histogram of one keypoint, computed by one wavefront with a
// kWaveLds-float LDS slice P; writes the 128 features to out.
template <int DT>
__device__ __forceinline__ void hist_one(const uint8_t* __restrict__ img, int32_t W, int32_t H, int64_t pitch,
                                         const bd_keypoint kp, float* __restrict__ out, float* P, int lane)
{
    if (!(finite_f(kp.x) && finite_f(kp.y) && finite_f(kp.scale) && finite_f(kp.angle) && kp.scale > 0.0f)) {
        out[lane] = 0.0f;
        out[lane + kWave] = 0.0f;
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

    // 1. resample the 34x34 patch.  Sample s = (i+1)*34 + (j+1) sits at patch
    // offset (j - 15.5, i - 15.5); its image position is the row origin
    // (kx - sb*uy, ky + sa*uy) plus (sa, sb) * ux, two FP64 FMAs per axis.
    // Three samples per lane are in flight at a time.
    const uint32_t upitch = (uint32_t)pitch;
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
            const int xa = min(max(xi, 0), wm1), xb = min(max(xi + 1, 0), wm1);
            const uint32_t ra = (uint32_t)min(max(yi, 0), hm1) * upitch;
            const uint32_t rb = (uint32_t)min(max(yi + 1, 0), hm1) * upitch;
            v[g][0] = pixel_at<DT>(img, ra, xa);
            v[g][1] = pixel_at<DT>(img, ra, xb);
            v[g][2] = pixel_at<DT>(img, rb, xa);
            v[g][3] = pixel_at<DT>(img, rb, xb);
        }
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            const float v00 = v[g][0] - base, v01 = v[g][1] - base;
            const float v10 = v[g][2] - base, v11 = v[g][3] - base;
            const float top = v00 + fxs[g] * (v01 - v00);
            const float bot = v10 + fxs[g] * (v11 - v10);
            if (sidx[g] < kSamples) P[sidx[g]] = top + fys[g] * (bot - top);
        }
    }
    wave_sync();

    // 2. gradients and votes
    const int j = lane & 31, half = lane >> 5;
    float acc[3][8];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[s][o] = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = half ? 31 - k : k;
        const int c = (i + 1) * kApron + (j + 1);
        const float gx = P[c + 1] - P[c - 1];
        const float gy = P[c + kApron] - P[c - kApron];
        const float m = __builtin_amdgcn_sqrtf(gx * gx + gy * gy);
        const float bo = orientation_bin(gx, gy);
        float tri[8];
#pragma unroll
        for (int o = 0; o < 8; ++o) tri[o] = fmaxf(0.0f, 1.0f - fabsf(bo - (float)o));
        tri[0] += fmaxf(0.0f, 1.0f - fabsf(bo - 8.0f));
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            if (slot_active(k, s)) {
                const float w = m * kRow.v[k][s];
#pragma unroll
                for (int o = 0; o < 8; ++o) acc[s][o] += w * tri[o];
            }
        }
    }
    wave_sync();

    // 3. cross-lane reduction through LDS: element e = slot*8 + o of lane l at e*64 + l
    const float gxj = kGauss.v[j];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int o = 0; o < 8; ++o) P[(s * 8 + o) * kWave + lane] = acc[s][o] * gxj;
    wave_sync();

    float h[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int b = lane + q * kWave;
        const int cy = b >> 5, cx = (b >> 3) & 3, o = b & 7;
        float sum = 0.0f;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int slot = hh ? 3 - cy : cy;
            if (slot > 2) continue;
            const float* src = P + (slot * 8 + o) * kWave + hh * 32;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int jj = 8 * cx - 4 + t;
                if (jj < 0 || jj > 31) continue;
                const float wx = fmaxf(0.0f, 1.0f - fabsf(((float)jj + 0.5f) * 0.125f - 0.5f - (float)cx));
                sum += wx * src[jj];
            }
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
                                                            float* __restrict__ hist)
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
    hist_one<DT>(img, W, H, pitch, kps[n], hist + (int64_t)n * 128, smem[wave], lane);
}

// Batch: units are blocks of four keypoints of every image in turn (pre is
// the prefix of ceil(n_kp / 4)); order entries are image-local; features are
// written to the flat array at the keypoint's global index.
__global__ __launch_bounds__(256) void hashsift_hist_batch(const BatchImage* __restrict__ imgs, int32_t n_img,
                                                           const int32_t* __restrict__ pre,
                                                           const bd_keypoint* __restrict__ kps,
                                                           const int32_t* __restrict__ order, float* __restrict__ hist)
{
    __shared__ float smem[kHistWaves][kWaveLds];
    const int lane = threadIdx.x % kWave;
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
        if (im.hs_dtype == BD_DTYPE_U8)
            hist_one<BD_DTYPE_U8>(im.img_hs, im.W, im.H, im.pitch_hs, kps[g], hist + (int64_t)g * 128, smem[wave], lane);
        else
            hist_one<BD_DTYPE_F32>(im.img_hs, im.W, im.H, im.pitch_hs, kps[g], hist + (int64_t)g * 128, smem[wave],
                                   lane);
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
    hist_one<BD_DTYPE_F32>(reinterpret_cast<const uint8_t*>(patches + (int64_t)i * 1024), 32, 32, 128, kp,
                           hist + (int64_t)i * 128, smem[wave], lane);
}

// ---------------------------------------------------------------- projection

constexpr int kProjKp = 16;      // keypoints per block (one MFMA row tile)
constexpr int kProjChunks = 4;   // 64-bit chunks per block, one per wavefront

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Largest |value| of a 128-float row held as 32 floats by each of the four
// lanes m, m+16, m+32, m+48.
__device__ __forceinline__ float row_maxabs(const float (&v)[32])
{
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < 32; ++i) m = fmaxf(m, fabsf(v[i]));
    m = fmaxf(m, __shfl_xor(m, 16, kWave));
    m = fmaxf(m, __shfl_xor(m, 32, kWave));
    return m;
}

// float8 e4m3 scale of a row: max|row| / 448 (1 for an all-zero row).
__device__ __forceinline__ float e4m3_scale(float maxabs) { return maxabs > 0.0f ? maxabs / 448.0f : 1.0f; }

// Eight consecutive values (starting at v[8s]) scaled by 1/scale, rounded to
// e4m3 (round to nearest even) and packed into 64 bits.
__device__ __forceinline__ long pack_e4m3(const float (&v)[32], int s, float scale)
{
    int lo = 0, hi = 0;
    float q[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) q[e] = fminf(fmaxf(v[8 * s + e] / scale, -448.0f), 448.0f);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(q[0], q[1], lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(q[2], q[3], lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(q[4], q[5], hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(q[6], q[7], hi, true);
    return (long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ bf16x8 pack_bf16(const float (&v)[32], int s)
{
    bf16x8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (__bf16)v[8 * s + e];
    return r;
}

// Wavefront-cooperative FP32 re-check of one (keypoint, bit) response from
// the unrounded operands: lane l multiplies elements 2l and 2l+1, and the 64
// partial sums are added by a fixed xor tree.  When that FP32 value is within
// 1e-6 of the threshold the same sum is redone in FP64.  Called by the whole
// wavefront with uniform arguments; every lane returns the response.
__device__ __forceinline__ float wave_dot_tree(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}
__device__ __forceinline__ double wave_dot_tree64(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <int N>
__device__ __forceinline__ void recheck_batch(const float* __restrict__ hist, const float* __restrict__ B,
                                              const float* __restrict__ t, const int (&kp)[N], const int (&bit)[N],
                                              int lane, float (&r)[N])
{
    float2 fv[N], bv[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        fv[c] = reinterpret_cast<const float2*>(hist + (int64_t)kp[c] * 128)[lane];
        bv[c] = reinterpret_cast<const float2*>(B + (int64_t)bit[c] * 128)[lane];
    }
#pragma unroll
    for (int c = 0; c < N; ++c) {
        r[c] = wave_dot_tree(fmaf(fv[c].y, bv[c].y, fv[c].x * bv[c].x)) - t[bit[c]];
        if (fabsf(r[c]) < 1e-6f) {
            const double p = (double)fv[c].x * (double)bv[c].x + (double)fv[c].y * (double)bv[c].y;
            r[c] = (float)(wave_dot_tree64(p) - (double)t[bit[c]]);
        }
    }
}

// grid = (ceil(n_kp / 16), ceil(n_words / 4)); wavefront w of a block computes
// the 64 responses of chunk blockIdx.y*4 + w for the block's 16 keypoints.
// Operands come straight from L2 (B is 128 or 256 KiB and shared by every
// block); lane (g, m) holds features 32g..32g+31 of keypoint row m and of
// B row m of each 16-bit subtile, so the k order of the MFMA chain is a
// permutation applied identically to both operands.
//   PREC = FP32: v_mfma_f32_16x16x4_f32, 32 steps per subtile.
//   PREC = BF16: operands rounded to bfloat16, v_mfma_f32_16x16x32_bf16.
//   PREC = FP8:  operands scaled per row (max|row| / 448) and rounded to
//                OCP e4m3, v_mfma_f32_16x16x32_fp8_fp8, response rescaled.
// With BF16/FP8 every response within `margin` of its threshold is
// recomputed from the unrounded operands (recheck_response) and counted.
template <int PREC>
__global__ __launch_bounds__(256) void hashsift_project_kernel(const float* __restrict__ hist,
                                                              const bd_keypoint* __restrict__ kps, int32_t n_kp,
                                                              const float* __restrict__ B,
                                                              const float* __restrict__ t, int32_t n_words,
                                                              float margin, uint64_t* __restrict__ codes,
                                                              float* __restrict__ resp,
                                                              uint32_t* __restrict__ recheck_count)
{
    const int lane = threadIdx.x % kWave;
    const int chunk = blockIdx.y * kProjChunks + threadIdx.x / kWave;
    if (chunk >= n_words) return;
    const int g = lane >> 4, m = lane & 15;
    const int kp0 = blockIdx.x * kProjKp;
    const int n_bits = n_words * 64;

    float a[32];
    {
        const int row = kp0 + m;
        if (row < n_kp) {
            const float4* src = reinterpret_cast<const float4*>(hist + (int64_t)row * 128 + 32 * g);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 v = src[q];
                a[4 * q] = v.x;
                a[4 * q + 1] = v.y;
                a[4 * q + 2] = v.z;
                a[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 32; ++q) a[q] = 0.0f;
        }
    }
    float b[4][32];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float4* brow = reinterpret_cast<const float4*>(B + (int64_t)(chunk * 64 + 16 * nt + m) * 128 + 32 * g);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float4 v = brow[q];
            b[nt][4 * q] = v.x;
            b[nt][4 * q + 1] = v.y;
            b[nt][4 * q + 2] = v.z;
            b[nt][4 * q + 3] = v.w;
        }
    }

    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float scale[4][4];  // per (subtile, register): factor applied to the accumulator
    if constexpr (PREC == BD_PREC_FP32) {
#pragma unroll
        for (int k = 0; k < 32; ++k)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[k], b[nt][k], acc[nt], 0, 0, 0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) scale[nt][i] = 1.0f;
    } else if constexpr (PREC == BD_PREC_BF16) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x8 av = pack_bf16(a, s);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, pack_bf16(b[nt], s), acc[nt], 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) scale[nt][i] = 1.0f;
    } else {
        const float sa = e4m3_scale(row_maxabs(a));  // scale of keypoint row m
        float sb[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) sb[nt] = e4m3_scale(row_maxabs(b[nt]));  // scale of B row 16nt + m
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const long av = pack_e4m3(a, s, sa);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, pack_e4m3(b[nt], s, sb[nt]), acc[nt], 0, 0, 0);
        }
        // the accumulator of register i belongs to keypoint row 4g + i, whose
        // scale lane 4g + i computed
        float sk[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) sk[i] = __shfl(sa, 4 * g + i, kWave);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) scale[nt][i] = sk[i] * sb[nt];
    }

    // lane holds D[kp = 4g + i][bit = m] of each 16-bit subtile nt
    float rv[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float tv = t[chunk * 64 + 16 * nt + m];
#pragma unroll
        for (int i = 0; i < 4; ++i) rv[nt][i] = acc[nt][i] * scale[nt][i] - tv;
    }
    if constexpr (PREC != BD_PREC_FP32) {
        // responses within the margin: the wavefront recomputes them one after
        // another (four candidates' operands in flight at a time)
        uint32_t rechecked = 0;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool need = fabsf(rv[nt][i]) < margin && kp0 + 4 * g + i < n_kp;
                uint64_t cand = __ballot(need);
                rechecked += (uint32_t)__popcll(cand);
                while (cand) {
                    constexpr int kB = 4;
                    int ln[kB], kp[kB], bit[kB];
                    int cnt = 0;
#pragma unroll
                    for (int c = 0; c < kB; ++c) {
                        const int L = cand ? (int)__builtin_ctzll(cand) : -1;
                        if (cand) cand &= cand - 1;
                        ln[c] = L;
                        const int Ls = L >= 0 ? L : ln[0];
                        kp[c] = kp0 + 4 * (Ls >> 4) + i;
                        bit[c] = chunk * 64 + 16 * nt + (Ls & 15);
                        cnt += L >= 0;
                    }
                    float r[kB];
                    recheck_batch<kB>(hist, B, t, kp, bit, lane, r);
#pragma unroll
                    for (int c = 0; c < kB; ++c)
                        if (c < cnt && lane == ln[c]) rv[nt][i] = r[c];
                }
            }
        }
        if (recheck_count && lane == 0 && rechecked) atomicAdd(recheck_count, rechecked);
    }
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
                valid = finite_f(k.x) && finite_f(k.y) && finite_f(k.scale) && finite_f(k.angle) && k.scale > 0.0f;
            }
            const int gq = lane >> 2, iq = lane & 3;
            uint64_t word = 0ull;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const uint64_t mk = iq == 0 ? mask[nt][0] : iq == 1 ? mask[nt][1] : iq == 2 ? mask[nt][2] : mask[nt][3];
                word |= ((mk >> (16 * gq)) & 0xffffull) << (16 * nt);
            }
            codes[(int64_t)kp * n_words + chunk] = valid ? word : 0ull;
        }
    }
}

}  // namespace

void launch_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                          const bd_keypoint* kps, int32_t n_kp, const int32_t* order, float* hist,
                          hipStream_t stream)
{
    const int blocks = xcd_grid((n_kp + kHistWaves - 1) / kHistWaves);
    const uint8_t* p = static_cast<const uint8_t*>(img);
    if (dtype == BD_DTYPE_U8)
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_U8>, dim3(blocks), dim3(kHistWaves * kWave), 0, stream,
                           p, W, H, img_pitch, kps, n_kp, order, hist);
    else
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_F32>, dim3(blocks), dim3(kHistWaves * kWave), 0,
                           stream, p, W, H, img_pitch, kps, n_kp, order, hist);
}

void launch_hashsift_hist_batch(const BatchImage* imgs, int32_t n_img, const int32_t* pre, const bd_keypoint* kps,
                                const int32_t* order, float* hist, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL(hashsift_hist_batch, dim3(grid), dim3(kHistWaves * kWave), 0, stream, imgs, n_img, pre, kps,
                       order, hist);
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
    const dim3 grid((n_kp + kProjKp - 1) / kProjKp, (n_words + kProjChunks - 1) / kProjChunks);
    const dim3 block(kProjChunks * kWave);
    if (precision == BD_PREC_BF16)
        hipLaunchKernelGGL(hashsift_project_kernel<BD_PREC_BF16>, grid, block, 0, stream, hist, kps, n_kp, B, t,
                           n_words, margin, codes, resp, recheck_count);
    else if (precision == BD_PREC_FP8)
        hipLaunchKernelGGL(hashsift_project_kernel<BD_PREC_FP8>, grid, block, 0, stream, hist, kps, n_kp, B, t,
                           n_words, margin, codes, resp, recheck_count);
    else
        hipLaunchKernelGGL(hashsift_project_kernel<BD_PREC_FP32>, grid, block, 0, stream, hist, kps, n_kp, B, t,
                           n_words, margin, codes, resp, recheck_count);
}

}  // namespace bd
