// HashSIFT (Sec. III-B): SIFT features f of the normalized 32x32 patch,
// then D = sgn(B [f; 1]) with the last column of B written as -t.
//
// hashsift_hist: one wavefront per keypoint.
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
// hashsift_project_fp32: responses r = B f - t on FP32 MFMA
// (v_mfma_f32_16x16x4_f32), 16 keypoints x 64 bits per wavefront step, B
// staged through LDS one 64-bit chunk at a time; the signs are packed into
// code words with 16 ballots per chunk.
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

__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <int DT>
__global__ __launch_bounds__(256) void hashsift_hist_kernel(const uint8_t* __restrict__ img, int32_t W,
                                                            int32_t H, int64_t pitch,
                                                            const bd_keypoint* __restrict__ kps,
                                                            int32_t n_kp, float* __restrict__ hist)
{
    __shared__ float smem[kHistWaves][kWaveLds];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int n = blockIdx.x * kHistWaves + wave;
    if (n >= n_kp) return;
    float* P = smem[wave];
    float* out = hist + (int64_t)n * 128;

    const bd_keypoint kp = kps[n];
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

    // 1. resample the 34x34 patch
    for (int s = lane; s < kSamples; s += kWave) {
        const int i = s / kApron - 1, j = s % kApron - 1;
        const double ux = j - 15.5, uy = i - 15.5;
        const double px = kx + (sa * ux - sb * uy);
        const double py = ky + (sb * ux + sa * uy);
        const double x0 = floor(px), y0 = floor(py);
        const float fx = (float)(px - x0), fy = (float)(py - y0);
        const int xa = (int)fmin(fmax(x0, 0.0), (double)(W - 1));
        const int xb = (int)fmin(fmax(x0 + 1.0, 0.0), (double)(W - 1));
        const int ya = (int)fmin(fmax(y0, 0.0), (double)(H - 1));
        const int yb = (int)fmin(fmax(y0 + 1.0, 0.0), (double)(H - 1));
        const float v00 = pixel<DT>(img, pitch, xa, ya) - base;
        const float v01 = pixel<DT>(img, pitch, xb, ya) - base;
        const float v10 = pixel<DT>(img, pitch, xa, yb) - base;
        const float v11 = pixel<DT>(img, pitch, xb, yb) - base;
        const float top = v00 + fx * (v01 - v00);
        const float bot = v10 + fx * (v11 - v10);
        P[s] = top + fy * (bot - top);
    }
    wave_sync();

    // 2. gradients and votes
    const int j = lane & 31, half = lane >> 5;
    float acc[3][8];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int o = 0; o < 8; ++o) acc[s][o] = 0.0f;
    constexpr float kBinScale = (float)(8.0 / (2.0 * 3.14159265358979323846));
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = half ? 31 - k : k;
        const int c = (i + 1) * kApron + (j + 1);
        const float gx = P[c + 1] - P[c - 1];
        const float gy = P[c + kApron] - P[c - kApron];
        const float m = sqrtf(gx * gx + gy * gy);
        float bo = atan2f(gy, gx) * kBinScale;
        if (bo < 0.0f) bo += 8.0f;
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

// ---------------------------------------------------------------- projection

constexpr int kProjKp = 64;          // keypoints per block (16 per wavefront)
constexpr int kBStride = 132;        // padded LDS row of B (floats)

typedef float floatx4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void hashsift_project_fp32_kernel(const float* __restrict__ hist,
                                                                   const bd_keypoint* __restrict__ kps,
                                                                   int32_t n_kp, const float* __restrict__ B,
                                                                   const float* __restrict__ t,
                                                                   int32_t n_words,
                                                                   uint64_t* __restrict__ codes,
                                                                   float* __restrict__ resp)
{
    __shared__ float Bs[64 * kBStride];
    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    const int g = lane >> 4, m = lane & 15;
    const int wave_kp = blockIdx.x * kProjKp + wave * 16;
    const int n_bits = n_words * 64;

    // A operand: row m of this wavefront's 16 keypoints, features 32g .. 32g+31
    float a[32];
    {
        const int row = wave_kp + m;
        if (row < n_kp) {
            const float4* src = reinterpret_cast<const float4*>(hist + (int64_t)row * 128 + 32 * g);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                float4 v = src[q];
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
    // validity of the keypoint whose word this lane stores (lanes 0..15)
    bool valid = false;
    if (lane < 16 && wave_kp + lane < n_kp) {
        valid = true;
        if (kps) {
            const bd_keypoint kp = kps[wave_kp + lane];
            valid = finite_f(kp.x) && finite_f(kp.y) && finite_f(kp.scale) && finite_f(kp.angle) && kp.scale > 0.0f;
        }
    }

    for (int chunk = 0; chunk < n_words; ++chunk) {
        __syncthreads();
        {
            const float4* src = reinterpret_cast<const float4*>(B + (int64_t)chunk * 64 * 128);
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int e = threadIdx.x + 256 * r;  // float4 index within the 64 x 128 chunk
                const int row = e >> 5, col = (e & 31) * 4;
                *reinterpret_cast<float4*>(&Bs[row * kBStride + col]) = src[e];
            }
        }
        __syncthreads();

        floatx4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            const float* brow = &Bs[(16 * nt + m) * kBStride + 32 * g];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 b = *reinterpret_cast<const float4*>(brow + 4 * q);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * q], b.x, acc[nt], 0, 0, 0);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * q + 1], b.y, acc[nt], 0, 0, 0);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * q + 2], b.z, acc[nt], 0, 0, 0);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[4 * q + 3], b.w, acc[nt], 0, 0, 0);
            }
        }

        // lane holds D[kp = 4g + i][bit = m] of each 16-bit subtile nt
        uint64_t mask[4][4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int bit = chunk * 64 + 16 * nt + m;
            const float tv = t[bit];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float r = acc[nt][i] - tv;
                if (resp) {
                    const int kp = wave_kp + 4 * g + i;
                    if (kp < n_kp) resp[(int64_t)kp * n_bits + bit] = r;
                }
                mask[nt][i] = __ballot(r > 0.0f);
            }
        }
        if (lane < 16) {
            const int gq = lane >> 2, iq = lane & 3;
            uint64_t word = 0ull;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const uint64_t mk = iq == 0 ? mask[nt][0] : iq == 1 ? mask[nt][1] : iq == 2 ? mask[nt][2] : mask[nt][3];
                word |= ((mk >> (16 * gq)) & 0xffffull) << (16 * nt);
            }
            const int kp = wave_kp + lane;
            if (kp < n_kp) codes[(int64_t)kp * n_words + chunk] = valid ? word : 0ull;
        }
    }
}

}  // namespace

void launch_hashsift_hist(const void* img, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch,
                          const bd_keypoint* kps, int32_t n_kp, float* hist, hipStream_t stream)
{
    const int blocks = (n_kp + kHistWaves - 1) / kHistWaves;
    const uint8_t* p = static_cast<const uint8_t*>(img);
    if (dtype == BD_DTYPE_U8)
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_U8>, dim3(blocks), dim3(kHistWaves * kWave), 0, stream,
                           p, W, H, img_pitch, kps, n_kp, hist);
    else
        hipLaunchKernelGGL(hashsift_hist_kernel<BD_DTYPE_F32>, dim3(blocks), dim3(kHistWaves * kWave), 0,
                           stream, p, W, H, img_pitch, kps, n_kp, hist);
}

void launch_hashsift_project_fp32(const float* hist, const bd_keypoint* kps, int32_t n_kp, const float* B,
                                  const float* t, int32_t n_words, uint64_t* codes, float* resp,
                                  hipStream_t stream)
{
    const int blocks = (n_kp + kProjKp - 1) / kProjKp;
    hipLaunchKernelGGL(hashsift_project_fp32_kernel, dim3(blocks), dim3(256), 0, stream, hist, kps, n_kp, B, t,
                       n_words, codes, resp);
}

}  // namespace bd
