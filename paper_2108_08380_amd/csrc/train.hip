// HashSIFT training (Sec. III-B): the projection B (with thresholds t, the
// last column of B [f; 1]) is learned by minimising the triplet ranking loss
// of the relaxed descriptors tanh(beta (B f - t)) with Adam, on batches of
// matched patch pairs whose negatives are the in-batch hardest ones (with
// anchor swap), every patch augmented by a small random rotation and scale,
// blur, illumination change and pixel noise.
//
// One training step is a fixed sequence of kernels on the caller's stream:
//   augment_kernel         2n patches (anchors, then positives) from the pool
//   hashsift_patch_kernel  their 128-d features
//   projection + tanh      relaxed descriptors of both halves (FP32 MFMA)
//   trl forward/backward   hardest negatives, loss, dL/dD
//   relaxed_hs_bwd         dL/dB, dL/dt summed over both halves
//   adam_kernel            the update of B and t
// The random draws of the augmentation are inputs.
#include <cmath>

#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kAugThreads = 256;
constexpr int kMaxBlurRadius = 12;  // sigma is clamped to 4

__device__ __forceinline__ int clamp31(int v) { return v < 0 ? 0 : (v > 31 ? 31 : v); }

// One block per output patch.  Output patch k (k < n: anchors, k >= n:
// positives) comes from pool pair batch[k mod n], anchor 2 batch + 0 or
// positive 2 batch + 1, with params / noise row 2 (k mod n) + (k >= n).
__global__ __launch_bounds__(kAugThreads) void augment_kernel(const float* __restrict__ pool, int32_t n_pairs,
                                                              const int32_t* __restrict__ batch, int32_t n,
                                                              const float* __restrict__ params,
                                                              const float* __restrict__ noise,
                                                              float* __restrict__ out)
{
    __shared__ float warp[1024];
    __shared__ float tmp[1024];
    __shared__ float w[2 * kMaxBlurRadius + 1];
    const int k = blockIdx.x, t = threadIdx.x;
    const int s = k % n, side = k / n;
    int pair = batch[s];
    pair = pair < 0 ? 0 : (pair >= n_pairs ? n_pairs - 1 : pair);  // out-of-range indices are clamped
    const float* src = pool + (int64_t)(2 * pair + side) * 1024;
    const int row = 2 * s + side;
    const float* pr = params + (int64_t)row * 5;
    double sa, ca;
    sincos((double)pr[0], &sa, &ca);
    const double sc = pr[1];
    const float gain = pr[2], bias = pr[3];
    float sigma = pr[4];
    sigma = sigma > 4.0f ? 4.0f : sigma;

    // 1. rotation and scale about the centre, bilinear with clamp-to-edge
    for (int e = t; e < 1024; e += kAugThreads) {
        const int i = e >> 5, j = e & 31;
        const double ux = j - 15.5, uy = i - 15.5;
        const double px = 15.5 + sc * (ca * ux - sa * uy);
        const double py = 15.5 + sc * (sa * ux + ca * uy);
        const double x0 = floor(px), y0 = floor(py);
        const float fx = (float)(px - x0), fy = (float)(py - y0);
        const int xi = (int)fmin(fmax(x0, -64.0), 64.0), yi = (int)fmin(fmax(y0, -64.0), 64.0);
        const int xa = clamp31(xi), xb = clamp31(xi + 1), ya = clamp31(yi), yb = clamp31(yi + 1);
        const float v00 = src[ya * 32 + xa], v01 = src[ya * 32 + xb];
        const float v10 = src[yb * 32 + xa], v11 = src[yb * 32 + xb];
        const float top = v00 + fx * (v01 - v00);
        const float bot = v10 + fx * (v11 - v10);
        warp[e] = top + fy * (bot - top);
    }
    // 2. separable Gaussian blur
    const int R = sigma > 0.0f ? (int)ceilf(3.0f * sigma) : 0;
    if (t <= 2 * R) w[t] = expf(-(float)((t - R) * (t - R)) / (2.0f * sigma * sigma));
    __syncthreads();
    if (R > 0) {
        float wsum = 0.0f;
        for (int d = 0; d <= 2 * R; ++d) wsum += w[d];
        const float inv = 1.0f / wsum;
        for (int e = t; e < 1024; e += kAugThreads) {
            const int i = e >> 5, j = e & 31;
            float acc = 0.0f;
            for (int d = -R; d <= R; ++d) acc = fmaf(w[d + R], warp[i * 32 + clamp31(j + d)], acc);
            tmp[e] = acc * inv;
        }
        __syncthreads();
        for (int e = t; e < 1024; e += kAugThreads) {
            const int i = e >> 5, j = e & 31;
            float acc = 0.0f;
            for (int d = -R; d <= R; ++d) acc = fmaf(w[d + R], tmp[clamp31(i + d) * 32 + j], acc);
            warp[e] = acc * inv;
        }
        __syncthreads();
    }
    // 3-5. illumination, noise, clipping
    const float* nz = noise + (int64_t)row * 1024;
    float* dst = out + (int64_t)k * 1024;
    for (int e = t; e < 1024; e += kAugThreads) {
        const float v = fmaf(gain, warp[e], bias) + nz[e];
        dst[e] = fminf(fmaxf(v, 0.0f), 1.0f);
    }
}

// Adam on one parameter array: g is the gradient; c1 = 1 - beta1^step,
// c2 = 1 - beta2^step.
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int32_t count,
                                                   float lr, float beta1, float beta2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void fill_one_kernel(float* p) { *p = 1.0f; }

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

size_t train_step_workspace(int32_t n, int32_t n_bits)
{
    const size_t n2 = 2 * (size_t)n, K = (size_t)n_bits;
    const size_t scratch = trl_workspace(n) > relaxed_hs_bwd_workspace(2 * n, n_bits)
                               ? trl_workspace(n)
                               : relaxed_hs_bwd_workspace(2 * n, n_bits);
    return al256(sizeof(float) * n2 * 1024) + al256(sizeof(float) * n2 * 128) + 2 * al256(sizeof(float) * n2 * K) +
           al256(sizeof(uint64_t) * n2 * (K / 64)) + al256(sizeof(float) * n2 * K) + al256(sizeof(int32_t) * n) +
           al256(sizeof(float) * n) + al256(sizeof(float) * 2) + al256(sizeof(float) * K * 129) + al256(scratch);
}

void launch_train_step(const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n, const float* params,
                       const float* noise, float* B, float* t, int32_t n_bits, float* adam_state, int32_t step,
                       float lr, float tau, float beta, float* loss, void* workspace, hipStream_t stream)
{
    const size_t n2 = 2 * (size_t)n, K = (size_t)n_bits;
    char* ws = static_cast<char*>(workspace);
    auto take = [&](size_t bytes) {
        void* p = ws;
        ws += al256(bytes);
        return p;
    };
    float* aug = static_cast<float*>(take(sizeof(float) * n2 * 1024));
    float* f = static_cast<float*>(take(sizeof(float) * n2 * 128));
    float* rho = static_cast<float*>(take(sizeof(float) * n2 * K));
    float* D = static_cast<float*>(take(sizeof(float) * n2 * K));
    uint64_t* codes = static_cast<uint64_t*>(take(sizeof(uint64_t) * n2 * (K / 64)));
    float* gD = static_cast<float*>(take(sizeof(float) * n2 * K));
    int32_t* neg = static_cast<int32_t*>(take(sizeof(int32_t) * n));
    float* hinge = static_cast<float*>(take(sizeof(float) * n));
    float* one = static_cast<float*>(take(sizeof(float) * 2));
    float* grad = static_cast<float*>(take(sizeof(float) * K * 129));  // dL/dB (K x 128), then dL/dt (K)
    void* scratch = take(0);

    hipLaunchKernelGGL(augment_kernel, dim3((int)n2), dim3(kAugThreads), 0, stream, pool, n_pairs, batch, n, params,
                       noise, aug);
    launch_hashsift_patch_features(aug, (int32_t)n2, f, stream);
    launch_hashsift_project(BD_PREC_FP32, f, nullptr, (int32_t)n2, B, t, n_bits / 64, 0.0f, codes, rho, nullptr,
                            stream);
    launch_tanh_scale(rho, (int64_t)n2 * n_bits, beta, D, stream);
    launch_trl_fwd(D, D + (size_t)n * K, n, n_bits, tau, loss, neg, hinge, scratch, stream);
    hipLaunchKernelGGL(fill_one_kernel, dim3(1), dim3(1), 0, stream, one);
    launch_trl_bwd(D, D + (size_t)n * K, n, n_bits, neg, hinge, one, gD, gD + (size_t)n * K, scratch, stream);
    launch_relaxed_hs_bwd(gD, D, f, (int32_t)n2, n_bits, beta, grad, grad + K * 128, scratch, stream);

    const double c1 = 1.0 - pow(0.9, (double)step), c2 = 1.0 - pow(0.999, (double)step);
    float* mB = adam_state;
    float* vB = mB + K * 128;
    float* mt = vB + K * 128;
    float* vt = mt + K;
    const int nB = (int)(K * 128);
    hipLaunchKernelGGL(adam_kernel, dim3((nB + 255) / 256), dim3(256), 0, stream, B, grad, mB, vB, nB, lr, 0.9f,
                       0.999f, 1e-8f, (float)c1, (float)c2);
    hipLaunchKernelGGL(adam_kernel, dim3(((int)K + 255) / 256), dim3(256), 0, stream, t, grad + K * 128, mt, vt,
                       (int)K, lr, 0.9f, 0.999f, 1e-8f, (float)c1, (float)c2);
}

void launch_augment(const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n, const float* params,
                    const float* noise, float* out, hipStream_t stream)
{
    hipLaunchKernelGGL(augment_kernel, dim3(2 * n), dim3(kAugThreads), 0, stream, pool, n_pairs, batch, n, params,
                       noise, out);
}

}  // namespace bd
