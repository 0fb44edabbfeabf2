// Differentiation extension (not proposed by the paper): relaxed descriptors
// tanh(beta * rho) for BAD and HashSIFT, the triplet ranking loss of
// Sec. III-A Eq. 1 / Sec. III-B Eq. 3 with in-batch hardest negatives and
// anchor swap, and hand-written backward kernels.
//
//   relaxed BAD:      rho_j = theta_j - (w1_j m1_j - w2_j m2_j), m = box means
//                     on the 32x32 patch (keypoint at its centre, scale 1)
//   relaxed HashSIFT: rho = B f - t (projection kernel), D = tanh(beta rho)
//   loss:             s(x, y) = D(x).D(y) / K,
//                     s_neg(i) = max(max_{j!=i} s(a_i, p_j), max_{j!=i} s(a_j, p_i)),
//                     L = mean_i [tau - s(a_i, p_i) + s_neg(i)]_+
//
// Every reduction has a fixed order (no floating-point atomics), so results
// are deterministic.  The hardest-negative search uses integer atomic max on
// packed (ordered value, reversed index) keys, which is order independent.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr int kWaves = 4;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------ relaxed BAD

// One wavefront per patch: an FP64 integral image of the patch in LDS (exact
// for float32 pixels in [0, 1]), then lane = pair for every 64-pair word.
__global__ __launch_bounds__(256) void relaxed_bad_fwd_kernel(const float* __restrict__ patches, int32_t n,
                                                              const bd_box_pair* __restrict__ pairs,
                                                              const float* __restrict__ w1,
                                                              const float* __restrict__ w2,
                                                              const float* __restrict__ theta, int32_t n_bits,
                                                              float beta, float* __restrict__ D,
                                                              float* __restrict__ m1, float* __restrict__ m2)
{
    __shared__ double ii_all[kWaves][33 * 33];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int i = blockIdx.x * kWaves + wave;
    if (i >= n) return;
    double* S = ii_all[wave];
    const float* patch = patches + (int64_t)i * 1024;
    if (lane < 33) S[lane] = 0.0;  // first row
    if (lane < 32) {               // row prefix sums
        double acc = 0.0;
        S[(lane + 1) * 33] = 0.0;
        for (int x = 0; x < 32; ++x) {
            acc += (double)patch[lane * 32 + x];
            S[(lane + 1) * 33 + x + 1] = acc;
        }
    }
    wave_sync();
    if (lane < 32) {  // column prefix sums
        double acc = 0.0;
        for (int y = 1; y <= 32; ++y) {
            acc += S[y * 33 + lane + 1];
            S[y * 33 + lane + 1] = acc;
        }
    }
    wave_sync();
    for (int w = 0; w < n_bits / kWave; ++w) {
        const int j = w * kWave + lane;
        const bd_box_pair pr = pairs[j];
        const int R = pr.radius > 15 ? 15 : pr.radius;
        const int c1x = min(max(16 + pr.x1, R), 31 - R), c1y = min(max(16 + pr.y1, R), 31 - R);
        const int c2x = min(max(16 + pr.x2, R), 31 - R), c2y = min(max(16 + pr.y2, R), 31 - R);
        const double s1 = S[(c1y + R + 1) * 33 + c1x + R + 1] - S[(c1y - R) * 33 + c1x + R + 1] -
                          S[(c1y + R + 1) * 33 + c1x - R] + S[(c1y - R) * 33 + c1x - R];
        const double s2 = S[(c2y + R + 1) * 33 + c2x + R + 1] - S[(c2y - R) * 33 + c2x + R + 1] -
                          S[(c2y + R + 1) * 33 + c2x - R] + S[(c2y - R) * 33 + c2x - R];
        const double area = (double)((2 * R + 1) * (2 * R + 1));
        const double a = s1 / area, b = s2 / area;
        const double rho = (double)theta[j] - ((double)w1[j] * a - (double)w2[j] * b);
        const int64_t o = (int64_t)i * n_bits + j;
        D[o] = tanhf(beta * (float)rho);
        if (m1) m1[o] = (float)a;
        if (m2) m2[o] = (float)b;
    }
}

// Parameter gradients: block (word, split) sums over its patch range in FP64,
// four wavefronts interleaved then combined in order; partial[split][3][K].
__global__ __launch_bounds__(256) void relaxed_bad_bwd_kernel(const float* __restrict__ gD,
                                                              const float* __restrict__ D,
                                                              const float* __restrict__ m1,
                                                              const float* __restrict__ m2, int32_t n,
                                                              int32_t n_bits, float beta, int32_t rows_per_split,
                                                              double* __restrict__ partial)
{
    __shared__ double red[kWaves][3][kWave];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int j = blockIdx.x * kWave + lane;
    const int r0 = blockIdx.y * rows_per_split, r1 = min(n, r0 + rows_per_split);
    double st = 0.0, s1 = 0.0, s2 = 0.0;
    for (int x = r0 + wave; x < r1; x += kWaves) {
        const int64_t o = (int64_t)x * n_bits + j;
        const double d = D[o];
        const double g = (double)gD[o] * (double)beta * (1.0 - d * d);
        st += g;
        s1 -= g * (double)m1[o];
        s2 += g * (double)m2[o];
    }
    red[wave][0][lane] = st;
    red[wave][1][lane] = s1;
    red[wave][2][lane] = s2;
    __syncthreads();
    if (wave == 0) {
        double a[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < kWaves; ++w)
            for (int q = 0; q < 3; ++q) a[q] += red[w][q][lane];
        for (int q = 0; q < 3; ++q) partial[((int64_t)blockIdx.y * 3 + q) * n_bits + j] = a[q];
    }
}

// outputs: g_theta (q = 0), g_w1 (q = 1), g_w2 (q = 2), summed over splits in order
__global__ __launch_bounds__(256) void relaxed_bad_reduce_kernel(const double* __restrict__ partial, int32_t splits,
                                                                 int32_t n_bits, float* __restrict__ g_w1,
                                                                 float* __restrict__ g_w2, float* __restrict__ g_theta)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 3 * n_bits) return;
    const int q = e / n_bits, j = e % n_bits;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += partial[((int64_t)s * 3 + q) * n_bits + j];
    float* out = q == 0 ? g_theta : (q == 1 ? g_w1 : g_w2);
    out[j] = (float)acc;
}

// ------------------------------------------------------------ relaxed HashSIFT

__global__ __launch_bounds__(256) void tanh_scale_kernel(const float* __restrict__ rho, int64_t count, float beta,
                                                         float* __restrict__ D)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) D[e] = tanhf(beta * rho[e]);
}

// dL/dB[j][k] = sum_x g[x][j] f[x][k], dL/dt[j] = -sum_x g[x][j] with
// g = dL/dD * beta * (1 - D^2).  Block (64-bit tile, split): thread t owns
// bits 4*(t/16) .. +3 of the tile and features 8*(t%16) .. +7 (32 FP64
// accumulators); 32 patches at a time are staged in LDS.
constexpr int kHsChunk = 32;
__global__ __launch_bounds__(256) void relaxed_hs_bwd_kernel(const float* __restrict__ gD, const float* __restrict__ D,
                                                             const float* __restrict__ f, int32_t n, int32_t n_bits,
                                                             float beta, int32_t rows_per_split,
                                                             double* __restrict__ partial)
{
    __shared__ float gs[kHsChunk][64];
    __shared__ float fs[kHsChunk][128];
    const int t = threadIdx.x;
    const int bit0 = blockIdx.x * 64;
    const int jb = 4 * (t / 16), kb = 8 * (t % 16);
    const int r0 = blockIdx.y * rows_per_split, r1 = min(n, r0 + rows_per_split);
    double acc[4][8];
    double gt[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
    for (int x0 = r0; x0 < r1; x0 += kHsChunk) {
        __syncthreads();
        for (int e = t; e < kHsChunk * 64; e += 256) {
            const int p = e / 64, j = e % 64, x = x0 + p;
            float g = 0.0f;
            if (x < r1) {
                const int64_t o = (int64_t)x * n_bits + bit0 + j;
                const float d = D[o];
                g = gD[o] * beta * (1.0f - d * d);
            }
            gs[p][j] = g;
        }
        for (int e = t; e < kHsChunk * 128; e += 256) {
            const int p = e / 128, k = e % 128, x = x0 + p;
            fs[p][k] = x < r1 ? f[(int64_t)x * 128 + k] : 0.0f;
        }
        __syncthreads();
        for (int p = 0; p < kHsChunk; ++p) {
            double gv[4], fv[8];
#pragma unroll
            for (int a = 0; a < 4; ++a) gv[a] = gs[p][jb + a];
#pragma unroll
            for (int b = 0; b < 8; ++b) fv[b] = fs[p][kb + b];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (kb == 0) gt[a] -= gv[a];
#pragma unroll
                for (int b = 0; b < 8; ++b) acc[a][b] = fma(gv[a], fv[b], acc[a][b]);
            }
        }
    }
    // partial[split][K*128 + K]
    double* out = partial + (int64_t)blockIdx.y * ((int64_t)n_bits * 129);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int b = 0; b < 8; ++b) out[(int64_t)(bit0 + jb + a) * 128 + kb + b] = acc[a][b];
        if (kb == 0) out[(int64_t)n_bits * 128 + bit0 + jb + a] = gt[a];
    }
}

__global__ __launch_bounds__(256) void relaxed_hs_reduce_kernel(const double* __restrict__ partial, int32_t splits,
                                                                int32_t n_bits, float* __restrict__ gB,
                                                                float* __restrict__ gt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)n_bits * 129;
    if (e >= per) return;
    double acc = 0.0;
    for (int s = 0; s < splits; ++s) acc += partial[(int64_t)s * per + e];
    if (e < (int64_t)n_bits * 128)
        gB[e] = (float)acc;
    else
        gt[e - (int64_t)n_bits * 128] = (float)acc;
}

// ------------------------------------------------------------ triplet loss, forward

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Order-preserving map of a float to u32 (larger float -> larger key).
__device__ __forceinline__ uint32_t ordered_bits(float v)
{
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
// key: value in the high word, reversed index in the low word, so the
// largest key is the largest value and, among equal values, the lowest index
__device__ __forceinline__ uint64_t pack_key(float v, int idx)
{
    return ((uint64_t)ordered_bits(v) << 32) | (uint64_t)(0xffffffffu - (uint32_t)idx);
}

__global__ __launch_bounds__(256) void trl_init_kernel(uint64_t* __restrict__ keys, int32_t count)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) keys[e] = 0ull;
}

__global__ __launch_bounds__(256) void zero_i32_kernel(int32_t* __restrict__ v, int32_t count)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) v[e] = 0;
}

// Similarity tiles S = A P^T / K on v_mfma_f32_16x16x4_f32: a block owns a
// 128x128 tile (four wavefronts of 64x64), K staged through LDS 32 at a time
// (rows padded to 36 floats).  The epilogue never stores S: it reduces each
// row's maximum over j != i (with its column) and each column's maximum over
// rows != column, and merges them into rowkey / colkey with 64-bit atomic
// max; diagonal entries go to diag.
constexpr int kTile = 128, kKc = 32, kLdsRow = 36;
__global__ __launch_bounds__(256) void trl_sim_kernel(const float* __restrict__ A, const float* __restrict__ P,
                                                      int32_t n, int32_t K, uint64_t* __restrict__ rowkey,
                                                      uint64_t* __restrict__ colkey, float* __restrict__ diag)
{
    __shared__ float As[kTile * kLdsRow];
    __shared__ float Ps[kTile * kLdsRow];
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    const int g = lane >> 4, m = lane & 15;
    const int wm = wave >> 1, wn = wave & 1;
    const int row0 = blockIdx.y * kTile, col0 = blockIdx.x * kTile;
    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < K; k0 += kKc) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {  // 128 rows x 32 floats = 1024 float4 per operand
            const int e = t + 256 * r, row = e >> 3, c4 = (e & 7) * 4;
            float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vp = va;
            if (row0 + row < n) va = *reinterpret_cast<const float4*>(A + (int64_t)(row0 + row) * K + k0 + c4);
            if (col0 + row < n) vp = *reinterpret_cast<const float4*>(P + (int64_t)(col0 + row) * K + k0 + c4);
            *reinterpret_cast<float4*>(&As[row * kLdsRow + c4]) = va;
            *reinterpret_cast<float4*>(&Ps[row * kLdsRow + c4]) = vp;
        }
        __syncthreads();
        // lane (g, m) supplies k = 8g .. 8g+7 of the chunk for row / column m of each 16-tile
        float a[4][8], b[4][8];
#pragma unroll
        for (int tm = 0; tm < 4; ++tm) {
            const float* src = &As[(wm * 64 + 16 * tm + m) * kLdsRow + 8 * g];
            const float4 lo = *reinterpret_cast<const float4*>(src), hi = *reinterpret_cast<const float4*>(src + 4);
            a[tm][0] = lo.x; a[tm][1] = lo.y; a[tm][2] = lo.z; a[tm][3] = lo.w;
            a[tm][4] = hi.x; a[tm][5] = hi.y; a[tm][6] = hi.z; a[tm][7] = hi.w;
        }
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) {
            const float* src = &Ps[(wn * 64 + 16 * tn + m) * kLdsRow + 8 * g];
            const float4 lo = *reinterpret_cast<const float4*>(src), hi = *reinterpret_cast<const float4*>(src + 4);
            b[tn][0] = lo.x; b[tn][1] = lo.y; b[tn][2] = lo.z; b[tn][3] = lo.w;
            b[tn][4] = hi.x; b[tn][5] = hi.y; b[tn][6] = hi.z; b[tn][7] = hi.w;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int tm = 0; tm < 4; ++tm)
#pragma unroll
                for (int tn = 0; tn < 4; ++tn)
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[tm][e], b[tn][e], acc[tm][tn], 0, 0, 0);
    }

    // lane (g, m) holds S[row = 16tm + 4g + i][col = 16tn + m] of the wavefront's 64x64 tile
    const float invK = 1.0f / (float)K;
    const int wrow = row0 + wm * 64, wcol = col0 + wn * 64;
    // row maxima over j != i
#pragma unroll
    for (int tm = 0; tm < 4; ++tm) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wrow + 16 * tm + 4 * g + i;
            uint64_t best = 0ull;
#pragma unroll
            for (int tn = 0; tn < 4; ++tn) {
                const int c = wcol + 16 * tn + m;
                const float v = acc[tm][tn][i] * invK;
                if (c < n && r < n) {
                    if (c == r)
                        diag[r] = v;
                    else {
                        const uint64_t k = pack_key(v, c);
                        best = k > best ? k : best;
                    }
                }
            }
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                const uint64_t o = __shfl_xor(best, d, kWave);
                best = o > best ? o : best;
            }
            if (m == 0 && r < n && best) atomicMax((unsigned long long*)&rowkey[r], (unsigned long long)best);
        }
    }
    // column maxima over rows != column
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
        const int c = wcol + 16 * tn + m;
        uint64_t best = 0ull;
#pragma unroll
        for (int tm = 0; tm < 4; ++tm)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = wrow + 16 * tm + 4 * g + i;
                if (r < n && c < n && r != c) {
                    const uint64_t k = pack_key(acc[tm][tn][i] * invK, r);
                    best = k > best ? k : best;
                }
            }
        for (int d = 16; d < 64; d <<= 1) {
            const uint64_t o = __shfl_xor(best, d, kWave);
            best = o > best ? o : best;
        }
        if (g == 0 && c < n && best) atomicMax((unsigned long long*)&colkey[c], (unsigned long long)best);
    }
}

// One block: hardest negative per sample (the row candidate wins ties),
// hinge values, and the mean loss summed in a fixed order.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void trl_finalize_kernel(const uint64_t* __restrict__ rowkey,
                                                                  const uint64_t* __restrict__ colkey,
                                                                  const float* __restrict__ diag, int32_t n, float tau,
                                                                  int32_t* __restrict__ neg, float* __restrict__ hinge,
                                                                  float* __restrict__ loss)
{
    __shared__ double part[kFinThreads];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int i = t; i < n; i += kFinThreads) {
        const uint64_t rk = rowkey[i], ck = colkey[i];
        const float rv = from_ordered((uint32_t)(rk >> 32)), cv = from_ordered((uint32_t)(ck >> 32));
        const int rj = (int)(0xffffffffu - (uint32_t)rk), cj = (int)(0xffffffffu - (uint32_t)ck);
        const bool use_row = rk != 0ull && (ck == 0ull || rv >= cv);
        const float sn = use_row ? rv : cv;
        const float h = (rk == 0ull && ck == 0ull) ? -1.0f : tau - diag[i] + sn;
        neg[i] = use_row ? rj : -1 - cj;
        hinge[i] = h;
        if (h > 0.0f) acc += (double)h;
    }
    part[t] = acc;
    __syncthreads();
    for (int s = kFinThreads / 2; s > 0; s >>= 1) {
        if (t < s) part[t] += part[t + s];
        __syncthreads();
    }
    if (t == 0) loss[0] = (float)(part[0] / (double)n);
}

// ------------------------------------------------------------ triplet loss, backward
//
// dL/dA[x] = c (-P[x] [x active] + P[j] [x active, row choice j] + sum_{i: col choice of i is x} P[i])
// dL/dP[x] = c (-A[x] [x active] + A[j] [x active, col choice j] + sum_{i: row choice of i is x} A[i])
// with c = dL/dloss / (n K).  The sums over other samples are gathered in
// ascending i from lists built by a stable counting sort.

// targets: tgt[0][i] = x for a column choice (feeds dL/dA[x]), tgt[1][i] = x for a row choice (feeds dL/dP[x])
__global__ __launch_bounds__(256) void trl_targets_kernel(const int32_t* __restrict__ neg,
                                                          const float* __restrict__ hinge, int32_t n,
                                                          int32_t* __restrict__ tgt, int32_t* __restrict__ count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ta = -1, tp = -1;
    if (hinge[i] > 0.0f) {
        const int c = neg[i];
        if (c >= 0) tp = c;
        else ta = -1 - c;
    }
    tgt[i] = ta;
    tgt[n + i] = tp;
    if (ta >= 0) atomicAdd(&count[ta], 1);
    if (tp >= 0) atomicAdd(&count[n + tp], 1);
}

// one block: exclusive scan of 2n counts into offsets
__global__ __launch_bounds__(1024) void trl_scan_kernel(const int32_t* __restrict__ count, int32_t total,
                                                        int32_t* __restrict__ offset)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (total + 1023) / 1024;
    const int b = t * per, e = min(total, b + per);
    int32_t s = 0;
    for (int i = b; i < e; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int32_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int i = b; i < e; ++i) {
        offset[i] = run;
        run += count[i];
    }
}

// list[offset[x] + rank] = i, rank = number of earlier samples with the same target (stable)
__global__ __launch_bounds__(256) void trl_fill_kernel(const int32_t* __restrict__ tgt, int32_t n,
                                                       const int32_t* __restrict__ offset, int32_t* __restrict__ list)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * n) return;
    const int side = e / n, i = e % n;
    const int x = tgt[side * n + i];
    if (x < 0) return;
    const int32_t* row = tgt + side * n;
    int rank = 0;
    for (int q = 0; q < i; ++q) rank += row[q] == x;
    list[offset[side * n + x] + rank] = i;
}

// one wavefront per sample x; lane covers columns lane, lane + 64, ...
__global__ __launch_bounds__(256) void trl_gather_kernel(const float* __restrict__ A, const float* __restrict__ P,
                                                         int32_t n, int32_t K, const int32_t* __restrict__ neg,
                                                         const float* __restrict__ hinge,
                                                         const int32_t* __restrict__ count,
                                                         const int32_t* __restrict__ offset,
                                                         const int32_t* __restrict__ list,
                                                         const float* __restrict__ grad_loss, float* __restrict__ gA,
                                                         float* __restrict__ gP)
{
    const int lane = threadIdx.x % kWave;
    const int x = blockIdx.x * kWaves + threadIdx.x / kWave;
    if (x >= n) return;
    const float c = grad_loss[0] / ((float)n * (float)K);
    const bool active = hinge[x] > 0.0f;
    const int choice = neg[x];
    const int la = offset[x], na = count[x];
    const int lp = offset[n + x], np = count[n + x];
    for (int k = lane; k < K; k += kWave) {
        float ga = 0.0f, gp = 0.0f;
        if (active) {
            ga -= P[(int64_t)x * K + k];
            gp -= A[(int64_t)x * K + k];
            if (choice >= 0)
                ga += P[(int64_t)choice * K + k];
            else
                gp += A[(int64_t)(-1 - choice) * K + k];
        }
        for (int q = 0; q < na; ++q) ga += P[(int64_t)list[la + q] * K + k];
        for (int q = 0; q < np; ++q) gp += A[(int64_t)list[lp + q] * K + k];
        gA[(int64_t)x * K + k] = c * ga;
        gP[(int64_t)x * K + k] = c * gp;
    }
}

int splits_for(int n, int rows_min) { return max(1, min(256, (n + rows_min - 1) / rows_min)); }

}  // namespace

// ---- launchers

void launch_relaxed_bad_fwd(const float* patches, int32_t n, const bd_box_pair* pairs, const float* w1,
                            const float* w2, const float* theta, int32_t n_bits, float beta, float* D, float* m1,
                            float* m2, hipStream_t stream)
{
    hipLaunchKernelGGL(relaxed_bad_fwd_kernel, dim3((n + kWaves - 1) / kWaves), dim3(kWaves * kWave), 0, stream,
                       patches, n, pairs, w1, w2, theta, n_bits, beta, D, m1, m2);
}

size_t relaxed_bad_bwd_workspace(int32_t n, int32_t n_bits)
{
    return sizeof(double) * 3 * (size_t)n_bits * (size_t)splits_for(n, 64);
}

void launch_relaxed_bad_bwd(const float* gD, const float* D, const float* m1, const float* m2, int32_t n,
                            int32_t n_bits, float beta, float* g_w1, float* g_w2, float* g_theta, void* workspace,
                            hipStream_t stream)
{
    const int splits = splits_for(n, 64);
    const int rps = (n + splits - 1) / splits;
    double* partial = static_cast<double*>(workspace);
    hipLaunchKernelGGL(relaxed_bad_bwd_kernel, dim3(n_bits / kWave, splits), dim3(kWaves * kWave), 0, stream, gD, D,
                       m1, m2, n, n_bits, beta, rps, partial);
    hipLaunchKernelGGL(relaxed_bad_reduce_kernel, dim3((3 * n_bits + 255) / 256), dim3(256), 0, stream, partial,
                       splits, n_bits, g_w1, g_w2, g_theta);
}

void launch_tanh_scale(const float* rho, int64_t count, float beta, float* D, hipStream_t stream)
{
    hipLaunchKernelGGL(tanh_scale_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, rho, count,
                       beta, D);
}

size_t relaxed_hs_bwd_workspace(int32_t n, int32_t n_bits)
{
    return sizeof(double) * (size_t)n_bits * 129 * (size_t)splits_for(n, 256);
}

void launch_relaxed_hs_bwd(const float* gD, const float* D, const float* f, int32_t n, int32_t n_bits, float beta,
                           float* gB, float* gt, void* workspace, hipStream_t stream)
{
    const int splits = splits_for(n, 256);
    const int rps = (n + splits - 1) / splits;
    double* partial = static_cast<double*>(workspace);
    hipLaunchKernelGGL(relaxed_hs_bwd_kernel, dim3(n_bits / 64, splits), dim3(256), 0, stream, gD, D, f, n, n_bits,
                       beta, rps, partial);
    const int64_t per = (int64_t)n_bits * 129;
    hipLaunchKernelGGL(relaxed_hs_reduce_kernel, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, stream, partial,
                       splits, n_bits, gB, gt);
}

size_t trl_workspace(int32_t n)
{
    // rowkey, colkey (u64), diag (f32); backward: tgt (2n), count (2n), offset (2n), list (2n) int32
    return sizeof(uint64_t) * 2 * (size_t)n + sizeof(float) * (size_t)n + sizeof(int32_t) * 8 * (size_t)n + 256;
}

void launch_trl_fwd(const float* A, const float* P, int32_t n, int32_t K, float tau, float* loss, int32_t* neg,
                    float* hinge, void* workspace, hipStream_t stream)
{
    uint64_t* rowkey = static_cast<uint64_t*>(workspace);
    uint64_t* colkey = rowkey + n;
    float* diag = reinterpret_cast<float*>(colkey + n);
    hipLaunchKernelGGL(trl_init_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, stream, rowkey, 2 * n);
    const int tiles = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(trl_sim_kernel, dim3(tiles, tiles), dim3(256), 0, stream, A, P, n, K, rowkey, colkey, diag);
    hipLaunchKernelGGL(trl_finalize_kernel, dim3(1), dim3(kFinThreads), 0, stream, rowkey, colkey, diag, n, tau, neg,
                       hinge, loss);
}

void launch_trl_bwd(const float* A, const float* P, int32_t n, int32_t K, const int32_t* neg, const float* hinge,
                    const float* grad_loss, float* gA, float* gP, void* workspace, hipStream_t stream)
{
    uint64_t* keys = static_cast<uint64_t*>(workspace);
    int32_t* tgt = reinterpret_cast<int32_t*>(reinterpret_cast<float*>(keys + 2 * n) + n);
    int32_t* count = tgt + 2 * n;
    int32_t* offset = count + 2 * n;
    int32_t* list = offset + 2 * n;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, stream, count, 2 * n);
    hipLaunchKernelGGL(trl_targets_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, neg, hinge, n, tgt, count);
    hipLaunchKernelGGL(trl_scan_kernel, dim3(1), dim3(1024), 0, stream, count, 2 * n, offset);
    hipLaunchKernelGGL(trl_fill_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, stream, tgt, n, offset, list);
    hipLaunchKernelGGL(trl_gather_kernel, dim3((n + kWaves - 1) / kWaves), dim3(kWaves * kWave), 0, stream, A, P, n,
                       K, neg, hinge, count, offset, list, grad_loss, gA, gP);
}

}  // namespace bd
