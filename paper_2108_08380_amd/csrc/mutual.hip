// Mutual nearest-neighbour matching with a distance-ratio filter: the
// Hamming MNN matcher of the paper's pipeline timing (Sec. IV, Table of
// pipeline steps).  Two k-NN passes (query -> train with k = 2, train ->
// query with k = 1) on the Hamming k-NN kernels, then one cross-check
// kernel per query.  Both passes break ties by the lowest index, so the
// result is deterministic and equals the definition exactly.
#include "bd_internal.hpp"

namespace bd {
namespace {

constexpr uint32_t kNoDist = 0xffffffffu;

// One thread per query: the nearest train code j must name the query back,
// and with max_ratio > 0 its distance must stay below max_ratio times the
// next distance (compared in double, as a product of exact integers and
// the ratio).
__global__ __launch_bounds__(256) void mutual_check_kernel(const int32_t* __restrict__ idx_qt,
                                                           const uint32_t* __restrict__ dist_qt,
                                                           const int32_t* __restrict__ idx_tq, int32_t n_q,
                                                           double max_ratio, int32_t* __restrict__ match,
                                                           uint32_t* __restrict__ dist, float* __restrict__ ratio)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_q) return;
    const int32_t j = idx_qt[2 * i];
    const uint32_t d1 = dist_qt[2 * i];
    const bool have_d2 = idx_qt[2 * i + 1] >= 0;
    const uint32_t d2 = dist_qt[2 * i + 1];
    bool ok = j >= 0 && idx_tq[j] == i;
    if (ok && max_ratio > 0.0 && have_d2) ok = (double)d1 < max_ratio * (double)d2;
    match[i] = ok ? j : -1;
    dist[i] = j >= 0 ? d1 : kNoDist;
    if (ratio) ratio[i] = !have_d2 ? 0.0f : (d2 == 0u ? 1.0f : (float)((double)d1 / (double)d2));
}

// Number of matches, one block, fixed-order reduction.
__global__ __launch_bounds__(1024) void mutual_count_kernel(const int32_t* __restrict__ match, int32_t n_q,
                                                            int32_t* __restrict__ count)
{
    __shared__ int32_t part[1024 / kWave];
    int32_t c = 0;
    for (int i = threadIdx.x; i < n_q; i += blockDim.x) c += match[i] >= 0;
    for (int d = kWave / 2; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
    if (threadIdx.x % kWave == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += part[w];
        *count = s;
    }
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

MutualPlan plan_mutual(int32_t n_q, int32_t n_t, int32_t n_words, int num_cus)
{
    MutualPlan p{};
    p.n_q = n_q;
    p.n_t = n_t;
    p.qt = plan_knn(n_q, n_t, n_words, 2, num_cus);
    p.tq = plan_knn(n_t, n_q, n_words, 1, num_cus);
    return p;
}

size_t MutualPlan::workspace_bytes() const
{
    const size_t part = qt.workspace_bytes() > tq.workspace_bytes() ? qt.workspace_bytes() : tq.workspace_bytes();
    return align256(sizeof(int32_t) * 2 * (size_t)n_q) * 2 + align256(sizeof(int32_t) * (size_t)n_t) * 2 +
           align256(part);
}

void launch_mutual(const MutualPlan& p, const uint64_t* query, const uint64_t* train, float max_ratio,
                   int32_t* match, uint32_t* dist, float* ratio, int32_t* count, void* workspace,
                   hipStream_t stream)
{
    char* ws = static_cast<char*>(workspace);
    int32_t* idx_qt = reinterpret_cast<int32_t*>(ws);
    ws += align256(sizeof(int32_t) * 2 * (size_t)p.n_q);
    uint32_t* dist_qt = reinterpret_cast<uint32_t*>(ws);
    ws += align256(sizeof(int32_t) * 2 * (size_t)p.n_q);
    int32_t* idx_tq = reinterpret_cast<int32_t*>(ws);
    ws += align256(sizeof(int32_t) * (size_t)p.n_t);
    uint32_t* dist_tq = reinterpret_cast<uint32_t*>(ws);
    ws += align256(sizeof(int32_t) * (size_t)p.n_t);
    if (p.n_q > 0) {
        launch_knn(p.qt, query, train, idx_qt, dist_qt, ws, stream);
        if (p.n_t > 0) launch_knn(p.tq, train, query, idx_tq, dist_tq, ws, stream);
        hipLaunchKernelGGL(mutual_check_kernel, dim3((p.n_q + 255) / 256), dim3(256), 0, stream, idx_qt, dist_qt,
                           idx_tq, p.n_q, (double)max_ratio, match, dist, ratio);
    }
    if (count) hipLaunchKernelGGL(mutual_count_kernel, dim3(1), dim3(1024), 0, stream, match, p.n_q, count);
}

}  // namespace bd
