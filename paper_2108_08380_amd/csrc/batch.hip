// Batched describe-and-match: many images of uneven sizes and keypoint
// counts, their BAD and HashSIFT codes and the per-pair Hamming k-NN, as one
// sequence of persistent launches captured into a HIP graph.
//
// Each stage is one persistent, XCD-aware kernel over the whole batch whose
// work units are counted per image (or per match problem) in prefix arrays
// built at creation: a block finds its image by binary search in the prefix,
// so large and small images share one launch and load-balance by units, not
// by image.  The graph holds only kernel nodes (no memset or copy nodes).
//
// The autotuner times each stage under a few grid sizes and, for the
// matcher, queries per lane and train rows per unit, on the caller's data,
// and keeps the fastest.  Every tuning gives the same codes and matches.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "bd_internal.hpp"

using namespace bd;

namespace {

constexpr size_t kAlign = 256;
constexpr int kKpPerUnit = 4;  // keypoints per block unit of BAD and the histogram

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct RunArgs {
    const bd_keypoint* kps;
    const bd_box_pair* pairs;
    const float* B;
    const float* t;
    uint64_t* bad_codes;
    uint64_t* hs_codes;
    int32_t* bad_idx;
    uint32_t* bad_dist;
    int32_t* hs_idx;
    uint32_t* hs_dist;
    bool operator==(const RunArgs& o) const { return std::memcmp(this, &o, sizeof *this) == 0; }
};

// One matcher (BAD or HashSIFT codes): its plan, device problem records and
// unit prefixes.
struct Matcher {
    int32_t n_words = 0;
    KnnBatchPlan plan{};
    BatchMatch* d_match = nullptr;
    int32_t* d_pre = nullptr;
    int32_t* d_merge_pre = nullptr;
    int64_t units = 0;
    size_t partial_elems = 0;  // u32 keys needed by the current plan
};

}  // namespace

struct bd_batch {
    bd_context* ctx = nullptr;
    int32_t n_img = 0, n_match = 0;
    int32_t bad_bits = 0, hs_bits = 0, precision = 0, k = 1;
    int32_t hs_dtypes = 0;  // bit (1 << dtype) for every HashSIFT source dtype present
    float margin = 0.0f;
    int64_t total_kp = 0;
    std::vector<BatchImage> images;
    std::vector<bd_batch_match> matches;
    std::vector<int32_t> match_out_off;  // result row of each match's first query

    void* arena = nullptr;  // integral images, tile tables, order, features, records, prefixes
    BatchImage* d_images = nullptr;
    int32_t* d_tile_pre = nullptr;
    int32_t* d_carry_pre = nullptr;
    int32_t* d_kpb_pre = nullptr;
    int32_t* d_order = nullptr;
    float* d_hist = nullptr;
    uint8_t* d_bad_table = nullptr;  // compiled BAD table, rebuilt at every run
    int32_t tile_units = 0, carry_units = 0, kpb_units = 0;

    Matcher bad_m, hs_m;
    uint32_t* d_partial = nullptr;  // shared by the two matchers (they run one after the other)
    size_t partial_cap = 0;         // u32 elements

    bd_batch_tuning tune{};

    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    RunArgs graph_args{};
};

namespace {

int hip_fail(const char* fn, const char* what, hipError_t e)
{
    return fail(e == hipErrorOutOfMemory ? BD_ENOMEM : BD_EDEVICE, "%s: %s: %s", fn, what, hipGetErrorString(e));
}

struct DeviceScope {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceScope(int device)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != device) err = hipSetDevice(device);
    }
    ~DeviceScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int grid_for(int64_t units, int blocks_per_cu, int num_cus)
{
    const int64_t cap = (int64_t)blocks_per_cu * (num_cus > 0 ? num_cus : 256);
    int64_t g = units < cap ? units : cap;
    if (g < 1) g = 1;
    return xcd_grid((int)g);
}

void drop_graph(bd_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

// Problem records and unit prefixes of one matcher under (qpl, rows).
void plan_matcher(const bd_batch* b, Matcher& m, int32_t qpl, int32_t rows, std::vector<BatchMatch>& recs,
                  std::vector<int32_t>& pre, std::vector<int32_t>& mpre)
{
    recs.assign(b->n_match, BatchMatch{});
    pre.assign(b->n_match + 1, 0);
    mpre.assign(b->n_match + 1, 0);
    const int qpw = knn_queries_per_unit(qpl, m.n_words);
    int64_t part = 0;
    for (int i = 0; i < b->n_match; ++i) {
        const BatchImage& q = b->images[b->matches[i].query_image];
        const BatchImage& t = b->images[b->matches[i].train_image];
        BatchMatch r{};
        r.q_off = q.kp_offset;
        r.n_q = q.n_kp;
        r.t_off = t.kp_offset;
        r.n_t = t.n_kp;
        r.out_off = b->match_out_off[i];
        r.splits = std::max(1, (t.n_kp + rows - 1) / rows);
        r.qgroups = (q.n_kp + qpw - 1) / qpw;
        r.part_off = part;
        if (r.splits > 1) part += (int64_t)r.splits * r.n_q * b->k;
        recs[i] = r;
        pre[i + 1] = pre[i] + r.splits * r.qgroups;
        mpre[i + 1] = mpre[i] + (r.splits > 1 ? (r.n_q + kWave - 1) / kWave : 0);
    }
    m.units = pre[b->n_match];
    m.partial_elems = (size_t)part;
    m.plan.n_words = m.n_words;
    m.plan.k = b->k;
    m.plan.qpl = qpl;
    m.plan.rows_per_split = rows;
    m.plan.merge_units = mpre[b->n_match];
}

// Uploads the matcher's records for its tuning (synchronous).
int apply_matcher(bd_batch* b, Matcher& m, int32_t qpl, int32_t rows, int32_t blocks_per_cu)
{
    const char* fn = "bd_batch";
    // the MFMA engine's keys number at most 64 tiles of 32 rows per unit
    if (qpl == 0 && (rows % 16 != 0 || rows > BD_BATCH_MFMA_MAX_ROWS))
        return fail(BD_EINVAL, "%s: rows per unit %d of the MFMA engine not a multiple of 16 up to %d", fn, rows,
                    BD_BATCH_MFMA_MAX_ROWS);
    std::vector<BatchMatch> recs;
    std::vector<int32_t> pre, mpre;
    plan_matcher(b, m, qpl, rows, recs, pre, mpre);
    if (m.partial_elems > b->partial_cap) return fail(BD_EINVAL, "%s: partial buffer too small for %d rows per unit", fn, rows);
    const int num_cus = b->ctx->num_cus;
    // lane-per-query units are wavefronts (four per block), MFMA units blocks
    m.plan.grid = grid_for(qpl == 0 ? m.units : (m.units + 3) / 4, blocks_per_cu, num_cus);
    m.plan.merge_grid = grid_for(m.plan.merge_units, 4, num_cus);
    hipError_t e = hipMemcpy(m.d_match, recs.data(), sizeof(BatchMatch) * recs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m.d_pre, pre.data(), sizeof(int32_t) * pre.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m.d_merge_pre, mpre.data(), sizeof(int32_t) * mpre.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(fn, "upload of match records", e);
    return BD_OK;
}

int apply_tuning(bd_batch* b, const bd_batch_tuning& t)
{
    drop_graph(b);
    b->tune = t;
    if (b->n_match > 0) {
        if (b->bad_bits)
            if (int rc = apply_matcher(b, b->bad_m, t.knn_qpl[0], t.knn_rows[0], t.knn_blocks_per_cu[0])) return rc;
        if (b->hs_bits)
            if (int rc = apply_matcher(b, b->hs_m, t.knn_qpl[1], t.knn_rows[1], t.knn_blocks_per_cu[1])) return rc;
    }
    return BD_OK;
}

int check_tuning(const bd_batch_tuning& t)
{
    const char* fn = "bd_batch_set_tuning";
    const int32_t* bpc[] = {&t.order_blocks_per_cu, &t.integral_blocks_per_cu, &t.bad_blocks_per_cu,
                            &t.hist_blocks_per_cu, &t.knn_blocks_per_cu[0], &t.knn_blocks_per_cu[1]};
    for (const int32_t* v : bpc)
        if (*v < 1 || *v > 64) return fail(BD_EINVAL, "%s: blocks per CU %d outside [1, 64]", fn, *v);
    for (int i = 0; i < 2; ++i) {
        if (t.knn_qpl[i] != 0 && t.knn_qpl[i] != 1 && t.knn_qpl[i] != 2 && t.knn_qpl[i] != 4)
            return fail(BD_EINVAL, "%s: queries per lane %d (0 for the MFMA engine, 1, 2 or 4)", fn, t.knn_qpl[i]);
        if (t.knn_rows[i] < BD_BATCH_MIN_ROWS || t.knn_rows[i] > BD_BATCH_MAX_ROWS)
            return fail(BD_EINVAL, "%s: rows per unit %d outside [%d, %d]", fn, t.knn_rows[i], BD_BATCH_MIN_ROWS,
                        BD_BATCH_MAX_ROWS);
        if (t.knn_qpl[i] == 0 && (t.knn_rows[i] % 16 != 0 || t.knn_rows[i] > BD_BATCH_MFMA_MAX_ROWS))
            return fail(BD_EINVAL, "%s: rows per unit %d of the MFMA engine not a multiple of 16 up to %d", fn,
                        t.knn_rows[i], BD_BATCH_MFMA_MAX_ROWS);
    }
    return BD_OK;
}

// ---- stages

enum Stage { kOrder, kIntegral, kBad, kHist, kProject, kMatchBad, kMatchHs, kStages };

void launch_stage(bd_batch* b, int stage, const RunArgs& a, hipStream_t s)
{
    const int cus = b->ctx->num_cus;
    switch (stage) {
        case kOrder:
            launch_keypoint_order_batch(b->d_images, b->n_img, a.kps, b->d_order,
                                        grid_for(b->n_img, b->tune.order_blocks_per_cu, cus), s);
            break;
        case kIntegral:
            if (b->bad_bits)
                launch_integral_batch(b->d_images, b->n_img, b->d_tile_pre, b->d_carry_pre,
                                      grid_for(std::max(b->tile_units, b->carry_units),
                                               b->tune.integral_blocks_per_cu, cus),
                                      s);
            break;
        case kBad:
            if (b->bad_bits) {
                launch_bad_compile(a.pairs, b->bad_bits, b->d_bad_table, s);
                launch_bad_compiled_batch(b->d_images, b->n_img, b->d_kpb_pre, a.kps, b->d_order, b->d_bad_table,
                                          b->bad_bits / 64, a.bad_codes,
                                          grid_for(b->kpb_units, b->tune.bad_blocks_per_cu, cus), b->ctx->invalid, s);
            }
            break;
        case kHist:
            if (b->hs_bits)
                launch_hashsift_hist_batch(b->d_images, b->n_img, b->hs_dtypes, b->d_kpb_pre, a.kps, b->d_order, b->d_hist,
                                           grid_for(b->kpb_units, b->tune.hist_blocks_per_cu, cus), b->ctx->invalid,
                                           s);
            break;
        case kProject:
            if (b->hs_bits)
                launch_hashsift_project(b->precision, b->d_hist, a.kps, (int32_t)b->total_kp, a.B, a.t,
                                        b->hs_bits / 64, b->margin, a.hs_codes, nullptr, nullptr, s);
            break;
        case kMatchBad:
            if (b->bad_bits && b->bad_m.units > 0)
                launch_knn_batch(b->bad_m.plan, b->bad_m.d_match, b->n_match, b->bad_m.d_pre, b->bad_m.d_merge_pre,
                                 a.bad_codes, b->d_partial, a.bad_idx, a.bad_dist, s);
            break;
        case kMatchHs:
            if (b->hs_bits && b->hs_m.units > 0)
                launch_knn_batch(b->hs_m.plan, b->hs_m.d_match, b->n_match, b->hs_m.d_pre, b->hs_m.d_merge_pre,
                                 a.hs_codes, b->d_partial, a.hs_idx, a.hs_dist, s);
            break;
    }
}

void enqueue_all(bd_batch* b, const RunArgs& a, hipStream_t s)
{
    if (b->total_kp == 0) return;
    for (int st = 0; st < kStages; ++st) launch_stage(b, st, a, s);
}

int check_run_args(const bd_batch* b, const RunArgs& a, const char* fn)
{
    if (b->total_kp == 0) return BD_OK;
    if (!a.kps) return fail(BD_EINVAL, "%s: null keypoints", fn);
    if (b->bad_bits && (!a.pairs || !a.bad_codes)) return fail(BD_EINVAL, "%s: null BAD table or code output", fn);
    if (b->hs_bits && (!a.B || !a.t || !a.hs_codes)) return fail(BD_EINVAL, "%s: null projection or code output", fn);
    const bool rows = !b->match_out_off.empty() && b->match_out_off.back() > 0;
    if (rows && b->bad_bits && (!a.bad_idx || !a.bad_dist)) return fail(BD_EINVAL, "%s: null BAD match output", fn);
    if (rows && b->hs_bits && (!a.hs_idx || !a.hs_dist)) return fail(BD_EINVAL, "%s: null HashSIFT match output", fn);
    return BD_OK;
}

RunArgs make_args(const bd_keypoint* kps, const bd_box_pair* pairs, const float* B, const float* t,
                  uint64_t* bad_codes, uint64_t* hs_codes, int32_t* bad_idx, uint32_t* bad_dist, int32_t* hs_idx,
                  uint32_t* hs_dist)
{
    RunArgs a;
    std::memset(&a, 0, sizeof a);
    a.kps = kps;
    a.pairs = pairs;
    a.B = B;
    a.t = t;
    a.bad_codes = bad_codes;
    a.hs_codes = hs_codes;
    a.bad_idx = bad_idx;
    a.bad_dist = bad_dist;
    a.hs_idx = hs_idx;
    a.hs_dist = hs_dist;
    return a;
}

int capture(bd_batch* b, const RunArgs& a, const char* fn)
{
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(fn, "hipStreamBeginCapture", e);
    enqueue_all(b, a, b->cap_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &graph);
    if (e != hipSuccess) return hip_fail(fn, "hipStreamEndCapture", e);
    e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return hip_fail(fn, "hipGraphInstantiate", e);
    }
    b->graph_args = a;
    return BD_OK;
}

// Mean time of `reps` back-to-back launches of one stage, in ms.
int time_stage(bd_batch* b, int stage, const RunArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps,
               float* ms)
{
    const char* fn = "bd_batch_autotune";
    launch_stage(b, stage, a, s);  // warm-up
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch_stage(b, stage, a, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(fn, "timing", e);
    float t = 0.0f;
    e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return hip_fail(fn, "hipEventElapsedTime", e);
    *ms = t / reps;
    return BD_OK;
}

}  // namespace

extern "C" {

int bd_batch_default_tuning(bd_batch_tuning* out)
{
    if (!out) return fail(BD_EINVAL, "bd_batch_default_tuning: null output");
    bd_batch_tuning t{};
    t.order_blocks_per_cu = 1;
    t.integral_blocks_per_cu = 8;
    t.bad_blocks_per_cu = 8;
    t.hist_blocks_per_cu = 4;
    for (int i = 0; i < 2; ++i) {
        t.knn_qpl[i] = 0;
        t.knn_rows[i] = 1024;
        t.knn_blocks_per_cu[i] = 2;
    }
    *out = t;
    return BD_OK;
}

int bd_batch_create(bd_context* ctx, const bd_batch_image* images, int32_t n_images, const bd_batch_match* matches,
                    int32_t n_matches, int32_t bad_bits, int32_t hs_bits, int32_t hs_precision, float hs_margin,
                    int32_t k, bd_batch** out)
{
    const char* fn = "bd_batch_create";
    if (!out) return fail(BD_EINVAL, "%s: null output pointer", fn);
    *out = nullptr;
    if (n_images < 1 || !images) return fail(BD_EINVAL, "%s: need at least one image", fn);
    if (n_matches < 0 || (n_matches > 0 && !matches)) return fail(BD_EINVAL, "%s: bad match list", fn);
    if (bad_bits != 0 && bad_bits != 256 && bad_bits != 512)
        return fail(BD_EUNSUPPORTED, "%s: bad_bits %d (0, 256 or 512)", fn, bad_bits);
    if (hs_bits != 0 && hs_bits != 256 && hs_bits != 512)
        return fail(BD_EUNSUPPORTED, "%s: hs_bits %d (0, 256 or 512)", fn, hs_bits);
    if (!bad_bits && !hs_bits) return fail(BD_EINVAL, "%s: neither descriptor enabled", fn);
    if (hs_bits) {
        if (hs_precision != BD_PREC_FP32 && hs_precision != BD_PREC_BF16 && hs_precision != BD_PREC_FP8)
            return fail(BD_EUNSUPPORTED, "%s: precision %d", fn, hs_precision);
        if (!(hs_margin >= 0.0f) || hs_margin > 1e30f) return fail(BD_EINVAL, "%s: margin must be finite and >= 0", fn);
    }
    if (n_matches > 0 && (k < 1 || k > 2)) return fail(BD_EUNSUPPORTED, "%s: k %d (1 or 2)", fn, k);

    std::vector<BatchImage> ims(n_images);
    int64_t total_kp = 0;
    for (int i = 0; i < n_images; ++i) {
        const bd_batch_image& s = images[i];
        if (s.W < 1 || s.H < 1) return fail(BD_EINVAL, "%s: image %d size %dx%d", fn, i, s.W, s.H);
        if (s.n_kp < 0) return fail(BD_EINVAL, "%s: image %d n_kp %d < 0", fn, i, s.n_kp);
        if (!s.img || s.pitch < s.W) return fail(BD_EINVAL, "%s: image %d null or pitch < W", fn, i);
        if ((int64_t)(s.H + 1) * (((int64_t)s.W + 1 + 63) / 64 * 64) >= ((int64_t)1 << 31))
            return fail(BD_EINVAL, "%s: image %d too large for a 32-bit indexed integral image", fn, i);
        BatchImage& b = ims[i];
        std::memset(&b, 0, sizeof b);
        b.img_u8 = s.img;
        b.pitch_u8 = s.pitch;
        if (s.hs_img) {
            if (s.hs_dtype != BD_DTYPE_U8 && s.hs_dtype != BD_DTYPE_F32)
                return fail(BD_EUNSUPPORTED, "%s: image %d HashSIFT dtype %d", fn, i, s.hs_dtype);
            const int64_t elem = s.hs_dtype == BD_DTYPE_U8 ? 1 : 4;
            if (s.hs_pitch < s.W * elem || (elem == 4 && s.hs_pitch % 4 != 0))
                return fail(BD_EINVAL, "%s: image %d HashSIFT pitch %lld", fn, i, (long long)s.hs_pitch);
            b.img_hs = static_cast<const uint8_t*>(s.hs_img);
            b.pitch_hs = s.hs_pitch;
            b.hs_dtype = s.hs_dtype;
        } else {
            b.img_hs = s.img;
            b.pitch_hs = s.pitch;
            b.hs_dtype = BD_DTYPE_U8;
        }
        if (hs_bits && !hashsift_image_fits(b.pitch_hs, s.H))
            return fail(BD_EINVAL, "%s: image %d HashSIFT image needs pitch < 2^24, H < 2^24, pitch * H <= 2^32", fn, i);
        b.W = s.W;
        b.H = s.H;
        b.kp_offset = (int32_t)total_kp;
        b.n_kp = s.n_kp;
        b.inv_cell = order_inv_cell(s.W, s.H);
        total_kp += s.n_kp;
        if (total_kp >= ((int64_t)1 << 31) / 512) return fail(BD_EINVAL, "%s: more than 2^22 keypoints in total", fn);
    }
    std::vector<bd_batch_match> mts(matches, matches + n_matches);
    std::vector<int32_t> out_off(n_matches + 1, 0);
    for (int i = 0; i < n_matches; ++i) {
        const bd_batch_match& m = mts[i];
        if (m.query_image < 0 || m.query_image >= n_images || m.train_image < 0 || m.train_image >= n_images)
            return fail(BD_EINVAL, "%s: match %d names image %d / %d of %d", fn, i, m.query_image, m.train_image,
                        n_images);
        const int64_t next = (int64_t)out_off[i] + ims[m.query_image].n_kp;
        if (next >= ((int64_t)1 << 31) / 2) return fail(BD_EINVAL, "%s: too many match rows", fn);
        out_off[i + 1] = (int32_t)next;
    }
    if (!ctx) return fail(BD_EINVAL, "%s: null context", fn);

    bd_batch* b = new (std::nothrow) bd_batch();
    if (!b) return fail(BD_ENOMEM, "%s: out of host memory", fn);
    b->ctx = ctx;
    b->n_img = n_images;
    for (const BatchImage& im : ims) b->hs_dtypes |= 1 << im.hs_dtype;
    b->n_match = n_matches;
    b->bad_bits = bad_bits;
    b->hs_bits = hs_bits;
    b->precision = hs_precision;
    b->margin = hs_margin;
    b->k = n_matches > 0 ? k : 1;
    b->total_kp = total_kp;
    b->matches = mts;
    b->match_out_off = out_off;
    b->bad_m.n_words = bad_bits / 64;
    b->hs_m.n_words = hs_bits / 64;

    // ---- arena layout
    std::vector<int32_t> tile_pre(n_images + 1, 0), carry_pre(n_images + 1, 0), kpb_pre(n_images + 1, 0);
    size_t bytes = 0;
    std::vector<size_t> ii_at(n_images), ws_at(n_images);
    for (int i = 0; i < n_images; ++i) {
        BatchImage& im = ims[i];
        kpb_pre[i + 1] = kpb_pre[i] + (im.n_kp + kKpPerUnit - 1) / kKpPerUnit;
        if (!bad_bits) continue;
        const IntegralPlan p = plan_integral(im.W, im.H);
        im.ii_pitch = ((int64_t)im.W + 1 + 63) / 64 * 64;
        im.strips = p.strips;
        im.slabs = p.slabs;
        im.col_pitch = p.col_pitch;
        im.aligned = (im.pitch_u8 % 4 == 0) && (reinterpret_cast<uintptr_t>(im.img_u8) % 4 == 0);
        ii_at[i] = bytes;
        bytes = align_up(bytes + sizeof(uint32_t) * (size_t)(im.H + 1) * (size_t)im.ii_pitch);
        ws_at[i] = bytes;
        bytes = align_up(bytes + p.workspace_bytes());
        tile_pre[i + 1] = tile_pre[i] + integral_tile_blocks(p);
        carry_pre[i + 1] = carry_pre[i] + integral_carry_blocks(p);
    }
    const size_t order_at = bytes;
    bytes = align_up(bytes + sizeof(int32_t) * (size_t)std::max<int64_t>(total_kp, 1));
    const size_t hist_at = bytes;
    if (hs_bits) bytes = align_up(bytes + sizeof(float) * 128 * (size_t)total_kp);
    const size_t table_at = bytes;
    if (bad_bits) bytes = align_up(bytes + bad_table_bytes(bad_bits));
    const size_t images_at = bytes;
    bytes = align_up(bytes + sizeof(BatchImage) * n_images);
    const size_t pre_at = bytes;
    bytes = align_up(bytes + sizeof(int32_t) * 3 * (n_images + 1));
    size_t match_at[2], mpre_at[2];
    for (int j = 0; j < 2; ++j) {
        match_at[j] = bytes;
        bytes = align_up(bytes + sizeof(BatchMatch) * std::max(n_matches, 1));
        mpre_at[j] = bytes;
        bytes = align_up(bytes + sizeof(int32_t) * 2 * (n_matches + 1));
    }

    // partial results: enough for the smallest rows per unit a tuning accepts
    size_t part_elems = 0;
    for (int i = 0; i < n_matches; ++i) {
        const int nq = ims[mts[i].query_image].n_kp, nt = ims[mts[i].train_image].n_kp;
        const int64_t splits = std::max(1, (nt + BD_BATCH_MIN_ROWS - 1) / BD_BATCH_MIN_ROWS);
        if (splits > 1) part_elems += (size_t)splits * nq * b->k;
    }

    DeviceScope dev(ctx->device);
    hipError_t e = dev.err;
    if (e != hipSuccess) {
        delete b;
        return hip_fail(fn, "hipSetDevice", e);
    }
    e = hipMalloc(&b->arena, bytes);
    if (e == hipSuccess && part_elems > 0) e = hipMalloc((void**)&b->d_partial, sizeof(uint32_t) * part_elems);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        bd_batch_destroy(b);
        return hip_fail(fn, "allocation", e);
    }
    b->partial_cap = part_elems;
    char* base = static_cast<char*>(b->arena);
    for (int i = 0; i < n_images && bad_bits; ++i) {
        BatchImage& im = ims[i];
        im.ii = reinterpret_cast<uint32_t*>(base + ii_at[i]);
        im.colsum = reinterpret_cast<uint32_t*>(base + ws_at[i]);
        im.rowsum = im.colsum + (size_t)im.strips * (size_t)im.col_pitch;
    }
    b->images = ims;
    b->d_order = reinterpret_cast<int32_t*>(base + order_at);
    b->d_hist = hs_bits ? reinterpret_cast<float*>(base + hist_at) : nullptr;
    b->d_bad_table = bad_bits ? reinterpret_cast<uint8_t*>(base + table_at) : nullptr;
    b->d_images = reinterpret_cast<BatchImage*>(base + images_at);
    b->d_tile_pre = reinterpret_cast<int32_t*>(base + pre_at);
    b->d_carry_pre = b->d_tile_pre + (n_images + 1);
    b->d_kpb_pre = b->d_carry_pre + (n_images + 1);
    b->tile_units = tile_pre[n_images];
    b->carry_units = carry_pre[n_images];
    b->kpb_units = kpb_pre[n_images];
    Matcher* ms[2] = {&b->bad_m, &b->hs_m};
    for (int j = 0; j < 2; ++j) {
        ms[j]->d_match = reinterpret_cast<BatchMatch*>(base + match_at[j]);
        ms[j]->d_pre = reinterpret_cast<int32_t*>(base + mpre_at[j]);
        ms[j]->d_merge_pre = ms[j]->d_pre + (n_matches + 1);
    }
    e = hipMemcpy(b->d_images, ims.data(), sizeof(BatchImage) * n_images, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_tile_pre, tile_pre.data(), sizeof(int32_t) * (n_images + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_carry_pre, carry_pre.data(), sizeof(int32_t) * (n_images + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_kpb_pre, kpb_pre.data(), sizeof(int32_t) * (n_images + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        bd_batch_destroy(b);
        return hip_fail(fn, "upload of image records", e);
    }
    bd_batch_tuning t;
    bd_batch_default_tuning(&t);
    if (int rc = apply_tuning(b, t)) {
        bd_batch_destroy(b);
        return rc;
    }
    *out = b;
    return BD_OK;
}

int bd_batch_destroy(bd_batch* b)
{
    if (!b) return BD_OK;
    int rc = BD_OK;
    {
        DeviceScope dev(b->ctx->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = fail(BD_EDEVICE, "bd_batch_destroy: %s", hipGetErrorString(e));
        drop_graph(b);
        if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
        if (b->d_partial) (void)hipFree(b->d_partial);
        if (b->arena) (void)hipFree(b->arena);
    }
    delete b;
    return rc;
}

int bd_batch_get_tuning(const bd_batch* b, bd_batch_tuning* out)
{
    if (!b || !out) return fail(BD_EINVAL, "bd_batch_get_tuning: null argument");
    *out = b->tune;
    return BD_OK;
}

int bd_batch_set_tuning(bd_batch* b, const bd_batch_tuning* t)
{
    if (!b || !t) return fail(BD_EINVAL, "bd_batch_set_tuning: null argument");
    if (int rc = check_tuning(*t)) return rc;
    DeviceScope dev(b->ctx->device);
    if (dev.err != hipSuccess) return hip_fail("bd_batch_set_tuning", "hipSetDevice", dev.err);
    hipError_t e = hipDeviceSynchronize();  // records may be in use by enqueued work
    if (e != hipSuccess) return hip_fail("bd_batch_set_tuning", "synchronize", e);
    return apply_tuning(b, *t);
}

int bd_batch_info(const bd_batch* b, int64_t* total_kp, int32_t* match_rows)
{
    if (!b) return fail(BD_EINVAL, "bd_batch_info: null batch");
    if (total_kp) *total_kp = b->total_kp;
    if (match_rows) *match_rows = b->match_out_off.back();
    return BD_OK;
}

int bd_batch_run(bd_batch* b, const bd_keypoint* kps, const bd_box_pair* pairs, const float* B, const float* t,
                 uint64_t* bad_codes, uint64_t* hs_codes, int32_t* bad_idx, uint32_t* bad_dist, int32_t* hs_idx,
                 uint32_t* hs_dist, int32_t use_graph, void* stream)
{
    const char* fn = "bd_batch_run";
    if (!b) return fail(BD_EINVAL, "%s: null batch", fn);
    const RunArgs a = make_args(kps, pairs, B, t, bad_codes, hs_codes, bad_idx, bad_dist, hs_idx, hs_dist);
    if (int rc = check_run_args(b, a, fn)) return rc;
    if (b->total_kp == 0) return BD_OK;
    DeviceScope dev(b->ctx->device);
    if (dev.err != hipSuccess) return hip_fail(fn, "hipSetDevice", dev.err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!use_graph) {
        enqueue_all(b, a, s);
        return check_launch(fn);
    }
    if (!b->exec || !(b->graph_args == a))
        if (int rc = capture(b, a, fn)) return rc;
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_fail(fn, "hipGraphLaunch", e);
    return BD_OK;
}

int bd_batch_autotune(bd_batch* b, const bd_keypoint* kps, const bd_box_pair* pairs, const float* B, const float* t,
                      uint64_t* bad_codes, uint64_t* hs_codes, int32_t* bad_idx, uint32_t* bad_dist,
                      int32_t* hs_idx, uint32_t* hs_dist, int32_t reps, void* stream)
{
    const char* fn = "bd_batch_autotune";
    if (!b) return fail(BD_EINVAL, "%s: null batch", fn);
    if (reps < 1 || reps > 1000) return fail(BD_EINVAL, "%s: reps %d outside [1, 1000]", fn, reps);
    const RunArgs a = make_args(kps, pairs, B, t, bad_codes, hs_codes, bad_idx, bad_dist, hs_idx, hs_dist);
    if (int rc = check_run_args(b, a, fn)) return rc;
    if (b->total_kp == 0) return BD_OK;
    DeviceScope dev(b->ctx->device);
    if (dev.err != hipSuccess) return hip_fail(fn, "hipSetDevice", dev.err);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(fn, "synchronize", e);
    drop_graph(b);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(fn, "hipEventCreate", e);
    }
    int rc = BD_OK;
    bd_batch_tuning best = b->tune;
    enqueue_all(b, a, s);  // every stage's inputs resident before stages are timed alone

    static const int kGridCands[] = {1, 2, 4, 8, 16};
    struct GridKnob {
        int stage;
        int32_t bd_batch_tuning::*field;
    };
    const GridKnob knobs[] = {{kOrder, &bd_batch_tuning::order_blocks_per_cu},
                              {kIntegral, &bd_batch_tuning::integral_blocks_per_cu},
                              {kBad, &bd_batch_tuning::bad_blocks_per_cu},
                              {kHist, &bd_batch_tuning::hist_blocks_per_cu}};
    for (const GridKnob& kn : knobs) {
        if ((kn.stage == kIntegral || kn.stage == kBad) && !b->bad_bits) continue;
        if (kn.stage == kHist && !b->hs_bits) continue;
        float best_ms = 1e30f;
        int32_t best_v = best.*kn.field;
        for (int v : kGridCands) {
            b->tune = best;
            b->tune.*kn.field = v;
            float ms = 0.0f;
            if ((rc = time_stage(b, kn.stage, a, s, e0, e1, reps, &ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_v = v;
            }
        }
        if (rc) break;
        best.*kn.field = best_v;
    }

    static const int kQpl[] = {0, 1, 2, 4};
    static const int kRows[] = {256, 512, 1024, 2048, 4096};
    static const int kKnnGrid[] = {2, 4, 8};
    for (int j = 0; j < 2 && rc == BD_OK && b->n_match > 0; ++j) {
        if ((j == 0 && !b->bad_bits) || (j == 1 && !b->hs_bits)) continue;
        Matcher& m = j == 0 ? b->bad_m : b->hs_m;
        const int stage = j == 0 ? kMatchBad : kMatchHs;
        float best_ms = 1e30f;
        int32_t bq = best.knn_qpl[j], br = best.knn_rows[j], bg = best.knn_blocks_per_cu[j];
        for (int q : kQpl) {
            for (int r : kRows) {
                if (q == 0 && r > BD_BATCH_MFMA_MAX_ROWS) continue;
                if ((rc = apply_matcher(b, m, q, r, bg))) break;
                float ms = 0.0f;
                if ((rc = time_stage(b, stage, a, s, e0, e1, reps, &ms))) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    bq = q;
                    br = r;
                }
            }
            if (rc) break;
        }
        for (int g : kKnnGrid) {
            if (rc || g == bg) continue;
            if ((rc = apply_matcher(b, m, bq, br, g))) break;
            float ms = 0.0f;
            if ((rc = time_stage(b, stage, a, s, e0, e1, reps, &ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best.knn_blocks_per_cu[j] = g;
            }
        }
        best.knn_qpl[j] = bq;
        best.knn_rows[j] = br;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        bd_batch_tuning d;
        bd_batch_default_tuning(&d);
        (void)apply_tuning(b, d);
        return rc;
    }
    rc = apply_tuning(b, best);
    if (rc) return rc;
    enqueue_all(b, a, s);  // leave the outputs of the chosen tuning in place
    return check_launch(fn);
}

}  // extern "C"
