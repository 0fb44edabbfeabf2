// C ABI: argument validation, context and workspace, dispatch to kernels.
//
// Every entry point validates its arguments on the host before it touches
// the HIP runtime, so argument errors are reported identically with or
// without a GPU.  Nothing here synchronizes except workspace growth and
// context destruction.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "bd_internal.hpp"

namespace bd {

namespace {
thread_local char g_error[512] = "";
}

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return code;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BD_EDEVICE, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
    return BD_OK;
}

namespace {
// Makes the context's device current for the allocation and restores the
// caller's current device afterwards.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int device)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != device) err = hipSetDevice(device);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

// Fixed device scratch for the entry points that allocate nothing.  Each
// device holds its own copy of the array from the first context created on
// it until the process ends; host code never uses the array's name as an
// address (that is a host-side stand-in), only the device address resolved
// once per device by hipGetSymbolAddress with that device current.
static __device__ __align__(256) uint8_t scratch[BD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int resolve_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(BD_EINVAL, "device %d beyond the scratch table", device);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return BD_OK;
    DeviceGuard guard(device);
    if (guard.err != hipSuccess) return fail(BD_EDEVICE, "hipSetDevice(%d): %s", device, hipGetErrorString(guard.err));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(BD_EDEVICE, "scratch address on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return BD_OK;
}

void* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

int reserve_workspace(bd_context* ctx, size_t bytes, hipStream_t stream, void** out)
{
    if (bytes == 0) {
        *out = ctx->workspace;
        return BD_OK;
    }
    if (bytes > ctx->workspace_bytes) {
        DeviceGuard guard(ctx->device);
        hipError_t e = guard.err;
        if (e != hipSuccess) return fail(BD_EDEVICE, "hipSetDevice(%d): %s", ctx->device, hipGetErrorString(e));
        if (ctx->workspace) {
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return fail(BD_EDEVICE, "workspace growth: stream sync failed: %s", hipGetErrorString(e));
            (void)hipFree(ctx->workspace);
            ctx->workspace = nullptr;
            ctx->workspace_bytes = 0;
        }
        const size_t want = (bytes + 0xFFFFF) & ~(size_t)0xFFFFF;  // whole MiB
        const char* inject = getenv("BD_TEST_FAIL_ALLOC");
        if (inject && inject[0] == '1') return fail(BD_ENOMEM, "workspace allocation of %zu bytes failed (injected)", want);
        void* p = nullptr;
        e = hipMalloc(&p, want);
        if (e != hipSuccess) return fail(BD_ENOMEM, "workspace allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
        ctx->workspace = p;
        ctx->workspace_bytes = want;
    }
    *out = ctx->workspace;
    return BD_OK;
}

}  // namespace bd

using namespace bd;

namespace {

bool is_supported_bits(int32_t n_bits) { return n_bits == 256 || n_bits == 512; }

int check_ctx(bd_context* ctx, const char* fn)
{
    if (!ctx) return fail(BD_EINVAL, "%s: null context", fn);
    return BD_OK;
}

}  // namespace

extern "C" {

const char* bd_last_error(void) { return bd::g_error; }

const char* bd_version(void) { return "bdesc 0.1 gfx950"; }

int bd_context_create(bd_context** out, int device)
{
    if (!out) return fail(BD_EINVAL, "bd_context_create: null output pointer");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return fail(BD_EDEVICE, "bd_context_create: no HIP device (%s)", e == hipSuccess ? "count 0" : hipGetErrorString(e));
    if (device < 0 || device >= count)
        return fail(BD_EINVAL, "bd_context_create: device %d out of range [0, %d)", device, count);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return fail(BD_EDEVICE, "bd_context_create: %s", hipGetErrorString(e));
    if (int rc = resolve_scratch(device)) return rc;
    bd_context* ctx = new (std::nothrow) bd_context();
    if (!ctx) return fail(BD_ENOMEM, "bd_context_create: out of host memory");
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    {
        DeviceGuard guard(device);
        e = guard.err;
        if (e == hipSuccess) e = hipMalloc((void**)&ctx->invalid, sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMemset(ctx->invalid, 0, sizeof(unsigned long long));
    }
    if (e != hipSuccess) {
        if (ctx->invalid) (void)hipFree(ctx->invalid);
        delete ctx;
        return fail(BD_ENOMEM, "bd_context_create: invalid-keypoint counter: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return BD_OK;
}

int bd_context_poll(bd_context* ctx, uint64_t* invalid_count)
{
    const char* fn = "bd_context_poll";
    if (!invalid_count) return fail(BD_EINVAL, "%s: null output pointer", fn);
    *invalid_count = 0;
    if (int rc = check_ctx(ctx, fn)) return rc;
    DeviceGuard guard(ctx->device);
    hipError_t e = guard.err;
    if (e == hipSuccess) e = hipDeviceSynchronize();
    unsigned long long v = 0;
    if (e == hipSuccess) e = hipMemcpy(&v, ctx->invalid, sizeof v, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(ctx->invalid, 0, sizeof v);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(BD_EDEVICE, "%s: %s", fn, hipGetErrorString(e));
    *invalid_count = v;
    return BD_OK;
}

int bd_context_destroy(bd_context* ctx)
{
    if (!ctx) return BD_OK;
    int rc = BD_OK;
    {
        DeviceGuard guard(ctx->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = fail(BD_EDEVICE, "bd_context_destroy: %s", hipGetErrorString(e));
        if (ctx->workspace) (void)hipFree(ctx->workspace);
        if (ctx->invalid) (void)hipFree(ctx->invalid);
    }
    delete ctx;
    return rc;
}

int bd_build_integral(bd_context* ctx, const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch,
                      uint32_t* ii, int64_t ii_pitch, void* stream)
{
    const char* fn = "bd_build_integral";
    if (W < 1 || H < 1) return fail(BD_EINVAL, "%s: image size %dx%d must be at least 1x1", fn, W, H);
    if (img_pitch < W) return fail(BD_EINVAL, "%s: img_pitch %lld < W %d", fn, (long long)img_pitch, W);
    if (ii_pitch < (int64_t)W + 1) return fail(BD_EINVAL, "%s: ii_pitch %lld < W+1", fn, (long long)ii_pitch);
    if (((int64_t)H + 1) * ii_pitch >= (int64_t)1 << 31)
        return fail(BD_EINVAL, "%s: integral image of %lld elements exceeds 2^31", fn, (long long)(((int64_t)H + 1) * ii_pitch));
    if (!img || !ii) return fail(BD_EINVAL, "%s: null image or output pointer", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const IntegralPlan plan = plan_integral(W, H);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, plan.workspace_bytes(), s, &ws)) return rc;
    launch_integral(plan, img, img_pitch, ii, ii_pitch, ws, s);
    return check_launch(fn);
}

namespace {

// The integral image, keypoint order and optional row-pair image of one
// view (bd_build_integral_order, bd_prepare_view).
int prepare_view(const char* fn, bd_context* ctx, const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch,
                 uint32_t* ii, int64_t ii_pitch, const bd_keypoint* kps, int32_t n_kp, int32_t* order,
                 const float* hs_img, int64_t hs_pitch, float* pairs, int64_t pairs_pitch, void* stream)
{
    if (W < 1 || H < 1) return fail(BD_EINVAL, "%s: image size %dx%d must be at least 1x1", fn, W, H);
    if (img_pitch < W) return fail(BD_EINVAL, "%s: img_pitch %lld < W %d", fn, (long long)img_pitch, W);
    if (ii_pitch < (int64_t)W + 1) return fail(BD_EINVAL, "%s: ii_pitch %lld < W+1", fn, (long long)ii_pitch);
    if (((int64_t)H + 1) * ii_pitch >= (int64_t)1 << 31)
        return fail(BD_EINVAL, "%s: integral image of %lld elements exceeds 2^31", fn, (long long)(((int64_t)H + 1) * ii_pitch));
    if (!img || !ii) return fail(BD_EINVAL, "%s: null image or output pointer", fn);
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!kps || !order)) return fail(BD_EINVAL, "%s: null keypoint or order pointer", fn);
    if (hs_img || pairs) {
        if (!hs_img || !pairs) return fail(BD_EINVAL, "%s: hs_img and pairs go together", fn);
        if (hs_pitch < 4 * (int64_t)W || hs_pitch % 4 != 0 || reinterpret_cast<uintptr_t>(hs_img) % 4 != 0)
            return fail(BD_EINVAL, "%s: hs_pitch %lld must be a multiple of 4 and >= 4 W", fn, (long long)hs_pitch);
        if (pairs_pitch < 8 * (int64_t)W || pairs_pitch % 8 != 0 || reinterpret_cast<uintptr_t>(pairs) % 8 != 0)
            return fail(BD_EINVAL, "%s: pairs_pitch %lld must be a multiple of 8 and >= 8 W", fn,
                        (long long)pairs_pitch);
        if (!hashsift_image_fits(pairs_pitch, H))
            return fail(BD_EINVAL, "%s: row-pair image needs pairs_pitch < 2^24, H < 2^24 and pairs_pitch * H <= 2^32",
                        fn);
    }
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const IntegralPlan plan = plan_integral(W, H);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, plan.workspace_bytes(), s, &ws)) return rc;
    if (n_kp == 0 && !hs_img)
        launch_integral(plan, img, img_pitch, ii, ii_pitch, ws, s);
    else
        launch_prepare_view(plan, img, img_pitch, ii, ii_pitch, ws, kps, n_kp, order, hs_img, hs_pitch / 4, pairs,
                            pairs_pitch / 8, s);
    return check_launch(fn);
}

}  // namespace

int bd_build_integral_order(bd_context* ctx, const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch,
                            uint32_t* ii, int64_t ii_pitch, const bd_keypoint* kps, int32_t n_kp, int32_t* order,
                            void* stream)
{
    return prepare_view("bd_build_integral_order", ctx, img, W, H, img_pitch, ii, ii_pitch, kps, n_kp, order, nullptr,
                        0, nullptr, 0, stream);
}

int bd_prepare_view(bd_context* ctx, const uint8_t* img, int32_t W, int32_t H, int64_t img_pitch, uint32_t* ii,
                    int64_t ii_pitch, const bd_keypoint* kps, int32_t n_kp, int32_t* order, const float* hs_img,
                    int64_t hs_pitch, float* pairs, int64_t pairs_pitch, void* stream)
{
    return prepare_view("bd_prepare_view", ctx, img, W, H, img_pitch, ii, ii_pitch, kps, n_kp, order, hs_img,
                        hs_pitch, pairs, pairs_pitch, stream);
}

int bd_keypoint_order(bd_context* ctx, const bd_keypoint* kps, int32_t n_kp, int32_t W, int32_t H,
                      int32_t* order, void* stream)
{
    const char* fn = "bd_keypoint_order";
    if (W < 1 || H < 1) return fail(BD_EINVAL, "%s: image size %dx%d must be at least 1x1", fn, W, H);
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!kps || !order)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_kp == 0) return BD_OK;
    launch_keypoint_order(kps, n_kp, W, H, order, static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int bd_describe_bad(bd_context* ctx, const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch,
                    const bd_keypoint* kps, int32_t n_kp, const int32_t* order, const bd_box_pair* pairs,
                    int32_t n_bits, uint64_t* codes, void* stream)
{
    const char* fn = "bd_describe_bad";
    if (!is_supported_bits(n_bits)) return fail(BD_EUNSUPPORTED, "%s: n_bits %d (256 or 512)", fn, n_bits);
    if (W < 1 || H < 1) return fail(BD_EINVAL, "%s: image size %dx%d must be at least 1x1", fn, W, H);
    if (ii_pitch < (int64_t)W + 1) return fail(BD_EINVAL, "%s: ii_pitch %lld < W+1", fn, (long long)ii_pitch);
    if (((int64_t)H + 1) * ii_pitch >= (int64_t)1 << 31) return fail(BD_EINVAL, "%s: integral image exceeds 2^31 elements", fn);
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!ii || !kps || !pairs || !codes)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_kp == 0) return BD_OK;
    launch_bad(ii, W, H, ii_pitch, kps, n_kp, order, pairs, n_bits / 64, codes, ctx->invalid,
               static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

}  // extern "C"

struct bd_bad_table {
    int device = 0;
    int32_t n_bits = 0;
    uint8_t* data = nullptr;  // device, bad_table_bytes(n_bits)
};

extern "C" {

int bd_bad_table_create(bd_context* ctx, const bd_box_pair* pairs, int32_t n_bits, bd_bad_table** out, void* stream)
{
    const char* fn = "bd_bad_table_create";
    if (!out) return fail(BD_EINVAL, "%s: null output pointer", fn);
    *out = nullptr;
    if (!is_supported_bits(n_bits)) return fail(BD_EUNSUPPORTED, "%s: n_bits %d (256 or 512)", fn, n_bits);
    if (!pairs) return fail(BD_EINVAL, "%s: null pairs", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    bd_bad_table* t = new (std::nothrow) bd_bad_table();
    if (!t) return fail(BD_ENOMEM, "%s: out of host memory", fn);
    t->device = ctx->device;
    t->n_bits = n_bits;
    DeviceGuard guard(ctx->device);
    hipError_t e = guard.err;
    if (e == hipSuccess) e = hipMalloc((void**)&t->data, bad_table_bytes(n_bits));
    if (e != hipSuccess) {
        delete t;
        return fail(BD_ENOMEM, "%s: allocation failed: %s", fn, hipGetErrorString(e));
    }
    launch_bad_compile(pairs, n_bits, t->data, static_cast<hipStream_t>(stream));
    if (int rc = check_launch(fn)) {
        (void)hipFree(t->data);
        delete t;
        return rc;
    }
    *out = t;
    return BD_OK;
}

int bd_bad_table_destroy(bd_bad_table* t)
{
    if (!t) return BD_OK;
    int rc = BD_OK;
    {
        DeviceGuard guard(t->device);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = fail(BD_EDEVICE, "bd_bad_table_destroy: %s", hipGetErrorString(e));
        (void)hipFree(t->data);
    }
    delete t;
    return rc;
}

int bd_describe_bad_table(bd_context* ctx, const uint32_t* ii, int32_t W, int32_t H, int64_t ii_pitch,
                          const bd_keypoint* kps, int32_t n_kp, const int32_t* order, const bd_bad_table* table,
                          uint64_t* codes, void* stream)
{
    const char* fn = "bd_describe_bad_table";
    if (!table) return fail(BD_EINVAL, "%s: null table", fn);
    if (W < 1 || H < 1) return fail(BD_EINVAL, "%s: image size %dx%d must be at least 1x1", fn, W, H);
    if (ii_pitch < (int64_t)W + 1) return fail(BD_EINVAL, "%s: ii_pitch %lld < W+1", fn, (long long)ii_pitch);
    if (((int64_t)H + 1) * ii_pitch >= (int64_t)1 << 31) return fail(BD_EINVAL, "%s: integral image exceeds 2^31 elements", fn);
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!ii || !kps || !codes)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (table->device != ctx->device) return fail(BD_EINVAL, "%s: table belongs to device %d", fn, table->device);
    if (n_kp == 0) return BD_OK;
    launch_bad_compiled(ii, W, H, ii_pitch, kps, n_kp, order, table->data, table->n_bits / 64, codes, ctx->invalid,
                        static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int check_image(const char* fn, int32_t dtype, int32_t W, int32_t H, int64_t img_pitch, const void* img)
{
    if (dtype != BD_DTYPE_U8 && dtype != BD_DTYPE_F32 && dtype != BD_DTYPE_F32_ROWPAIR)
        return fail(BD_EUNSUPPORTED, "%s: dtype %d", fn, dtype);
    if (W < 1 || H < 1) return fail(BD_EINVAL, "%s: image size %dx%d must be at least 1x1", fn, W, H);
    const int64_t elem = dtype == BD_DTYPE_U8 ? 1 : dtype == BD_DTYPE_F32 ? 4 : 8;
    if (img_pitch < W * elem) return fail(BD_EINVAL, "%s: img_pitch %lld < row bytes", fn, (long long)img_pitch);
    if (dtype == BD_DTYPE_F32 && img_pitch % 4 != 0) return fail(BD_EINVAL, "%s: f32 img_pitch must be a multiple of 4", fn);
    if (dtype == BD_DTYPE_F32_ROWPAIR && (img_pitch % 8 != 0 || reinterpret_cast<uintptr_t>(img) % 8 != 0))
        return fail(BD_EINVAL, "%s: row-pair image and img_pitch must be 8-byte aligned", fn);
    if (!hashsift_image_fits(img_pitch, H))
        return fail(BD_EINVAL, "%s: image needs img_pitch < 2^24, H < 2^24 and img_pitch * H <= 2^32", fn);
    return BD_OK;
}

int check_projection(const char* fn, int32_t n_bits, int32_t precision, float margin)
{
    if (!is_supported_bits(n_bits)) return fail(BD_EUNSUPPORTED, "%s: n_bits %d (256 or 512)", fn, n_bits);
    if (precision != BD_PREC_FP32 && precision != BD_PREC_BF16 && precision != BD_PREC_FP8)
        return fail(BD_EUNSUPPORTED, "%s: precision %d", fn, precision);
    if (!(margin >= 0.0f) || margin > 1e30f) return fail(BD_EINVAL, "%s: margin must be finite and >= 0", fn);
    return BD_OK;
}

int bd_hashsift_features(bd_context* ctx, const void* img, int32_t dtype, int32_t W, int32_t H,
                         int64_t img_pitch, const bd_keypoint* kps, int32_t n_kp, const int32_t* order,
                         float* hist, void* stream)
{
    const char* fn = "bd_hashsift_features";
    if (int rc = check_image(fn, dtype, W, H, img_pitch, img)) return rc;
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!img || !kps || !hist)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_kp == 0) return BD_OK;
    launch_hashsift_hist(img, dtype, W, H, img_pitch, kps, n_kp, order, hist, ctx->invalid,
                         static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int bd_hashsift_project(bd_context* ctx, const float* hist, const bd_keypoint* kps, int32_t n_kp, const float* B,
                        const float* t, int32_t n_bits, int32_t precision, float margin, uint64_t* codes,
                        float* resp_out, uint32_t* recheck_count, void* stream)
{
    const char* fn = "bd_hashsift_project";
    if (int rc = check_projection(fn, n_bits, precision, margin)) return rc;
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!hist || !B || !t || !codes)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_kp == 0) return BD_OK;
    launch_hashsift_project(precision, hist, kps, n_kp, B, t, n_bits / 64, margin, codes, resp_out, recheck_count,
                            static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int bd_describe_hashsift(bd_context* ctx, const void* img, int32_t dtype, int32_t W, int32_t H,
                         int64_t img_pitch, const bd_keypoint* kps, int32_t n_kp, const int32_t* order,
                         const float* B, const float* t, int32_t n_bits, int32_t precision, float margin,
                         uint64_t* codes, float* hist_out, float* resp_out, uint32_t* recheck_count, void* stream)
{
    const char* fn = "bd_describe_hashsift";
    if (int rc = check_projection(fn, n_bits, precision, margin)) return rc;
    if (int rc = check_image(fn, dtype, W, H, img_pitch, img)) return rc;
    if (n_kp < 0) return fail(BD_EINVAL, "%s: n_kp %d < 0", fn, n_kp);
    if (n_kp > 0 && (!img || !kps || !B || !t || !codes)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_kp == 0) return BD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* hist = hist_out;
    if (!hist) {
        void* ws = nullptr;
        if (int rc = reserve_workspace(ctx, sizeof(float) * 128 * (size_t)n_kp, s, &ws)) return rc;
        hist = static_cast<float*>(ws);
    }
    launch_hashsift_hist(img, dtype, W, H, img_pitch, kps, n_kp, order, hist, ctx->invalid, s);
    launch_hashsift_project(precision, hist, kps, n_kp, B, t, n_bits / 64, margin, codes, resp_out, recheck_count, s);
    return check_launch(fn);
}

int bd_match_hamming_knn(bd_context* ctx, const uint64_t* query, int32_t n_q, const uint64_t* train,
                         int32_t n_t, int32_t n_words, int32_t k, int32_t* idx, uint32_t* dist, void* stream)
{
    const char* fn = "bd_match_hamming_knn";
    if (n_words < 1 || n_words > 8) return fail(BD_EUNSUPPORTED, "%s: n_words %d (1..8)", fn, n_words);
    if (k < 1 || k > 2) return fail(BD_EUNSUPPORTED, "%s: k %d (1 or 2)", fn, k);
    if (n_q < 0 || n_t < 0) return fail(BD_EINVAL, "%s: negative count", fn);
    if (n_q > 0 && (!query || !idx || !dist)) return fail(BD_EINVAL, "%s: null query or output pointer", fn);
    if (n_q > 0 && n_t > 0 && !train) return fail(BD_EINVAL, "%s: null train pointer", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_q == 0) return BD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const KnnPlan plan = plan_knn(n_q, n_t, n_words, k, ctx->num_cus);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, plan.workspace_bytes(), s, &ws)) return rc;
    launch_knn(plan, query, train, idx, dist, ws, s);
    return check_launch(fn);
}

int bd_match_hamming_knn_noalloc(bd_context* ctx, const uint64_t* query, int32_t n_q, const uint64_t* train,
                                 int32_t n_t, int32_t n_words, int32_t k, int32_t* idx, uint32_t* dist, void* stream)
{
    const char* fn = "bd_match_hamming_knn_noalloc";
    if (n_words < 1 || n_words > 8) return fail(BD_EUNSUPPORTED, "%s: n_words %d (1..8)", fn, n_words);
    if (k < 1 || k > 2) return fail(BD_EUNSUPPORTED, "%s: k %d (1 or 2)", fn, k);
    if (n_q < 0 || n_t < 0) return fail(BD_EINVAL, "%s: negative count", fn);
    if (n_q > 0 && (!query || !idx || !dist)) return fail(BD_EINVAL, "%s: null query or output pointer", fn);
    if (n_q > 0 && n_t > 0 && !train) return fail(BD_EINVAL, "%s: null train pointer", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_q == 0) return BD_OK;
    // the same plan, hence the same kernels and launch shapes, as bd_match_hamming_knn
    const KnnPlan plan = plan_knn(n_q, n_t, n_words, k, ctx->num_cus);
    const size_t need = plan.workspace_bytes();
    if (need > (size_t)BD_NOALLOC_SCRATCH_BYTES)
        return fail(BD_EINVAL, "%s: %d queries x %d train codes need %zu bytes of scratch, above the fixed %d", fn,
                    n_q, n_t, need, (int)BD_NOALLOC_SCRATCH_BYTES);
    void* ws = scratch_of(ctx->device);
    if (!ws) return fail(BD_EDEVICE, "%s: no scratch resolved for device %d", fn, ctx->device);
    // every per-split slot is written before the merge reads it: nothing to clear
    launch_knn(plan, query, train, idx, dist, ws, static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int bd_match_mutual(bd_context* ctx, const uint64_t* query, int32_t n_q, const uint64_t* train, int32_t n_t,
                    int32_t n_words, float max_ratio, int32_t* match, uint32_t* dist, float* ratio, int32_t* count,
                    void* stream)
{
    const char* fn = "bd_match_mutual";
    if (n_words < 1 || n_words > 8) return fail(BD_EUNSUPPORTED, "%s: n_words %d (1..8)", fn, n_words);
    if (n_q < 0 || n_t < 0) return fail(BD_EINVAL, "%s: negative count", fn);
    if (!(max_ratio >= 0.0f) || max_ratio > 1e30f) return fail(BD_EINVAL, "%s: max_ratio must be finite and >= 0", fn);
    if (n_q > 0 && (!query || !match || !dist)) return fail(BD_EINVAL, "%s: null query or output pointer", fn);
    if (n_q > 0 && n_t > 0 && !train) return fail(BD_EINVAL, "%s: null train pointer", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_q == 0 && !count) return BD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const MutualPlan plan = plan_mutual(n_q, n_t, n_words, ctx->num_cus);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, plan.workspace_bytes(), s, &ws)) return rc;
    launch_mutual(plan, query, train, max_ratio, match, dist, ratio, count, ws, s);
    return check_launch(fn);
}

int bd_find_threshold(bd_context* ctx, const uint8_t* patches, int32_t n_triplets, const int32_t* s_ap,
                      const int32_t* s_an, float tau, const bd_box_pair* cands, int32_t n_cands, int32_t* best_bin,
                      float* best_theta, double* best_loss, void* stream)
{
    const char* fn = "bd_find_threshold";
    if (n_triplets < 0 || n_cands < 0) return fail(BD_EINVAL, "%s: negative count", fn);
    if (n_triplets > (1 << 24)) return fail(BD_EINVAL, "%s: more than 2^24 triplets", fn);
    const float tau2 = 2.0f * tau;
    if (!(tau2 == tau2) || tau2 != (float)(int)tau2 || fabsf(tau) > 65536.0f)
        return fail(BD_EINVAL, "%s: tau must be a multiple of 1/2 with |tau| <= 65536", fn);
    if (n_cands > 0 && (!cands || !best_bin)) return fail(BD_EINVAL, "%s: null candidate or output pointer", fn);
    if (n_cands > 0 && n_triplets > 0 && (!patches || !s_ap || !s_an))
        return fail(BD_EINVAL, "%s: null triplet input", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n_cands == 0) return BD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, select_workspace(n_cands), s, &ws)) return rc;
    launch_find_threshold(patches, nullptr, n_triplets, s_ap, s_an, (int)tau2, cands, n_cands, best_bin,
                          best_theta, best_loss, ws, ctx->num_cus, s);
    return check_launch(fn);
}

int bd_select_features(bd_context* ctx, const uint8_t* pool, int32_t n_pairs, const int32_t* samples,
                       int32_t n_sample, const bd_box_pair* cands, int32_t n_cands, int32_t n_bits, float tau,
                       bd_box_pair* table, int32_t* chosen, int32_t* chosen_bin, double* round_loss,
                       uint64_t* pool_codes, void* stream)
{
    const char* fn = "bd_select_features";
    if (n_bits < 1 || n_bits > 512) return fail(BD_EUNSUPPORTED, "%s: n_bits %d (1..512)", fn, n_bits);
    if (n_pairs < 2 || n_sample < 2 || n_sample > n_pairs)
        return fail(BD_EINVAL, "%s: need 2 <= n_sample <= n_pairs (got %d, %d)", fn, n_sample, n_pairs);
    if (n_pairs > (1 << 22) || n_sample > (1 << 22)) return fail(BD_EINVAL, "%s: more than 2^22 pairs", fn);
    if (n_cands < 1) return fail(BD_EINVAL, "%s: n_cands %d < 1", fn, n_cands);
    const float tau2 = 2.0f * tau;
    if (!(tau2 == tau2) || tau2 != (float)(int)tau2 || fabsf(tau) > 65536.0f)
        return fail(BD_EINVAL, "%s: tau must be a multiple of 1/2 with |tau| <= 65536", fn);
    if (!pool || !samples || !cands || !table) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, select_features_workspace(n_pairs, n_sample, n_cands, n_bits, ctx->num_cus),
                                   s, &ws))
        return rc;
    launch_select_features(pool, n_pairs, samples, n_sample, cands, n_cands, n_bits, (int)tau2, table, chosen,
                           chosen_bin, round_loss, pool_codes, ws, ctx->num_cus, s);
    return check_launch(fn);
}

int bd_hashsift_patch_features(bd_context* ctx, const float* patches, int32_t n, float* hist, void* stream)
{
    const char* fn = "bd_hashsift_patch_features";
    if (n < 0) return fail(BD_EINVAL, "%s: n %d < 0", fn, n);
    if (n > 0 && (!patches || !hist)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n == 0) return BD_OK;
    launch_hashsift_patch_features(patches, n, hist, static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

static int check_relaxed(const char* fn, int32_t n, int32_t n_bits, float beta)
{
    if (n_bits < 64 || n_bits % 64 != 0 || n_bits > 4096)
        return fail(BD_EUNSUPPORTED, "%s: n_bits %d (a multiple of 64 up to 4096)", fn, n_bits);
    if (n < 0) return fail(BD_EINVAL, "%s: n %d < 0", fn, n);
    if (!(beta > 0.0f) || beta > 1e30f) return fail(BD_EINVAL, "%s: beta must be finite and > 0", fn);
    return BD_OK;
}

int bd_relaxed_bad_fwd(bd_context* ctx, const float* patches, int32_t n, const bd_box_pair* pairs, const float* w1,
                       const float* w2, const float* theta, int32_t n_bits, float beta, float* D, float* m1, float* m2,
                       void* stream)
{
    const char* fn = "bd_relaxed_bad_fwd";
    if (int rc = check_relaxed(fn, n, n_bits, beta)) return rc;
    if (n > 0 && (!patches || !pairs || !w1 || !w2 || !theta || !D)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n == 0) return BD_OK;
    launch_relaxed_bad_fwd(patches, n, pairs, w1, w2, theta, n_bits, beta, D, m1, m2, static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int bd_relaxed_bad_bwd(bd_context* ctx, const float* gD, const float* D, const float* m1, const float* m2, int32_t n,
                       int32_t n_bits, float beta, float* g_w1, float* g_w2, float* g_theta, void* stream)
{
    const char* fn = "bd_relaxed_bad_bwd";
    if (int rc = check_relaxed(fn, n, n_bits, beta)) return rc;
    if (!g_w1 || !g_w2 || !g_theta) return fail(BD_EINVAL, "%s: null gradient output", fn);
    if (n > 0 && (!gD || !D || !m1 || !m2)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, relaxed_bad_bwd_workspace(n > 0 ? n : 1, n_bits), s, &ws)) return rc;
    launch_relaxed_bad_bwd(gD, D, m1, m2, n, n_bits, beta, g_w1, g_w2, g_theta, ws, s);
    return check_launch(fn);
}

int bd_relaxed_hashsift_fwd(bd_context* ctx, const float* f, int32_t n, const float* B, const float* t, int32_t n_bits,
                            float beta, float* rho, float* D, void* stream)
{
    const char* fn = "bd_relaxed_hashsift_fwd";
    if (int rc = check_relaxed(fn, n, n_bits, beta)) return rc;
    if (n_bits != 256 && n_bits != 512) return fail(BD_EUNSUPPORTED, "%s: n_bits %d (256 or 512)", fn, n_bits);
    if (n > 0 && (!f || !B || !t || !D)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    if (n == 0) return BD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* r = rho;
    void* ws = nullptr;
    const size_t codes_bytes = sizeof(uint64_t) * (size_t)n * (size_t)(n_bits / 64);
    const size_t rho_bytes = rho ? 0 : sizeof(float) * (size_t)n * (size_t)n_bits;
    if (int rc = reserve_workspace(ctx, codes_bytes + rho_bytes, s, &ws)) return rc;
    uint64_t* codes = static_cast<uint64_t*>(ws);
    if (!r) r = reinterpret_cast<float*>(codes + (size_t)n * (size_t)(n_bits / 64));
    launch_hashsift_project(BD_PREC_FP32, f, nullptr, n, B, t, n_bits / 64, 0.0f, codes, r, nullptr, s);
    launch_tanh_scale(r, (int64_t)n * n_bits, beta, D, s);
    return check_launch(fn);
}

int bd_relaxed_hashsift_bwd(bd_context* ctx, const float* gD, const float* D, const float* f, int32_t n,
                            int32_t n_bits, float beta, float* gB, float* gt, void* stream)
{
    const char* fn = "bd_relaxed_hashsift_bwd";
    if (int rc = check_relaxed(fn, n, n_bits, beta)) return rc;
    if (!gB || !gt) return fail(BD_EINVAL, "%s: null gradient output", fn);
    if (n > 0 && (!gD || !D || !f)) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, relaxed_hs_bwd_workspace(n > 0 ? n : 1, n_bits), s, &ws)) return rc;
    launch_relaxed_hs_bwd(gD, D, f, n, n_bits, beta, gB, gt, ws, s);
    return check_launch(fn);
}

int bd_trl_hnm_fwd(bd_context* ctx, const float* A, const float* P, int32_t n, int32_t n_bits, float tau, float* loss,
                   int32_t* neg, float* hinge, void* stream)
{
    const char* fn = "bd_trl_hnm_fwd";
    if (n_bits < 64 || n_bits % 64 != 0 || n_bits > 4096)
        return fail(BD_EUNSUPPORTED, "%s: n_bits %d (a multiple of 64 up to 4096)", fn, n_bits);
    if (n < 1) return fail(BD_EINVAL, "%s: n %d < 1", fn, n);
    if (!(tau == tau) || tau > 1e30f || tau < -1e30f) return fail(BD_EINVAL, "%s: tau must be finite", fn);
    if (!A || !P || !loss || !neg || !hinge) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, trl_workspace(n), s, &ws)) return rc;
    launch_trl_fwd(A, P, n, n_bits, tau, loss, neg, hinge, ws, s);
    return check_launch(fn);
}

int bd_trl_hnm_bwd(bd_context* ctx, const float* A, const float* P, int32_t n, int32_t n_bits, const int32_t* neg,
                   const float* hinge, const float* grad_loss, float* gA, float* gP, void* stream)
{
    const char* fn = "bd_trl_hnm_bwd";
    if (n_bits < 64 || n_bits % 64 != 0 || n_bits > 4096)
        return fail(BD_EUNSUPPORTED, "%s: n_bits %d (a multiple of 64 up to 4096)", fn, n_bits);
    if (n < 1) return fail(BD_EINVAL, "%s: n %d < 1", fn, n);
    if (!A || !P || !neg || !hinge || !grad_loss || !gA || !gP) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, trl_workspace(n), s, &ws)) return rc;
    launch_trl_bwd(A, P, n, n_bits, neg, hinge, grad_loss, gA, gP, ws, s);
    return check_launch(fn);
}

int bd_augment_patches(bd_context* ctx, const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n,
                       const float* params, const float* noise, float* out, void* stream)
{
    const char* fn = "bd_augment_patches";
    if (n_pairs < 1 || n < 1) return fail(BD_EINVAL, "%s: need n_pairs >= 1 and n >= 1", fn);
    if (!pool || !batch || !params || !noise || !out) return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    launch_augment(pool, n_pairs, batch, n, params, noise, out, static_cast<hipStream_t>(stream));
    return check_launch(fn);
}

int bd_hashsift_train_step(bd_context* ctx, const float* pool, int32_t n_pairs, const int32_t* batch, int32_t n,
                           const float* params, const float* noise, float* B, float* t, int32_t n_bits,
                           float* adam_state, int32_t step, float lr, float tau, float beta, float* loss,
                           void* stream)
{
    const char* fn = "bd_hashsift_train_step";
    if (n_bits != 256 && n_bits != 512) return fail(BD_EUNSUPPORTED, "%s: n_bits %d (256 or 512)", fn, n_bits);
    if (n_pairs < 2 || n < 2) return fail(BD_EINVAL, "%s: need n_pairs >= 2 and n >= 2", fn);
    if (n > (1 << 20)) return fail(BD_EINVAL, "%s: batch of %d pairs exceeds 2^20", fn, n);
    if (step < 1) return fail(BD_EINVAL, "%s: step %d (counts from 1)", fn, step);
    if (!(lr > 0.0f) || lr > 1e30f || !(beta > 0.0f) || beta > 1e30f || !(tau == tau) || fabsf(tau) > 1e30f)
        return fail(BD_EINVAL, "%s: lr and beta must be finite and > 0, tau finite", fn);
    if (!pool || !batch || !params || !noise || !B || !t || !adam_state || !loss)
        return fail(BD_EINVAL, "%s: null pointer argument", fn);
    if (int rc = check_ctx(ctx, fn)) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* ws = nullptr;
    if (int rc = reserve_workspace(ctx, train_step_workspace(n, n_bits), s, &ws)) return rc;
    launch_train_step(pool, n_pairs, batch, n, params, noise, B, t, n_bits, adam_state, step, lr, tau, beta, loss,
                      ws, s);
    return check_launch(fn);
}

}  // extern "C"
