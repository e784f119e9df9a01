// Context, scratch arena and error reporting of libdressi.
#include "dressi_internal.h"

#include <cstdio>
#include <new>

int dressi_fail(dressi_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int dressi_hip_check(dressi_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return DRESSI_OK;
    return dressi_fail(ctx, DRESSI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int dressi_launch_check(dressi_ctx *ctx, const char *what) {
    return dressi_hip_check(ctx, hipGetLastError(), what);
}

extern "C" int dressi_create(dressi_ctx **out, int device) {
    if (!out) return DRESSI_EINVAL;
    *out = nullptr;
    dressi_ctx *ctx = new (std::nothrow) dressi_ctx();
    if (!ctx) return DRESSI_ENOMEM;
    ctx->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&ctx->status, 4 * sizeof(int64_t));
    if (e == hipSuccess) e = hipMemset(ctx->status, 0, 4 * sizeof(int64_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (ctx->status) (void)hipFree(ctx->status);
        delete ctx;
        return DRESSI_EHIP;
    }
    if (dressi_softras_noalloc_setup(device) != DRESSI_OK) {
        (void)hipFree(ctx->status);
        delete ctx;
        return DRESSI_EHIP;
    }
    *out = ctx;
    return DRESSI_OK;
}

extern "C" int dressi_destroy(dressi_ctx *ctx) {
    if (!ctx) return DRESSI_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->status) (void)hipFree(ctx->status);
    if (ctx->counters) (void)hipFree(ctx->counters);
    for (void *p : ctx->retired) (void)hipFree(p);
    delete ctx;
    return DRESSI_OK;
}

extern "C" const char *dressi_last_error(const dressi_ctx *ctx) {
    return ctx ? ctx->err.c_str() : "null context";
}

static int grow(dressi_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->scratch_bytes) return DRESSI_OK;
    size_t nb = bytes + bytes / 4 + (1 << 20);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return dressi_hip_check(ctx, e, "synchronize before scratch growth");
    void *p = nullptr;
    e = hipMalloc(&p, nb);
    if (e != hipSuccess)
        return dressi_fail(ctx, DRESSI_ENOMEM, "scratch allocation of " + std::to_string(nb) +
                                                   " bytes failed: " + hipGetErrorString(e));
    // the old arena is retired, not freed: graphs captured earlier use it
    if (ctx->scratch) ctx->retired.push_back(ctx->scratch);
    ctx->scratch = p;
    ctx->scratch_bytes = nb;
    return DRESSI_OK;
}

int dressi_scratch(dressi_ctx *ctx, size_t bytes, hipStream_t stream) {
    if (bytes <= ctx->scratch_bytes) return DRESSI_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return dressi_hip_check(ctx, e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return dressi_fail(ctx, DRESSI_ENOMEM,
                           "scratch too small during stream capture: need " + std::to_string(bytes) +
                               " bytes, call dressi_reserve before capturing");
    return grow(ctx, bytes);
}

int dressi_counters(dressi_ctx *ctx, size_t n, hipStream_t stream) {
    if (n <= ctx->counters_n) return DRESSI_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return dressi_hip_check(ctx, e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return dressi_fail(ctx, DRESSI_ENOMEM, "counter array too small during stream capture: "
                                               "run the call once before capturing");
    size_t nn = n + n / 4 + 4096;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return dressi_hip_check(ctx, e, "synchronize before counter growth");
    int32_t *p = nullptr;
    e = hipMalloc(&p, nn * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(p, 0, nn * sizeof(int32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (p) (void)hipFree(p);
        return dressi_fail(ctx, DRESSI_ENOMEM, std::string("counter allocation failed: ") + hipGetErrorString(e));
    }
    // retired like the arena (the kernels keep a retired array at zero)
    if (ctx->counters) ctx->retired.push_back(ctx->counters);
    ctx->counters = p;
    ctx->counters_n = nn;
    return DRESSI_OK;
}

extern "C" int dressi_reserve(dressi_ctx *ctx, size_t bytes, int64_t bin_entries) {
    if (!ctx) return DRESSI_EINVAL;
    if (bin_entries > ctx->bin_capacity) ctx->bin_capacity = bin_entries;
    return grow(ctx, bytes);
}

extern "C" int dressi_tune(dressi_ctx *ctx, int key, int64_t value) {
    if (!ctx) return DRESSI_EINVAL;
    switch (key) {
    case DRESSI_TUNE_BIN_CAPACITY:
        if (value < 0 || value > (1 << 26)) return dressi_fail(ctx, DRESSI_EINVAL, "tune: bad bin capacity");
        ctx->bin_capacity = value;   // 0 = automatic
        return DRESSI_OK;
    case DRESSI_TUNE_HARD_RASTER:
        if (value < 0 || value > 3) return dressi_fail(ctx, DRESSI_EINVAL, "tune: hard raster is 0, 1, 2 or 3");
        ctx->hard_raster = (int)value;
        return DRESSI_OK;
    case DRESSI_TUNE_HYBRID_WEIGHT:
        if (value < 1 || value > 1024) return dressi_fail(ctx, DRESSI_EINVAL, "tune: hybrid weight is 1..1024");
        ctx->hybrid_weight = (int)value;
        return DRESSI_OK;
    case DRESSI_TUNE_EMPTY_SLOTS:
        if (value != 0 && value != 1) return dressi_fail(ctx, DRESSI_EINVAL, "tune: empty slots is 0 or 1");
        ctx->skip_empty = (int)value;
        return DRESSI_OK;
    case DRESSI_TUNE_IV_ROWS:
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return dressi_fail(ctx, DRESSI_EINVAL, "tune: gather rows is 0, 1, 2 or 4");
        ctx->iv_rows = (int)value;
        return DRESSI_OK;
    default:
        return dressi_fail(ctx, DRESSI_EINVAL, "tune: unknown key");
    }
}

extern "C" int dressi_check_status(dressi_ctx *ctx, int64_t *needed, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    int64_t h[4];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(h, ctx->status, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dressi_hip_check(ctx, e, "reading device status");
    if (needed) *needed = h[1];
    if (h[0]) {
        // clear with a tiny fill kernel rather than a memset (capture friendly)
        dressi_fill_i32(reinterpret_cast<int32_t *>(ctx->status), 0, 8, s);
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return dressi_hip_check(ctx, e, "clearing device status");
        return dressi_fail(ctx, DRESSI_EOVERFLOW,
                           "tile-bin capacity exceeded: " + std::to_string(h[1]) +
                               " triangles per tile needed; call dressi_reserve and rerun");
    }
    return DRESSI_OK;
}

// ---------------------------------------------------------------------------
// kernel timing (eager runs only; never enable while capturing a graph)
// ---------------------------------------------------------------------------
namespace {
struct Prof {
    bool on = false;
    int cap = 0, used = 0;
    hipEvent_t *ev = nullptr;
    const char **names = nullptr;
};
Prof g_prof;

void prof_free() {
    for (int i = 0; i < 2 * g_prof.cap; i++) (void)hipEventDestroy(g_prof.ev[i]);
    delete[] g_prof.ev;
    delete[] g_prof.names;
    g_prof = Prof();
}
}  // namespace

bool dr_prof_slot(const char *name, hipEvent_t *start, hipEvent_t *stop) {
    if (!g_prof.on || g_prof.used >= g_prof.cap) return false;
    int i = g_prof.used++;
    g_prof.names[i] = name;
    *start = g_prof.ev[2 * i];
    *stop = g_prof.ev[2 * i + 1];
    return true;
}

extern "C" int dressi_profile_start(int max_launches) {
    prof_free();
    if (max_launches <= 0) return DRESSI_OK;
    g_prof.ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches];
    g_prof.names = new (std::nothrow) const char *[max_launches];
    if (!g_prof.ev || !g_prof.names) {
        prof_free();
        return DRESSI_ENOMEM;
    }
    for (int i = 0; i < 2 * max_launches; i++) {
        if (hipEventCreate(&g_prof.ev[i]) != hipSuccess) {
            g_prof.cap = i / 2;
            prof_free();
            return DRESSI_EHIP;
        }
        g_prof.cap = (i + 1) / 2;
    }
    g_prof.cap = max_launches;
    g_prof.on = true;
    return DRESSI_OK;
}

extern "C" int dressi_profile_read(const char **names, float *ms, int max) {
    int n = g_prof.used < max ? g_prof.used : max;
    for (int i = 0; i < n; i++) {
        if (hipEventSynchronize(g_prof.ev[2 * i + 1]) != hipSuccess) return DRESSI_EHIP;
        float t = 0.0f;
        if (hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess) return DRESSI_EHIP;
        names[i] = g_prof.names[i];
        ms[i] = t;
    }
    g_prof.used = 0;
    return n;
}
