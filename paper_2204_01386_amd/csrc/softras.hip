// HardSoftRas blend (§3.4.3, BuildBlend) and its backward for gfx950.
//
// Edge mask: the hard stencil S^H of the front layer, its 4-neighbour
// boundary (both sides), and an L-infinity dilation of radius
// rho = ceil(delta*W) - 1 done as a row pass then a column pass, integer
// exact.  The column pass is fused with the per-pixel blend.
#include "dressi_internal.h"

#include <mutex>

__device__ __forceinline__ bool front_hard(const int32_t *tri_id, const float *dist, int64_t o) {
    if (tri_id[o] < 0) return false;
    if (!dist) return true;
    return !signbit(dist[o]);
}

// S^H boundary: pixels whose S^H differs from an in-image 4-neighbour
__global__ void k_boundary(const int32_t *__restrict__ tri_id, const float *__restrict__ dist,
                           int B, int K, int H, int W, uint8_t *__restrict__ bnd) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t N = (int64_t)H * W;
    if (gid >= (int64_t)B * N) return;
    int b = (int)(gid / N);
    int p = (int)(gid - (int64_t)b * N);
    int y = p / W, x = p - y * W;
    int64_t o = (int64_t)b * K * N + p;
    bool s = front_hard(tri_id, dist, o);
    bool e = false;
    if (x > 0) e |= front_hard(tri_id, dist, o - 1) != s;
    if (x < W - 1) e |= front_hard(tri_id, dist, o + 1) != s;
    if (y > 0) e |= front_hard(tri_id, dist, o - W) != s;
    if (y < H - 1) e |= front_hard(tri_id, dist, o + W) != s;
    bnd[gid] = e ? 1 : 0;
}

// row pass of the dilation: any boundary pixel within |dx| <= rho
__global__ void k_dilate_rows(const uint8_t *__restrict__ bnd, int B, int H, int W, int rho,
                              uint8_t *__restrict__ rows) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t N = (int64_t)H * W;
    if (gid >= (int64_t)B * N) return;
    int64_t rowbase = gid - (gid % W);
    int x = (int)(gid % W);
    int a = max(x - rho, 0), e = min(x + rho, W - 1);
    uint8_t v = 0;
    for (int q = a; q <= e && !v; q++) v = bnd[rowbase + q];
    rows[gid] = v;
}

// column pass of the dilation, written out as the edge mask itself (the blend
// fuses this pass; the banded rasterizer needs the mask before any blend)
__global__ void k_dilate_cols(const uint8_t *__restrict__ rows, int B, int H, int W, int rho,
                              uint8_t *__restrict__ edge) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t N = (int64_t)H * W;
    if (gid >= (int64_t)B * N) return;
    int b = (int)(gid / N);
    int p = (int)(gid - (int64_t)b * N);
    int y = p / W, x = p - y * W;
    int a = max(y - rho, 0), e = min(y + rho, H - 1);
    const uint8_t *col = rows + (int64_t)b * N + x;
    uint8_t v = 0;
    for (int q = a; q <= e && !v; q++) v = col[(int64_t)q * W];
    edge[gid] = v;
}

void dressi_edge_mask(const int32_t *tri_id, const float *dist, int B, int K, int H, int W, int rho,
                      uint8_t *bnd, uint8_t *rows, uint8_t *edge, hipStream_t st) {
    const int64_t n = (int64_t)B * H * W;
    if (n == 0) return;
    const int g = (int)((n + 255) / 256);
    DR_LAUNCH("k_boundary", (k_boundary), g, 256, 0, st, tri_id, dist, B, K, H, W, bnd);
    DR_LAUNCH("k_dilate_rows", (k_dilate_rows), g, 256, 0, st, bnd, B, H, W, rho, rows);
    DR_LAUNCH("k_dilate_cols", (k_dilate_cols), g, 256, 0, st, rows, B, H, W, rho, edge);
}

// sigmoid(x) and 1 - sigmoid(x) = sigmoid(-x), each to full relative
// precision: the complement is never formed by subtracting from 1, which
// would lose it where the sigmoid is near 1 (its derivative w (1 - w) and
// the silhouette's product of complements use it).
__device__ __forceinline__ float sigmoid_pair(float x, float &q) {
    if (x >= 0.0f) {
        const float e = expf(-x), w = 1.0f / (1.0f + e);
        q = e * w;
        return w;
    }
    const float e = expf(x);
    q = 1.0f / (1.0f + e);
    return e * q;
}

template <int K>
__global__ void k_blend(const float *__restrict__ color, const float *__restrict__ dist,
                        const int32_t *__restrict__ tri_id, int B, int H, int W, int Cc,
                        float inv_sigma, int mode, int rho, const uint8_t *__restrict__ rows,
                        float *__restrict__ out_color, float *__restrict__ out_sil,
                        uint8_t *__restrict__ edge) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t N = (int64_t)H * W;
    if (gid >= (int64_t)B * N) return;
    int b = (int)(gid / N);
    int p = (int)(gid - (int64_t)b * N);
    int y = p / W, x = p - y * W;
    uint8_t E;
    if (mode == DRESSI_BLEND_SOFTRAS) E = 1;
    else if (mode == DRESSI_BLEND_HARD || rho < 0) E = 0;
    else {
        E = 0;
        int a = max(y - rho, 0), e = min(y + rho, H - 1);
        const uint8_t *col = rows + (int64_t)b * N + x;
        for (int q = a; q <= e && !E; q++) E = col[(int64_t)q * W];
    }
    edge[gid] = E;
    float *oc = out_color + gid * Cc;
    const int64_t o1 = (int64_t)b * K * N + p;
    if (!E) {
        bool sh = front_hard(tri_id, dist, o1);
        const float *c1 = color + o1 * Cc;
        for (int c = 0; c < Cc; c++) oc[c] = sh ? c1[c] : 0.0f;
        out_sil[gid] = sh ? 1.0f : 0.0f;
        return;
    }
    float w[K];
    float Wsum = 0.0f, prod = 1.0f;
    int nS = 0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        int64_t o = o1 + (int64_t)k * N;
        w[k] = 0.0f;
        if (tri_id[o] < 0) continue;
        float d = dist ? dist[o] : 0.0f;
        float q;
        w[k] = sigmoid_pair(d * inv_sigma, q);
        nS++;
        Wsum += w[k];
        prod *= q;
    }
    float inv = nS > 0 ? 1.0f / Wsum : 0.0f;
    for (int c = 0; c < Cc; c++) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < K; k++)
            if (w[k] != 0.0f) s += w[k] * color[(o1 + (int64_t)k * N) * Cc + c];
        oc[c] = s * inv;
    }
    out_sil[gid] = 1.0f - prod;
}

template <int K>
__global__ void k_blend_bwd(const float *__restrict__ color, const float *__restrict__ dist,
                            const int32_t *__restrict__ tri_id, int B, int H, int W, int Cc,
                            float inv_sigma, const uint8_t *__restrict__ edge,
                            const float *__restrict__ grad_color, const float *__restrict__ grad_sil,
                            float *__restrict__ grad_layer, float *__restrict__ grad_dist, int skip_empty) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t N = (int64_t)H * W;
    if (gid >= (int64_t)B * N) return;
    int b = (int)(gid / N);
    int p = (int)(gid - (int64_t)b * N);
    const int64_t o1 = (int64_t)b * K * N + p;
    const float *gc = grad_color + gid * Cc;
    float gs = grad_sil ? grad_sil[gid] : 0.0f;
    if (!edge[gid]) {
        bool sh = front_hard(tri_id, dist, o1);
#pragma unroll
        for (int k = 0; k < K; k++) {
            int64_t o = o1 + (int64_t)k * N;
            if (skip_empty && tri_id[o] < 0) continue;
            float *gl = grad_layer + o * Cc;
            for (int c = 0; c < Cc; c++) gl[c] = (k == 0 && sh) ? gc[c] : 0.0f;
            if (grad_dist) grad_dist[o] = 0.0f;
        }
        return;
    }
    float w[K], q[K];   // w_k and its complement 1 - w_k
    bool S[K];
    float Wsum = 0.0f;
#pragma unroll
    for (int k = 0; k < K; k++) {
        int64_t o = o1 + (int64_t)k * N;
        S[k] = tri_id[o] >= 0;
        q[k] = 1.0f;
        w[k] = S[k] ? sigmoid_pair((dist ? dist[o] : 0.0f) * inv_sigma, q[k]) : 0.0f;
        Wsum += w[k];
    }
    float inv = Wsum > 0.0f ? 1.0f / Wsum : 0.0f;
    // g_w_k = g_c . (C_k - I_c) / W + g_s prod_{j != k} (1 - w_j)
    float gw[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        float others = 1.0f;
#pragma unroll
        for (int j = 0; j < K; j++)
            if (j != k && S[j]) others *= q[j];
        gw[k] = gs * others;
    }
    for (int c = 0; c < Cc; c++) {
        float ic = 0.0f;
#pragma unroll
        for (int k = 0; k < K; k++)
            if (S[k]) ic += w[k] * color[(o1 + (int64_t)k * N) * Cc + c];
        ic *= inv;
#pragma unroll
        for (int k = 0; k < K; k++) {
            int64_t o = o1 + (int64_t)k * N;
            if (S[k]) {
                grad_layer[o * Cc + c] = gc[c] * w[k] * inv;
                gw[k] += gc[c] * (color[o * Cc + c] - ic) * inv;
            } else if (!skip_empty) {
                grad_layer[o * Cc + c] = 0.0f;
            }
        }
    }
    if (grad_dist) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            int64_t o = o1 + (int64_t)k * N;
            if (S[k] || !skip_empty) grad_dist[o] = S[k] ? gw[k] * w[k] * q[k] * inv_sigma : 0.0f;
        }
    }
}

static int check_softras(dressi_ctx *ctx, const void *color, const void *tid, int B, int K, int H,
                         int W, int Cc, float sigma, int mode) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || K < 1 || K > DRESSI_MAX_K || H < 0 || W < 0)
        return dressi_fail(ctx, DRESSI_EINVAL, "softras: bad dimensions");
    if (Cc < 1 || Cc > 16) return dressi_fail(ctx, DRESSI_EINVAL, "softras: Cc must be 1..16");
    if (mode < DRESSI_BLEND_HSR || mode > DRESSI_BLEND_HARD)
        return dressi_fail(ctx, DRESSI_EINVAL, "softras: bad mode");
    if (mode != DRESSI_BLEND_HARD && !(sigma > 0.0f))
        return dressi_fail(ctx, DRESSI_EINVAL, "softras: sigma must be > 0");
    if ((int64_t)B * H * W > 0 && (!color || !tid)) return dressi_fail(ctx, DRESSI_EINVAL, "softras: null input");
    return DRESSI_OK;
}

#define KDISPATCH(K, ...)                                  \
    switch (K) {                                           \
    case 1: { constexpr int KK = 1; __VA_ARGS__; } break;  \
    case 2: { constexpr int KK = 2; __VA_ARGS__; } break;  \
    case 3: { constexpr int KK = 3; __VA_ARGS__; } break;  \
    case 4: { constexpr int KK = 4; __VA_ARGS__; } break;  \
    default: { constexpr int KK = 5; __VA_ARGS__; } break; \
    }

// The edge mask and blend, given the two one-byte-per-pixel planes the edge
// mask needs (bnd: the boundary, rows: its row-dilated form; unused when the
// mode needs no dilation).  Shared by dressi_softras and its allocation-free
// variant.
static void softras_launch(const float *color, const float *dist, const int32_t *tri_id, int B, int K, int H,
                           int W, int Cc, float sigma, int rho, int mode, uint8_t *bnd, uint8_t *rows,
                           float *out_color, float *out_sil, uint8_t *edge_mask, hipStream_t st) {
    const int64_t n = (int64_t)B * H * W;
    const int g = (int)((n + 255) / 256);
    if (rows) {
        DR_LAUNCH("k_boundary", (k_boundary), g, 256, 0, st, tri_id, dist, B, K, H, W, bnd);
        DR_LAUNCH("k_dilate_rows", (k_dilate_rows), g, 256, 0, st, bnd, B, H, W, rho, rows);
    }
    const float inv_sigma = mode == DRESSI_BLEND_HARD ? 0.0f : 1.0f / sigma;
    KDISPATCH(K, DR_LAUNCH("k_blend", (k_blend<KK>), g, 256, 0, st, color, dist, tri_id, B, H, W, Cc, inv_sigma, mode,
                                                 rho, rows, out_color, out_sil, edge_mask));
}

static bool softras_needs_planes(int mode, float delta, int W, int *rho) {
    *rho = mode == DRESSI_BLEND_HSR ? (int)ceilf(delta * (float)W) - 1 : 0;
    return (mode == DRESSI_BLEND_HSR || mode == DRESSI_BLEND_AA) && *rho >= 0;
}

extern "C" int dressi_softras(dressi_ctx *ctx, const float *color, const float *dist,
                              const int32_t *tri_id, int B, int K, int H, int W, int Cc,
                              float sigma, float delta, int mode, float *out_color, float *out_sil,
                              uint8_t *edge_mask, void *stream) {
    int rc = check_softras(ctx, color, tri_id, B, K, H, W, Cc, sigma, mode);
    if (rc) return rc;
    int64_t n = (int64_t)B * H * W;
    if (n == 0) return DRESSI_OK;
    if (!out_color || !out_sil || !edge_mask)
        return dressi_fail(ctx, DRESSI_EINVAL, "softras: null output");
    hipStream_t st = (hipStream_t)stream;
    int rho = 0;
    uint8_t *bnd = nullptr, *rows = nullptr;
    if (softras_needs_planes(mode, delta, W, &rho)) {
        Carver c;
        size_t o_b = c.take((size_t)n);
        size_t o_r = c.take((size_t)n);
        rc = dressi_scratch(ctx, c.off, st);
        if (rc) return rc;
        bnd = at<uint8_t>(ctx->scratch, o_b);
        rows = at<uint8_t>(ctx->scratch, o_r);
    }
    softras_launch(color, dist, tri_id, B, K, H, W, Cc, sigma, rho, mode, bnd, rows, out_color, out_sil,
                   edge_mask, st);
    return dressi_launch_check(ctx, "softras");
}

// ---------------------------------------------------------------------------
// Allocation-free variant of dressi_softras: the two edge-mask planes live in
// a fixed device array of the library instead of the context's arena.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// its device address is looked up once per device (with that device current)
// when the library is set up on it, and only that address is passed on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[2 * (size_t)DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS];

#define NOALLOC_MAX_DEVICES 64
static std::mutex g_noalloc_mu;
static uint8_t *g_noalloc_ptr[NOALLOC_MAX_DEVICES];

// Called by dressi_create with `device` current.
int dressi_softras_noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return DRESSI_EINVAL;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return DRESSI_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return DRESSI_EHIP;
    g_noalloc_ptr[device] = static_cast<uint8_t *>(p);
    return DRESSI_OK;
}

extern "C" int dressi_softras_noalloc(dressi_ctx *ctx, const float *color, const float *dist,
                                      const int32_t *tri_id, int B, int K, int H, int W, int Cc,
                                      float sigma, float delta, int mode, float *out_color, float *out_sil,
                                      uint8_t *edge_mask, void *stream) {
    int rc = check_softras(ctx, color, tri_id, B, K, H, W, Cc, sigma, mode);
    if (rc) return rc;
    int64_t n = (int64_t)B * H * W;
    if (n == 0) return DRESSI_OK;
    if (!out_color || !out_sil || !edge_mask)
        return dressi_fail(ctx, DRESSI_EINVAL, "softras_noalloc: null output");
    if (n > DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS)
        return dressi_fail(ctx, DRESSI_EINVAL,
                           "softras_noalloc: B*H*W = " + std::to_string(n) + " exceeds the fixed scratch's " +
                               std::to_string((int64_t)DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS) +
                               " pixels; use dressi_softras");
    uint8_t *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) base = g_noalloc_ptr[ctx->device];
    }
    if (!base)
        return dressi_fail(ctx, DRESSI_EHIP, "softras_noalloc: the fixed scratch of this device was not set up");
    int rho = 0;
    uint8_t *bnd = nullptr, *rows = nullptr;
    if (softras_needs_planes(mode, delta, W, &rho)) {
        bnd = base;
        rows = base + DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS;
    }
    softras_launch(color, dist, tri_id, B, K, H, W, Cc, sigma, rho, mode, bnd, rows, out_color, out_sil,
                   edge_mask, (hipStream_t)stream);
    return dressi_launch_check(ctx, "softras_noalloc");
}

extern "C" int dressi_softras_bwd(dressi_ctx *ctx, const float *color, const float *dist,
                                  const int32_t *tri_id, int B, int K, int H, int W, int Cc,
                                  float sigma, const uint8_t *edge_mask, const float *grad_color,
                                  const float *grad_sil, float *grad_layer_color, float *grad_dist,
                                  void *stream) {
    int rc = check_softras(ctx, color, tri_id, B, K, H, W, Cc, sigma > 0.0f ? sigma : 1.0f,
                           DRESSI_BLEND_HSR);
    if (rc) return rc;
    int64_t n = (int64_t)B * H * W;
    if (n == 0) return DRESSI_OK;
    if (!edge_mask || !grad_color || !grad_layer_color)
        return dressi_fail(ctx, DRESSI_EINVAL, "softras_bwd: null edge_mask, grad_color or grad_layer_color");
    hipStream_t st = (hipStream_t)stream;
    float inv_sigma = sigma > 0.0f ? 1.0f / sigma : 0.0f;
    int g = (int)((n + 255) / 256);
    KDISPATCH(K, DR_LAUNCH("k_blend_bwd", (k_blend_bwd<KK>), g, 256, 0, st, color, dist, tri_id, B, H, W, Cc, inv_sigma,
                                                     edge_mask, grad_color, grad_sil,
                                                     grad_layer_color, grad_dist, ctx->skip_empty));
    return dressi_launch_check(ctx, "softras_bwd");
}
