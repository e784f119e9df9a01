// The optimisation loop around the render step (§4.1: vertex positions, then
// the albedo texture, each optimised with Adam; a scheduled Laplacian
// regulariser on the positions), for gfx950.
//
// Adam is one streaming pass over the parameter and its moments.  Its step
// count and bias corrections live in a small device state advanced by a
// one-thread kernel, so a captured graph replays successive steps.  The
// Laplacian is a gather over the vertex->corner adjacency: one pass for
// delta_v (summed in double, in corner order), one for the transposed
// product, and a fixed-order reduction for the regulariser's value, so every
// result is bitwise reproducible.
#include "dressi_internal.h"

// The step counter t (steps taken) and the bias corrections 1 - beta^t of the
// step in progress.
struct AdamState {
    int32_t t;
    float c1, c2, pad;
};
static_assert(sizeof(AdamState) == DRESSI_ADAM_STATE_BYTES, "Adam state size");

__global__ void k_adam_tick(AdamState *__restrict__ s, float b1, float b2) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    AdamState n;
    n.t = s->t + 1;
    n.c1 = (float)(1.0 - pow((double)b1, (double)n.t));
    n.c2 = (float)(1.0 - pow((double)b2, (double)n.t));
    n.pad = 0.0f;
    *s = n;
}

__device__ __forceinline__ float adam_one(float &p, float g, float &m, float &v, float lr, float b1, float b2,
                                          float eps, float c1, float c2) {
    m = b1 * m + (1.0f - b1) * g;
    v = b2 * v + (1.0f - b2) * (g * g);
    const float mh = m / c1, vh = v / c2;
    p = p - lr * mh / (sqrtf(vh) + eps);
    return p;
}

// VEC: four elements per thread through 16-byte loads (n a multiple of 4,
// every pointer 16-byte aligned).
template <bool VEC>
__global__ void __launch_bounds__(256)
    k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
           int64_t n, float lr, float b1, float b2, float eps, const AdamState *__restrict__ s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float c1 = s->c1, c2 = s->c2;
    if (VEC) {
        if (4 * i >= n) return;
        float4 P = reinterpret_cast<float4 *>(p)[i], G = reinterpret_cast<const float4 *>(g)[i];
        float4 M = reinterpret_cast<float4 *>(m)[i], Vv = reinterpret_cast<float4 *>(v)[i];
        adam_one(P.x, G.x, M.x, Vv.x, lr, b1, b2, eps, c1, c2);
        adam_one(P.y, G.y, M.y, Vv.y, lr, b1, b2, eps, c1, c2);
        adam_one(P.z, G.z, M.z, Vv.z, lr, b1, b2, eps, c1, c2);
        adam_one(P.w, G.w, M.w, Vv.w, lr, b1, b2, eps, c1, c2);
        reinterpret_cast<float4 *>(p)[i] = P;
        reinterpret_cast<float4 *>(m)[i] = M;
        reinterpret_cast<float4 *>(v)[i] = Vv;
    } else {
        if (i >= n) return;
        float P = p[i], M = m[i], Vv = v[i];
        adam_one(P, g[i], M, Vv, lr, b1, b2, eps, c1, c2);
        p[i] = P;
        m[i] = M;
        v[i] = Vv;
    }
}

extern "C" int dressi_adam(dressi_ctx *ctx, float *param, const float *grad, float *m, float *v, int64_t n,
                           float lr, float beta1, float beta2, float eps, void *state, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (n < 0) return dressi_fail(ctx, DRESSI_EINVAL, "adam: negative size");
    if (!state) return dressi_fail(ctx, DRESSI_EINVAL, "adam: null state");
    if (n > 0 && (!param || !grad || !m || !v)) return dressi_fail(ctx, DRESSI_EINVAL, "adam: null pointer");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return dressi_fail(ctx, DRESSI_EINVAL, "adam: betas must lie in [0, 1) and eps be positive");
    if (((uintptr_t)state & 15u) != 0) return dressi_fail(ctx, DRESSI_EINVAL, "adam: state not 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    AdamState *s = static_cast<AdamState *>(state);
    DR_LAUNCH("k_adam_tick", (k_adam_tick), 1, 64, 0, st, s, beta1, beta2);
    if (n > 0) {
        const bool vec = n % 4 == 0 && ((((uintptr_t)param | (uintptr_t)grad | (uintptr_t)m | (uintptr_t)v) & 15u) == 0);
        const int64_t nt = vec ? n / 4 : n;
        const int nb = (int)((nt + 255) / 256);
        if (vec)
            DR_LAUNCH("k_adam", (k_adam<true>), nb, 256, 0, st, param, grad, m, v, n, lr, beta1, beta2, eps, s);
        else
            DR_LAUNCH("k_adam", (k_adam<false>), nb, 256, 0, st, param, grad, m, v, n, lr, beta1, beta2, eps, s);
    }
    return dressi_launch_check(ctx, "adam");
}

// ---------------------------------------------------------------------------
// Laplacian regulariser
// ---------------------------------------------------------------------------
#define LAP_BS 256

__device__ __forceinline__ double3 ld3d(const float *__restrict__ p, int v) {
    return make_double3(p[3 * (int64_t)v], p[3 * (int64_t)v + 1], p[3 * (int64_t)v + 2]);
}

// delta_v = p_v - (sum over v's fan triangles of their two other corners) /
// (2 |fan|), summed in double in corner order; w_v = 1 / (2 |fan|) (0 for a
// vertex in no triangle, whose delta is 0).  Each block writes the sum of
// |delta|^2 of its vertices (fixed tree order) to part[block].
__global__ void __launch_bounds__(LAP_BS)
    k_lap_delta(const float *__restrict__ pos, const int32_t *__restrict__ tris, Adjacency A, int V,
                float4 *__restrict__ dw, double *__restrict__ part) {
    __shared__ double red[LAP_BS];
    const int v = blockIdx.x * LAP_BS + threadIdx.x;
    double sq = 0.0;
    if (v < V) {
        const int lo = A.offsets[v], hi = A.offsets[v + 1];
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int k = lo; k < hi; k++) {
            const int c = A.corners[k];
            const int t = c / 3, i = c - 3 * t;
            const int a = tris[3 * (int64_t)t + (i + 1) % 3], b = tris[3 * (int64_t)t + (i + 2) % 3];
            const double3 pa = ld3d(pos, a), pb = ld3d(pos, b);
            sx += pa.x + pb.x;
            sy += pa.y + pb.y;
            sz += pa.z + pb.z;
        }
        float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (hi > lo) {
            const double w = 0.5 / (double)(hi - lo);
            const double3 pv = ld3d(pos, v);
            const double dx = pv.x - w * sx, dy = pv.y - w * sy, dz = pv.z - w * sz;
            sq = dx * dx + dy * dy + dz * dz;
            o = make_float4((float)dx, (float)dy, (float)dz, (float)w);
        }
        dw[v] = o;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = LAP_BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__device__ __forceinline__ double lap_weight(float lam0, float gamma, const AdamState *s) {
    return (double)lam0 * (s ? pow((double)gamma, (double)s->t) : 1.0);
}

// grad_out[u] = grad_in[u] + 2 lam / V * (delta_u - sum over u's fan
// triangles t, over t's two other corners v, of w_v delta_v), the transpose
// of delta = (I - A) p applied to delta.  grad_in may be grad_out (each
// thread reads its own entries before writing them).
__global__ void __launch_bounds__(LAP_BS)
    k_lap_grad(const int32_t *__restrict__ tris, Adjacency A, int V, const float4 *__restrict__ dw, float lam0,
               float gamma, const AdamState *__restrict__ s, const float *grad_in, float *grad_out) {
    const int u = blockIdx.x * LAP_BS + threadIdx.x;
    if (u >= V) return;
    const int lo = A.offsets[u], hi = A.offsets[u + 1];
    const float4 du = dw[u];
    double ax = du.x, ay = du.y, az = du.z;
    for (int k = lo; k < hi; k++) {
        const int c = A.corners[k];
        const int t = c / 3, i = c - 3 * t;
#pragma unroll
        for (int j = 1; j <= 2; j++) {
            const float4 d = dw[tris[3 * (int64_t)t + (i + j) % 3]];
            ax -= (double)d.w * d.x;
            ay -= (double)d.w * d.y;
            az -= (double)d.w * d.z;
        }
    }
    const double sc = 2.0 * lap_weight(lam0, gamma, s) / (double)V;
    float gx = (float)(sc * ax), gy = (float)(sc * ay), gz = (float)(sc * az);
    if (grad_in) {
        gx += grad_in[3 * (int64_t)u];
        gy += grad_in[3 * (int64_t)u + 1];
        gz += grad_in[3 * (int64_t)u + 2];
    }
    grad_out[3 * (int64_t)u] = gx;
    grad_out[3 * (int64_t)u + 1] = gy;
    grad_out[3 * (int64_t)u + 2] = gz;
}

// value = lam / V * (sum of the block partials, in a fixed tree order)
__global__ void __launch_bounds__(LAP_BS)
    k_lap_value(const double *__restrict__ part, int nb, int V, float lam0, float gamma,
                const AdamState *__restrict__ s, float *__restrict__ value) {
    __shared__ double red[LAP_BS];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += LAP_BS) a += part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int k = LAP_BS / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) value[0] = (float)(lap_weight(lam0, gamma, s) / (double)V * red[0]);
}

extern "C" int dressi_laplacian_reg(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                                    const int32_t *adj, float lam0, float gamma, const void *adam_state,
                                    const float *grad_in, float *grad_out, float *value, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0 || T < 0) return dressi_fail(ctx, DRESSI_EINVAL, "laplacian_reg: bad dimensions");
    if (V == 0) {
        if (value) dressi_fill_f32(value, 0.0f, 1, (hipStream_t)stream);
        return dressi_launch_check(ctx, "laplacian_reg");
    }
    if (!pos || (T > 0 && !tris) || (!grad_out && !value))
        return dressi_fail(ctx, DRESSI_EINVAL, "laplacian_reg: null pointer");
    if (adam_state && ((uintptr_t)adam_state & 15u) != 0)
        return dressi_fail(ctx, DRESSI_EINVAL, "laplacian_reg: state not 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int nb = (V + LAP_BS - 1) / LAP_BS;
    Carver c;
    size_t o_adj = adj ? 0 : c.take(adjacency_buf_bytes(V, T));
    size_t o_tmp = adj ? 0 : c.take(dressi_adjacency_tmp_bytes(V, T));
    size_t o_dw = c.take(sizeof(float4) * (size_t)V);
    size_t o_part = c.take(sizeof(double) * (size_t)nb);
    int rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    void *S = ctx->scratch;
    const int32_t *ab = adj;
    if (!ab) {
        int32_t *buf = at<int32_t>(S, o_adj);
        dressi_build_adjacency_into(tris, T, V, buf, at<void>(S, o_tmp), st);
        ab = buf;
    }
    Adjacency A = adjacency_view(ab, V);
    float4 *dw = at<float4>(S, o_dw);
    double *part = at<double>(S, o_part);
    const AdamState *s = static_cast<const AdamState *>(adam_state);
    DR_LAUNCH("k_lap_delta", (k_lap_delta), nb, LAP_BS, 0, st, pos, tris, A, V, dw, part);
    if (grad_out)
        DR_LAUNCH("k_lap_grad", (k_lap_grad), nb, LAP_BS, 0, st, tris, A, V, dw, lam0, gamma, s, grad_in, grad_out);
    if (value) DR_LAUNCH("k_lap_value", (k_lap_value), 1, LAP_BS, 0, st, part, nb, V, lam0, gamma, s, value);
    return dressi_launch_check(ctx, "laplacian_reg");
}

// laplacian_reg with the adjacency built internally
size_t dr_need_optim(const dressi_limits &l) {
    const int V = std::max(l.V, 0), T = std::max(l.T, 0);
    Carver c;
    c.take(adjacency_buf_bytes(V, T));
    c.take(dressi_adjacency_tmp_bytes(V, T));
    c.take(sizeof(float4) * (size_t)V);
    c.take(sizeof(double) * (size_t)((V + LAP_BS - 1) / LAP_BS));
    return c.off;
}
