// Bilinear texture sampling and its backward (the inverse-UV texture of
// §3.3.2, Algorithm 1) for gfx950.
//
// Forward and d/dcoord: one lane per pixel.  Texture gradient: per slice
// (view, layer) an inverse-UV plane of int32 pixel indices is cleared to -1
// and every covered pixel does an integer atomicMax of its index into the
// cell its coordinate falls in (the "last writer" of the paper's sequential
// loop is the largest index).  Then one lane per texel gathers the kept
// pixels of the distinct in-range cells of its 3x3 neighbourhood in every
// slice, in a fixed order.  No float atomics.
#include "dressi_internal.h"

struct Taps {
    int ok;
    int face;
    int x0, x1, y0, y1;
    float fx, fy;
};

// s = u*n - 1/2 (float), taps floor(s) + {0,1}, wrapped or clamped
__device__ __forceinline__ void taps1d(float u, int n, int wrap, int &a, int &b, float &f) {
    float s = u * (float)n;
    s = s - 0.5f;
    float fl = floorf(s);
    f = s - fl;
    a = (int)fl;
    b = a + 1;
    if (wrap == DRESSI_WRAP_REPEAT) {
        a %= n;
        if (a < 0) a += n;
        b %= n;
        if (b < 0) b += n;
    } else {
        a = min(max(a, 0), n - 1);
        b = min(max(b, 0), n - 1);
    }
}

__device__ __forceinline__ int cell1d(float u, int n, int wrap) {
    float p = u * (float)n;
    int c = (int)floorf(p);
    if (wrap == DRESSI_WRAP_REPEAT) {
        c %= n;
        if (c < 0) c += n;
    } else {
        c = min(max(c, 0), n - 1);
    }
    return c;
}

// major-axis cube mapping (faces +X,-X,+Y,-Y,+Z,-Z; ties prefer x then y)
__device__ __forceinline__ int cube_face(float x, float y, float z, float &u, float &v, float &sc,
                                         float &tc, float &ma) {
    float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int f;
    if (ax >= ay && ax >= az) {
        ma = ax;
        if (x >= 0.0f) { f = 0; sc = -z; tc = -y; }
        else { f = 1; sc = z; tc = -y; }
    } else if (ay >= az) {
        ma = ay;
        if (y >= 0.0f) { f = 2; sc = x; tc = z; }
        else { f = 3; sc = x; tc = -z; }
    } else {
        ma = az;
        if (z >= 0.0f) { f = 4; sc = x; tc = -y; }
        else { f = 5; sc = -x; tc = -y; }
    }
    if (!(ma > 0.0f)) return -1;
    float us = sc / ma, vs = tc / ma;
    u = (us + 1.0f) * 0.5f;
    v = (vs + 1.0f) * 0.5f;
    return f;
}

__device__ __forceinline__ Taps make_taps(const dressi_tex_desc &td, const float *q) {
    Taps t;
    t.ok = 0;
    float u, v;
    int wu = td.wrap_u, wv = td.wrap_v;
    t.face = 0;
    if (td.kind == DRESSI_TEX_CUBE) {
        float sc, tc, ma;
        int f = cube_face(q[0], q[1], q[2], u, v, sc, tc, ma);
        if (f < 0) return t;
        t.face = f;
        wu = wv = DRESSI_WRAP_CLAMP;
    } else {
        u = q[0];
        v = q[1];
    }
    taps1d(u, td.Wt, wu, t.x0, t.x1, t.fx);
    taps1d(v, td.Ht, wv, t.y0, t.y1, t.fy);
    t.ok = 1;
    return t;
}

__global__ void k_tex_fwd(const float *__restrict__ tex, dressi_tex_desc td,
                          const float *__restrict__ coord, const int32_t *__restrict__ tri_id,
                          int64_t n, float *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int Ct = td.Ct;
    const int cd = td.kind == DRESSI_TEX_CUBE ? 3 : 2;
    float *y = out + i * Ct;
    Taps t;
    t.ok = 0;
    if (!tri_id || tri_id[i] >= 0) t = make_taps(td, coord + i * cd);
    if (!t.ok) {
        for (int c = 0; c < Ct; c++) y[c] = 0.0f;
        return;
    }
    const int64_t face = (int64_t)t.face * td.Ht * td.Wt;
    const float *p00 = tex + (face + (int64_t)t.y0 * td.Wt + t.x0) * Ct;
    const float *p01 = tex + (face + (int64_t)t.y0 * td.Wt + t.x1) * Ct;
    const float *p10 = tex + (face + (int64_t)t.y1 * td.Wt + t.x0) * Ct;
    const float *p11 = tex + (face + (int64_t)t.y1 * td.Wt + t.x1) * Ct;
    float w00 = (1.0f - t.fy) * (1.0f - t.fx), w01 = (1.0f - t.fy) * t.fx;
    float w10 = t.fy * (1.0f - t.fx), w11 = t.fy * t.fx;
    if (Ct == 4) {
        float4 a = *reinterpret_cast<const float4 *>(p00), b = *reinterpret_cast<const float4 *>(p01);
        float4 c = *reinterpret_cast<const float4 *>(p10), d = *reinterpret_cast<const float4 *>(p11);
        float4 r;
        r.x = w00 * a.x + w01 * b.x + w10 * c.x + w11 * d.x;
        r.y = w00 * a.y + w01 * b.y + w10 * c.y + w11 * d.y;
        r.z = w00 * a.z + w01 * b.z + w10 * c.z + w11 * d.z;
        r.w = w00 * a.w + w01 * b.w + w10 * c.w + w11 * d.w;
        *reinterpret_cast<float4 *>(y) = r;
        return;
    }
    for (int c = 0; c < Ct; c++) y[c] = w00 * p00[c] + w01 * p01[c] + w10 * p10[c] + w11 * p11[c];
}

// Per pixel: d out / d coord and, when `inv` is given, the inverse-UV record
// (the pixel index written into its cell with atomicMax).
__global__ void k_tex_bwd_pixel(const float *__restrict__ tex, dressi_tex_desc td,
                                const float *__restrict__ coord, const int32_t *__restrict__ tri_id,
                                int64_t npix, int S, const float *__restrict__ grad_out,
                                float *__restrict__ grad_coord, int32_t *__restrict__ inv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * npix) return;
    const int Ct = td.Ct;
    const bool cube = td.kind == DRESSI_TEX_CUBE;
    const int cd = cube ? 3 : 2;
    const float *q = coord + i * cd;
    Taps t;
    t.ok = 0;
    bool covered = !tri_id || tri_id[i] >= 0;
    if (covered) t = make_taps(td, q);
    if (inv && covered && t.ok) {
        int s = (int)(i / npix);
        int pix = (int)(i - (int64_t)s * npix);
        int cx, cy;
        if (cube) {
            float u, v, sc, tc, ma;
            cube_face(q[0], q[1], q[2], u, v, sc, tc, ma);
            cx = cell1d(u, td.Wt, DRESSI_WRAP_CLAMP);
            cy = cell1d(v, td.Ht, DRESSI_WRAP_CLAMP);
        } else {
            cx = cell1d(q[0], td.Wt, td.wrap_u);
            cy = cell1d(q[1], td.Ht, td.wrap_v);
        }
        int64_t cells = (int64_t)(cube ? 6 : 1) * td.Ht * td.Wt;
        atomicMax(&inv[(int64_t)s * cells + ((int64_t)t.face * td.Ht + cy) * td.Wt + cx], pix);
    }
    if (!grad_coord) return;
    float *gc = grad_coord + i * cd;
    if (!t.ok) {
        for (int j = 0; j < cd; j++) gc[j] = 0.0f;
        return;
    }
    const int64_t face = (int64_t)t.face * td.Ht * td.Wt;
    const float *p00 = tex + (face + (int64_t)t.y0 * td.Wt + t.x0) * Ct;
    const float *p01 = tex + (face + (int64_t)t.y0 * td.Wt + t.x1) * Ct;
    const float *p10 = tex + (face + (int64_t)t.y1 * td.Wt + t.x0) * Ct;
    const float *p11 = tex + (face + (int64_t)t.y1 * td.Wt + t.x1) * Ct;
    const float *g = grad_out + i * Ct;
    float du = 0.0f, dv = 0.0f;
    for (int c = 0; c < Ct; c++) {
        du += g[c] * ((1.0f - t.fy) * (p01[c] - p00[c]) + t.fy * (p11[c] - p10[c]));
        dv += g[c] * ((1.0f - t.fx) * (p10[c] - p00[c]) + t.fx * (p11[c] - p01[c]));
    }
    du *= (float)td.Wt;
    dv *= (float)td.Ht;
    if (!cube) {
        gc[0] = du;
        gc[1] = dv;
        return;
    }
    // u = (sc/ma + 1)/2 with ma = |major component|
    float u, v, sc, tc, ma;
    int f = cube_face(q[0], q[1], q[2], u, v, sc, tc, ma);
    float gs = 0.5f * du / ma, gt = 0.5f * dv / ma;
    float gm = -0.5f * (du * sc + dv * tc) / (ma * ma);
    float g3[3] = {0.0f, 0.0f, 0.0f};
    // component index and sign of sc, tc and the major axis per face
    switch (f) {
    case 0: g3[2] -= gs; g3[1] -= gt; g3[0] += gm; break;
    case 1: g3[2] += gs; g3[1] -= gt; g3[0] -= gm; break;
    case 2: g3[0] += gs; g3[2] += gt; g3[1] += gm; break;
    case 3: g3[0] += gs; g3[2] -= gt; g3[1] -= gm; break;
    case 4: g3[0] += gs; g3[1] -= gt; g3[2] += gm; break;
    default: g3[0] -= gs; g3[1] -= gt; g3[2] -= gm; break;
    }
    gc[0] = g3[0];
    gc[1] = g3[1];
    gc[2] = g3[2];
}

// Texture gradient through the inverse UV.  One 16x16 block of texels per
// workgroup: per slice the 18x18 cells around the block are staged in LDS
// (wrapped, or -1 outside a clamped texture); blocks whose cells are all
// empty skip the slice.  Each texel then visits its 3x3 cells in row-major
// order and adds the kept pixel's gradient times that pixel's bilinear
// weight on the texel.
#define IV_T 16
#define IV_H (IV_T + 2)
template <int CT>
__global__ void __launch_bounds__(IV_T * IV_T)
    k_invuv_gather(dressi_tex_desc td, const float *__restrict__ coord, int64_t npix, int S,
                   const int32_t *__restrict__ inv, const float *__restrict__ grad_out,
                   float *__restrict__ grad_tex) {
    __shared__ int cells[IV_H * IV_H];
    const int Ht = td.Ht, Wt = td.Wt, Ct = CT > 0 ? CT : td.Ct;
    const bool cube = td.kind == DRESSI_TEX_CUBE;
    const int F = cube ? 6 : 1;
    const int wu = cube ? DRESSI_WRAP_CLAMP : td.wrap_u;
    const int wv = cube ? DRESSI_WRAP_CLAMP : td.wrap_v;
    const int cd = cube ? 3 : 2;
    const int f = blockIdx.z;
    const int bx0 = blockIdx.x * IV_T, by0 = blockIdx.y * IV_T;
    const int lx = threadIdx.x % IV_T, ly = threadIdx.x / IV_T;
    const int tx = bx0 + lx, ty = by0 + ly;
    const bool mine = tx < Wt && ty < Ht;
    const int64_t cells_all = (int64_t)F * Ht * Wt;
    float acc[16];
#pragma unroll
    for (int c = 0; c < 16; c++) acc[c] = 0.0f;
    for (int s = 0; s < S; s++) {
        const int32_t *iv = inv + (int64_t)s * cells_all + (int64_t)f * Ht * Wt;
        int found = 0;
        for (int h = threadIdx.x; h < IV_H * IV_H; h += IV_T * IV_T) {
            int cy = by0 - 1 + h / IV_H, cx = bx0 - 1 + h % IV_H;
            bool ok = true;
            if (wv == DRESSI_WRAP_REPEAT) cy = ((cy % Ht) + Ht) % Ht;
            else ok = cy >= 0 && cy < Ht;
            if (wu == DRESSI_WRAP_REPEAT) cx = ((cx % Wt) + Wt) % Wt;
            else ok = ok && cx >= 0 && cx < Wt;
            int v = ok ? iv[(int64_t)cy * Wt + cx] : -1;
            cells[h] = v;
            found |= v >= 0;
        }
        if (!__syncthreads_or(found)) continue;
        if (mine) {
#pragma unroll
            for (int dy = 0; dy < 3; dy++) {
#pragma unroll
                for (int dx = 0; dx < 3; dx++) {
                    int i = cells[(ly + dy) * IV_H + lx + dx];
                    if (i < 0) continue;
                    int64_t o = (int64_t)s * npix + i;
                    Taps t = make_taps(td, coord + o * cd);
                    if (!t.ok || t.face != f) continue;
                    float w = 0.0f;
                    if (t.y0 == ty && t.x0 == tx) w += (1.0f - t.fy) * (1.0f - t.fx);
                    if (t.y0 == ty && t.x1 == tx) w += (1.0f - t.fy) * t.fx;
                    if (t.y1 == ty && t.x0 == tx) w += t.fy * (1.0f - t.fx);
                    if (t.y1 == ty && t.x1 == tx) w += t.fy * t.fx;
                    if (w == 0.0f) continue;
                    const float *g = grad_out + o * Ct;
#pragma unroll
                    for (int c = 0; c < 16; c++)
                        if (c < Ct) acc[c] += w * g[c];
                }
            }
        }
        __syncthreads();
    }
    if (!mine) return;
    float *gt = grad_tex + ((int64_t)f * Ht * Wt + (int64_t)ty * Wt + tx) * Ct;
    if (Ct == 4) {
        *reinterpret_cast<float4 *>(gt) = make_float4(acc[0], acc[1], acc[2], acc[3]);
        return;
    }
#pragma unroll
    for (int c = 0; c < 16; c++)
        if (c < Ct) gt[c] = acc[c];
}

static int check_tex(dressi_ctx *ctx, const void *tex, const dressi_tex_desc *td, const void *coord,
                     const void *tid, int S, int H, int W) {
    if (!ctx) return DRESSI_EINVAL;
    if (!td) return dressi_fail(ctx, DRESSI_EINVAL, "texture: null descriptor");
    if (td->kind != DRESSI_TEX_2D && td->kind != DRESSI_TEX_CUBE)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: bad kind");
    if (td->Ht < 1 || td->Wt < 1 || td->Ct < 1 || td->Ct > 16)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: bad texture shape (Ct must be 1..16)");
    if (td->kind == DRESSI_TEX_CUBE && td->Ht != td->Wt)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: cube faces must be square");
    if (td->kind == DRESSI_TEX_2D) {
        for (int w : {td->wrap_u, td->wrap_v})
            if (w != DRESSI_WRAP_REPEAT && w != DRESSI_WRAP_CLAMP)
                return dressi_fail(ctx, DRESSI_EINVAL, "texture: bad wrap mode");
    }
    if (S < 0 || H < 0 || W < 0) return dressi_fail(ctx, DRESSI_EINVAL, "texture: bad dimensions");
    if ((int64_t)S * H * W > 0 && (!tex || !coord))
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: null input");
    if ((int64_t)H * W >= (1ll << 31)) return dressi_fail(ctx, DRESSI_EINVAL, "texture: slice too large");
    return DRESSI_OK;
}

extern "C" int dressi_texture(dressi_ctx *ctx, const float *tex, const dressi_tex_desc *td,
                              const float *coord, const int32_t *tri_id, int S, int H, int W,
                              float *out, void *stream) {
    int rc = check_tex(ctx, tex, td, coord, tri_id, S, H, W);
    if (rc) return rc;
    int64_t n = (int64_t)S * H * W;
    if (n == 0) return DRESSI_OK;
    if (!out) return dressi_fail(ctx, DRESSI_EINVAL, "texture: null out");
    hipStream_t st = (hipStream_t)stream;
    DR_LAUNCH("k_tex_fwd", (k_tex_fwd), (int)((n + 255) / 256), 256, 0, st, tex, *td, coord, tri_id, n, out);
    return dressi_launch_check(ctx, "texture");
}

extern "C" int dressi_texture_bwd(dressi_ctx *ctx, const float *tex, const dressi_tex_desc *td,
                                  const float *coord, const int32_t *tri_id, int S, int H, int W,
                                  const float *grad_out, float *grad_tex, float *grad_coord,
                                  void *stream) {
    int rc = check_tex(ctx, tex, td, coord, tri_id, S, H, W);
    if (rc) return rc;
    int64_t npix = (int64_t)H * W, n = (int64_t)S * npix;
    if (n > 0 && !grad_out) return dressi_fail(ctx, DRESSI_EINVAL, "texture_bwd: null grad_out");
    if (grad_tex && !tri_id)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_bwd: the texture gradient needs tri_id");
    if (grad_tex && td->kind == DRESSI_TEX_2D &&
        ((td->wrap_u == DRESSI_WRAP_REPEAT && td->Wt < 3) || (td->wrap_v == DRESSI_WRAP_REPEAT && td->Ht < 3)))
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_bwd: repeat wrap needs at least 3 texels");
    hipStream_t st = (hipStream_t)stream;
    int32_t *inv = nullptr;
    int64_t cells = (int64_t)(td->kind == DRESSI_TEX_CUBE ? 6 : 1) * td->Ht * td->Wt;
    if (grad_tex) {
        Carver c;
        size_t o_inv = c.take(sizeof(int32_t) * (size_t)cells * (S > 0 ? S : 1));
        rc = dressi_scratch(ctx, c.off, st);
        if (rc) return rc;
        inv = at<int32_t>(ctx->scratch, o_inv);
        if (n > 0) dressi_fill_i32(inv, -1, cells * S, st);
    }
    if (n > 0 && (grad_coord || inv))
        DR_LAUNCH("k_tex_bwd_pixel", (k_tex_bwd_pixel), (int)((n + 255) / 256), 256, 0, st, tex, *td, coord,
                  tri_id, npix, S, grad_out, grad_coord, inv);
    if (grad_tex) {
        dim3 g((unsigned)((td->Wt + IV_T - 1) / IV_T), (unsigned)((td->Ht + IV_T - 1) / IV_T),
               (unsigned)(td->kind == DRESSI_TEX_CUBE ? 6 : 1));
        if (td->Ct == 4)
            DR_LAUNCH("k_invuv_gather", (k_invuv_gather<4>), g, IV_T * IV_T, 0, st, *td, coord, npix, S, inv,
                      grad_out, grad_tex);
        else if (td->Ct == 3)
            DR_LAUNCH("k_invuv_gather", (k_invuv_gather<3>), g, IV_T * IV_T, 0, st, *td, coord, npix, S, inv,
                      grad_out, grad_tex);
        else if (td->Ct == 7)
            DR_LAUNCH("k_invuv_gather", (k_invuv_gather<7>), g, IV_T * IV_T, 0, st, *td, coord, npix, S, inv,
                      grad_out, grad_tex);
        else
            DR_LAUNCH("k_invuv_gather", (k_invuv_gather<0>), g, IV_T * IV_T, 0, st, *td, coord, npix, S, inv,
                      grad_out, grad_tex);
    }
    return dressi_launch_check(ctx, "texture_bwd");
}
