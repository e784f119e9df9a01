// Bilinear texture taps shared by the sampler (texture.hip) and the packed
// single-layer pass (shade.hip): tap positions and fractions of a coordinate,
// the bilinear combination and its derivative in the coordinate, written once
// so that both compute the same values.
#pragma once
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

// Number of 2-D faces or layers of a texture.
__host__ __device__ __forceinline__ int tex_faces(const dressi_tex_desc &td) {
    return td.kind == DRESSI_TEX_CUBE ? 6 : (td.kind == DRESSI_TEX_2D_ARRAY ? td.layers : 1);
}

// Layer of fragment i of a texture array (its triangle's layer), 0 otherwise.
__device__ __forceinline__ int tex_layer(const dressi_tex_desc &td, const int32_t *__restrict__ tri_id,
                                         int64_t i) {
    return td.kind == DRESSI_TEX_2D_ARRAY ? td.tri_layer[tri_id[i]] : 0;
}

__device__ __forceinline__ Taps make_taps(const dressi_tex_desc &td, const float *q, int layer = 0) {
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
        t.face = layer;
    }
    taps1d(u, td.Wt, wu, t.x0, t.x1, t.fx);
    taps1d(v, td.Ht, wv, t.y0, t.y1, t.fy);
    t.ok = 1;
    return t;
}

// Record of a registered pixel for the inverse-UV gather of an RGBA texture
// (32 bytes): its taps packed as x0 | x1 << 16 and y0 | y1 << 16 and its
// bilinear fractions, then the gradient of its sample.  The gather reads a
// kept pixel's record instead of its coordinate and gradient.
__device__ __forceinline__ void invrec_put(int4 *__restrict__ r, const Taps &t, const float *g) {
    r[0] = make_int4(t.x0 | (t.x1 << 16), t.y0 | (t.y1 << 16), __float_as_int(t.fx), __float_as_int(t.fy));
    r[1] = make_int4(__float_as_int(g[0]), __float_as_int(g[1]), __float_as_int(g[2]), __float_as_int(g[3]));
}

// CT channels per texel or pixel (CT = 0: Ct at run time, at most 16).
// Multiples of 4 are moved as float4 (16-byte aligned rows).
template <int CT>
__device__ __forceinline__ void ldv(const float *__restrict__ p, float *v, int Ct) {
    if constexpr (CT > 0 && CT % 4 == 0) {
#pragma unroll
        for (int q = 0; q < CT / 4; q++) {
            const float4 a = reinterpret_cast<const float4 *>(p)[q];
            v[4 * q] = a.x; v[4 * q + 1] = a.y; v[4 * q + 2] = a.z; v[4 * q + 3] = a.w;
        }
    } else if constexpr (CT > 0) {
#pragma unroll
        for (int c = 0; c < CT; c++) v[c] = p[c];
    } else {
#pragma unroll
        for (int c = 0; c < 16; c++)
            if (c < Ct) v[c] = p[c];
    }
}

template <int CT>
__device__ __forceinline__ void stv(float *__restrict__ p, const float *v, int Ct) {
    if constexpr (CT > 0 && CT % 4 == 0) {
#pragma unroll
        for (int q = 0; q < CT / 4; q++)
            reinterpret_cast<float4 *>(p)[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else if constexpr (CT > 0) {
#pragma unroll
        for (int c = 0; c < CT; c++) p[c] = v[c];
    } else {
#pragma unroll
        for (int c = 0; c < 16; c++)
            if (c < Ct) p[c] = v[c];
    }
}

#define TEX_NC(CT) ((CT) > 0 ? (CT) : 16)

// Bilinear combination of the four taps (channels CT, or Ct when CT = 0).
template <int CT>
__device__ __forceinline__ void tex_bilinear(const float *__restrict__ tex, const dressi_tex_desc &td,
                                             const Taps &t, float *r, int Ct) {
    const int64_t face = (int64_t)t.face * td.Ht * td.Wt;
    float a[TEX_NC(CT)], b[TEX_NC(CT)], c4[TEX_NC(CT)], d[TEX_NC(CT)];
    ldv<CT>(tex + (face + (int64_t)t.y0 * td.Wt + t.x0) * Ct, a, Ct);
    ldv<CT>(tex + (face + (int64_t)t.y0 * td.Wt + t.x1) * Ct, b, Ct);
    ldv<CT>(tex + (face + (int64_t)t.y1 * td.Wt + t.x0) * Ct, c4, Ct);
    ldv<CT>(tex + (face + (int64_t)t.y1 * td.Wt + t.x1) * Ct, d, Ct);
    const float w00 = (1.0f - t.fy) * (1.0f - t.fx), w01 = (1.0f - t.fy) * t.fx;
    const float w10 = t.fy * (1.0f - t.fx), w11 = t.fy * t.fx;
#pragma unroll
    for (int c = 0; c < TEX_NC(CT); c++) r[c] = w00 * a[c] + w01 * b[c] + w10 * c4[c] + w11 * d[c];
}

// The four taps' texels (channels CT, or Ct when CT = 0).
template <int CT>
__device__ __forceinline__ void tex_taps_load(const float *__restrict__ tex, const dressi_tex_desc &td,
                                              const Taps &t, int Ct, float *p00, float *p01, float *p10,
                                              float *p11) {
    const int64_t face = (int64_t)t.face * td.Ht * td.Wt;
    ldv<CT>(tex + (face + (int64_t)t.y0 * td.Wt + t.x0) * Ct, p00, Ct);
    ldv<CT>(tex + (face + (int64_t)t.y0 * td.Wt + t.x1) * Ct, p01, Ct);
    ldv<CT>(tex + (face + (int64_t)t.y1 * td.Wt + t.x0) * Ct, p10, Ct);
    ldv<CT>(tex + (face + (int64_t)t.y1 * td.Wt + t.x1) * Ct, p11, Ct);
}

// d (g . sample) / d (u, v) on the taps' face from its texels: the bilinear
// derivative in the texel grid times the texture's size.
template <int CT>
__device__ __forceinline__ void tex_dcoord_texels(const dressi_tex_desc &td, const Taps &t, const float *p00,
                                                  const float *p01, const float *p10, const float *p11,
                                                  const float *g, int Ct, float &du, float &dv) {
    du = 0.0f;
    dv = 0.0f;
#pragma unroll
    for (int c = 0; c < TEX_NC(CT); c++) {
        if (CT == 0 && c >= Ct) break;
        du += g[c] * ((1.0f - t.fy) * (p01[c] - p00[c]) + t.fy * (p11[c] - p10[c]));
        dv += g[c] * ((1.0f - t.fx) * (p10[c] - p00[c]) + t.fx * (p11[c] - p01[c]));
    }
    du *= (float)td.Wt;
    dv *= (float)td.Ht;
}

// The same, loading the texels.
template <int CT>
__device__ __forceinline__ void tex_dcoord(const float *__restrict__ tex, const dressi_tex_desc &td,
                                           const Taps &t, const float *g, int Ct, float &du, float &dv) {
    float p00[TEX_NC(CT)], p01[TEX_NC(CT)], p10[TEX_NC(CT)], p11[TEX_NC(CT)];
    tex_taps_load<CT>(tex, td, t, Ct, p00, p01, p10, p11);
    tex_dcoord_texels<CT>(td, t, p00, p01, p10, p11, g, Ct, du, dv);
}
