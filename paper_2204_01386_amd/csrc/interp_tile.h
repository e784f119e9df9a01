// Pieces of the per-tile interpolation adjoint shared by its own kernel
// (interp.hip) and the packed geometry adjoint (raster.hip): one fragment's
// staging and barycentric gradient, and one triangle record's sums, written
// once so that both compute the same values.
#pragma once
#include "dressi_internal.h"

#define IB_CH 16   // channels per pass of the per-triangle gather

// Row of C floats; CC = C at compile time (0: run time), 8-byte aligned rows
// with an even CC are read in pairs, odd ones one float at a time.
template <int CC>
__device__ __forceinline__ void ld_row(const float *src, float *v, int C) {
    if constexpr (CC > 0 && (CC & 1) == 0) {
#pragma unroll
        for (int c = 0; c < CC; c += 2) {
            const float2 q = *reinterpret_cast<const float2 *>(src + c);
            v[c] = q.x;
            v[c + 1] = q.y;
        }
    } else if constexpr (CC > 0) {
#pragma unroll
        for (int c = 0; c < CC; c++) v[c] = src[c];
    }
}

// LDS row stride of a fragment: odd, so that lanes writing consecutive rows
// fall in distinct banks
__host__ __device__ static inline int ib_stride(int C) { return (C + 2) | 1; }

// One fragment o (triangle t) of the per-tile interpolation adjoint: stages
// (b0, b1, g_0..g_{C-1}) in its LDS row `dst`, forms the barycentric gradient
// `acc` (gb_in[o] plus g . (a0 - a2), g . (a1 - a2)) and writes it to
// grad_bary.  Returns false for an empty slot skipped under the empty-slot
// knob (nothing staged or written).
// The arithmetic of ib_fragment (CC > 0) from its loaded values: bary w, the
// output gradient row gv and the corners' attribute rows r0, r1, r2 (used
// only when ok); acc enters as gb_in[o].
template <int CC>
__device__ __forceinline__ void ib_fragment_math(bool ok, int t, float2 w, const float *gv, const float *r0,
                                                 const float *r1, const float *r2, float *dst, float2 &acc) {
    if (ok) {
        dst[0] = w.x;
        dst[1] = w.y;
        float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
        for (int c = 0; c < CC; c++) {
            dst[2 + c] = gv[c];
            g0 += gv[c] * (r0[c] - r2[c]);
            g1 += gv[c] * (r1[c] - r2[c]);
        }
        acc.x += g0;
        acc.y += g1;
    } else if (t >= 0) {
        // a fragment whose attribute triangle is invalid contributes nothing
        dst[0] = 0.0f;
        dst[1] = 0.0f;
#pragma unroll
        for (int c = 0; c < CC; c++) dst[2 + c] = 0.0f;
    }
}

template <int CC>
__device__ __forceinline__ bool ib_fragment(const float *__restrict__ ab, int Va, int C,
                                            const int32_t *__restrict__ attr_tris, int T, int t, int64_t o,
                                            const float2 *__restrict__ bary, const float *__restrict__ grad_out,
                                            const float2 *__restrict__ gb_in, float2 *__restrict__ grad_bary,
                                            float *dst, int skip_empty, float2 &acc) {
    int v0 = -1, v1 = -1, v2 = -1;
    if (t >= 0 && t < T) {
        v0 = attr_tris[3 * (int64_t)t];
        v1 = attr_tris[3 * (int64_t)t + 1];
        v2 = attr_tris[3 * (int64_t)t + 2];
    }
    if (skip_empty && t < 0) return false;
    bool ok = v0 >= 0 && v0 < Va && v1 >= 0 && v1 < Va && v2 >= 0 && v2 < Va;
    acc = gb_in ? gb_in[o] : make_float2(0.0f, 0.0f);
    const float *g = grad_out + o * C;
    if constexpr (CC > 0) {
        float gv[CC], r0[CC], r1[CC], r2[CC];
        float2 w = make_float2(0.0f, 0.0f);
        if (ok) {
            w = bary[o];
            ld_row<CC>(g, gv, C);
            ld_row<CC>(ab + (int64_t)v0 * C, r0, C);
            ld_row<CC>(ab + (int64_t)v1 * C, r1, C);
            ld_row<CC>(ab + (int64_t)v2 * C, r2, C);
        }
        ib_fragment_math<CC>(ok, t, w, gv, r0, r1, r2, dst, acc);
        if (grad_bary) grad_bary[o] = acc;
        return true;
    }
    if (ok) {
        float2 w = bary[o];
        dst[0] = w.x;
        dst[1] = w.y;
        const float *a0 = ab + (int64_t)v0 * C, *a1 = ab + (int64_t)v1 * C, *a2 = ab + (int64_t)v2 * C;
        float g0 = 0.0f, g1 = 0.0f;
        for (int c = 0; c < C; c++) {
            float gc = g[c];
            dst[2 + c] = gc;
            g0 += gc * (a0[c] - a2[c]);
            g1 += gc * (a1[c] - a2[c]);
        }
        acc.x += g0;
        acc.y += g1;
    } else if (t >= 0) {
        // a fragment whose attribute triangle is invalid contributes nothing
        dst[0] = 0.0f;
        dst[1] = 0.0f;
        for (int c = 0; c < C; c++) dst[2 + c] = 0.0f;
    }
    if (grad_bary) grad_bary[o] = acc;
    return true;
}

// One record of the per-tile sums: the fragments [j0, j1) of the tile's
// sorted list (one triangle), b_i g_c summed in list order into dst[3][C].
// frag: the tile's sorted fragment list (in global memory or an LDS copy)
__device__ __forceinline__ void ib_record(const float *vals, int S, int C, const uint16_t *frag,
                                          int j0, int j1, float *__restrict__ dst) {
    for (int c0 = 0; c0 < C; c0 += IB_CH) {
        float acc[3][IB_CH];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int c = 0; c < IB_CH; c++) acc[i][c] = 0.0f;
        for (int j = j0; j < j1; j++) {
            const float *v = vals + (int)frag[j] * S;
            float w0 = v[0], w1 = v[1], w2 = 1.0f - w0 - w1;
#pragma unroll
            for (int c = 0; c < IB_CH; c++) {
                if (c0 + c < C) {
                    float gc = v[2 + c0 + c];
                    acc[0][c] += w0 * gc;
                    acc[1][c] += w1 * gc;
                    acc[2][c] += w2 * gc;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int c = 0; c < IB_CH; c++)
                if (c0 + c < C) dst[i * C + c0 + c] = acc[i][c];
    }
}
