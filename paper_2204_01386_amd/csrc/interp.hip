// Attribute interpolation (BuildInterpolate) and its backward for gfx950.
//
// Forward: one lane per (pixel, layer) fragment; memory bound.
// Backward: grad_bary is elementwise; grad_attr is a deterministic gather:
// fragments are sorted per tile by triangle id (shared with the rasterizer
// backward) and each tile sums b_i * g per triangle into one record; then per
// attribute vertex and channel, every corner's records are summed in tile
// order (through the triangle->tile transpose) and the corners in ascending
// order.  No float atomics.
#include "interp_tile.h"

#include <algorithm>


// One lane per fragment; the block's outputs (256 fragments x C channels, a
// contiguous range) are staged in LDS and written back with coalesced float4
// stores.  CC = C at compile time (0: run time).
template <int CC>
__global__ void __launch_bounds__(256)
    k_interp(const float *__restrict__ attr, int Ba, int Va, int C_, const int32_t *__restrict__ attr_tris,
             int T, const int32_t *__restrict__ tri_id, const float2 *__restrict__ bary, int64_t per_view,
             int64_t n, float *__restrict__ out, int skip_empty) {
    extern __shared__ float stage[];   // [256 * C]
    const int C = CC > 0 ? CC : C_;
    const int64_t o0 = (int64_t)blockIdx.x * 256;
    const int64_t o = o0 + threadIdx.x;
    float *y = stage + threadIdx.x * C;
    const int t = o < n ? tri_id[o] : -1;
    // empty fragments left unwritten: a block without a fragment stores nothing
    if (skip_empty && !__syncthreads_or(t >= 0)) return;
    if (o < n) {
        int v0 = -1, v1 = -1, v2 = -1;
        if (t >= 0 && t < T) {
            v0 = attr_tris[3 * (int64_t)t];
            v1 = attr_tris[3 * (int64_t)t + 1];
            v2 = attr_tris[3 * (int64_t)t + 2];
        }
        if (v0 < 0 || v0 >= Va || v1 < 0 || v1 >= Va || v2 < 0 || v2 >= Va) {
            for (int c = 0; c < C; c++) y[c] = 0.0f;
        } else {
            int b = (int)(o / per_view);
            const float *a = attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
            float2 w = bary[o];
            float w2 = 1.0f - w.x - w.y;
            const float *a0 = a + (int64_t)v0 * C, *a1 = a + (int64_t)v1 * C, *a2 = a + (int64_t)v2 * C;
            if constexpr (CC > 0) {
#pragma unroll
                for (int c = 0; c < CC; c++) y[c] = w.x * a0[c] + w.y * a1[c] + w2 * a2[c];
            } else {
                for (int c = 0; c < C; c++) y[c] = w.x * a0[c] + w.y * a1[c] + w2 * a2[c];
            }
        }
    }
    __syncthreads();
    // the block's outputs are out[o0 * C, (o0 + cnt) * C)
    const int64_t cnt = min((int64_t)256, n - o0);
    const int64_t nf = cnt * C;
    float *dst = out + o0 * C;
    if (((o0 * C) & 3) == 0 && (((uintptr_t)out) & 15) == 0) {
        const int64_t n4 = nf >> 2;
        for (int64_t i = threadIdx.x; i < n4; i += 256)
            reinterpret_cast<float4 *>(dst)[i] = reinterpret_cast<const float4 *>(stage)[i];
        for (int64_t i = (n4 << 2) + threadIdx.x; i < nf; i += 256) dst[i] = stage[i];
    } else {
        for (int64_t i = threadIdx.x; i < nf; i += 256) dst[i] = stage[i];
    }
}

// Wide attributes (C > 32): one lane per fragment writing its row directly.
__global__ void k_interp_wide(const float *__restrict__ attr, int Ba, int Va, int C,
                              const int32_t *__restrict__ attr_tris, int T, const int32_t *__restrict__ tri_id,
                              const float2 *__restrict__ bary, int64_t per_view, int64_t n,
                              float *__restrict__ out, int skip_empty) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    float *y = out + o * C;
    int t = tri_id[o];
    if (skip_empty && t < 0) return;
    int v0 = -1, v1 = -1, v2 = -1;
    if (t >= 0 && t < T) {
        v0 = attr_tris[3 * (int64_t)t];
        v1 = attr_tris[3 * (int64_t)t + 1];
        v2 = attr_tris[3 * (int64_t)t + 2];
    }
    if (v0 < 0 || v0 >= Va || v1 < 0 || v1 >= Va || v2 < 0 || v2 >= Va) {
        for (int c = 0; c < C; c++) y[c] = 0.0f;
        return;
    }
    int b = (int)(o / per_view);
    const float *a = attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
    float2 w = bary[o];
    float w2 = 1.0f - w.x - w.y;
    const float *a0 = a + (int64_t)v0 * C, *a1 = a + (int64_t)v1 * C, *a2 = a + (int64_t)v2 * C;
    for (int c = 0; c < C; c++) y[c] = w.x * a0[c] + w.y * a1[c] + w2 * a2[c];
}

static int check_interp(dressi_ctx *ctx, const void *attr, int Ba, int Va, int C, const void *at,
                        int T, const void *tid, const void *bary, int B, int K, int H, int W) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || K < 1 || K > DRESSI_MAX_K || H < 0 || W < 0 || T < 0 || Va < 0)
        return dressi_fail(ctx, DRESSI_EINVAL, "interpolate: bad dimensions");
    if (C < 1 || C > 64) return dressi_fail(ctx, DRESSI_EINVAL, "interpolate: C must be 1..64");
    if (!(Ba == 1 || Ba == B)) return dressi_fail(ctx, DRESSI_EINVAL, "interpolate: Ba must be 1 or B");
    if ((int64_t)B * K * H * W > 0 && (!attr || !at || !tid || !bary))
        return dressi_fail(ctx, DRESSI_EINVAL, "interpolate: null input");
    return DRESSI_OK;
}

extern "C" int dressi_interpolate(dressi_ctx *ctx, const float *attr, int Ba, int Va, int C,
                                  const int32_t *attr_tris, int T, const int32_t *tri_id,
                                  const float *bary, int B, int K, int H, int W, float *out,
                                  void *stream) {
    int rc = check_interp(ctx, attr, Ba, Va, C, attr_tris, T, tri_id, bary, B, K, H, W);
    if (rc) return rc;
    int64_t n = (int64_t)B * K * H * W;
    if (n == 0) return DRESSI_OK;
    if (!out) return dressi_fail(ctx, DRESSI_EINVAL, "interpolate: null out");
    hipStream_t st = (hipStream_t)stream;
    const int g = (int)((n + 255) / 256);
    const size_t sh = sizeof(float) * 256 * (size_t)C;
    const float2 *b2 = reinterpret_cast<const float2 *>(bary);
    const int64_t pv = (int64_t)K * H * W;
    switch (C) {
    case 2: DR_LAUNCH("k_interp", (k_interp<2>), g, 256, sh, st, attr, Ba, Va, C, attr_tris, T, tri_id, b2, pv, n, out, ctx->skip_empty); break;
    case 6: DR_LAUNCH("k_interp", (k_interp<6>), g, 256, sh, st, attr, Ba, Va, C, attr_tris, T, tri_id, b2, pv, n, out, ctx->skip_empty); break;
    case 9: DR_LAUNCH("k_interp", (k_interp<9>), g, 256, sh, st, attr, Ba, Va, C, attr_tris, T, tri_id, b2, pv, n, out, ctx->skip_empty); break;
    default:
        if (C <= 32)
            DR_LAUNCH("k_interp", (k_interp<0>), g, 256, sh, st, attr, Ba, Va, C, attr_tris, T, tri_id, b2, pv, n,
                      out, ctx->skip_empty);
        else
            DR_LAUNCH("k_interp", (k_interp_wide), g, 256, 0, st, attr, Ba, Va, C, attr_tris, T, tri_id, b2, pv, n,
                      out, ctx->skip_empty);
        break;
    }
    return dressi_launch_check(ctx, "interpolate");
}

// grad_bary: g . (a0 - a2), g . (a1 - a2)
__global__ void k_interp_bwd_bary(const float *__restrict__ attr, int Ba, int Va, int C,
                                  const int32_t *__restrict__ attr_tris, int T,
                                  const int32_t *__restrict__ tri_id, int64_t per_view, int64_t n,
                                  const float *__restrict__ grad_out, const float2 *__restrict__ gb_in,
                                  float2 *__restrict__ grad_bary, int skip_empty) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    int t = tri_id[o];
    if (skip_empty && t < 0) return;
    int v0 = -1, v1 = -1, v2 = -1;
    if (t >= 0 && t < T) {
        v0 = attr_tris[3 * (int64_t)t];
        v1 = attr_tris[3 * (int64_t)t + 1];
        v2 = attr_tris[3 * (int64_t)t + 2];
    }
    float2 acc = gb_in ? gb_in[o] : make_float2(0.0f, 0.0f);
    if (v0 < 0 || v0 >= Va || v1 < 0 || v1 >= Va || v2 < 0 || v2 >= Va) {
        grad_bary[o] = acc;
        return;
    }
    int b = (int)(o / per_view);
    const float *a = attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
    const float *a0 = a + (int64_t)v0 * C, *a1 = a + (int64_t)v1 * C, *a2 = a + (int64_t)v2 * C;
    const float *g = grad_out + o * C;
    float g0 = 0.0f, g1 = 0.0f;
    for (int c = 0; c < C; c++) {
        float gc = g[c];
        g0 += gc * (a0[c] - a2[c]);
        g1 += gc * (a1[c] - a2[c]);
    }
    grad_bary[o] = make_float2(acc.x + g0, acc.y + g1);
}

// per tile: every fragment's (b0, b1, g_0..g_{C-1}) in LDS; each triangle's
// fragments (consecutive in the tile's sorted list) are summed into one
// record of b_i g_c for its three corners.  Also writes grad_bary.
template <int CC>
__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    k_interp_bwd_tile(const float *__restrict__ attr, int Ba, int Va, int C,
                      const int32_t *__restrict__ attr_tris, int T, const int32_t *__restrict__ tri_id,
                      const float2 *__restrict__ bary, int K, int H, int W, int ntx, int nt, FragLists fl,
                      const float *__restrict__ grad_out, const float2 *__restrict__ gb_in,
                      float2 *__restrict__ grad_bary, float *__restrict__ partial, int skip_empty) {
    extern __shared__ float vals[];   // [K*256][ib_stride(C)]
    __shared__ uint16_t sfrag[DRESSI_MAX_K * DRESSI_TILE_PIX];   // the tile's sorted fragment list
    if (CC > 0) C = CC;
    // several views: XCD-aware order (each XCD whole views); one view keeps the
    // default interleave, which balances uneven work over the image
    const int bt = (int)gridDim.x > nt ? (int)xcd_block() : (int)blockIdx.x;
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    // the tile's lists are read before the fragments' adjoints, not after
    // the barrier (in bounds whatever the counts: K*256 slots each)
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX * K;
    const int nf = fl.n_frag[bt];
    const int nr = fl.n_rec[bt];
    const int np = K * DRESSI_TILE_PIX;
    for (int i = p; i < np; i += DRESSI_TILE_PIX) sfrag[i] = fl.frag[base + i];
    const int rs0 = fl.rec_start[base + p];
    const int rs1 = p + 1 < np ? fl.rec_start[base + p + 1] : 0;
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + p / DRESSI_TILE;
    const int S = ib_stride(C);
    const float *ab = attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
    if (x < W && y < H) {
        for (int k = 0; k < K; k++) {
            int64_t o = (((int64_t)b * K + k) * H + y) * W + x;
            float2 acc;
            ib_fragment<CC>(ab, Va, C, attr_tris, T, tri_id[o], o, bary, grad_out, gb_in, grad_bary,
                            vals + (k * DRESSI_TILE_PIX + p) * S, skip_empty, acc);
        }
    }
    __syncthreads();
    for (int r = p; r < nr; r += DRESSI_TILE_PIX) {
        const int j0 = r == p ? rs0 : fl.rec_start[base + r];
        const int j1 = (r + 1 < nr) ? (r == p ? rs1 : fl.rec_start[base + r + 1]) : nf;
        ib_record(vals, S, C, sfrag, j0, j1, partial + (base + r) * 3 * C);
    }
}

// Four lanes per (shared or per-view attribute set, vertex, channel); lane j
// takes the vertex's corners j, j+4, ... in ascending order, sums each
// corner's tile records over views and tiles in order and adds the corner
// sum to its own; the four lane sums are combined in a fixed butterfly order.
#define IBV_LANES 4
__global__ void k_interp_bwd_vertex(int B, int Ba, int Va, int T, int K, int C, TriTiles tt,
                                    const float *__restrict__ partial, Adjacency adj,
                                    float *__restrict__ grad_attr) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t oi = gid / IBV_LANES;   // output element (ba, v, c)
    const int slot = (int)(gid - oi * IBV_LANES);
    const bool live = oi < (int64_t)Ba * Va * C;
    float s = 0.0f;
    if (live) {
        const int c = (int)(oi % C);
        const int64_t bv = oi / C;
        const int ba = (int)(bv / Va), v = (int)(bv - (int64_t)ba * Va);
        const int b0 = (Ba == 1) ? 0 : ba, b1 = (Ba == 1) ? B : ba + 1;
        for (int j = adj.offsets[v] + slot; j < adj.offsets[v + 1]; j += IBV_LANES) {
            const int cr = adj.corners[j];
            const int t = cr / 3, i = cr - 3 * t;
            float a = 0.0f;
            for (int b = b0; b < b1; b++) {
                const int64_t key = (int64_t)b * T + t;
                for (int e = tt.offsets[key]; e < tt.offsets[key + 1]; e++) {
                    const int2 ent = tt.entries[e];
                    a += partial[((int64_t)ent.x * DRESSI_TILE_PIX * K + ent.y) * 3 * C + i * C + c];
                }
            }
            s += a;
        }
    }
#pragma unroll
    for (int m = 1; m < IBV_LANES; m <<= 1) s += __shfl_xor(s, m, 64);
    if (live && slot == 0) grad_attr[oi] = s;
}

// The same sums for a vertex's CC channels at once: one group of IBV_LANES
// lanes per (view, vertex) walks its corners and their tile lists once and
// loads each record's CC channels together, instead of one walk per channel.
// Every channel is summed over the same terms in the same order as above, so
// the results are bitwise those of k_interp_bwd_vertex.
template <int CC>
__global__ void k_interp_bwd_vertex_c(int B, int Ba, int Va, int T, int K, TriTiles tt,
                                      const float *__restrict__ partial, Adjacency adj,
                                      float *__restrict__ grad_attr) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t bv = gid / IBV_LANES;   // (ba, v)
    const int slot = (int)(gid - bv * IBV_LANES);
    const bool live = bv < (int64_t)Ba * Va;
    float s[CC];
#pragma unroll
    for (int c = 0; c < CC; c++) s[c] = 0.0f;
    if (live) {
        const int ba = (int)(bv / Va), v = (int)(bv - (int64_t)ba * Va);
        const int b0 = (Ba == 1) ? 0 : ba, b1 = (Ba == 1) ? B : ba + 1;
        for (int j = adj.offsets[v] + slot; j < adj.offsets[v + 1]; j += IBV_LANES) {
            const int cr = adj.corners[j];
            const int t = cr / 3, i = cr - 3 * t;
            float a[CC];
#pragma unroll
            for (int c = 0; c < CC; c++) a[c] = 0.0f;
            for (int b = b0; b < b1; b++) {
                const int64_t key = (int64_t)b * T + t;
                for (int e = tt.offsets[key]; e < tt.offsets[key + 1]; e++) {
                    const int2 ent = tt.entries[e];
                    const float *pp = partial + ((int64_t)ent.x * DRESSI_TILE_PIX * K + ent.y) * 3 * CC + i * CC;
#pragma unroll
                    for (int c = 0; c < CC; c++) a[c] += pp[c];
                }
            }
#pragma unroll
            for (int c = 0; c < CC; c++) s[c] += a[c];
        }
    }
#pragma unroll
    for (int c = 0; c < CC; c++) {
#pragma unroll
        for (int m = 1; m < IBV_LANES; m <<= 1) s[c] += __shfl_xor(s[c], m, 64);
    }
    if (live && slot == 0) {
#pragma unroll
        for (int c = 0; c < CC; c++) grad_attr[bv * CC + c] = s[c];
    }
}

// Per-tile interpolation adjoint (k_interp_bwd_tile): grad_bary and each
// tile's per-triangle records of b_i g (`part`), which the per-vertex sums
// read.  Shared by dressi_interpolate_bwd and dressi_geometry_bwd.
void dr_interp_bwd_tiles(const float *attr, int Ba, int Va, int C, const int32_t *attr_tris, int T,
                         const int32_t *tri_id, const float *bary, int B, int K, int H, int W, const FragLists &fl,
                         const float *grad_out, const float *grad_bary_in, float *grad_bary, float *part,
                         int skip_empty, hipStream_t st) {
    const int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    if ((int64_t)B * nt > 0) {
        const size_t lds = sizeof(float) * (size_t)ib_stride(C) * DRESSI_TILE_PIX * K;
        const bool al8 = (((uintptr_t)attr | (uintptr_t)grad_out) & 7u) == 0;
        const float2 *b2 = reinterpret_cast<const float2 *>(bary);
        const float2 *gbi = reinterpret_cast<const float2 *>(grad_bary_in);
        float2 *gbo = reinterpret_cast<float2 *>(grad_bary);
        if (al8 && C == 6)
            DR_LAUNCH("k_interp_bwd_tile", (k_interp_bwd_tile<6>), B * nt, DRESSI_TILE_PIX, lds, st, attr, Ba,
                      Va, C, attr_tris, T, tri_id, b2, K, H, W, ntx, nt, fl, grad_out, gbi, gbo, part,
                      skip_empty);
        else if (al8 && C == 2)
            DR_LAUNCH("k_interp_bwd_tile", (k_interp_bwd_tile<2>), B * nt, DRESSI_TILE_PIX, lds, st, attr, Ba,
                      Va, C, attr_tris, T, tri_id, b2, K, H, W, ntx, nt, fl, grad_out, gbi, gbo, part,
                      skip_empty);
        else if (C == 9)
            DR_LAUNCH("k_interp_bwd_tile", (k_interp_bwd_tile<9>), B * nt, DRESSI_TILE_PIX, lds, st, attr, Ba,
                      Va, C, attr_tris, T, tri_id, b2, K, H, W, ntx, nt, fl, grad_out, gbi, gbo, part,
                      skip_empty);
        else
            DR_LAUNCH("k_interp_bwd_tile", (k_interp_bwd_tile<0>), B * nt, DRESSI_TILE_PIX, lds, st, attr, Ba,
                      Va, C, attr_tris, T, tri_id, b2, K, H, W, ntx, nt, fl, grad_out, gbi, gbo, part,
                      skip_empty);
    }
}

extern "C" int dressi_interpolate_bwd(dressi_ctx *ctx, const float *attr, int Ba, int Va, int C,
                                      const int32_t *attr_tris, int T, const int32_t *tri_id,
                                      const float *bary, int B, int K, int H, int W,
                                      const float *grad_out, const float *grad_bary_in,
                                      const void *frag_index, const int32_t *adj, float *grad_attr,
                                      float *grad_bary, void *stream) {
    int rc = check_interp(ctx, attr, Ba, Va, C, attr_tris, T, tri_id, bary, B, K, H, W);
    if (rc) return rc;
    int64_t n = (int64_t)B * K * H * W;
    if (n > 0 && !grad_out) return dressi_fail(ctx, DRESSI_EINVAL, "interpolate_bwd: null grad_out");
    hipStream_t st = (hipStream_t)stream;
    if (grad_attr && Va > 0 && ib_stride(C) * K > 160)
        return dressi_fail(ctx, DRESSI_EINVAL, "interpolate_bwd: ((C + 2) | 1) * K must be at most 160 with grad_attr");
    if (grad_attr && Va > 0) {
        int ntx = tiles_x(W), nt = ntx * tiles_y(H);
        Carver c;
        size_t o_fi = frag_index ? 0 : c.take(dressi_fragindex_bytes(B, K, H, W, T));
        size_t o_adj = adj ? 0 : c.take(adjacency_buf_bytes(Va, T));
        size_t o_tmp = c.take(std::max(frag_index ? (size_t)0 : dressi_fragindex_tmp_bytes(B, K, H, W, T),
                                       adj ? (size_t)0 : dressi_adjacency_tmp_bytes(Va, T)));
        size_t o_part = c.take(sizeof(float) * (size_t)B * nt * DRESSI_TILE_PIX * K * 3 * C);
        rc = dressi_scratch(ctx, c.off, st);
        if (rc) return rc;
        if (!frag_index) {
            rc = dressi_counters(ctx, (size_t)B * T, st);
            if (rc) return rc;
        }
        void *S = ctx->scratch;
        void *fi = const_cast<void *>(frag_index);
        if (!fi) {
            fi = at<void>(S, o_fi);
            dressi_build_fragindex(tri_id, B, K, H, W, T, fi, at<void>(S, o_tmp), ctx->counters, st);
        }
        FragLists fl;
        TriTiles tt;
        dressi_fragindex_view(fi, B, K, H, W, T, fl, tt);
        const int32_t *ab = adj;
        if (!ab) {
            int32_t *buf = at<int32_t>(S, o_adj);
            dressi_build_adjacency_into(attr_tris, T, Va, buf, at<void>(S, o_tmp), st);
            ab = buf;
        }
        Adjacency A = adjacency_view(ab, Va);
        float *part = at<float>(S, o_part);
        dr_interp_bwd_tiles(attr, Ba, Va, C, attr_tris, T, tri_id, bary, B, K, H, W, fl, grad_out, grad_bary_in,
                            grad_bary, part, ctx->skip_empty, st);
        const int64_t nv = (int64_t)Ba * Va, gv = (nv * IBV_LANES + 255) / 256;
        if (C == 6)
            DR_LAUNCH("k_interp_bwd_vertex", (k_interp_bwd_vertex_c<6>), (int)gv, 256, 0, st, B, Ba, Va, T, K, tt,
                      part, A, grad_attr);
        else if (C == 9)
            DR_LAUNCH("k_interp_bwd_vertex", (k_interp_bwd_vertex_c<9>), (int)gv, 256, 0, st, B, Ba, Va, T, K, tt,
                      part, A, grad_attr);
        else if (C == 3)
            DR_LAUNCH("k_interp_bwd_vertex", (k_interp_bwd_vertex_c<3>), (int)gv, 256, 0, st, B, Ba, Va, T, K, tt,
                      part, A, grad_attr);
        else {
            int64_t ng = (int64_t)Ba * Va * C;
            DR_LAUNCH("k_interp_bwd_vertex", (k_interp_bwd_vertex), (int)((ng * IBV_LANES + 255) / 256), 256, 0,
                      st, B, Ba, Va, T, K, C, tt, part, A, grad_attr);
        }
    } else if (grad_bary && n > 0) {
        DR_LAUNCH("k_interp_bwd_bary", (k_interp_bwd_bary), (int)((n + 255) / 256), 256, 0, st,
                  attr, Ba, Va, C, attr_tris, T, tri_id, (int64_t)K * H * W, n, grad_out,
                  reinterpret_cast<const float2 *>(grad_bary_in), reinterpret_cast<float2 *>(grad_bary),
                  ctx->skip_empty);
    }
    return dressi_launch_check(ctx, "interpolate_bwd");
}

// interpolate_bwd with grad_attr, the fragment index and adjacency built
// internally (the largest of its calls)
size_t dr_need_interp(const dressi_limits &l) {
    const int B = l.B, K = std::max(l.K, 1), H = l.H, W = l.W, T = l.T, Va = l.Va, C = l.C;
    if (B <= 0 || H <= 0 || W <= 0 || Va <= 0 || C <= 0) return 0;
    const int nt = tiles_x(W) * tiles_y(H);
    Carver c;
    c.take(dressi_fragindex_bytes(B, K, H, W, T));
    c.take(adjacency_buf_bytes(Va, T));
    c.take(std::max(dressi_fragindex_tmp_bytes(B, K, H, W, T), dressi_adjacency_tmp_bytes(Va, T)));
    c.take(sizeof(float) * (size_t)B * nt * DRESSI_TILE_PIX * K * 3 * C);
    return c.off;
}
