// Vertex transform, per-vertex attribute assembly (vertex normals), deferred
// shading and the L2 image loss, forward and backward, for gfx950.
//
// All of these are memory-bound elementwise or gather kernels.  Per-vertex
// sums over incident faces go through the vertex->corner adjacency, each
// vertex's corners split over a fixed group of lanes combined in a fixed
// order, and the loss is reduced in a fixed tree order, so every result is
// bitwise reproducible.
#include "texcore.h"

// ---------------------------------------------------------------------------
// transform
// ---------------------------------------------------------------------------
// With vert_view (uneven batches, B = 1), vertex v uses the matrix of its own view.
__global__ void k_transform(const float *__restrict__ pos, const float *__restrict__ mvp,
                            const int32_t *__restrict__ vert_view, int B, int V, float4 *__restrict__ out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)B * V) return;
    int b = (int)(gid / V), v = (int)(gid - (int64_t)b * V);
    const float *M = mvp + 16 * (int64_t)(vert_view ? vert_view[v] : b);
    float x = pos[3 * (int64_t)v], y = pos[3 * (int64_t)v + 1], z = pos[3 * (int64_t)v + 2];
    out[gid] = clip_of(M, x, y, z);
}

__global__ void k_transform_bwd(const float *__restrict__ mvp, const int32_t *__restrict__ vert_view, int B,
                                int V, const float4 *__restrict__ g, float *__restrict__ grad_pos) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    for (int b = 0; b < B; b++) {
        const float *M = mvp + 16 * (int64_t)(vert_view ? vert_view[v] : b);
        float4 q = g[(int64_t)b * V + v];
        gx += M[0] * q.x + M[4] * q.y + M[8] * q.z + M[12] * q.w;
        gy += M[1] * q.x + M[5] * q.y + M[9] * q.z + M[13] * q.w;
        gz += M[2] * q.x + M[6] * q.y + M[10] * q.z + M[14] * q.w;
    }
    grad_pos[3 * (int64_t)v] = gx;
    grad_pos[3 * (int64_t)v + 1] = gy;
    grad_pos[3 * (int64_t)v + 2] = gz;
}

extern "C" int dressi_transform(dressi_ctx *ctx, const float *pos, const float *mvp, int B, int V,
                                float *pos_clip, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || V < 0) return dressi_fail(ctx, DRESSI_EINVAL, "transform: bad dimensions");
    if ((int64_t)B * V == 0) return DRESSI_OK;
    if (!pos || !mvp || !pos_clip) return dressi_fail(ctx, DRESSI_EINVAL, "transform: null pointer");
    int64_t n = (int64_t)B * V;
    DR_LAUNCH("k_transform", (k_transform), (int)((n + 255) / 256), 256, 0, (hipStream_t)stream, pos, mvp,
              nullptr, B, V, reinterpret_cast<float4 *>(pos_clip));
    return dressi_launch_check(ctx, "transform");
}

extern "C" int dressi_transform_batched(dressi_ctx *ctx, const float *pos, const int32_t *vert_view,
                                        const float *mvp, int V, float *pos_clip, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0) return dressi_fail(ctx, DRESSI_EINVAL, "transform_batched: bad dimensions");
    if (V == 0) return DRESSI_OK;
    if (!pos || !vert_view || !mvp || !pos_clip)
        return dressi_fail(ctx, DRESSI_EINVAL, "transform_batched: null pointer");
    DR_LAUNCH("k_transform", (k_transform), (V + 255) / 256, 256, 0, (hipStream_t)stream, pos, mvp, vert_view, 1,
              V, reinterpret_cast<float4 *>(pos_clip));
    return dressi_launch_check(ctx, "transform_batched");
}

extern "C" int dressi_transform_batched_bwd(dressi_ctx *ctx, const float *mvp, const int32_t *vert_view, int V,
                                            const float *grad_clip, float *grad_pos, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0) return dressi_fail(ctx, DRESSI_EINVAL, "transform_batched_bwd: bad dimensions");
    if (V == 0) return DRESSI_OK;
    if (!mvp || !vert_view || !grad_clip || !grad_pos)
        return dressi_fail(ctx, DRESSI_EINVAL, "transform_batched_bwd: null pointer");
    DR_LAUNCH("k_transform_bwd", (k_transform_bwd), (V + 255) / 256, 256, 0, (hipStream_t)stream, mvp, vert_view,
              1, V, reinterpret_cast<const float4 *>(grad_clip), grad_pos);
    return dressi_launch_check(ctx, "transform_batched_bwd");
}

extern "C" int dressi_transform_bwd(dressi_ctx *ctx, const float *mvp, int B, int V,
                                    const float *grad_clip, float *grad_pos, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || V < 0) return dressi_fail(ctx, DRESSI_EINVAL, "transform_bwd: bad dimensions");
    if (V == 0) return DRESSI_OK;
    if (!grad_pos || (B > 0 && (!mvp || !grad_clip)))
        return dressi_fail(ctx, DRESSI_EINVAL, "transform_bwd: null pointer");
    DR_LAUNCH("k_transform_bwd", (k_transform_bwd), (V + 255) / 256, 256, 0, (hipStream_t)stream, mvp, nullptr,
              B, V, reinterpret_cast<const float4 *>(grad_clip), grad_pos);
    return dressi_launch_check(ctx, "transform_bwd");
}

// ---------------------------------------------------------------------------
// per-vertex attributes: (normal, position[, tangent])
// ---------------------------------------------------------------------------
__device__ __forceinline__ float3 ld3(const float *p) { return make_float3(p[0], p[1], p[2]); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return make_float3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return make_float3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 normalize3(float3 a) {
    float l = sqrtf(dot3(a, a));
    return l > 0.0f ? (1.0f / l) * a : make_float3(0.0f, 0.0f, 0.0f);
}
// gradient of normalize(a): (g - (g.n) n) / |a|
__device__ __forceinline__ float3 normalize3_bwd(float3 a, float3 g) {
    float l = sqrtf(dot3(a, a));
    if (!(l > 0.0f)) return make_float3(0.0f, 0.0f, 0.0f);
    float3 n = (1.0f / l) * a;
    return (1.0f / l) * (g - dot3(g, n) * n);
}

// Per-vertex sums over incident faces use VA_LANES lanes per vertex: lane j
// takes the vertex's corners j, j + VA_LANES, ... in ascending order and the
// lane sums are combined in a fixed butterfly order (the same in every lane).
#define VA_LANES 8

__device__ __forceinline__ float3 lanes_sum(float3 s) {
#pragma unroll
    for (int m = 1; m < VA_LANES; m <<= 1) {
        s.x += __shfl_xor(s.x, m, 64);
        s.y += __shfl_xor(s.y, m, 64);
        s.z += __shfl_xor(s.z, m, 64);
    }
    return s;
}

struct dbl3 {
    double x, y, z;
};

// Face normals, their sums and the normalisation run in double (the vertex
// normal is rounded to float once, at the end): the shading downstream has
// max(0, .) kinks whose side should not depend on the summation order.
// the face normal (u x v in double) from the corners' positions pa, pb, pc
__device__ __forceinline__ dbl3 face_normal_rows(const float *pa, const float *pb, const float *pc) {
    const double p0x = pa[0], p0y = pa[1], p0z = pa[2];
    const double ux = pb[0] - p0x, uy = pb[1] - p0y, uz = pb[2] - p0z;
    const double vx = pc[0] - p0x, vy = pc[1] - p0y, vz = pc[2] - p0z;
    return dbl3{uy * vz - uz * vy, uz * vx - ux * vz, ux * vy - uy * vx};
}
__device__ __forceinline__ dbl3 face_normal_d(const float *pos, const int32_t *tris, int t, int V) {
    const int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    if (a < 0 || a >= V || b < 0 || b >= V || c < 0 || c >= V) return dbl3{0.0, 0.0, 0.0};
    return face_normal_rows(pos + 3 * (int64_t)a, pos + 3 * (int64_t)b, pos + 3 * (int64_t)c);
}

// sum of the (area-weighted) normals of the faces around v (every lane of the
// vertex gets it; lanes with live = false contribute nothing)
__device__ __forceinline__ dbl3 vertex_acc(const float *pos, const int32_t *tris, const Adjacency &adj,
                                          int v, int V, bool live, int slot) {
    dbl3 s{0.0, 0.0, 0.0};
    if (live)
        for (int j = adj.offsets[v] + slot; j < adj.offsets[v + 1]; j += VA_LANES) {
            const dbl3 f = face_normal_d(pos, tris, adj.corners[j] / 3, V);
            s.x += f.x;
            s.y += f.y;
            s.z += f.z;
        }
#pragma unroll
    for (int m = 1; m < VA_LANES; m <<= 1) {
        s.x += __shfl_xor(s.x, m, 64);
        s.y += __shfl_xor(s.y, m, 64);
        s.z += __shfl_xor(s.z, m, 64);
    }
    return s;
}

__global__ void k_vertex_attrs(const float *__restrict__ pos, const int32_t *__restrict__ tris,
                               const float *__restrict__ extra, Adjacency adj, int V, int C,
                               float *__restrict__ out) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = (int)(gid / VA_LANES), slot = (int)(gid % VA_LANES);
    const bool live = v < V;
    const dbl3 a = vertex_acc(pos, tris, adj, v, V, live, slot);
    if (!live || slot != 0) return;
    const double l = sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
    const double il = l > 0.0 ? 1.0 / l : 0.0;
    float *o = out + (int64_t)v * C;
    o[0] = (float)(a.x * il); o[1] = (float)(a.y * il); o[2] = (float)(a.z * il);
    o[3] = pos[3 * (int64_t)v]; o[4] = pos[3 * (int64_t)v + 1]; o[5] = pos[3 * (int64_t)v + 2];
    if (C == 9) {
        o[6] = extra[3 * (int64_t)v]; o[7] = extra[3 * (int64_t)v + 1]; o[8] = extra[3 * (int64_t)v + 2];
    }
}

// The vertex attributes of k_vertex_attrs and the clip positions of
// k_transform in one launch, with the arithmetic of both: the vertex's lanes
// sum its face normals as above; lane j transforms it for the views j, j +
// VA_LANES, ... (with vert_view, lane 0 for its own view) and lane 0 writes
// its attribute row.
__device__ __forceinline__ void vertex_stage(int64_t gid, const float *__restrict__ pos,
                                             const int32_t *__restrict__ tris, const float *__restrict__ extra,
                                             const Adjacency &adj, int V, int C, float *__restrict__ out,
                                             const float *__restrict__ mvp, const int32_t *__restrict__ vert_view,
                                             int B, float4 *__restrict__ pos_clip) {
    const int v = (int)(gid / VA_LANES), slot = (int)(gid % VA_LANES);
    const bool live = v < V;
    const dbl3 a = vertex_acc(pos, tris, adj, v, V, live, slot);
    if (!live) return;
    const float x = pos[3 * (int64_t)v], y = pos[3 * (int64_t)v + 1], z = pos[3 * (int64_t)v + 2];
    const int nb = vert_view ? 1 : B;
    for (int b = slot; b < nb; b += VA_LANES)
        pos_clip[(int64_t)b * V + v] = clip_of(mvp + 16 * (int64_t)(vert_view ? vert_view[v] : b), x, y, z);
    if (slot != 0) return;
    const double l = sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
    const double il = l > 0.0 ? 1.0 / l : 0.0;
    float *o = out + (int64_t)v * C;
    o[0] = (float)(a.x * il); o[1] = (float)(a.y * il); o[2] = (float)(a.z * il);
    o[3] = x; o[4] = y; o[5] = z;
    if (C == 9) {
        o[6] = extra[3 * (int64_t)v]; o[7] = extra[3 * (int64_t)v + 1]; o[8] = extra[3 * (int64_t)v + 2];
    }
}

__global__ void k_vertex_stage(const float *__restrict__ pos, const int32_t *__restrict__ tris,
                               const float *__restrict__ extra, Adjacency adj, int V, int C,
                               float *__restrict__ out, const float *__restrict__ mvp,
                               const int32_t *__restrict__ vert_view, int B, float4 *__restrict__ pos_clip) {
    vertex_stage((int64_t)blockIdx.x * blockDim.x + threadIdx.x, pos, tris, extra, adj, V, C, out, mvp, vert_view,
                 B, pos_clip);
}

// The vertex stage (B views, no vert_view) and the binless hard rasterizer's
// merge in one launch: the first `nrb` workgroups merge the (view, triangle)
// pairs, each lane transforming its triangle's three corners itself with the
// vertex stage's arithmetic (so that the merge does not wait for the stage's
// positions and its keys are those of the stored positions); the rest run
// the vertex stage.
__global__ void __launch_bounds__(256)
    k_vertex_raster_direct(const float *__restrict__ pos, const int32_t *__restrict__ tris,
                           const float *__restrict__ extra, Adjacency adj, int V, int C, float *__restrict__ out,
                           const float *__restrict__ mvp, int B, float4 *__restrict__ pos_clip, int T, int H, int W,
                           int cull, unsigned long long *__restrict__ zbuf, int nrb) {
    if ((int)blockIdx.x >= nrb) {
        vertex_stage((int64_t)(blockIdx.x - nrb) * blockDim.x + threadIdx.x, pos, tris, extra, adj, V, C, out, mvp,
                     nullptr, B, pos_clip);
        return;
    }
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)B * T) return;
    const int b = (int)(gid / T), t = (int)(gid - (int64_t)b * T);
    const int32_t *tv = tris + 3 * (int64_t)t;
    const int v0 = tv[0], v1 = tv[1], v2 = tv[2];
    if (v0 < 0 || v0 >= V || v1 < 0 || v1 >= V || v2 < 0 || v2 >= V) return;
    const float *M = mvp + 16 * (int64_t)b;
    const int vid[3] = {v0, v1, v2};
    float q[9];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        q[3 * i] = pos[3 * (int64_t)vid[i]];
        q[3 * i + 1] = pos[3 * (int64_t)vid[i] + 1];
        q[3 * i + 2] = pos[3 * (int64_t)vid[i] + 2];
    }
    float4 p[3];
#pragma unroll
    for (int i = 0; i < 3; i++) p[i] = clip_of(M, q[3 * i], q[3 * i + 1], q[3 * i + 2]);
    const TriSetup s = dr_setup_pts(p, H, W, 0, 0, cull, 0);
    if (!(s.meta & 1)) return;
    dr_direct_merge(s, t, W, zbuf + (int64_t)b * H * W);
}

void dr_vertex_raster_direct(const float *pos, const int32_t *tris, const float *extra, const int32_t *adj, int V,
                             int C, float *vattr, const float *mvp, int B, float *pos_clip, int T, int H, int W,
                             int cull, unsigned long long *zbuf, hipStream_t st) {
    const int nrb = (int)(((int64_t)B * T + 255) / 256);
    const int nvb = (int)(((int64_t)V * VA_LANES + 255) / 256);
    if (nrb + nvb == 0) return;
    DR_LAUNCH("k_vertex_raster_direct", (k_vertex_raster_direct), nrb + nvb, 256, 0, st, pos, tris, extra,
              adjacency_view(adj, V), V, C, vattr, mvp, B, reinterpret_cast<float4 *>(pos_clip), T, H, W, cull, zbuf,
              nrb);
}

// gradient w.r.t. the un-normalised vertex normal sum
__global__ void k_vertex_attrs_bwd1(const float *__restrict__ pos, const int32_t *__restrict__ tris,
                                    Adjacency adj, int V, int C, const float *__restrict__ g,
                                    float *__restrict__ gacc) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = (int)(gid / VA_LANES), slot = (int)(gid % VA_LANES);
    const bool live = v < V;
    const dbl3 a = vertex_acc(pos, tris, adj, v, V, live, slot);
    if (!live || slot != 0) return;
    // (g - (g.n) n) / |a| with n = a / |a|
    const double l = sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (l > 0.0) {
        const double il = 1.0 / l;
        const double nx = a.x * il, ny = a.y * il, nz = a.z * il;
        const double gx = g[(int64_t)v * C], gy = g[(int64_t)v * C + 1], gz = g[(int64_t)v * C + 2];
        const double gn = gx * nx + gy * ny + gz * nz;
        rx = (gx - gn * nx) * il;
        ry = (gy - gn * ny) * il;
        rz = (gz - gn * nz) * il;
    }
    gacc[3 * (int64_t)v] = (float)rx;
    gacc[3 * (int64_t)v + 1] = (float)ry;
    gacc[3 * (int64_t)v + 2] = (float)rz;
}

// per vertex: the corner gradients of the cross products of its faces
// (n = e1 x e2: ge1 = e2 x gn, ge2 = gn x e1; corner 0 gets -(ge1 + ge2),
// corner 1 ge1, corner 2 ge2), lane-split as above, then the position column
// and grad_pos_in
__global__ void k_vertex_attrs_bwd2(const float *__restrict__ pos, const int32_t *__restrict__ tris,
                                    Adjacency adj, int V, int C, const float *__restrict__ g,
                                    const float *__restrict__ gin, const float *__restrict__ gacc,
                                    float *__restrict__ grad_pos) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int v = (int)(gid / VA_LANES), slot = (int)(gid % VA_LANES);
    const bool live = v < V;
    float3 s = make_float3(0.0f, 0.0f, 0.0f);
    if (live) {
        for (int j = adj.offsets[v] + slot; j < adj.offsets[v + 1]; j += VA_LANES) {
            int cr = adj.corners[j];
            int t = cr / 3, i = cr - 3 * t;
            int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
            if (a < 0 || a >= V || b < 0 || b >= V || c < 0 || c >= V) continue;
            float3 gn = ld3(gacc + 3 * (int64_t)a) + ld3(gacc + 3 * (int64_t)b) + ld3(gacc + 3 * (int64_t)c);
            float3 p0 = ld3(pos + 3 * (int64_t)a);
            float3 e1 = ld3(pos + 3 * (int64_t)b) - p0, e2 = ld3(pos + 3 * (int64_t)c) - p0;
            float3 g1 = cross3(e2, gn), g2 = cross3(gn, e1);
            if (i == 0) s = s - (g1 + g2);
            else if (i == 1) s = s + g1;
            else s = s + g2;
        }
    }
    s = lanes_sum(s);
    if (!live || slot != 0) return;
    s = s + ld3(g + (int64_t)v * C + 3);
    if (gin) s = s + ld3(gin + 3 * (int64_t)v);
    grad_pos[3 * (int64_t)v] = s.x;
    grad_pos[3 * (int64_t)v + 1] = s.y;
    grad_pos[3 * (int64_t)v + 2] = s.z;
}

// The per-vertex part of the geometry adjoint of one image (B = K = 1), eight
// lanes per vertex.  Attribute gradient: lanes 0-3 take the corners j, j + 4,
// ... and are combined as k_interp_bwd_vertex_c combines its four;
// clip-space gradient: all eight take the corners j, j + 8, ... as
// k_rast_bwd_vertex does; then the transform adjoint of k_transform_bwd, and
// the first pass of the vertex-normal adjoint (k_vertex_attrs_bwd1: the
// gradient of the un-normalised normal sum, recomputed over the same lanes).
// Each corner's triangle's tile records are summed in tile order through the
// triangle -> tile lists, so every value is summed over the same terms in
// the same order as those kernels.
#define GV_LANES 8
static_assert(GV_LANES == VA_LANES, "the normal sums use the vertex-attribute lanes");
template <int CC>
__global__ void __launch_bounds__(256)
    k_geo_vertex(const float *__restrict__ pos, const int32_t *__restrict__ tris, const float4 *__restrict__ pos_clip,
                 Viewports vp, int V, int H, int W, TriTiles tt, const float *__restrict__ ipart,
                 const float *__restrict__ rpart, Adjacency adj, const float *__restrict__ mvp,
                 const int32_t *__restrict__ vert_view, float *__restrict__ grad_attr,
                 float4 *__restrict__ grad_pos_clip, float *__restrict__ grad_pos_t, float *__restrict__ gacc) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t v = gid / GV_LANES;
    const int lane = (int)(gid - v * GV_LANES);
    const bool live = v < V;
    float s[CC];
#pragma unroll
    for (int c = 0; c < CC; c++) s[c] = 0.0f;
    float gx = 0.0f, gy = 0.0f, gw = 0.0f;
    dbl3 nacc{0.0, 0.0, 0.0};
    // one view: the transform's matrix is read before the walk rather than
    // after it (uniform: scalar registers)
    float M[16];
    if (!vert_view) {
#pragma unroll
        for (int k = 0; k < 16; k++) M[k] = mvp[k];
    }
    if (live) {
        const int j0 = adj.offsets[v], j1 = adj.offsets[v + 1];
        const float4 p = pos_clip[v];
        const double iw = 1.0 / (double)p.w, xn = (double)(p.x / p.w), yn = (double)(p.y / p.w);
        // One walk for all three sums, so that their loads overlap.  Lane L
        // takes the corners L, L + 8, ... for the clip-space gradient and the
        // normal sum; lanes 0-3 also take the corners L, L + 4, L + 8, ... for
        // the attribute gradient, here as the pairs (j, j + 4) of each step:
        // every sum sees its terms in the order of its own kernel.
        for (int j = j0 + lane; j < j1; j += GV_LANES) {
            // both corners, then both triangles' list bounds, each pair
            // loaded together (the second corner from j itself when unused)
            const bool two = lane < 4 && j + 4 < j1;
            const int c = adj.corners[j];
            const int cb = adj.corners[j + 4 < j1 ? j + 4 : j];
            const int c2 = two ? cb : c;
            const int t = c / 3, i = c - 3 * t;
            const int t2 = c2 / 3, i2 = c2 - 3 * t2;
            const int e0 = tt.offsets[t], e1 = tt.offsets[t + 1];
            const int f0 = tt.offsets[t2], f1 = tt.offsets[t2 + 1];
            // the face normal's corner positions, loaded beside the records
            // and combined after them (row 0 for an invalid corner)
            const int va = tris[3 * t], vb = tris[3 * t + 1], vc = tris[3 * t + 2];
            const bool nok = !(va < 0 || va >= V || vb < 0 || vb >= V || vc < 0 || vc >= V);
            float pa[3], pb[3], pc[3];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                pa[k] = pos[3 * (int64_t)(nok ? va : 0) + k];
                pb[k] = pos[3 * (int64_t)(nok ? vb : 0) + k];
                pc[k] = pos[3 * (int64_t)(nok ? vc : 0) + k];
            }
            // triangle t's tile records: its clip-space sum on every lane and,
            // on lanes 0-3, the attribute sum of corner i; beside them, the
            // second corner's attribute sum (each sum in its own list order)
            float a[CC], b[CC];
#pragma unroll
            for (int q = 0; q < CC; q++) a[q] = b[q] = 0.0f;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            const int n1 = e1 - e0, n2 = two ? f1 - f0 : 0;
            for (int k = 0; k < n1 || k < n2; k++) {
                // both lists' entries and their rows loaded without a branch
                // (entry 0 past a list's end, lanes 4-7 the record's first
                // attribute slice), then added where they count: the sums
                // start at +0 and so never hold -0, which makes adding +0 a
                // no-op
                const bool in1 = k < n1, in2 = k < n2, at1 = in1 && lane < 4;
                const int2 ent = tt.entries[in1 ? e0 + k : 0];
                const int2 ent2 = tt.entries[in2 ? f0 + k : 0];
                const int64_t rix = (int64_t)ent.x * DRESSI_TILE_PIX + ent.y;
                const int64_t rix2 = (int64_t)ent2.x * DRESSI_TILE_PIX + ent2.y;
                const float *pp = ipart + rix * 3 * CC + (lane < 4 ? i * CC : 0);
                const float *pp2 = ipart + rix2 * 3 * CC + i2 * CC;
                const float *r = rpart + rix * 9 + 3 * i;
                float v[CC], v2[CC];
#pragma unroll
                for (int q = 0; q < CC; q++) {
                    v[q] = pp[q];
                    v2[q] = pp2[q];
                }
                const float r0 = r[0], r1 = r[1], r2 = r[2];
#pragma unroll
                for (int q = 0; q < CC; q++) {
                    a[q] += at1 ? v[q] : 0.0f;
                    b[q] += in2 ? v2[q] : 0.0f;
                }
                a0 += in1 ? (double)r0 : 0.0;
                a1 += in1 ? (double)r1 : 0.0;
                a2 += in1 ? (double)r2 : 0.0;
            }
            if (lane < 4) {
#pragma unroll
                for (int q = 0; q < CC; q++) s[q] += a[q];
            }
            if (two) {
#pragma unroll
                for (int q = 0; q < CC; q++) s[q] += b[q];
            }
            const dbl3 f = nok ? face_normal_rows(pa, pb, pc) : dbl3{0.0, 0.0, 0.0};
            nacc.x += f.x;
            nacc.y += f.y;
            nacc.z += f.z;
            // a triangle without fragments adds nothing (as in k_rast_bwd_vertex)
            if (e0 == e1) continue;
            const int4 q = dr_viewport(vp, t, H, W);
            const double hw = 0.5 * (double)q.z, hh = 0.5 * (double)q.w;
            gx += (float)(a0 * hw * iw);
            gy += (float)(-a1 * hh * iw);
            gw += (float)((-a0 * hw * xn + a1 * hh * yn) * iw + a2);
        }
    }
#pragma unroll
    for (int c = 0; c < CC; c++) {
#pragma unroll
        for (int m = 1; m < 4; m <<= 1) s[c] += __shfl_xor(s[c], m, 64);
    }
#pragma unroll
    for (int m = 1; m < GV_LANES; m <<= 1) {
        gx += __shfl_xor(gx, m, 64);
        gy += __shfl_xor(gy, m, 64);
        gw += __shfl_xor(gw, m, 64);
        // the normal sum's butterfly, as in vertex_acc
        nacc.x += __shfl_xor(nacc.x, m, 64);
        nacc.y += __shfl_xor(nacc.y, m, 64);
        nacc.z += __shfl_xor(nacc.z, m, 64);
    }
    if (!live || lane != 0) return;
#pragma unroll
    for (int c = 0; c < CC; c++) grad_attr[v * CC + c] = s[c];
    const float4 q = make_float4(gx, gy, 0.0f, gw);
    grad_pos_clip[v] = q;
    if (vert_view) {
        const float *Mp = mvp + 16 * (int64_t)vert_view[v];
#pragma unroll
        for (int k = 0; k < 16; k++) M[k] = Mp[k];
    }
    float hx = 0.0f, hy = 0.0f, hz = 0.0f;
    hx += M[0] * q.x + M[4] * q.y + M[8] * q.z + M[12] * q.w;
    hy += M[1] * q.x + M[5] * q.y + M[9] * q.z + M[13] * q.w;
    hz += M[2] * q.x + M[6] * q.y + M[10] * q.z + M[14] * q.w;
    grad_pos_t[3 * v] = hx;
    grad_pos_t[3 * v + 1] = hy;
    grad_pos_t[3 * v + 2] = hz;
    // (g - (g.n) n) / |a| with n = a / |a|, g the normal's gradient
    const double l = sqrt(nacc.x * nacc.x + nacc.y * nacc.y + nacc.z * nacc.z);
    double rx = 0.0, ry = 0.0, rz = 0.0;
    if (l > 0.0) {
        const double il = 1.0 / l;
        const double nx = nacc.x * il, ny = nacc.y * il, nz = nacc.z * il;
        const double ggx = s[0], ggy = s[1], ggz = s[2];
        const double gn = ggx * nx + ggy * ny + ggz * nz;
        rx = (ggx - gn * nx) * il;
        ry = (ggy - gn * ny) * il;
        rz = (ggz - gn * nz) * il;
    }
    gacc[3 * v] = (float)rx;
    gacc[3 * v + 1] = (float)ry;
    gacc[3 * v + 2] = (float)rz;
}

// The per-vertex kernel above, then the second pass of the vertex-normal
// adjoint (k_vertex_attrs_bwd2): the world-position gradient.
void dr_geo_vertex(int Cv, const float *pos, const int32_t *tris, const float *pos_clip, Viewports vp, int V, int H,
                   int W, TriTiles tt, const float *ipart, const float *rpart, Adjacency adj, const float *mvp,
                   const int32_t *vert_view, float *grad_attr, float *grad_pos_clip, float *grad_pos_t, float *gacc,
                   float *grad_pos, hipStream_t st) {
    const int g = (int)(((int64_t)V * GV_LANES + 255) / 256);
    const float4 *pc4 = reinterpret_cast<const float4 *>(pos_clip);
    float4 *gpc = reinterpret_cast<float4 *>(grad_pos_clip);
    if (Cv == 6)
        DR_LAUNCH("k_geo_vertex", (k_geo_vertex<6>), g, 256, 0, st, pos, tris, pc4, vp, V, H, W, tt, ipart, rpart,
                  adj, mvp, vert_view, grad_attr, gpc, grad_pos_t, gacc);
    else
        DR_LAUNCH("k_geo_vertex", (k_geo_vertex<9>), g, 256, 0, st, pos, tris, pc4, vp, V, H, W, tt, ipart, rpart,
                  adj, mvp, vert_view, grad_attr, gpc, grad_pos_t, gacc);
    const int nb = (int)(((int64_t)V * VA_LANES + 255) / 256);
    DR_LAUNCH("k_vertex_attrs_bwd2", (k_vertex_attrs_bwd2), nb, 256, 0, st, pos, tris, adj, V, Cv, grad_attr,
              grad_pos_t, gacc, grad_pos);
}


extern "C" int dressi_vertex_attrs(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                                   const float *extra, const int32_t *adj, float *out, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0 || T < 0) return dressi_fail(ctx, DRESSI_EINVAL, "vertex_attrs: bad dimensions");
    if (V == 0) return DRESSI_OK;
    if (!pos || !out || (T > 0 && !tris)) return dressi_fail(ctx, DRESSI_EINVAL, "vertex_attrs: null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int32_t *ab = adj;
    if (!ab) {
        Carver c;
        size_t o_adj = c.take(adjacency_buf_bytes(V, T));
        size_t o_tmp = c.take(dressi_adjacency_tmp_bytes(V, T));
        int rc = dressi_scratch(ctx, c.off, st);
        if (rc) return rc;
        int32_t *buf = at<int32_t>(ctx->scratch, o_adj);
        dressi_build_adjacency_into(tris, T, V, buf, at<void>(ctx->scratch, o_tmp), st);
        ab = buf;
    }
    Adjacency A = adjacency_view(ab, V);
    int C = extra ? 9 : 6;
    const int nb = (int)(((int64_t)V * VA_LANES + 255) / 256);
    DR_LAUNCH("k_vertex_attrs", (k_vertex_attrs), nb, 256, 0, st, pos, tris, extra, A, V, C, out);
    return dressi_launch_check(ctx, "vertex_attrs");
}

extern "C" int dressi_vertex_stage(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                                   const float *extra, const int32_t *adj, const float *mvp,
                                   const int32_t *vert_view, int B, float *vattr, float *pos_clip, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0 || T < 0 || B < 1 || (vert_view && B != 1))
        return dressi_fail(ctx, DRESSI_EINVAL, "vertex_stage: bad dimensions (B >= 1; 1 with vert_view)");
    if (V == 0) return DRESSI_OK;
    if (!pos || !vattr || !mvp || !pos_clip || (T > 0 && !tris))
        return dressi_fail(ctx, DRESSI_EINVAL, "vertex_stage: null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int32_t *ab = adj;
    if (!ab) {
        Carver c;
        size_t o_adj = c.take(adjacency_buf_bytes(V, T));
        size_t o_tmp = c.take(dressi_adjacency_tmp_bytes(V, T));
        int rc = dressi_scratch(ctx, c.off, st);
        if (rc) return rc;
        int32_t *buf = at<int32_t>(ctx->scratch, o_adj);
        dressi_build_adjacency_into(tris, T, V, buf, at<void>(ctx->scratch, o_tmp), st);
        ab = buf;
    }
    const int nb = (int)(((int64_t)V * VA_LANES + 255) / 256);
    DR_LAUNCH("k_vertex_stage", (k_vertex_stage), nb, 256, 0, st, pos, tris, extra, adjacency_view(ab, V), V,
              extra ? 9 : 6, vattr, mvp, vert_view, B, reinterpret_cast<float4 *>(pos_clip));
    return dressi_launch_check(ctx, "vertex_stage");
}

extern "C" int dressi_vertex_attrs_bwd(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V,
                                       int T, int C, const int32_t *adj, const float *grad_out,
                                       const float *grad_pos_in, float *grad_pos, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0 || T < 0 || (C != 6 && C != 9))
        return dressi_fail(ctx, DRESSI_EINVAL, "vertex_attrs_bwd: bad dimensions (C must be 6 or 9)");
    if (V == 0) return DRESSI_OK;
    if (!pos || !grad_out || !grad_pos || (T > 0 && !tris))
        return dressi_fail(ctx, DRESSI_EINVAL, "vertex_attrs_bwd: null pointer");
    hipStream_t st = (hipStream_t)stream;
    Carver c;
    size_t o_adj = adj ? 0 : c.take(adjacency_buf_bytes(V, T));
    size_t o_tmp = adj ? 0 : c.take(dressi_adjacency_tmp_bytes(V, T));
    size_t o_ga = c.take(sizeof(float) * 3 * (size_t)V);
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
    float *ga = at<float>(S, o_ga);
    const int nb = (int)(((int64_t)V * VA_LANES + 255) / 256);
    DR_LAUNCH("k_vertex_attrs_bwd1", (k_vertex_attrs_bwd1), nb, 256, 0, st, pos, tris, A, V, C, grad_out, ga);
    DR_LAUNCH("k_vertex_attrs_bwd2", (k_vertex_attrs_bwd2), nb, 256, 0, st, pos, tris, A, V, C, grad_out,
              grad_pos_in, ga, grad_pos);
    return dressi_launch_check(ctx, "vertex_attrs_bwd");
}

// ---------------------------------------------------------------------------
// deferred shading
// ---------------------------------------------------------------------------
// The shading chain runs in double from the float G-buffer values and is
// rounded once at the outputs.  Its results feed discrete decisions: the
// reflection direction selects a cube face, texels and an inverse-UV cell,
// and n.l and r.v pick a side of the max(0, .) kinks.  Computed in double
// from the same float inputs, those choices do not depend on the order of
// the arithmetic, so they coincide with a double-precision reference.
__constant__ double c_light[3] = {0.40824829046386302, 0.40824829046386302, 0.81649658092772603};

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 ldd3(const float *p) { return d3{p[0], p[1], p[2]}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return d3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dotd(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 crossd(d3 a, d3 b) {
    return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 normalized(d3 a) {
    const double l = sqrt(dotd(a, a));
    return l > 0.0 ? (1.0 / l) * a : d3{0.0, 0.0, 0.0};
}
// gradient of normalize(a): (g - (g.n) n) / |a|
__device__ __forceinline__ d3 normalized_bwd(d3 a, d3 g) {
    const double l = sqrt(dotd(a, a));
    if (!(l > 0.0)) return d3{0.0, 0.0, 0.0};
    const d3 n = (1.0 / l) * a;
    return (1.0 / l) * (g - dotd(g, n) * n);
}

struct ShadeState {
    d3 nin, nh, t, tp, th, bh, m, u, np;   // normal-map chain (np = shading normal)
    d3 vv, vh;                              // view vector and its direction
    double ndl, rv, spec, base, kd;
    d3 r;
    double a[4];
    d3 e;
};

__device__ __forceinline__ void shade_forward(int mode, const dressi_frag_in &in, const float *eye,
                                              int64_t i, bool need_view, ShadeState &s) {
    s.nin = ldd3(in.normal + i * in.normal_stride);
    s.nh = normalized(s.nin);
    s.np = s.nh;
    if (in.tangent && in.nmap) {
        s.t = ldd3(in.tangent + i * in.tangent_stride);
        s.m = ldd3(in.nmap + i * in.nmap_stride);
        s.tp = s.t - dotd(s.t, s.nh) * s.nh;
        s.th = normalized(s.tp);
        s.bh = crossd(s.nh, s.th);
        s.u = s.m.x * s.th + s.m.y * s.bh + s.m.z * s.nh;
        s.np = normalized(s.u);
    }
    if (need_view) {
        s.vv = ldd3(eye) - ldd3(in.pos + i * in.pos_stride);
        s.vh = normalized(s.vv);
    }
    const d3 L{c_light[0], c_light[1], c_light[2]};
    s.ndl = dotd(s.np, L);
    s.kd = mode == DRESSI_SHADE_LAMBERT ? 0.9 : 0.8;
    s.base = 0.1 + s.kd * fmax(s.ndl, 0.0);
    s.spec = 0.0;
    s.rv = 0.0;
    if (mode != DRESSI_SHADE_LAMBERT) {
        s.r = (2.0 * s.ndl) * s.np - L;
        s.rv = dotd(s.r, s.vh);
        if (s.rv > 0.0) {
            const double r2 = s.rv * s.rv, r4 = r2 * r2, r8 = r4 * r4, r16 = r8 * r8;
            s.spec = r16 * r16;
        }
    }
    const float *ap = in.albedo + i * in.albedo_stride;
    s.a[0] = ap[0]; s.a[1] = ap[1]; s.a[2] = ap[2];
    s.a[3] = in.albedo_channels > 3 ? ap[3] : 0.0;
    s.e = d3{0.0, 0.0, 0.0};
    if (mode == DRESSI_SHADE_PHONG_ENV && in.env) s.e = ldd3(in.env + i * in.env_stride);
}

// The colour of a shaded fragment, rounded once to float.
__device__ __forceinline__ void shade_color(int mode, const ShadeState &s, float *c) {
    double add = 0.0;
    if (mode != DRESSI_SHADE_LAMBERT) add = 0.2 * s.a[3] * s.spec;
    const double env = mode == DRESSI_SHADE_PHONG_ENV ? 0.5 * s.a[3] : 0.0;
    c[0] = (float)(s.a[0] * s.base + add + env * s.e.x);
    c[1] = (float)(s.a[1] * s.base + add + env * s.e.y);
    c[2] = (float)(s.a[2] * s.base + add + env * s.e.z);
}

__global__ void k_shade(int mode, dressi_frag_in in, const float *__restrict__ eye,
                        const int32_t *__restrict__ tri_id, int64_t N, int64_t Npv,
                        float *__restrict__ color, float *__restrict__ dir, int skip_empty) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (tri_id[i] < 0) {
        if (skip_empty) return;
        if (color) { color[3 * i] = 0.0f; color[3 * i + 1] = 0.0f; color[3 * i + 2] = 0.0f; }
        if (dir) { dir[3 * i] = 0.0f; dir[3 * i + 1] = 0.0f; dir[3 * i + 2] = 0.0f; }
        return;
    }
    const int64_t e = in.tri_eye ? (int64_t)in.tri_eye[tri_id[i]] : i / Npv;
    ShadeState s;
    shade_forward(mode, in, eye + 3 * e, i, mode != DRESSI_SHADE_LAMBERT || dir != nullptr, s);
    if (dir) {
        const d3 d = (2.0 * dotd(s.np, s.vh)) * s.np - s.vh;
        dir[3 * i] = (float)d.x; dir[3 * i + 1] = (float)d.y; dir[3 * i + 2] = (float)d.z;
    }
    if (color) shade_color(mode, s, color + 3 * i);
}

__device__ __forceinline__ void st3(float *p, int64_t i, int stride, d3 v) {
    float *q = p + i * stride;
    q[0] = (float)v.x; q[1] = (float)v.y; q[2] = (float)v.z;
}

// Adjoint of one covered fragment's shading: the gradient g of its colour
// (and grad_dir, NULL = 0, of its environment direction) to every non-NULL
// member of gr at fragment i; s is the fragment's forward state.
__device__ __forceinline__ void shade_bwd_frag(int mode, const dressi_frag_in &in, const ShadeState &s, d3 g,
                                               const float *__restrict__ grad_dir, const dressi_frag_grad &gr,
                                               int64_t i, bool need_geo) {
    const d3 Z{0.0, 0.0, 0.0};
    const double gsum = g.x + g.y + g.z;
    if (gr.albedo) {
        float *q = gr.albedo + i * gr.albedo_stride;
        q[0] = (float)(g.x * s.base); q[1] = (float)(g.y * s.base); q[2] = (float)(g.z * s.base);
        if (in.albedo_channels > 3) {
            double ga = 0.0;
            if (mode != DRESSI_SHADE_LAMBERT) ga += 0.2 * s.spec * gsum;
            if (mode == DRESSI_SHADE_PHONG_ENV) ga += 0.5 * dotd(g, s.e);
            q[3] = (float)ga;
        }
    }
    if (gr.env) st3(gr.env, i, gr.env_stride, mode == DRESSI_SHADE_PHONG_ENV ? (0.5 * s.a[3]) * g : Z);
    if (!need_geo) return;
    const d3 L{c_light[0], c_light[1], c_light[2]};
    d3 gnp = Z, gvh = Z;
    const double gdot = g.x * s.a[0] + g.y * s.a[1] + g.z * s.a[2];
    if (s.ndl > 0.0) gnp = (s.kd * gdot) * L;
    if (mode != DRESSI_SHADE_LAMBERT && s.rv > 0.0) {
        const double r2 = s.rv * s.rv, r4 = r2 * r2, r8 = r4 * r4, r16 = r8 * r8;
        const double r31 = r16 * r8 * r4 * r2 * s.rv;
        const double grv = 0.2 * s.a[3] * gsum * 32.0 * r31;
        const d3 gr_ = grv * s.vh;
        gvh = gvh + grv * s.r;
        gnp = gnp + (2.0 * s.ndl) * gr_ + (2.0 * dotd(gr_, s.np)) * L;
    }
    if (grad_dir) {
        const d3 gd = ldd3(grad_dir + 3 * i);
        const double d = dotd(s.np, s.vh), gdn = dotd(gd, s.np);
        gnp = gnp + (2.0 * d) * gd + (2.0 * gdn) * s.vh;
        gvh = gvh + (2.0 * gdn) * s.np - gd;
    }
    if (gr.pos) {
        const d3 gvv = (mode != DRESSI_SHADE_LAMBERT || grad_dir) ? normalized_bwd(s.vv, gvh) : Z;
        st3(gr.pos, i, gr.pos_stride, d3{-gvv.x, -gvv.y, -gvv.z});
    }
    if (in.tangent && in.nmap) {
        const d3 gu = normalized_bwd(s.u, gnp);
        if (gr.nmap) st3(gr.nmap, i, gr.nmap_stride, d3{dotd(gu, s.th), dotd(gu, s.bh), dotd(gu, s.nh)});
        d3 gth = s.m.x * gu, gbh = s.m.y * gu, gnh = s.m.z * gu;
        gnh = gnh + crossd(s.th, gbh);
        gth = gth + crossd(gbh, s.nh);
        const d3 gtp = normalized_bwd(s.tp, gth);
        const double d = dotd(s.t, s.nh);
        const double gd = -dotd(gtp, s.nh);
        if (gr.tangent) st3(gr.tangent, i, gr.tangent_stride, gtp + gd * s.nh);
        gnh = gnh + (-d) * gtp + gd * s.t;
        if (gr.normal) st3(gr.normal, i, gr.normal_stride, normalized_bwd(s.nin, gnh));
    } else {
        if (gr.normal) st3(gr.normal, i, gr.normal_stride, normalized_bwd(s.nin, gnp));
        if (gr.tangent) st3(gr.tangent, i, gr.tangent_stride, Z);
        if (gr.nmap) st3(gr.nmap, i, gr.nmap_stride, Z);
    }
}

__global__ void k_shade_bwd(int mode, dressi_frag_in in, const float *__restrict__ eye,
                            const int32_t *__restrict__ tri_id, int64_t N, int64_t Npv,
                            const float *__restrict__ grad_color, const float *__restrict__ grad_dir,
                            dressi_frag_grad gr, int skip_empty) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const d3 Z{0.0, 0.0, 0.0};
    if (tri_id[i] < 0) {
        if (skip_empty) return;
        if (gr.normal) st3(gr.normal, i, gr.normal_stride, Z);
        if (gr.pos) st3(gr.pos, i, gr.pos_stride, Z);
        if (gr.tangent) st3(gr.tangent, i, gr.tangent_stride, Z);
        if (gr.nmap) st3(gr.nmap, i, gr.nmap_stride, Z);
        if (gr.env) st3(gr.env, i, gr.env_stride, Z);
        if (gr.albedo) {
            float *q = gr.albedo + i * gr.albedo_stride;
            for (int c = 0; c < in.albedo_channels; c++) q[c] = 0.0f;
        }
        return;
    }
    const int64_t e = in.tri_eye ? (int64_t)in.tri_eye[tri_id[i]] : i / Npv;
    bool need_geo = gr.normal || gr.pos || gr.tangent || gr.nmap;
    ShadeState s;
    shade_forward(mode, in, eye + 3 * e, i, mode != DRESSI_SHADE_LAMBERT || grad_dir != nullptr, s);
    const d3 g = grad_color ? ldd3(grad_color + 3 * i) : Z;
    shade_bwd_frag(mode, in, s, g, grad_dir, gr, i, need_geo);
}

static int check_shade(dressi_ctx *ctx, int mode, const dressi_frag_in *in, const float *eye,
                       const int32_t *tri_id, int B, int64_t Npv) {
    if (!ctx) return DRESSI_EINVAL;
    if (mode < DRESSI_SHADE_LAMBERT || mode > DRESSI_SHADE_PHONG_ENV)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade: bad mode");
    if (!in || B < 0 || Npv < 0) return dressi_fail(ctx, DRESSI_EINVAL, "shade: bad arguments");
    if ((int64_t)B * Npv == 0) return DRESSI_OK;
    if (!in->normal || !in->albedo || !eye || !tri_id)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade: normal, albedo, eye and tri_id are required");
    if (in->albedo_channels != 3 && in->albedo_channels != 4)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade: albedo_channels must be 3 or 4");
    if (mode != DRESSI_SHADE_LAMBERT && (!in->pos || in->albedo_channels != 4))
        return dressi_fail(ctx, DRESSI_EINVAL, "shade: Phong modes need pos and rgba albedo");
    if ((in->tangent == nullptr) != (in->nmap == nullptr))
        return dressi_fail(ctx, DRESSI_EINVAL, "shade: tangent and nmap go together");
    return DRESSI_OK;
}

extern "C" int dressi_shade(dressi_ctx *ctx, int mode, const dressi_frag_in *in, const float *eye,
                            const int32_t *tri_id, int B, int64_t Npv, float *color, float *dir,
                            void *stream) {
    int rc = check_shade(ctx, mode, in, eye, tri_id, B, Npv);
    if (rc) return rc;
    int64_t N = (int64_t)B * Npv;
    if (N == 0) return DRESSI_OK;
    if (dir && !in->pos) return dressi_fail(ctx, DRESSI_EINVAL, "shade: dir needs pos");
    if (color && mode == DRESSI_SHADE_PHONG_ENV && !in->env)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade: PHONG_ENV colour needs the environment sample");
    DR_LAUNCH("k_shade", (k_shade), (int)((N + 255) / 256), 256, 0, (hipStream_t)stream, mode, *in, eye, tri_id, N, Npv,
                                                                      color, dir, ctx->skip_empty);
    return dressi_launch_check(ctx, "shade");
}

extern "C" int dressi_shade_bwd(dressi_ctx *ctx, int mode, const dressi_frag_in *in, const float *eye,
                                const int32_t *tri_id, int B, int64_t Npv, const float *grad_color,
                                const float *grad_dir, const dressi_frag_grad *grad, void *stream) {
    int rc = check_shade(ctx, mode, in, eye, tri_id, B, Npv);
    if (rc) return rc;
    if (!grad) return dressi_fail(ctx, DRESSI_EINVAL, "shade_bwd: null grad");
    int64_t N = (int64_t)B * Npv;
    if (N == 0) return DRESSI_OK;
    if (grad_dir && !in->pos) return dressi_fail(ctx, DRESSI_EINVAL, "shade_bwd: grad_dir needs pos");
    if (mode == DRESSI_SHADE_PHONG_ENV && !in->env && (grad->albedo || grad->normal || grad->pos))
        return dressi_fail(ctx, DRESSI_EINVAL, "shade_bwd: PHONG_ENV needs the environment sample");
    DR_LAUNCH("k_shade_bwd", (k_shade_bwd), (int)((N + 255) / 256), 256, 0, (hipStream_t)stream, mode, *in, eye, tri_id, N, Npv,
                                                                          grad_color, grad_dir, *grad, ctx->skip_empty);
    return dressi_launch_check(ctx, "shade_bwd");
}

// ---------------------------------------------------------------------------
// L2 loss with a fixed-order reduction
// ---------------------------------------------------------------------------
#define LOSS_BS 256
#define LOSS_PER_THREAD 4
#define LOSS_MAX_BLOCKS 4096

// Squared differences (and their gradients) of a contiguous range of pixels
// per block, reduced in a fixed tree order to one partial per block; a second
// one-block kernel adds the partials in block order.  No atomics, no fences.
__global__ void __launch_bounds__(LOSS_BS)
    k_loss_l2(const float *__restrict__ color, const float *__restrict__ sil,
              const float *__restrict__ target, const float *__restrict__ weight, int64_t n, int64_t per_block,
              float inv, float *__restrict__ grad_color, float *__restrict__ grad_sil,
              float *__restrict__ partial) {
    __shared__ float red[LOSS_BS];
    float acc = 0.0f;
    const int64_t i0 = (int64_t)blockIdx.x * per_block, i1 = min(n, i0 + per_block);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += LOSS_BS) {
        float4 t = reinterpret_cast<const float4 *>(target)[i];
        float d0 = color[3 * i] - t.x, d1 = color[3 * i + 1] - t.y, d2 = color[3 * i + 2] - t.z;
        float d3 = sil[i] - t.w;
        const float sq = d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
        // per-pixel weight (uneven batches: 1 / (4 H_i W_i) of the pixel's view), else uniform
        const float w = weight ? weight[i] : inv;
        acc += weight ? w * sq : sq;
        if (grad_color) {
            grad_color[3 * i] = 2.0f * w * d0;
            grad_color[3 * i + 1] = 2.0f * w * d1;
            grad_color[3 * i + 2] = 2.0f * w * d2;
        }
        if (grad_sil) grad_sil[i] = 2.0f * w * d3;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = LOSS_BS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// The same with four pixels per thread and 16-byte accesses (every base
// 16-byte aligned, per_block a multiple of 4 * LOSS_BS); a block's last
// pixels that do not fill a quad are taken by its first thread.  Each pixel's
// terms are formed exactly as above.
__device__ __forceinline__ float loss_px(float c0, float c1, float c2, float s, float4 t, float w, bool wt,
                                         float &g0, float &g1, float &g2, float &g3, float &acc) {
    float d0 = c0 - t.x, d1 = c1 - t.y, d2 = c2 - t.z;
    float d3 = s - t.w;
    const float sq = d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
    acc += wt ? w * sq : sq;
    g0 = 2.0f * w * d0;
    g1 = 2.0f * w * d1;
    g2 = 2.0f * w * d2;
    g3 = 2.0f * w * d3;
    return sq;
}

__global__ void __launch_bounds__(LOSS_BS)
    k_loss_l2_v4(const float *__restrict__ color, const float *__restrict__ sil,
                 const float *__restrict__ target, const float *__restrict__ weight, int64_t n,
                 int64_t per_block, float inv, float *__restrict__ grad_color, float *__restrict__ grad_sil,
                 float *__restrict__ partial) {
    __shared__ float red[LOSS_BS];
    float acc = 0.0f;
    const bool wt = weight != nullptr;
    const int64_t i0 = (int64_t)blockIdx.x * per_block, i1 = min(n, i0 + per_block);
    const int64_t q1 = i0 + (i1 - i0) / 4 * 4;
    for (int64_t i = i0 + 4 * (int64_t)threadIdx.x; i < q1; i += 4 * LOSS_BS) {
        const float4 *c4 = reinterpret_cast<const float4 *>(color + 3 * i);
        const float4 ca = c4[0], cb = c4[1], cc = c4[2];
        const float4 s4 = *reinterpret_cast<const float4 *>(sil + i);
        const float4 *t4 = reinterpret_cast<const float4 *>(target) + i;
        const float4 ta = t4[0], tb = t4[1], tc = t4[2], td = t4[3];
        const float4 w4 = wt ? *reinterpret_cast<const float4 *>(weight + i) : make_float4(inv, inv, inv, inv);
        float g[12], gs[4];
        loss_px(ca.x, ca.y, ca.z, s4.x, ta, w4.x, wt, g[0], g[1], g[2], gs[0], acc);
        loss_px(ca.w, cb.x, cb.y, s4.y, tb, w4.y, wt, g[3], g[4], g[5], gs[1], acc);
        loss_px(cb.z, cb.w, cc.x, s4.z, tc, w4.z, wt, g[6], g[7], g[8], gs[2], acc);
        loss_px(cc.y, cc.z, cc.w, s4.w, td, w4.w, wt, g[9], g[10], g[11], gs[3], acc);
        if (grad_color) {
            float4 *o = reinterpret_cast<float4 *>(grad_color + 3 * i);
            o[0] = make_float4(g[0], g[1], g[2], g[3]);
            o[1] = make_float4(g[4], g[5], g[6], g[7]);
            o[2] = make_float4(g[8], g[9], g[10], g[11]);
        }
        if (grad_sil) *reinterpret_cast<float4 *>(grad_sil + i) = make_float4(gs[0], gs[1], gs[2], gs[3]);
    }
    if (threadIdx.x == 0) {
        for (int64_t i = q1; i < i1; i++) {
            const float w = wt ? weight[i] : inv;
            float g0, g1, g2, g3;
            loss_px(color[3 * i], color[3 * i + 1], color[3 * i + 2], sil[i],
                    reinterpret_cast<const float4 *>(target)[i], w, wt, g0, g1, g2, g3, acc);
            if (grad_color) {
                grad_color[3 * i] = g0;
                grad_color[3 * i + 1] = g1;
                grad_color[3 * i + 2] = g2;
            }
            if (grad_sil) grad_sil[i] = g3;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = LOSS_BS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(LOSS_BS)
    k_loss_sum(const float *__restrict__ partial, int nb, float scale, float *__restrict__ loss) {
    static_assert(LOSS_BS == 256, "loss_sum_block is one 256-lane workgroup");
    __shared__ float red[LOSS_BS];
    loss_sum_block(LossJob{partial, nb, scale, loss}, red);
}

extern "C" int dressi_loss_l2(dressi_ctx *ctx, const float *color, const float *sil, const float *target,
                              const float *weight, int B, int H, int W, float *loss, float *grad_color,
                              float *grad_sil, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || H < 0 || W < 0) return dressi_fail(ctx, DRESSI_EINVAL, "loss_l2: bad dimensions");
    int64_t n = (int64_t)B * H * W;
    if (!loss) return dressi_fail(ctx, DRESSI_EINVAL, "loss_l2: null loss");
    if (n > 0 && (!color || !sil || !target)) return dressi_fail(ctx, DRESSI_EINVAL, "loss_l2: null input");
    hipStream_t st = (hipStream_t)stream;
    // blocks of at least LOSS_PER_THREAD pixels per thread, at most LOSS_MAX_BLOCKS
    int64_t per = (int64_t)LOSS_BS * LOSS_PER_THREAD;
    int64_t nb = (n + per - 1) / per;
    if (nb > LOSS_MAX_BLOCKS) {
        nb = LOSS_MAX_BLOCKS;
        per = (n + nb - 1) / nb;
        per = (per + 4 * LOSS_BS - 1) / (4 * LOSS_BS) * (4 * LOSS_BS);
        nb = (n + per - 1) / per;
    }
    if (nb < 1) nb = 1;
    Carver c;
    size_t o_p = c.take(sizeof(float) * (size_t)nb);
    int rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    float *partial = at<float>(ctx->scratch, o_p);
    float inv = 1.0f / (4.0f * (float)(n > 0 ? n : 1));
    const uintptr_t al = (uintptr_t)color | (uintptr_t)sil | (uintptr_t)target | (uintptr_t)weight |
                         (uintptr_t)grad_color | (uintptr_t)grad_sil;
    if ((al & 15u) == 0)
        DR_LAUNCH("k_loss_l2", (k_loss_l2_v4), (int)nb, LOSS_BS, 0, st, color, sil, target, weight, n, per, inv,
                  grad_color, grad_sil, partial);
    else
        DR_LAUNCH("k_loss_l2", (k_loss_l2), (int)nb, LOSS_BS, 0, st, color, sil, target, weight, n, per, inv,
                  grad_color, grad_sil, partial);
    DR_LAUNCH("k_loss_sum", (k_loss_sum), 1, LOSS_BS, 0, st, partial, (int)nb, weight ? 1.0f : inv, loss);
    return dressi_launch_check(ctx, "loss_l2");
}

// vertex_attrs(_bwd) with the adjacency built internally, and the loss's
// block partials
size_t dr_need_shade(const dressi_limits &l) {
    Carver c;
    c.take(adjacency_buf_bytes(std::max(l.V, 0), std::max(l.T, 0)));
    c.take(dressi_adjacency_tmp_bytes(std::max(l.V, 0), std::max(l.T, 0)));
    c.take(sizeof(float) * 3 * (size_t)std::max(l.V, 0));
    // the loss partials: LOSS_MAX_BLOCKS (dressi_loss_l2) or one per 256
    // pixels, at most 65536 (dressi_packed_backward, then the split parts of
    // its texel gather when it gathers)
    const size_t pix = (size_t)std::max(l.B, 0) * std::max(l.H, 0) * std::max(l.W, 0);
    Carver pb;
    pb.take(sizeof(float) * std::min<size_t>((pix + 255) / 256, 65536));
    if (l.tex_cells > 0) pb.take(dressi_invuv_part_bytes(l.tex_cells, 4, std::max(l.B, 1)));
    return std::max({c.off, sizeof(float) * (size_t)LOSS_MAX_BLOCKS, pb.off});
}

// ---------------------------------------------------------------------------
// packed single-layer pass
// ---------------------------------------------------------------------------
// Stage packing (§3.3.3) of a single-layer hard image (K = 1; the blend has
// no edge, so the image is the front fragment's colour where one is present):
// one lane per pixel runs the interpolation, texture and shading stages and
// the blend in the forward, and the loss, blend and shading adjoints, the
// texture-coordinate adjoint with its inverse-UV registration and the
// coordinate's barycentric adjoint in the backward.  Every per-fragment
// value is produced by the same device code as the separate stages.

// Corners of triangle t in a [T, 3] index buffer over Va entries; false when
// t or a corner is out of range (the stages then give zeros).
__device__ __forceinline__ bool tri_corners(const int32_t *__restrict__ tris, int T, int Va, int t, int &v0,
                                            int &v1, int &v2) {
    v0 = v1 = v2 = -1;
    if (t >= 0 && t < T) {
        v0 = tris[3 * (int64_t)t];
        v1 = tris[3 * (int64_t)t + 1];
        v2 = tris[3 * (int64_t)t + 2];
    }
    return !(v0 < 0 || v0 >= Va || v1 < 0 || v1 >= Va || v2 < 0 || v2 >= Va);
}

// CV attribute channels (6: normal, position; 9: + colour); TEX: Phong with a
// 2-D RGBA albedo texture, else Lambert with the vertex colour.
template <int CV, bool TEX>
__global__ void __launch_bounds__(256)
    k_packed_fwd(int mode, dressi_packed_scene sc, const int32_t *__restrict__ tri_id,
                 const float2 *__restrict__ bary, int64_t npix, int64_t n, float *__restrict__ gbuf,
                 float *__restrict__ uvbuf, float *__restrict__ samp, float *__restrict__ color,
                 float *__restrict__ sil, uint8_t *__restrict__ edge, int32_t *__restrict__ inv, int64_t ncells,
                 int skip_empty, ListJob lj, int nmain) {
    // workgroups past the pass's own run a list-building job of the step
    if ((int)blockIdx.x >= nmain) {
        list_job_block(lj, (int)blockIdx.x - nmain);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (inv) {
        // the backward's inverse-UV map starts at -1 (16-byte aligned, int4 rows)
        const int64_t stride = (int64_t)nmain * blockDim.x;
        for (int64_t c = i; c < ncells / 4; c += stride)
            reinterpret_cast<int4 *>(inv)[c] = make_int4(-1, -1, -1, -1);
        for (int64_t c = ncells / 4 * 4 + i; c < ncells; c += stride) inv[c] = -1;
    }
    if (i >= n) return;
    const int t = tri_id[i];
    if (t < 0) {
        edge[i] = 0;
        color[3 * i] = 0.0f; color[3 * i + 1] = 0.0f; color[3 * i + 2] = 0.0f;
        sil[i] = 0.0f;
        if (skip_empty) return;
#pragma unroll
        for (int c = 0; c < CV; c++) gbuf[i * CV + c] = 0.0f;
        if (TEX) {
            uvbuf[2 * i] = 0.0f; uvbuf[2 * i + 1] = 0.0f;
            reinterpret_cast<float4 *>(samp)[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        return;
    }
    // Every load is issued before the first store (the outputs may alias the
    // inputs as far as the compiler knows, so a store would hold back each
    // later load): the corners, the barycentrics, the camera and the texture
    // layer together, then the attribute and coordinate rows, then the taps.
    const float2 w = bary[i];
    const bool view = mode != DRESSI_SHADE_LAMBERT;
    int v0 = -1, v1 = -1, v2 = -1, u0 = -1, u1 = -1, u2 = -1, layer = 0;
    float eye[3] = {0.0f, 0.0f, 0.0f};
    if (t < sc.T) {
        const int32_t *tv = sc.tris + 3 * (int64_t)t;
        v0 = tv[0]; v1 = tv[1]; v2 = tv[2];
        if (TEX) {
            const int32_t *uv = sc.uv_tris + 3 * (int64_t)t;
            u0 = uv[0]; u1 = uv[1]; u2 = uv[2];
            if (sc.td.kind == DRESSI_TEX_2D_ARRAY) layer = sc.td.tri_layer[t];
        }
    }
    const bool oka = !(v0 < 0 || v0 >= sc.V || v1 < 0 || v1 >= sc.V || v2 < 0 || v2 >= sc.V);
    const bool oku = TEX && !(u0 < 0 || u0 >= sc.Vuv || u1 < 0 || u1 >= sc.Vuv || u2 < 0 || u2 >= sc.Vuv);
    const float w2 = 1.0f - w.x - w.y;
    float ga[CV];
    float smp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float q[2] = {0.0f, 0.0f};
    // The attribute and coordinate rows are loaded without a branch (from row
    // 0 for an invalid corner, whose result is then replaced by zero), so that
    // all their loads are in flight together.
    if (sc.V > 0 && (!TEX || sc.Vuv > 0)) {
        const float *a0 = sc.vattr + (int64_t)(oka ? v0 : 0) * CV, *a1 = sc.vattr + (int64_t)(oka ? v1 : 0) * CV,
                    *a2 = sc.vattr + (int64_t)(oka ? v2 : 0) * CV;
        float A0[CV], A1[CV], A2[CV];
#pragma unroll
        for (int c = 0; c < CV; c++) {
            A0[c] = a0[c];
            A1[c] = a1[c];
            A2[c] = a2[c];
        }
        float P0[2] = {0.0f, 0.0f}, P1[2] = {0.0f, 0.0f}, P2[2] = {0.0f, 0.0f};
        if (TEX) {
            const float *p0 = sc.uv + 2 * (int64_t)(oku ? u0 : 0), *p1 = sc.uv + 2 * (int64_t)(oku ? u1 : 0),
                        *p2 = sc.uv + 2 * (int64_t)(oku ? u2 : 0);
#pragma unroll
            for (int c = 0; c < 2; c++) {
                P0[c] = p0[c];
                P1[c] = p1[c];
                P2[c] = p2[c];
            }
        }
#pragma unroll
        for (int c = 0; c < CV; c++) ga[c] = oka ? w.x * A0[c] + w.y * A1[c] + w2 * A2[c] : 0.0f;
        if (TEX) {
#pragma unroll
            for (int c = 0; c < 2; c++) q[c] = oku ? w.x * P0[c] + w.y * P1[c] + w2 * P2[c] : 0.0f;
        }
    } else {
#pragma unroll
        for (int c = 0; c < CV; c++) ga[c] = 0.0f;
    }
    // the camera beside the taps (shading needs it last)
    if (view) {
        const int64_t e = sc.tri_eye ? (int64_t)sc.tri_eye[t] : i / npix;
        eye[0] = sc.eye[3 * e]; eye[1] = sc.eye[3 * e + 1]; eye[2] = sc.eye[3 * e + 2];
    }
    if (TEX) {
        const Taps tp = make_taps(sc.td, q, layer);
        if (tp.ok) tex_bilinear<4>(sc.tex, sc.td, tp, smp, 4);
    }
    dressi_frag_in in{};
    in.normal = ga;
    in.pos = ga + 3;
    in.albedo = TEX ? smp : ga + 6;
    in.albedo_channels = TEX ? 4 : 3;
    ShadeState s;
    shade_forward(mode, in, eye, 0, view, s);
    edge[i] = 0;
#pragma unroll
    for (int c = 0; c < CV; c++) gbuf[i * CV + c] = ga[c];
    if (TEX) {
        uvbuf[2 * i] = q[0];
        uvbuf[2 * i + 1] = q[1];
        reinterpret_cast<float4 *>(samp)[i] = make_float4(smp[0], smp[1], smp[2], smp[3]);
    }
    shade_color(mode, s, color + 3 * i);
    sil[i] = 1.0f;
}

template <int CV, bool TEX>
__global__ void __launch_bounds__(256)
    k_packed_bwd(int mode, dressi_packed_scene sc, const int32_t *__restrict__ tri_id, int64_t npix, int64_t n,
                 const float *__restrict__ gbuf, const float *__restrict__ uvbuf, const float *__restrict__ samp,
                 const float *__restrict__ color, const float *__restrict__ sil, const float4 *__restrict__ target,
                 const float *__restrict__ weight, float w_uniform, float *__restrict__ grad_color,
                 float *__restrict__ grad_sil, float *__restrict__ g_gbuf, float *__restrict__ g_samp,
                 float2 *__restrict__ g_bary_uv, int32_t *__restrict__ inv, int4 *__restrict__ rec,
                 float *__restrict__ partial, int skip_empty, ListJob lj, int nmain) {
    // workgroups past the pass's own run a list-building job of the step
    if ((int)blockIdx.x >= nmain) {
        list_job_block(lj, (int)blockIdx.x - nmain);
        return;
    }
    __shared__ float red[256];
    float acc = 0.0f;
    // one pixel per lane (grid-stride when the image has more pixels than the
    // grid has lanes: each lane's loss terms are added in pixel order)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)nmain * blockDim.x) {
        // L2 loss term and its gradient (the loss stage's arithmetic)
        const float4 tg = target[i];
        const float d0 = color[3 * i] - tg.x, d1 = color[3 * i + 1] - tg.y, d2 = color[3 * i + 2] - tg.z;
        const float d3_ = sil[i] - tg.w;
        const float sq = d0 * d0 + d1 * d1 + d2 * d2 + d3_ * d3_;
        // per-pixel weight (uneven batches), else uniform
        const float w = weight ? weight[i] : w_uniform;
        acc += weight ? w * sq : sq;
        const float g0 = 2.0f * w * d0, g1 = 2.0f * w * d1, g2 = 2.0f * w * d2;
        const int t = tri_id[i];
        if (t < 0) {
            if (grad_color) {
                grad_color[3 * i] = g0; grad_color[3 * i + 1] = g1; grad_color[3 * i + 2] = g2;
            }
            if (grad_sil) grad_sil[i] = 2.0f * w * d3_;
            if (!skip_empty) {
                if (g_gbuf) {
#pragma unroll
                    for (int c = 0; c < CV; c++) g_gbuf[i * CV + c] = 0.0f;
                }
                if (TEX) {
                    reinterpret_cast<float4 *>(g_samp)[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    if (g_bary_uv) g_bary_uv[i] = make_float2(0.0f, 0.0f);
                }
            }
            continue;
        }
        // Every load of the fragment is issued before its first store (the
        // outputs may alias the inputs as far as the compiler knows, so a
        // store would hold back each later load): its G-buffer row, sample and
        // coordinate, its corners' coordinate indices, the texture layer and
        // the camera; then the corners' coordinates beside the taps' texels.
        // The shading adjoint writes into registers, stored at the end.
        const bool view = mode != DRESSI_SHADE_LAMBERT;
        const bool texg = TEX && (inv || g_bary_uv || rec);
        float gv[CV];
#pragma unroll
        for (int c = 0; c < CV; c++) gv[c] = gbuf[i * CV + c];
        float sm[4] = {0.0f, 0.0f, 0.0f, 0.0f}, q[2] = {0.0f, 0.0f};
        int u0 = -1, u1 = -1, u2 = -1, layer = 0;
        if (TEX) {
            const float4 a4 = reinterpret_cast<const float4 *>(samp)[i];
            sm[0] = a4.x; sm[1] = a4.y; sm[2] = a4.z; sm[3] = a4.w;
            if (texg) {
                q[0] = uvbuf[2 * i];
                q[1] = uvbuf[2 * i + 1];
                if (t < sc.T) {
                    const int32_t *ut = sc.uv_tris + 3 * (int64_t)t;
                    u0 = ut[0]; u1 = ut[1]; u2 = ut[2];
                    if (sc.td.kind == DRESSI_TEX_2D_ARRAY) layer = sc.td.tri_layer[t];
                }
            }
        }
        // the taps' texels, the corners' coordinates (from row 0 for an
        // invalid corner, whose result is then zero) and the camera together
        Taps tp;
        tp.ok = 0;
        float t00[4], t01[4], t10[4], t11[4];
        bool oku = false;
        float P0[2] = {0.0f, 0.0f}, P1[2] = {0.0f, 0.0f}, P2[2] = {0.0f, 0.0f};
        if (texg) {
            tp = make_taps(sc.td, q, layer);
            if (tp.ok && g_bary_uv) tex_taps_load<4>(sc.tex, sc.td, tp, 4, t00, t01, t10, t11);
            oku = !(u0 < 0 || u0 >= sc.Vuv || u1 < 0 || u1 >= sc.Vuv || u2 < 0 || u2 >= sc.Vuv);
            if (sc.Vuv > 0) {
                const float *p0 = sc.uv + 2 * (int64_t)(oku ? u0 : 0), *p1 = sc.uv + 2 * (int64_t)(oku ? u1 : 0),
                            *p2 = sc.uv + 2 * (int64_t)(oku ? u2 : 0);
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    P0[c] = p0[c];
                    P1[c] = p1[c];
                    P2[c] = p2[c];
                }
            }
        }
        float eye[3] = {0.0f, 0.0f, 0.0f};
        if (view) {
            const int64_t e = sc.tri_eye ? (int64_t)sc.tri_eye[t] : i / npix;
            eye[0] = sc.eye[3 * e]; eye[1] = sc.eye[3 * e + 1]; eye[2] = sc.eye[3 * e + 2];
        }
        // the hard blend passes the colour gradient to the front layer unchanged
        dressi_frag_in in{};
        in.normal = gv;
        in.pos = gv + 3;
        in.albedo = TEX ? sm : gv + 6;
        in.albedo_channels = TEX ? 4 : 3;
        ShadeState s;
        shade_forward(mode, in, eye, 0, view, s);
        // without g_gbuf only the albedo sample's gradient (texture-only steps)
        float lg[CV], gs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < CV; c++) lg[c] = 0.0f;
        dressi_frag_grad gr{};
        if (g_gbuf) {
            gr.normal = lg;
            gr.pos = lg + 3;
        }
        gr.albedo = TEX ? gs : (g_gbuf ? lg + 6 : nullptr);
        shade_bwd_frag(mode, in, s, d3{g0, g1, g2}, nullptr, gr, 0, g_gbuf != nullptr);
        float2 gb = make_float2(0.0f, 0.0f);
        if (texg) {
            float du = 0.0f, dv = 0.0f;
            if (tp.ok && g_bary_uv) tex_dcoord_texels<4>(sc.td, tp, t00, t01, t10, t11, gs, 4, du, dv);
            if (tp.ok && inv) {
                const int cx = cell1d(q[0], sc.td.Wt, sc.td.wrap_u);
                const int cy = cell1d(q[1], sc.td.Ht, sc.td.wrap_v);
                const int64_t sl = i / npix;
                const int64_t cells = (int64_t)tex_faces(sc.td) * sc.td.Ht * sc.td.Wt;
                atomicMax(&inv[sl * cells + ((int64_t)tp.face * sc.td.Ht + cy) * sc.td.Wt + cx],
                          (int)(i - sl * npix));
            }
            if (tp.ok && rec) invrec_put(rec + 2 * i, tp, gs);
            // barycentric adjoint of the interpolated coordinate
            if (oku) {
                const float gq[2] = {du, dv};
                float a = 0.0f, b = 0.0f;
#pragma unroll
                for (int c = 0; c < 2; c++) {
                    a += gq[c] * (P0[c] - P2[c]);
                    b += gq[c] * (P1[c] - P2[c]);
                }
                gb = make_float2(0.0f + a, 0.0f + b);
            }
        }
        if (grad_color) {
            grad_color[3 * i] = g0; grad_color[3 * i + 1] = g1; grad_color[3 * i + 2] = g2;
        }
        if (grad_sil) grad_sil[i] = 2.0f * w * d3_;
        if (g_gbuf) {
#pragma unroll
            for (int c = 0; c < CV; c++) g_gbuf[i * CV + c] = lg[c];
        }
        if (TEX) {
            reinterpret_cast<float4 *>(g_samp)[i] = make_float4(gs[0], gs[1], gs[2], gs[3]);
            if (texg && g_bary_uv) g_bary_uv[i] = gb;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    // a second launch adds the partials: an agent-scope fence per workgroup
    // (for a last-workgroup sum) writes back the XCD's L2 and costs far more
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

static bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
#define PACKED_MAX_BLOCKS 65536   // loss partials of the packed backward, at most

static int check_packed(dressi_ctx *ctx, const dressi_packed_scene *sc, int B, int H, int W, const char *what) {
    if (!ctx) return DRESSI_EINVAL;
    std::string w(what);
    if (!sc || B < 0 || H < 0 || W < 0 || sc->V < 0 || sc->T < 0) return dressi_fail(ctx, DRESSI_EINVAL, w + ": bad arguments");
    if (sc->mode == DRESSI_SHADE_LAMBERT) {
        if (sc->Cv != 9) return dressi_fail(ctx, DRESSI_EINVAL, w + ": Lambert takes 9 attribute channels");
    } else if (sc->mode == DRESSI_SHADE_PHONG) {
        if (sc->Cv != 6) return dressi_fail(ctx, DRESSI_EINVAL, w + ": Phong takes 6 attribute channels");
        if (!sc->uv || !sc->uv_tris || !sc->tex || sc->Vuv < 0)
            return dressi_fail(ctx, DRESSI_EINVAL, w + ": Phong needs uv, uv_tris and the albedo texture");
        if ((sc->td.kind != DRESSI_TEX_2D && sc->td.kind != DRESSI_TEX_2D_ARRAY) || sc->td.Ct != 4 ||
            sc->td.Ht < 1 || sc->td.Wt < 1 || !al16(sc->tex))
            return dressi_fail(ctx, DRESSI_EINVAL,
                               w + ": the albedo must be a 16-byte aligned 2-D RGBA texture or texture array");
        if (sc->td.kind == DRESSI_TEX_2D_ARRAY && (sc->td.layers < 1 || !sc->td.tri_layer))
            return dressi_fail(ctx, DRESSI_EINVAL, w + ": a texture array needs layers and tri_layer");
        if (sc->td.wrap_u < DRESSI_WRAP_REPEAT || sc->td.wrap_u > DRESSI_WRAP_CLAMP ||
            sc->td.wrap_v < DRESSI_WRAP_REPEAT || sc->td.wrap_v > DRESSI_WRAP_CLAMP)
            return dressi_fail(ctx, DRESSI_EINVAL, w + ": bad wrap mode");
    } else {
        return dressi_fail(ctx, DRESSI_EINVAL, w + ": mode must be Lambert or Phong");
    }
    if ((int64_t)B * H * W > 0 && (!sc->vattr || !sc->tris || !sc->eye))
        return dressi_fail(ctx, DRESSI_EINVAL, w + ": null vattr, tris or eye");
    return DRESSI_OK;
}

extern "C" int dressi_packed_forward(dressi_ctx *ctx, const dressi_packed_scene *sc, const int32_t *tri_id,
                                     const float *bary, int B, int H, int W, float *gbuf, float *uvbuf,
                                     float *samp, float *color, float *sil, uint8_t *edge, int32_t *inv,
                                     void *stream) {
    int rc = check_packed(ctx, sc, B, H, W, "packed_forward");
    if (rc) return rc;
    const int64_t npix = (int64_t)H * W, n = (int64_t)B * npix;
    const bool tex = sc->mode == DRESSI_SHADE_PHONG;
    if (inv && !tex) return dressi_fail(ctx, DRESSI_EINVAL, "packed_forward: inv is for the textured (Phong) pass");
    if (inv && !al16(inv)) return dressi_fail(ctx, DRESSI_EINVAL, "packed_forward: inv must be 16-byte aligned");
    if (n == 0) return DRESSI_OK;
    if (!tri_id || !bary || !gbuf || !color || !sil || !edge || (tex && (!uvbuf || !samp)))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_forward: null input or output");
    if (tex && !al16(samp)) return dressi_fail(ctx, DRESSI_EINVAL, "packed_forward: samp must be 16-byte aligned");
    const int64_t ncells = inv ? (int64_t)B * tex_faces(sc->td) * sc->td.Ht * sc->td.Wt : 0;
    hipStream_t st = (hipStream_t)stream;
    const int g = (int)((n + 255) / 256);
    const float2 *b2 = reinterpret_cast<const float2 *>(bary);
    const ListJob lj = dr_take_list_job(ctx);
    if (tex)
        DR_LAUNCH("k_packed_fwd", (k_packed_fwd<6, true>), g + lj.nb, 256, 0, st, sc->mode, *sc, tri_id, b2, npix, n,
                  gbuf, uvbuf, samp, color, sil, edge, inv, ncells, ctx->skip_empty, lj, g);
    else
        DR_LAUNCH("k_packed_fwd", (k_packed_fwd<9, false>), g + lj.nb, 256, 0, st, sc->mode, *sc, tri_id, b2, npix,
                  n, gbuf, uvbuf, samp, color, sil, edge, inv, ncells, ctx->skip_empty, lj, g);
    return dressi_launch_check(ctx, "packed_forward");
}

size_t dr_packed_bwd_scratch(const dressi_packed_scene *sc, int B, int H, int W, bool grad_tex) {
    const int64_t n = (int64_t)B * H * W;
    const int64_t nb = n > 0 ? std::min<int64_t>((n + 255) / 256, PACKED_MAX_BLOCKS) : 1;
    Carver c;
    c.take(sizeof(float) * (size_t)nb);
    const int64_t cells =
        sc->mode == DRESSI_SHADE_PHONG ? (int64_t)tex_faces(sc->td) * sc->td.Ht * sc->td.Wt : 0;
    if (grad_tex) c.take(dressi_invuv_part_bytes(cells, 4, B));
    return c.off;
}

extern "C" int dressi_packed_backward(dressi_ctx *ctx, const dressi_packed_scene *sc, const int32_t *tri_id,
                                      int B, int H, int W, const float *gbuf, const float *uvbuf,
                                      const float *samp, const float *color, const float *sil,
                                      const float *target, const float *weight, float *loss, float *grad_color,
                                      float *grad_sil, float *grad_gbuf, float *grad_samp, float *grad_bary_uv,
                                      int32_t *inv, void *inv_rec, float *grad_tex, void *stream) {
    int rc = check_packed(ctx, sc, B, H, W, "packed_backward");
    if (rc) return rc;
    const int64_t npix = (int64_t)H * W, n = (int64_t)B * npix;
    const bool tex = sc->mode == DRESSI_SHADE_PHONG;
    if (!loss) return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: null loss");
    if (inv && !tex) return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: inv is for the textured (Phong) pass");
    if (inv_rec && (!tex || !al16(inv_rec)))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: inv_rec is for the textured pass, 16-byte aligned");
    if (grad_tex && (!inv || !inv_rec || !al16(grad_tex)))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: grad_tex needs inv, inv_rec and 16-byte alignment");
    if (grad_tex && ((sc->td.wrap_u == DRESSI_WRAP_REPEAT && sc->td.Wt < 3) ||
                     (sc->td.wrap_v == DRESSI_WRAP_REPEAT && sc->td.Ht < 3)))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: repeat wrap needs at least 3 texels");
    if (n > 0 && (!tri_id || !gbuf || !color || !sil || !target || (!tex && !grad_gbuf) ||
                  (tex && (!uvbuf || !samp || !grad_samp))))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: null input or output");
    if (n > 0 && (!al16(target) || (tex && (!al16(samp) || !al16(grad_samp)))))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_backward: target, samp and grad_samp must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = n > 0 ? std::min<int64_t>((n + 255) / 256, PACKED_MAX_BLOCKS) : 1;
    Carver c;
    const size_t o_p = c.take(sizeof(float) * (size_t)nb);
    const int64_t cells = tex ? (int64_t)tex_faces(sc->td) * sc->td.Ht * sc->td.Wt : 0;
    const size_t o_g = grad_tex ? c.take(dressi_invuv_part_bytes(cells, 4, B)) : 0;
    if ((rc = dressi_scratch(ctx, c.off, st))) return rc;
    float *partial = at<float>(ctx->scratch, o_p);
    const float w = 1.0f / (4.0f * (float)(n > 0 ? n : 1));
    const float4 *t4 = reinterpret_cast<const float4 *>(target);
    float2 *gb = reinterpret_cast<float2 *>(grad_bary_uv);
    if (n == 0) {
        dressi_fill_f32(partial, 0.0f, 1, st);
    } else {
        const ListJob job = dr_take_list_job(ctx);
        if (tex)
            DR_LAUNCH("k_packed_bwd", (k_packed_bwd<6, true>), (int)nb + job.nb, 256, 0, st, sc->mode, *sc, tri_id,
                      npix, n, gbuf, uvbuf, samp, color, sil, t4, weight, w, grad_color, grad_sil, grad_gbuf,
                      grad_samp, gb, inv, static_cast<int4 *>(inv_rec), partial, ctx->skip_empty, job, (int)nb);
        else
            DR_LAUNCH("k_packed_bwd", (k_packed_bwd<9, false>), (int)nb + job.nb, 256, 0, st, sc->mode, *sc, tri_id,
                      npix, n, gbuf, uvbuf, samp, color, sil, t4, weight, w, grad_color, grad_sil, grad_gbuf,
                      grad_samp, gb, inv, nullptr, partial, ctx->skip_empty, job, (int)nb);
    }
    const LossJob lj{partial, (int)nb, weight ? 1.0f : w, loss};
    if (grad_tex) {
        // the texel gather, with the loss's last sum in an extra workgroup of its launch
        dr_gather_invrec(sc->td, B, npix, inv, static_cast<const int4 *>(inv_rec), at<float>(ctx->scratch, o_g),
                         grad_tex, st, ctx->iv_rows, lj, dr_take_list_job(ctx));
    } else {
        DR_LAUNCH("k_loss_sum", (k_loss_sum), 1, LOSS_BS, 0, st, lj.partial, lj.nb, lj.scale, lj.loss);
    }
    return dressi_launch_check(ctx, "packed_backward");
}
