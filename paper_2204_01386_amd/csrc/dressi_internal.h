// Internal declarations of libdressi (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dressi.h"

#define DRESSI_TILE 16          // screen tile edge in pixels (one lane per pixel)
#define DRESSI_TILE_PIX 256     // pixels per tile
#define DRESSI_MAX_K 5
#define DRESSI_SUBPIX 256       // 8 sub-pixel bits

struct dressi_ctx {
    int device = 0;
    void *scratch = nullptr;    // device arena, reused by every call on this context
    size_t scratch_bytes = 0;
    int64_t bin_capacity = 0;   // triangles per screen tile bin (0 = automatic)
    int hard_raster = 0;        // hard rasterization: 0 triangle-parallel, 1 pixel-parallel, 2 per tile
    int hybrid_weight = 24;     // strategy 2's cost ratio, in sixteenths
    int skip_empty = 0;         // 1: per-fragment outputs of empty slots left unwritten
    int iv_rows = 0;            // texel rows per lane of the inverse-UV gather (0 = automatic)
    int64_t *status = nullptr;  // device: [0] overflow flag, [1] bin capacity needed
    int32_t *counters = nullptr;  // device counters kept at zero between calls
    size_t counters_n = 0;
    // Arenas and counter arrays replaced by larger ones.  A graph captured
    // before the growth still holds their addresses, so they stay allocated
    // (and the counters zero) until dressi_destroy.
    std::vector<void *> retired;
    std::string err;
    // list-building jobs for the next capable launches, taken in order (a
    // whole step only)
    const struct ListJob *list_job = nullptr;
    int n_list_jobs = 0;
};

// ---------------------------------------------------------------------------
// host helpers (context.hip)
// ---------------------------------------------------------------------------
int dressi_fail(dressi_ctx *ctx, int code, const std::string &msg);
int dressi_hip_check(dressi_ctx *ctx, hipError_t e, const char *what);
// Makes sure the arena holds `bytes`; grows it outside stream capture,
// fails with DRESSI_ENOMEM while `stream` is capturing.
int dressi_scratch(dressi_ctx *ctx, size_t bytes, hipStream_t stream);
int dressi_launch_check(dressi_ctx *ctx, const char *what);
// The blend's edge mask (softras.hip): S^H from layer 0 of tri_id (hard where
// the sign bit of dist is clear, all present fragments when dist is NULL),
// its 4-neighbour boundary `bnd`, the row pass `rows` and the mask `edge`
// (L-infinity dilation of radius rho >= 0), one byte per pixel [B,H,W].
void dressi_edge_mask(const int32_t *tri_id, const float *dist, int B, int K, int H, int W, int rho,
                      uint8_t *bnd, uint8_t *rows, uint8_t *edge, hipStream_t st);
// Scratch each file's entry points need at the given limits (the largest
// call, with every optional index built internally); for dressi_limits.
size_t dr_need_raster(const dressi_limits &l, int64_t cap);   // raster.hip
size_t dr_need_interp(const dressi_limits &l);                // interp.hip
size_t dr_need_texture(const dressi_limits &l);               // texture.hip
size_t dr_packed_bwd_scratch(const dressi_packed_scene *sc, int B, int H, int W, bool grad_tex);
size_t dr_need_shade(const dressi_limits &l);                 // shade.hip
size_t dr_need_optim(const dressi_limits &l);                 // optim.hip
size_t dr_need_pbs(const dressi_limits &l);                   // pbs.hip
int64_t dr_tile_capacity(const dressi_limits &l);             // raster.hip
// Looks up, once per device, the device address of the fixed scratch of
// dressi_softras_noalloc (softras.hip); `device` must be current.
int dressi_softras_noalloc_setup(int device);
// Makes sure ctx->counters holds at least n int32 counters, all zero.  The
// kernels that use them count up and then back down (or reset what they
// read), so they are zero again when a call ends.  Grows only outside
// stream capture.
int dressi_counters(dressi_ctx *ctx, size_t n, hipStream_t stream);

// Optional per-kernel timing with HIP events (eager runs only): every launch
// goes through DR_LAUNCH.  While the profiler is on (dressi_profile_start) the
// launch takes a start/stop event pair that the runtime stamps from the
// kernel's own dispatch (hipExtLaunchKernelGGL), so the measured time is the
// kernel's execution alone; otherwise it costs one branch.
bool dr_prof_slot(const char *name, hipEvent_t *start, hipEvent_t *stop);
#define DR_LAUNCH(NAME, KERN, GRID, BLOCK, SHMEM, STREAM, ...)                  \
    do {                                                                        \
        hipEvent_t dr_e0_ = nullptr, dr_e1_ = nullptr;                          \
        if (dr_prof_slot(NAME, &dr_e0_, &dr_e1_))                               \
            hipExtLaunchKernelGGL(KERN, dim3(GRID), dim3(BLOCK), SHMEM, STREAM, \
                                  dr_e0_, dr_e1_, 0, __VA_ARGS__);              \
        else                                                                    \
            hipLaunchKernelGGL(KERN, dim3(GRID), dim3(BLOCK), SHMEM, STREAM,    \
                               __VA_ARGS__);                                    \
    } while (0)

// Inverse-UV gather: slices whose cell halos are loaded together, and the
// split of the slices over the grid for small textures (with its scratch of
// partial sums).
#define DRESSI_IV_SG 1     // slices staged together by the inverse-UV gather
#define DRESSI_IV_PART 4   // slices per part when a small texture's slices are split over the grid
static inline int dressi_invuv_nsplit(int64_t cells, int S) {
    return (cells < (1 << 19) && S > DRESSI_IV_PART) ? (S + DRESSI_IV_PART - 1) / DRESSI_IV_PART : 1;
}
static inline size_t dressi_invuv_part_bytes(int64_t cells, int Ct, int S) {
    int ns = dressi_invuv_nsplit(cells, S);
    return ns > 1 ? sizeof(float) * (size_t)cells * Ct * ns : 0;
}

// The last step of a loss: its per-block partials added by one 256-lane
// workgroup (lane i takes the partials i, i + 256, ... in order, eight loads
// in flight, then a fixed tree), loss[0] = scale * sum.  `red` is 256 floats
// of LDS.  Used by k_loss_sum and, riding in the texel gather's launch, by
// the packed backward.
struct LossJob {
    const float *partial;
    int nb;
    float scale;
    float *loss;   // NULL: no job
};
__device__ __forceinline__ void loss_sum_block(const LossJob &j, float *red) {
    float a = 0.0f;
    for (int i = threadIdx.x; i < j.nb; i += 8 * 256) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = i + q * 256 < j.nb ? j.partial[i + q * 256] : 0.0f;
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (i + q * 256 < j.nb) a += v[q];
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) j.loss[0] = red[0] * j.scale;
}

// Texel gather from per-pixel records (texture.hip), with an optional loss
// job in an extra workgroup of its launch; part: scratch of
// dressi_invuv_part_bytes(cells, 4, S).
struct ListJob;
void dr_gather_invrec(const dressi_tex_desc &td, int S, int64_t npix, const int32_t *inv, const int4 *rec,
                      float *part, float *grad_tex, hipStream_t st, int rows, LossJob lj, const ListJob &job);

// Bump allocator over the arena: carve(n) returns 256-byte aligned offsets.
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};
template <class T> static inline T *at(void *base, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

// ---------------------------------------------------------------------------
// primitives (prims.hip)
// ---------------------------------------------------------------------------
void dressi_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void dressi_fill_f32(float *p, float v, int64_t n, hipStream_t s);
// Exclusive scan of n int32 counts into out[0..n] (out[n] = total); `tmp`
// needs dressi_scan_tmp_bytes(n).  out may alias nothing.
size_t dressi_scan_tmp_bytes(int64_t n);
void dressi_exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *tmp, hipStream_t s);

// vertex -> corner adjacency: offsets [V+1], corners [3T] (corner = 3t+i),
// stored in one int32 buffer of V+1+3T entries (offsets first)
struct Adjacency {
    int32_t *offsets;
    int32_t *corners;
};
static inline Adjacency adjacency_view(const int32_t *buf, int V) {
    Adjacency a;
    a.offsets = const_cast<int32_t *>(buf);
    a.corners = const_cast<int32_t *>(buf) + V + 1;
    return a;
}
static inline size_t adjacency_buf_bytes(int V, int T) { return sizeof(int32_t) * ((size_t)V + 1 + 3 * (size_t)T); }
size_t dressi_adjacency_tmp_bytes(int V, int T);
void dressi_build_adjacency_into(const int32_t *tris, int T, int V, int32_t *buf, void *tmp,
                                 hipStream_t s);

// ---------------------------------------------------------------------------
// fragment index (raster.hip): the fragments of each tile sorted by triangle
// id, and its transpose (the tiles of each triangle).  Used by every
// deterministic backward reduction; built once per rasterization.
// ---------------------------------------------------------------------------
struct FragLists {
    int32_t *n_frag;    // [B*nTiles] valid fragments in the tile
    int32_t *n_rec;     // [B*nTiles] distinct triangles in the tile
    uint16_t *frag;     // [B*nTiles*256*K] local fragment index k*256 + pixel, sorted
    int32_t *rec_tri;   // [B*nTiles*256*K] distinct triangle ids, ascending
    int32_t *rec_start; // [B*nTiles*256*K] first sorted fragment of each triangle
};
// for every (view, triangle) the tiles in which it has fragments, as
// (tile index b*nTiles+tile, record index) pairs in ascending tile order
struct TriTiles {
    int32_t *offsets;   // [B*T+1]
    int2 *entries;      // [B*nTiles*256*K]
};
// Per-tile interpolation adjoint (interp.hip): grad_bary and each tile's
// per-triangle records of b_i g in `part` [B*nTiles*256*K][3][C].
void dr_interp_bwd_tiles(const float *attr, int Ba, int Va, int C, const int32_t *attr_tris, int T,
                         const int32_t *tri_id, const float *bary, int B, int K, int H, int W, const FragLists &fl,
                         const float *grad_out, const float *grad_bary_in, float *grad_bary, float *part,
                         int skip_empty, hipStream_t st);
size_t dressi_fragindex_bytes(int B, int K, int H, int W, int T);
void dressi_fragindex_view(void *base, int B, int K, int H, int W, int T, FragLists &fl, TriTiles &tt);
size_t dressi_fragindex_tmp_bytes(int B, int K, int H, int W, int T);
void dressi_build_fragindex(const int32_t *tri_id, int B, int K, int H, int W, int T, void *base,
                            void *tmp, int32_t *zero_counts, hipStream_t s);

// MI355X dispatches the workgroups of a grid to its 8 XCDs round-robin
// (workgroup i on XCD i mod 8), and each XCD has its own L2.  The logical
// block index below gives every XCD one contiguous range of the grid, so
// workgroups that touch neighbouring pixels or tiles (and share triangles,
// attributes and texels) run behind the same L2.  A bijection of [0, nb).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}
__device__ __forceinline__ int64_t xcd_block() { return xcd_block(blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------------------
// The workgroup bodies of the kernels that turn the per-tile records of a
// fragment index into its triangle -> tile lists (the counts' scan, the
// fill and the ranking; prims.hip and raster.hip), as jobs that the extra
// workgroups of another stage's launch can run: a whole step launches them
// beside independent kernels (ListJob; bid, nb: the workgroup and the
// workgroup count the job is run with).  256 lanes a workgroup.
// ---------------------------------------------------------------------------
template <int BS>
__device__ __forceinline__ int block_exclusive_scan(int v, int &total, int *wsum) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int s = (lane < BS / 64) ? wsum[lane] : 0;
#pragma unroll
        for (int o = 1; o < BS / 64; o <<= 1) {
            int y = __shfl_up(s, o, 64);
            if (lane >= o) s += y;
        }
        if (lane < BS / 64) wsum[lane] = s;
    }
    __syncthreads();
    int base = wid ? wsum[wid - 1] : 0;
    total = wsum[BS / 64 - 1];
    __syncthreads();
    return base + x - v;
}

#define SCAN_BS 256
#define SCAN_PER 4
#define SCAN_CHUNK (SCAN_BS * SCAN_PER)
#define SCAN_DIRECT_MAX 2048   // chunks the one-pass apply adds up before its own
#define TT_SHORT 32

// the sum of each chunk of SCAN_CHUNK counts
__device__ __forceinline__ void scan_reduce_block(const int32_t *in, int64_t n, int32_t *block_sums, int bid) {
    __shared__ int wsum[SCAN_BS / 64];
    int64_t base = (int64_t)bid * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++)
        if (base + j < n) s += in[base + j];
    int total;
    block_exclusive_scan<SCAN_BS>(s, total, wsum);
    if (threadIdx.x == 0) block_sums[bid] = total;
}

// the exclusive scan of one chunk, after adding up the sums of the chunks
// before it (nb chunks; the last writes the total to out[n])
__device__ __forceinline__ void scan_apply_direct_block(const int32_t *in, int32_t *out, int64_t n,
                                                        const int32_t *block_sums, int bid, int nb) {
    __shared__ int wsum[SCAN_BS / 64];
    int pre = 0;
    for (int j = threadIdx.x; j < bid; j += SCAN_BS) pre += block_sums[j];
    int offset;
    block_exclusive_scan<SCAN_BS>(pre, offset, wsum);
    int64_t base = (int64_t)bid * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
    int v[SCAN_PER];
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        s += v[j];
    }
    int total;
    int ex = block_exclusive_scan<SCAN_BS>(s, total, wsum) + offset;
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
    if (bid == nb - 1 && threadIdx.x == SCAN_BS - 1) out[n] = ex;
}

// One tile's records into their (view, triangle) lists, unsorted: each takes
// a slot by counting its list's counter back down (which leaves the counters
// at zero for the next call); the last entry placed of a list longer than
// TT_SHORT queues it for the merge sort.  Several views: XCD-aware order
// (each XCD whole views); one view keeps the default interleave.
__device__ __forceinline__ void tt_fill_block(const FragLists &fl, int K, int T, int nt,
                                              const int32_t *__restrict__ offsets, int32_t *__restrict__ counts,
                                              int2 *__restrict__ entries, int32_t *__restrict__ nlong,
                                              int64_t *__restrict__ longk, int cap, int bid, int nb) {
    const int bt = nb > nt ? (int)xcd_block(bid, nb) : bid;
    const int b = bt / nt;
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX * K;
    const int n = fl.n_rec[bt];
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        int t = fl.rec_tri[base + r];
        if (t < 0 || t >= T) continue;
        int64_t bt_t = (int64_t)b * T + t;
        const int c = atomicSub(&counts[bt_t], 1);
        int slot = offsets[bt_t] + c - 1;
        entries[slot] = make_int2(bt, r);
        if (c == 1 && offsets[bt_t + 1] - offsets[bt_t] > TT_SHORT) {
            const int q = atomicAdd(nlong, 1);
            if (q < cap) longk[q] = bt_t;
        }
    }
}

// The lists in ascending tile order.  Short lists: one thread per entry,
// whose place is the number of its list's entries from lower tiles (a
// triangle has at most one record per tile).  Long lists: one workgroup per
// queued list, a bottom-up merge sort by tile from the list's stretch of
// `unsorted`, ping-ponging between its stretches of `sbuf` and `entries`
// (runs of width 1, 2, 4, ...; an entry's place in its merged pair of runs
// is its rank in its own run plus the number of smaller tiles in the other,
// by binary search).  `unsorted` is only read, so the short lists' threads
// never see a list being sorted.
__device__ __forceinline__ void tt_rank_block(const FragLists &fl, int K, int T, int nt,
                                              const int32_t *__restrict__ offsets,
                                              const int2 *__restrict__ unsorted, int2 *__restrict__ entries,
                                              int2 *__restrict__ sbuf, int64_t nkeys,
                                              const int32_t *__restrict__ nlong, const int64_t *__restrict__ longk,
                                              int cap, int bid, int nb) {
    const int nq = min(*nlong, cap);
    for (int q = bid; q < nq; q += nb) {
        const int64_t key = longk[q];
        const int lo = offsets[key], n = offsets[key + 1] - lo;
        for (int i = threadIdx.x; i < n; i += blockDim.x) sbuf[lo + i] = unsorted[lo + i];
        __syncthreads();
        int2 *src = sbuf + lo, *dst = entries + lo;
        for (int w = 1; w < n; w <<= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int2 x = src[i];
                const int r = i / w;
                const int own = r * w, base = (r & ~1) * w;
                const int ps = (r ^ 1) * w, pe = min(ps + w, n);
                int a = ps, z = max(ps, pe);
                while (a < z) {
                    const int mid = (a + z) >> 1;
                    if (src[mid].x < x.x) a = mid + 1;
                    else z = mid;
                }
                dst[base + (i - own) + (a - ps)] = x;
            }
            __syncthreads();
            int2 *tswap = src;
            src = dst;
            dst = tswap;
        }
        if (src != entries + lo)
            for (int i = threadIdx.x; i < n; i += blockDim.x) entries[lo + i] = src[i];
        __syncthreads();
    }
    const int64_t total = offsets[nkeys];   // the number of entries (the scan's total)
    for (int64_t e = (int64_t)bid * blockDim.x + threadIdx.x; e < total; e += (int64_t)nb * blockDim.x) {
        const int2 ent = unsorted[e];
        const int t = fl.rec_tri[(int64_t)ent.x * DRESSI_TILE_PIX * K + ent.y];
        const int64_t key = (int64_t)(ent.x / nt) * T + t;
        const int lo = offsets[key], hi = offsets[key + 1];
        if (hi - lo > TT_SHORT) continue;   // a long list, sorted above
        int rank = 0;
        for (int j = lo; j < hi; j++) rank += unsorted[j].x < ent.x;
        entries[lo + rank] = ent;
    }
}

enum { LJ_NONE = 0, LJ_SCAN_REDUCE, LJ_SCAN_APPLY, LJ_TT_FILL, LJ_TT_RANK };
// One job's arguments.  in: the record counts [n] (the scan's input); out:
// the lists' offsets [n + 1] (the scan's output, which the fill and the
// ranking read); n: the number of (view, triangle) keys; sums: the chunk
// sums; the rest as k_tt_fill and k_tt_rank take them.
struct ListJob {
    int kind = LJ_NONE;
    int nb = 0;                         // workgroups
    const int32_t *in = nullptr;
    int32_t *out = nullptr;
    int64_t n = 0;
    int32_t *sums = nullptr;
    FragLists fl{};
    int K = 1, T = 0, nt = 1, cap = 0;
    int32_t *counts = nullptr, *nlong = nullptr;
    int2 *unsorted = nullptr, *entries = nullptr, *sbuf = nullptr;
    int64_t *longk = nullptr;
};
__device__ __forceinline__ void list_job_block(const ListJob &j, int bid) {
    if (bid >= j.nb) return;
    switch (j.kind) {
    case LJ_SCAN_REDUCE: scan_reduce_block(j.in, j.n, j.sums, bid); break;
    case LJ_SCAN_APPLY: scan_apply_direct_block(j.in, j.out, j.n, j.sums, bid, j.nb); break;
    case LJ_TT_FILL:
        tt_fill_block(j.fl, j.K, j.T, j.nt, j.out, j.counts, j.unsorted, j.nlong, j.longk, j.cap, bid, j.nb);
        break;
    case LJ_TT_RANK:
        tt_rank_block(j.fl, j.K, j.T, j.nt, j.out, j.unsorted, j.entries, j.sbuf, j.n, j.nlong, j.longk, j.cap, bid,
                      j.nb);
        break;
    default: break;
    }
}
// the job the step's next capable launch takes (none outside a whole step)
static inline ListJob dr_take_list_job(dressi_ctx *ctx) {
    ListJob j;
    if (ctx->n_list_jobs > 0) {
        j = *ctx->list_job++;
        ctx->n_list_jobs--;
    }
    return j;
}
// runs the jobs not taken yet as launches of their own (raster.hip)
void dr_flush_list_jobs(dressi_ctx *ctx, hipStream_t st);

__host__ __device__ static inline int tiles_x(int W) { return (W + DRESSI_TILE - 1) / DRESSI_TILE; }
__host__ __device__ static inline int tiles_y(int H) { return (H + DRESSI_TILE - 1) / DRESSI_TILE; }

// ---------------------------------------------------------------------------
// Triangle setup shared by the forward and backward kernels (device code).
// The arithmetic order below is part of the interface contract (the decisions
// it feeds must be reproducible by any conforming implementation):
//   x_px = (x/w + 1) * (W/2), y_px = (1 - y/w) * (H/2) in float, snapped with
//   round-to-nearest-even to 1/256 px; twice the signed area in int64; the
//   vertex order is normalised so the area is positive (1 <-> 2 swapped);
//   zero area or a vertex with w <= 0 drops the triangle.
// ---------------------------------------------------------------------------
struct TriSetup {
    int X[3], Y[3];   // snapped fixed-point coordinates, normalised order
    float zn[3];      // z/w
    float w[3];       // clip w
    float Af;         // twice the area as float
    int meta;         // bit0 valid, bits1-3 edge owns zero, bits 4-9 corner of vertex i
    int box0, box1;   // pixel bbox: x0 | x1 << 16, y0 | y1 << 16 (hard or soft)
    // for the soft rasterizer's culling tests
    int hbox0, hbox1; // pixels whose centres lie in the vertex box, as box0/box1 (signed halves)
    int zlb;          // float bits of a lower bound of the hard keys (>= 0)
    float elen[3];    // sqrtf of the squared length (fixed-point units) of edge i, opposite vertex i
    int pad[2];
};
static_assert(sizeof(TriSetup) == 96, "setup record is 96 bytes");

__device__ __forceinline__ bool dr_snap(float c, float w, float half, bool is_y, int &out) {
    float n = c / w;
    float p = is_y ? (1.0f - n) * half : (n + 1.0f) * half;
    float f = p * 256.0f;
    if (!(fabsf(f) < 4194304.0f)) return false;
    out = (int)rintf(f);
    return true;
}

__device__ __forceinline__ int floor_div256(int v) { return v >> 8; }  // arithmetic shift floors

// Views of an uneven batch: triangle t belongs to view tri_view[t], drawn in
// the rectangle views[v] = (x0, y0, W, H) of one image.  A null tri_view
// means one view covering the whole H x W image.
struct Viewports {
    const int32_t *tri_view;
    const int4 *views;
};

__device__ __forceinline__ int4 dr_viewport(const Viewports &vp, int t, int H, int W) {
    if (!vp.tri_view) return make_int4(0, 0, W, H);
    return vp.views[vp.tri_view[t]];
}

// Per-vertex part of the geometry adjoint of one image (shade.hip): both
// vertex sums, the transform adjoint and the vertex-normal adjoint, writing
// grad_attr, grad_pos_clip and the world-position gradient grad_pos
// (grad_pos_t and gacc: scratch of 3V floats each).
// The vertex stage of B views (vattr [V,C], pos_clip [B,V,4]) and the binless
// hard rasterizer's merge into the zero-kept per-pixel keys zbuf [B,H,W] in
// one launch (shade.hip); adj: the vertex -> corner adjacency buffer.
void dr_vertex_raster_direct(const float *pos, const int32_t *tris, const float *extra, const int32_t *adj, int V,
                             int C, float *vattr, const float *mvp, int B, float *pos_clip, int T, int H, int W,
                             int cull, unsigned long long *zbuf, hipStream_t st);

void dr_geo_vertex(int Cv, const float *pos, const int32_t *tris, const float *pos_clip, Viewports vp, int V, int H,
                   int W, TriTiles tt, const float *ipart, const float *rpart, Adjacency adj, const float *mvp,
                   const int32_t *vert_view, float *grad_attr, float *grad_pos_clip, float *grad_pos_t, float *gacc,
                   float *grad_pos, hipStream_t st);

// Builds the record of triangle `tv` (three vertex ids) for a view of H x W
// pixels placed at pixel (ox, oy) of the image (0, 0 for a whole image):
// coordinates are snapped in the view's own frame, then moved by the integer
// offset, and the boxes are clamped to the view.  `margin` extends the pixel
// bbox (soft reach).  cull = 1 drops faces clockwise in NDC.  Here from the
// three vertices' clip-space positions p, already loaded; dr_setup below
// loads them.
__device__ __forceinline__ TriSetup dr_setup_pts(const float4 *p, int H, int W, int ox, int oy, int cull,
                                                 int margin) {
    TriSetup s;
    s.meta = 0;
    s.box0 = 1;      // empty box (x0 = 1 > x1 = 0)
    s.box1 = 1;
    s.hbox0 = s.hbox1 = 1;
    s.zlb = 0;
    s.elen[0] = s.elen[1] = s.elen[2] = 0.0f;
    s.pad[0] = s.pad[1] = 0;
    int X[3], Y[3];
    float hw = 0.5f * (float)W, hh = 0.5f * (float)H;
    // the three vertices' tests are combined into one branch
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        X[i] = Y[i] = 0;
        ok = ok & (p[i].w > 0.0f);
        ok = ok & dr_snap(p[i].x, p[i].w, hw, false, X[i]);
        ok = ok & dr_snap(p[i].y, p[i].w, hh, true, Y[i]);
        X[i] += DRESSI_SUBPIX * ox;
        Y[i] += DRESSI_SUBPIX * oy;
    }
    if (!ok) return s;
    int64_t A2 = (int64_t)(X[1] - X[0]) * (int64_t)(Y[2] - Y[0]) -
                 (int64_t)(X[2] - X[0]) * (int64_t)(Y[1] - Y[0]);
    if (A2 == 0) return s;
    if (cull && A2 > 0) return s;
    int o1 = 1, o2 = 2;
    if (A2 < 0) { o1 = 2; o2 = 1; A2 = -A2; }
    const int ord[3] = {0, o1, o2};
    int xmin = 0x7fffffff, xmax = -0x7fffffff, ymin = 0x7fffffff, ymax = -0x7fffffff;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        int c = ord[i];
        s.X[i] = X[c];
        s.Y[i] = Y[c];
        s.zn[i] = p[c].z / p[c].w;
        s.w[i] = p[c].w;
        s.meta |= c << (4 + 2 * i);
        xmin = min(xmin, X[c]); xmax = max(xmax, X[c]);
        ymin = min(ymin, Y[c]); ymax = max(ymax, Y[c]);
    }
    s.Af = (float)A2;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        int a = (i + 1) % 3, b = (i + 2) % 3;
        int dx = s.X[b] - s.X[a], dy = s.Y[b] - s.Y[a];
        if (dy < 0 || (dy == 0 && dx > 0)) s.meta |= 1 << (1 + i);
    }
    // pixels with centre 256x+128 inside [xmin, xmax]
    int x0 = -floor_div256(-(xmin - 128)) - margin;   // ceil
    int x1 = floor_div256(xmax - 128) + margin;
    int y0 = -floor_div256(-(ymin - 128)) - margin;
    int y1 = floor_div256(ymax - 128) + margin;
    {
        int hx0 = x0 + margin, hx1 = x1 - margin, hy0 = y0 + margin, hy1 = y1 - margin;
        hx0 = min(max(hx0, ox - 1), ox + W); hx1 = min(max(hx1, ox - 1), ox + W);
        hy0 = min(max(hy0, oy - 1), oy + H); hy1 = min(max(hy1, oy - 1), oy + H);
        s.hbox0 = (hx0 & 0xffff) | (hx1 << 16);
        s.hbox1 = (hy0 & 0xffff) | (hy1 << 16);
        float zmin = fminf(fminf(s.zn[0], s.zn[1]), s.zn[2]);
        float zlb = 0.5f * zmin - 1e-6f;
        s.zlb = zlb > 0.0f ? __float_as_int(zlb) : 0;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            int a = (i + 1) % 3, c = (i + 2) % 3;
            double ex = (double)(s.X[c] - s.X[a]), ey = (double)(s.Y[c] - s.Y[a]);
            s.elen[i] = sqrtf((float)(ex * ex + ey * ey));
        }
    }
    x0 = max(x0, ox); y0 = max(y0, oy);
    x1 = min(x1, ox + W - 1); y1 = min(y1, oy + H - 1);
    if (x0 > x1 || y0 > y1) return s;
    s.box0 = x0 | (x1 << 16);
    s.box1 = y0 | (y1 << 16);
    s.meta |= 1;
    return s;
}

// dr_setup_pts of vertices v0, v1, v2 of pc, loaded before any test so that
// their loads are in flight together (the indices are valid: every caller
// checks them).
__device__ __forceinline__ TriSetup dr_setup(const float4 *pc, int v0, int v1, int v2, int H, int W, int ox, int oy,
                                             int cull, int margin) {
    const float4 p[3] = {pc[v0], pc[v1], pc[v2]};
    return dr_setup_pts(p, H, W, ox, oy, cull, margin);
}

// dr_setup of triangle `tv` (three vertex indices), empty when an index is
// outside [0, V)
__device__ __forceinline__ TriSetup dr_setup_tri(const float4 *pc, const int32_t *tv, int V, int H, int W, int ox,
                                                 int oy, int cull, int margin) {
    const int v0 = tv[0], v1 = tv[1], v2 = tv[2];
    if ((unsigned)v0 >= (unsigned)V || (unsigned)v1 >= (unsigned)V || (unsigned)v2 >= (unsigned)V) {
        TriSetup s;
        s.meta = 0;
        s.box0 = s.box1 = 1;
        s.hbox0 = s.hbox1 = 1;
        return s;
    }
    return dr_setup(pc, v0, v1, v2, H, W, ox, oy, cull, margin);
}

__device__ __forceinline__ int dr_corner(int meta, int i) { return (meta >> (4 + 2 * i)) & 3; }

// Clip-space position M p of object-space point (x, y, z) for a row-major 4x4
// matrix M: the one expression every transform uses, so that recomputed
// positions are bitwise those of the transform.
__device__ __forceinline__ float4 clip_of(const float *M, float x, float y, float z) {
    float4 o;
    o.x = M[0] * x + M[1] * y + M[2] * z + M[3];
    o.y = M[4] * x + M[5] * y + M[6] * z + M[7];
    o.z = M[8] * x + M[9] * y + M[10] * z + M[11];
    o.w = M[12] * x + M[13] * y + M[14] * z + M[15];
    return o;
}

// Integer products in double.  Snapped coordinates satisfy |X|, |Y| < 2^22
// before a view's offset (below 2^23 with it) and pixel centres are below
// 2^23, so every difference is below 2^25, every product or sum of two
// products below 2^51: all exact in a double's 53-bit significand.  The results (and their conversions to float) are therefore the
// same as with 64-bit integers, at FP64 FMA rate instead of emulated 64-bit
// integer multiplies.
//
// Edge function of the edge opposite vertex i at fixed-point (px, py).
__device__ __forceinline__ double dr_edge(const int *X, const int *Y, int i, int px, int py) {
    int a = (i == 2) ? 0 : i + 1;
    int b = (i == 0) ? 2 : i - 1;
    double ex = (double)(X[b] - X[a]), ey = (double)(Y[b] - Y[a]);
    double qx = (double)(px - X[a]), qy = (double)(py - Y[a]);
    return ex * qy - ey * qx;
}

// Segment distance (fixed-point units, float) of edge i, from exact integers.
template <typename TE>
__device__ __forceinline__ float dr_segdist(const int *X, const int *Y, int i, int px, int py,
                                            TE E) {
    int a = (i == 2) ? 0 : i + 1;
    int b = (i == 0) ? 2 : i - 1;
    double ex = (double)(X[b] - X[a]), ey = (double)(Y[b] - Y[a]);
    double qx = (double)(px - X[a]), qy = (double)(py - Y[a]);
    double dot = qx * ex + qy * ey;
    double len2 = ex * ex + ey * ey;
    if (dot <= 0.0) return sqrtf((float)(qx * qx + qy * qy));
    if (dot >= len2) {
        double rx = (double)(px - X[b]), ry = (double)(py - Y[b]);
        return sqrtf((float)(rx * rx + ry * ry));
    }
    return (float)(E < 0 ? -E : E) / sqrtf((float)len2);
}

// Normalised distance (pixels / W) to the triangle and the nearest edge
// (lowest index on ties).
template <typename TE>
__device__ __forceinline__ float dr_distnorm(const int *X, const int *Y, int px, int py,
                                             const TE *E, float scale, int &nearest) {
    float best = dr_segdist(X, Y, 0, px, py, E[0]);
    nearest = 0;
    float d1 = dr_segdist(X, Y, 1, px, py, E[1]);
    if (d1 < best) { best = d1; nearest = 1; }
    float d2 = dr_segdist(X, Y, 2, px, py, E[2]);
    if (d2 < best) { best = d2; nearest = 2; }
    return best / scale;
}

template <typename TE>
__device__ __forceinline__ float dr_depth(const TriSetup &s, const TE *E) {
    float l1 = (float)E[1] / s.Af;
    float l2 = (float)E[2] / s.Af;
    float d1 = s.zn[1] - s.zn[0];
    float d2 = s.zn[2] - s.zn[0];
    float t1 = l1 * d1;
    float t2 = l2 * d2;
    float z = s.zn[0] + t1;
    return z + t2;
}

// The binless hard rasterizer's merge of one set-up triangle t (K = 1): each
// covered pixel centre of its box with depth in (0, 1) takes the 64-bit
// maximum of ~(depth bits << 32 | t) in zb (one view, H x W), so that the
// nearest fragment, then the lowest id, wins.
__device__ __forceinline__ void dr_direct_merge(const TriSetup &s, int t, int W, unsigned long long *zb) {
    const int x0 = s.box0 & 0xffff, x1 = s.box0 >> 16, y0 = s.box1 & 0xffff, y1 = s.box1 >> 16;
    for (int y = y0; y <= y1; y++) {
        const int py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
        for (int x = x0; x <= x1; x++) {
            const int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2;
            double E[3];
            bool in = true;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                E[i] = dr_edge(s.X, s.Y, i, px, py);
                bool own = (s.meta >> (1 + i)) & 1;
                in = in && (E[i] > 0 || (E[i] == 0 && own));
            }
            if (!in) continue;
            const float z = dr_depth(s, E);
            if (!(z > 0.0f && z < 1.0f)) continue;
            const unsigned long long v = ((unsigned long long)__float_as_uint(0.5f * z) << 32) | (unsigned)t;
            atomicMax(&zb[(int64_t)y * W + x], ~v);
        }
    }
}
