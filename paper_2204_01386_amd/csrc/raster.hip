// Rasterization forward and backward for gfx950.
//
// Forward (Algorithm 2 and the Shift equation of §3.4.2, depth peeling with K
// buffers): one kernel sets up every triangle (snap to 8 sub-pixel bits,
// orientation, top-left ownership, box) and appends it to the fixed-capacity
// bins of the 16x16 tiles its box covers; one workgroup per tile then
// rasterizes.  Hard rasterization (r = 0) is triangle-parallel: each lane
// walks one binned triangle's pixels in the tile and merges its fragments
// into per-pixel LDS slots with 64-bit atomicMin, K passes for K layers.  Soft
// rasterization (r > 0) is pixel-parallel: each lane keeps its pixel's K best
// fragments in registers while the tile's triangles stream through LDS.  Both
// select, independently of the visiting order, the K smallest distinct keys
// with the smallest triangle id at each key.
//
// Backward: the fragments of every tile are sorted by triangle id (wavefront
// sorts merged by rank in LDS) into per-tile records; per-record sums of the
// screen-space vertex gradients are formed in LDS; per vertex, each of its
// corners sums its records over the tiles in a fixed order and the corners
// are combined in a fixed order.  No float atomics: results are bitwise
// reproducible.
#include "interp_tile.h"

#include <algorithm>
#include <type_traits>
#include <cfloat>

// ---------------------------------------------------------------------------
// setup, counting and bin fill
//
// Neighbouring triangle ids are mostly neighbours on screen, so the lanes of
// a wavefront tend to hit the same few tiles.  Counting and filling are
// aggregated per wavefront: one atomic per distinct tile and wave, the lanes
// that share the tile take consecutive slots (ballot + popcount).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// next tile of a lane's tile rectangle in row-major order, -1 when done
__device__ __forceinline__ int next_tile(int cur, int tx0, int tx1, int ty1, int ntx) {
    int ty = cur / ntx, tx = cur - ty * ntx;
    if (tx < tx1) return cur + 1;
    if (ty < ty1) return (ty + 1) * ntx + tx0;
    return -1;
}

// One pass: every triangle is set up and appended to the bins of the tiles
// its box covers.  Each bin has a fixed capacity; its counter (kept at zero
// between calls, reset by the rasterizer after reading it) gives the slot.
__global__ void k_setup_bin(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris,
                            Viewports vp, int B, int V, int T, int H, int W, int cull, int margin, int ntx,
                            int nt, int cap, TriSetup *__restrict__ setup, int32_t *__restrict__ counts,
                            int32_t *__restrict__ bins, unsigned long long *__restrict__ status) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cur = -1, tx0 = 0, tx1 = 0, ty1 = 0, b = 0, t = 0;
    if (gid < (int64_t)B * T) {
        b = (int)(gid / T);
        t = (int)(gid - (int64_t)b * T);
        const int32_t *tv = tris + 3 * (int64_t)t;
        int v0 = tv[0], v1 = tv[1], v2 = tv[2];
        TriSetup s;
        if (v0 < 0 || v0 >= V || v1 < 0 || v1 >= V || v2 < 0 || v2 >= V) {
            s.meta = 0;
            s.box0 = s.box1 = 1;
            s.hbox0 = s.hbox1 = 1;
        } else {
            const int4 q = dr_viewport(vp, t, H, W);
            s = dr_setup(pos_clip + (int64_t)b * V, v0, v1, v2, q.w, q.z, q.x, q.y, cull, margin);
        }
        setup[gid] = s;
        if (s.meta & 1) {
            tx0 = (s.box0 & 0xffff) / DRESSI_TILE;
            tx1 = (s.box0 >> 16) / DRESSI_TILE;
            int ty0 = (s.box1 & 0xffff) / DRESSI_TILE;
            ty1 = (s.box1 >> 16) / DRESSI_TILE;
            cur = ty0 * ntx + tx0;
        }
    }
    // Rounds: in each round every lane with tiles left takes its next tile.
    // Lanes are grouped by tile with ballots (ALU only), then every group's
    // first lane issues one atomicAdd for the whole group - all groups in the
    // same instruction - and the lanes take consecutive slots.
    const unsigned long long below = (1ull << lane_id()) - 1ull;
    int worst = 0;
    unsigned long long active = __ballot(cur >= 0);
    while (active) {
        int leader = -1, rank = 0, gsize = 0;
        unsigned long long todo = active;
        while (todo) {
            int src = __ffsll((long long)todo) - 1;
            int key_tile = __shfl(cur, src, 64);
            int key_b = __shfl(b, src, 64);
            unsigned long long same = __ballot(cur >= 0 && cur == key_tile && b == key_b);
            if ((same >> lane_id()) & 1ull) {
                leader = src;
                rank = __popcll(same & below);
                gsize = __popcll(same);
            }
            todo &= ~same;
        }
        int base = 0;
        if (cur >= 0 && leader == lane_id())
            base = atomicAdd(&counts[(int64_t)b * nt + cur], gsize);
        base = __shfl(base, leader < 0 ? 0 : leader, 64);
        if (cur >= 0) {
            int64_t bt = (int64_t)b * nt + cur;
            int slot = base + rank;
            if (slot < cap) bins[bt * cap + slot] = t;
            else worst = max(worst, slot + 1);
            cur = next_tile(cur, tx0, tx1, ty1, ntx);
        }
        active = __ballot(cur >= 0);
    }
    if (worst > 0) {
        atomicMax(&status[0], 1ull);
        atomicMax(&status[1], (unsigned long long)worst);
    }
}

// ---------------------------------------------------------------------------
// fine rasterizer: one 16x16 tile per workgroup; each lane takes one binned
// triangle and walks the pixels of its box inside the tile, merging fragment
// keys into a per-pixel LDS slot with a 64-bit atomicMin of
// (key bits << 32 | triangle id).  Keys are positive floats, whose bit
// patterns order like the values, so the slot ends as the smallest key and the
// smallest id at that key, independently of the visiting order.  Layer k > 0
// repeats the pass keeping only keys strictly above the pixel's layer k-1 key
// (depth peeling, PeelDepth's "discard if key <= previous").
// ---------------------------------------------------------------------------
#define RS_EMPTY 0xffffffffffffffffull

template <bool SOFT>
__device__ __forceinline__ void raster_tri_in_tile(const TriSetup &s, int t, int tx, int ty,
                                                   float r, float dscale,
                                                   unsigned long long *slot, const float *prev) {
    int x0 = max(s.box0 & 0xffff, tx * DRESSI_TILE), x1 = min(s.box0 >> 16, tx * DRESSI_TILE + DRESSI_TILE - 1);
    int y0 = max(s.box1 & 0xffff, ty * DRESSI_TILE), y1 = min(s.box1 >> 16, ty * DRESSI_TILE + DRESSI_TILE - 1);
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
            float key;
            if (in) {
                float z = dr_depth(s, E);
                if (!(z > 0.0f && z < 1.0f)) continue;
                key = 0.5f * z;
            } else {
                if (!SOFT) continue;
                int ne;
                float dn = dr_distnorm(s.X, s.Y, px, py, E, dscale, ne);
                if (!(dn <= r)) continue;
                float h = 0.5f * dn;
                key = h + 0.5f;
            }
            int p = (y - ty * DRESSI_TILE) * DRESSI_TILE + (x - tx * DRESSI_TILE);
            if (!(key > prev[p])) continue;
            unsigned long long v = ((unsigned long long)__float_as_uint(key) << 32) | (unsigned)t;
            atomicMin(&slot[p], v);
        }
    }
}

// One fragment of triangle t (set up as s) at pixel centre (px, py):
// triangle id, perspective-correct (b0, b1) and, for soft rasterization, the
// signed normalised distance (+ for a hard fragment, - for a soft one).
template <bool SOFT>
__device__ __forceinline__ void resolve_frag(const TriSetup &s, int t, int px, int py, float key, float dscale,
                                             int64_t o, int32_t *__restrict__ tri_id, float2 *__restrict__ bary,
                                             float *__restrict__ dist) {
    double E[3];
#pragma unroll
    for (int i = 0; i < 3; i++) E[i] = dr_edge(s.X, s.Y, i, px, py);
    // perspective-correct b_i = (l_i / w_i) / sum_j (l_j / w_j) with
    // l_i = E_i / 2A: the area cancels, and multiplying through by
    // w0 w1 w2 leaves one division.  In double: soft fragments
    // extrapolate and the sum can come close to zero for grazing triangles.
    const double w0 = s.w[0], w1 = s.w[1], w2 = s.w[2];
    const double q0 = E[0] * (w1 * w2), q1 = E[1] * (w0 * w2), q2 = E[2] * (w0 * w1);
    const double iQ = 1.0 / (q0 + q1 + q2);
    double b0 = q0 * iQ, b1 = q1 * iQ, b2 = q2 * iQ;
    bool swapped = dr_corner(s.meta, 1) == 2;
    tri_id[o] = t;
    bary[o] = make_float2((float)b0, (float)(swapped ? b2 : b1));
    if (SOFT) {
        int ne;
        float dn = dr_distnorm(s.X, s.Y, px, py, E, dscale, ne);
        dist[o] = key < 0.5f ? dn : -dn;
    }
}

// Writes the K layers of one pixel (resolve_frag for each found layer).
template <int K, bool SOFT>
__device__ __forceinline__ void resolve_store(const TriSetup *__restrict__ sv, const float *key,
                                              const int *id, int b, int x, int y, int px, int py,
                                              int H, int W, float dscale, int32_t *__restrict__ tri_id,
                                              float2 *__restrict__ bary, float *__restrict__ dist) {
    if (x >= W || y >= H) return;
#pragma unroll
    for (int k = 0; k < K; k++) {
        int64_t o = (((int64_t)b * K + k) * H + y) * W + x;
        int t = id[k];
        if (t < 0) {
            tri_id[o] = -1;
            bary[o] = make_float2(0.0f, 0.0f);
            if (SOFT) dist[o] = 0.0f;
            continue;
        }
        resolve_frag<SOFT>(sv[t], t, px, py, key[k], dscale, o, tri_id, bary, dist);
    }
}

template <int K, bool SOFT>
__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    k_raster(const TriSetup *__restrict__ setup, int32_t *__restrict__ counts,
             const int32_t *__restrict__ bins, int cap, int T, int H, int W, int ntx, int nt,
             float r, int32_t *__restrict__ tri_id, float2 *__restrict__ bary,
             float *__restrict__ dist) {
    __shared__ unsigned long long slot[DRESSI_TILE_PIX];
    __shared__ float prev[DRESSI_TILE_PIX];
    const int bt = (int)xcd_block();
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + (p / DRESSI_TILE);
    const int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2;
    const int py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
    const float dscale = (float)W * 256.0f;
    const TriSetup *sv = setup + (int64_t)b * T;
    const int32_t *bin = bins + (int64_t)bt * cap;
    // the bin's first entries are read beside its count, not after it (in
    // bounds whatever the count: the bin has `cap` slots; entries past the
    // count are never used), one dependent load fewer
    const int t_first = p < cap ? bin[p] : -1;
    int nbin = counts[bt];
    if (nbin > cap) nbin = cap;

    float key[K];
    int id[K];
    prev[p] = 0.0f;
#pragma unroll
    for (int k = 0; k < K; k++) {
        slot[p] = RS_EMPTY;
        __syncthreads();
        for (int c0 = 0; c0 < nbin; c0 += DRESSI_TILE_PIX) {
            if (c0 + p < nbin) {
                int t = c0 == 0 ? t_first : bin[c0 + p];
                TriSetup s = sv[t];
                raster_tri_in_tile<SOFT>(s, t, tx, ty, r, dscale, slot, prev);
            }
        }
        __syncthreads();
        unsigned long long v = slot[p];
        if (v == RS_EMPTY) {
            key[k] = 2.0f;
            id[k] = -1;
        } else {
            key[k] = __uint_as_float((unsigned)(v >> 32));
            id[k] = (int)(v & 0xffffffffu);
        }
        prev[p] = key[k];   // an empty layer (2.0) blocks every later key
        __syncthreads();
    }
    if (p == 0) counts[bt] = 0;   // every lane has read it before the first barrier
    resolve_store<K, SOFT>(sv, key, id, b, x, y, px, py, H, W, dscale, tri_id, bary, dist);
}

// ---------------------------------------------------------------------------
// soft rasterizer (r > 0): one 16x16 tile per workgroup, one lane per pixel,
// each wavefront a 16x4 strip.  Each lane keeps its pixel's list of the K
// smallest distinct keys (smallest id at each key), sorted in registers: one
// pass over the tile's triangles selects exactly what K passes of depth
// peeling select, with no atomics.  A soft reach of several pixels gives every
// binned triangle many candidate pixels in the tile, which suits
// pixel-parallel evaluation.
//
// The tile's bin is staged through LDS, 256 triangles at a time, with the
// per-tile data the tests need.  A wavefront then tests 64 staged triangles at
// once (one per lane) and evaluates only the survivors, one at a time across
// its 64 pixels.  The bin is walked three times, nearest triangles first, so
// that the lists fill with near fragments early and cull more of the rest:
// (0) triangles whose vertex box covers pixel centres of the strip, (1) those
// at most RL_NEAR pixels away, (2) the others.  Every culling test is exact by
// construction (bounds carry rounding margins):
//  * the soft box misses the strip;
//  * the smallest key the triangle can give the strip (half its lowest vertex
//    depth in walk 0, else the soft key of the L-infinity pixel gap between
//    its vertex box and the strip) is above every lane's current K-th key;
//  * per lane, a soft candidate is dropped before its segment distances when
//    the line distance of an edge it lies outside of already rules it out.
// Edge functions (and the segment-distance products) are evaluated with
// 24-bit integer multiplies when staging has shown that every pixel-to-vertex
// difference over the tile and every edge vector is below 2^15 in magnitude
// (then every product and sum of two products fits in 32 bits, exactly);
// otherwise in the exact double form.  Workgroups take the tiles in an
// XCD-aware order (each XCD one contiguous range), so the setup records of
// neighbouring tiles are read through one L2.
// ---------------------------------------------------------------------------
#define RL_BATCH 256
#define RL_NEAR 2

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int lo16(int v) { return (int)(short)(v & 0xffff); }
__device__ __forceinline__ int hi16(int v) { return v >> 16; }

// Smallest segment distance (fixed-point units) from the pixel centre to the
// triangle: the same value as the minimum of the three segment distances in
// their usual form, computed without branches.  Every integer product and sum
// is exact in double; el[i] is sqrtf of edge i's squared length.
template <typename TE>
__device__ __forceinline__ float rl_segmin(const TriSetup &s, const TE *E, const float *el, int px, int py) {
    double qx[3], qy[3], dv[3];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        qx[v] = (double)(px - s.X[v]);
        qy[v] = (double)(py - s.Y[v]);
        dv[v] = qx[v] * qx[v] + qy[v] * qy[v];
    }
    float d[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int a = (i + 1) % 3, b = (i + 2) % 3;
        const double ex = (double)(s.X[b] - s.X[a]), ey = (double)(s.Y[b] - s.Y[a]);
        const double dot = qx[a] * ex + qy[a] * ey;
        const double len2 = ex * ex + ey * ey;
        const bool va = dot <= 0.0, vb = dot >= len2;
        const float sv = sqrtf((float)(va ? dv[a] : dv[b]));        // nearest point: a vertex
        const float si = (float)(E[i] < 0 ? -E[i] : E[i]) / el[i];  // nearest point inside the edge
        d[i] = (va || vb) ? sv : si;
    }
    float best = d[0];
    if (d[1] < best) best = d[1];
    if (d[2] < best) best = d[2];
    return best;
}

// The same value when every coordinate difference over the tile is below
// 2^15 in magnitude: products and sums of two products then stay below 2^31
// and 24-bit integer multiplies give them exactly.  q[v] = (px - X_v, py - Y_v).
__device__ __forceinline__ float rl_segmin_i(const int *qx, const int *qy, const int *ex, const int *ey,
                                             const int *len2, const int *E, const float *el) {
    int dv[3];
#pragma unroll
    for (int v = 0; v < 3; v++) dv[v] = __mul24(qx[v], qx[v]) + __mul24(qy[v], qy[v]);
    float d[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int a = (i + 1) % 3, b = (i + 2) % 3;
        const int dot = __mul24(qx[a], ex[i]) + __mul24(qy[a], ey[i]);
        const bool va = dot <= 0, vb = dot >= len2[i];
        const float sv = sqrtf((float)(va ? dv[a] : dv[b]));
        const float si = (float)(E[i] < 0 ? -E[i] : E[i]) / el[i];
        d[i] = (va || vb) ? sv : si;
    }
    float best = d[0];
    if (d[1] < best) best = d[1];
    if (d[2] < best) best = d[2];
    return best;
}

// Merges the candidate fragment of triangle t at this lane's pixel.  MAYHARD
// is false when no pixel centre of the wavefront can be inside the triangle.
// Edge vectors of the 32-bit path: edge i (opposite vertex i) runs from
// vertex i+1 to vertex i+2 (mod 3); every component is below 2^15 there.
__device__ __forceinline__ void rl_edges(const TriSetup &s, int *ex, int *ey) {
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int a = (i + 1) % 3, c = (i + 2) % 3;
        ex[i] = s.X[c] - s.X[a];
        ey[i] = s.Y[c] - s.Y[a];
    }
}

// One staged triangle (slot e of the batch) rasterized over its pixels in the
// tile, hard fragments only, merged into the tile's per-pixel slots: the same
// edge values (32-bit or exact double), depth and key as rl_merge.
__device__ __forceinline__ void rl_tri_in_tile(int e, const int2 *sfi, const int2 *sbox,
                                               const int4 *sxy0, const int2 *sxy1, const float4 *sz, int tx,
                                               int ty, unsigned long long *slot) {
    const int fl = sfi[e].x;
    if (!(fl & 1)) return;
    const int2 bx = sbox[e];
    const int x0 = max(bx.x & 0xffff, tx * DRESSI_TILE), x1 = min(bx.x >> 16, tx * DRESSI_TILE + DRESSI_TILE - 1);
    const int y0 = max(bx.y & 0xffff, ty * DRESSI_TILE), y1 = min(bx.y >> 16, ty * DRESSI_TILE + DRESSI_TILE - 1);
    if (x0 > x1 || y0 > y1) return;
    const int t = sfi[e].y;
    const int4 q0 = sxy0[e];
    const int2 q1 = sxy1[e];
    const float4 z4 = sz[e];
    TriSetup s;
    s.X[0] = q0.x; s.X[1] = q0.y; s.X[2] = q0.z;
    s.Y[0] = q0.w; s.Y[1] = q1.x; s.Y[2] = q1.y;
    s.zn[0] = z4.x; s.zn[1] = z4.y; s.zn[2] = z4.z;
    s.Af = z4.w;
    s.meta = fl & 0xffff;
    const bool own0 = (s.meta >> 1) & 1, own1 = (s.meta >> 2) & 1, own2 = (s.meta >> 3) & 1;
    const bool small = fl >> 16;
    int ex[3], ey[3];
    rl_edges(s, ex, ey);
    for (int y = y0; y <= y1; y++) {
        const int py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
        for (int x = x0; x <= x1; x++) {
            const int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2;
            float z;
            if (small) {
                int E[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    const int a = (i + 1) % 3;
                    E[i] = __mul24(ex[i], py - s.Y[a]) - __mul24(ey[i], px - s.X[a]);
                }
                if (!((E[0] > 0 || (E[0] == 0 && own0)) && (E[1] > 0 || (E[1] == 0 && own1)) &&
                      (E[2] > 0 || (E[2] == 0 && own2))))
                    continue;
                z = dr_depth(s, E);
            } else {
                double E[3];
#pragma unroll
                for (int i = 0; i < 3; i++) E[i] = dr_edge(s.X, s.Y, i, px, py);
                if (!((E[0] > 0 || (E[0] == 0 && own0)) && (E[1] > 0 || (E[1] == 0 && own1)) &&
                      (E[2] > 0 || (E[2] == 0 && own2))))
                    continue;
                z = dr_depth(s, E);
            }
            if (!(z > 0.0f && z < 1.0f)) continue;
            const float key = 0.5f * z;
            const int pp = (y - ty * DRESSI_TILE) * DRESSI_TILE + (x - tx * DRESSI_TILE);
            const unsigned long long v = ((unsigned long long)__float_as_uint(key) << 32) | (unsigned)t;
            atomicMin(&slot[pp], v);
        }
    }
}

template <int K, bool MAYHARD, typename TE, bool SOFT = true>
__device__ __forceinline__ void rl_merge(const TriSetup &s, const TE *E, const float *el, int t, int px,
                                         int py, float dscale, float r, float reach, float *key, int *id,
                                         const int *qx = nullptr, const int *qy = nullptr,
                                         const int *ex = nullptr, const int *ey = nullptr,
                                         const int *len2 = nullptr) {
    bool in = MAYHARD;
    if (MAYHARD) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            bool own = (s.meta >> (1 + i)) & 1;
            in = in && (E[i] > 0 || (E[i] == 0 && own));
        }
    }
    float kf;
    if (in) {
        float z = dr_depth(s, E);
        if (!(z > 0.0f && z < 1.0f)) return;
        kf = 0.5f * z;
    } else {
        if (!SOFT) return;
        // The distance to the triangle is at least the distance -E_i / |e_i|
        // to the line of any edge the pixel lies outside of.  A soft fragment
        // enters the list only if its key 0.5 + dn/2 is at most the list's
        // last key, so it needs dn <= 2 (last - 0.5) (+ one rounding of the
        // key) and dn <= r.  The bound is compared with a relative margin far
        // above the float rounding of either side, so every fragment dropped
        // here would also fail the exact tests below.
        const float lim = fminf(reach, (2.0f * (key[K - 1] - 0.5f) + 2.4e-7f) * dscale * 1.001f);
        if ((E[0] < 0 && (float)(-E[0]) > lim * el[0]) || (E[1] < 0 && (float)(-E[1]) > lim * el[1]) ||
            (E[2] < 0 && (float)(-E[2]) > lim * el[2]))
            return;
        float best;
        if constexpr (std::is_integral<TE>::value)
            best = rl_segmin_i(qx, qy, ex, ey, len2, E, el);
        else
            best = rl_segmin(s, E, el, px, py);
        float dn = best / dscale;
        if (!(dn <= r)) return;
        float h = 0.5f * dn;
        kf = h + 0.5f;
    }
    if (!(kf <= key[K - 1])) return;
    bool same = false;
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (kf == key[k]) {
            id[k] = min(id[k], t);
            same = true;
        }
    }
    if (same) return;
    // insert below the first larger key; the largest entry drops out
#pragma unroll
    for (int k = K - 1; k > 0; k--) {
        if (kf < key[k - 1]) {
            key[k] = key[k - 1];
            id[k] = id[k - 1];
        } else if (kf < key[k]) {
            key[k] = kf;
            id[k] = t;
        }
    }
    if (kf < key[0]) {
        key[0] = kf;
        id[0] = t;
    }
}

// HYB (hard, K = 1): every staged batch is rasterized either pixel-parallel
// (the list walk below) or triangle-parallel (one lane per staged triangle,
// walking its pixels in the tile and merging into a per-pixel LDS slot with a
// 64-bit atomicMin, as k_raster does), whichever the batch's estimated cost
// favours: the pixel-parallel walk costs about one iteration per (triangle,
// wavefront strip it touches), the triangle-parallel one, per wavefront, the
// largest pixel count of its lanes' triangles.  The slot and the register list
// are merged at the end; both keep the smallest key and the smallest id at
// that key, so the choice never changes the result.
// hyb_w: the cost of a pixel-parallel triangle step relative to a
// triangle-parallel pixel step, in sixteenths (a tuning knob).

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Edge-band soft rasterization (BAND != 0).  Outside the blend's edge mask E
// the image is S^H C_1 and the silhouette S^H (§3.4.3), so only the front
// hard fragment of a pixel reaches the image or a gradient there.  The
// banded contract keeps, outside E, layer 0 if it is hard and nothing else,
// and the full K layers inside E.  BAND = 1 is its first pass: every tile,
// covering triangles only, hard fragments only, writing layer 0 (the front
// hard fragment, with its distance) and empty layers 1..K-1; E is then built
// from that layer 0 (its S^H equals the full form's); BAND = 2 is the second
// pass: tiles with a pixel in E rasterize fully (the full form's walks) and
// write the K layers of their E pixels; other tiles exit at once.
template <int K, bool SOFT, bool HYB = false, int BAND = 0>
__global__ void __launch_bounds__(DRESSI_TILE_PIX) __attribute__((amdgpu_waves_per_eu(SOFT ? 7 : 5)))
    k_raster_list(const TriSetup *__restrict__ setup, int32_t *__restrict__ counts,
                  const int32_t *__restrict__ bins, int cap, int T, int H, int W, int ntx, int nt,
                  float r, int32_t *__restrict__ tri_id, float2 *__restrict__ bary,
                  float *__restrict__ dist, int hyb_w, const uint8_t *__restrict__ band, int keep_counts) {
    static_assert(BAND == 0 || SOFT, "banding is for soft rasterization");
    constexpr bool SM = SOFT && BAND != 1;   // soft fragments merged
    constexpr int KL = BAND == 1 ? 1 : K;    // layers kept in registers
    // staged triangles (structure of arrays)
    __shared__ int2 sfi[RL_BATCH];      // meta | 32-bit-exact flag << 16, triangle id
    __shared__ int2 sbox[RL_BATCH];     // soft box
    __shared__ int2 shb[RL_BATCH];      // pixels with centres in the vertex box
    __shared__ int szlb[RL_BATCH];      // lower bound of the hard keys (float bits)
    __shared__ float4 sel[RL_BATCH];    // sqrtf of the squared edge lengths
    __shared__ int4 sxy0[RL_BATCH];     // X0 X1 X2 Y0
    __shared__ int2 sxy1[RL_BATCH];     // Y1 Y2
    __shared__ float4 sz[RL_BATCH];     // zn0 zn1 zn2 Af
    // triangle-parallel batches (HYB): per-pixel slot and the batch costs,
    // double-buffered by batch parity
    __shared__ unsigned long long sslot[HYB ? DRESSI_TILE_PIX : 1];
    __shared__ int scost[2][2];
    static_assert(!HYB || (K == 1 && !SOFT), "the hybrid strategy is for one hard layer");
    const int bt = (int)xcd_block();
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    const int lane = p & 63;
    const int lx = p & (DRESSI_TILE - 1), ly = p / DRESSI_TILE;
    const int x = tx * DRESSI_TILE + lx;
    const int y = ty * DRESSI_TILE + ly;
    const int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2;
    const int py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
    const float dscale = (float)W * 256.0f;
    const float reach = r * dscale * 1.001f;   // conservative, in fixed-point units
    const TriSetup *__restrict__ sv = setup + (int64_t)b * T;
    const int32_t *__restrict__ bin = bins + (int64_t)bt * cap;
    // this lane's wavefront: pixels [wx0, wx1] x [wy0, wy1]
    const int wx0 = tx * DRESSI_TILE, wx1 = wx0 + DRESSI_TILE - 1;
    const int wy0 = ty * DRESSI_TILE + (p / 64) * (64 / DRESSI_TILE);
    const int wy1 = wy0 + 64 / DRESSI_TILE - 1;
    const int px0 = DRESSI_SUBPIX * wx0 + DRESSI_SUBPIX / 2;                 // tile's first pixel centre
    const int py0 = DRESSI_SUBPIX * (ty * DRESSI_TILE) + DRESSI_SUBPIX / 2;
    // the first batch of the bin is read beside its count (as in k_raster)
    const int t_first = p < cap ? bin[p] : -1;
    int nbin = counts[bt];
    if (nbin > cap) nbin = cap;
    bool inE = true;   // this lane's pixel is in the edge mask (the second banded pass)
    if (BAND == 2) {
        inE = x < W && y < H && band[((int64_t)b * H + y) * W + x] != 0;
        if (!__syncthreads_or(inE)) {
            if (p == 0) counts[bt] = 0;
            return;
        }
    }
    const bool waveE = BAND != 2 || __ballot(inE) != 0ull;

    float key[KL];
    int id[KL];
#pragma unroll
    for (int k = 0; k < KL; k++) {
        key[k] = 2.0f;   // empty: above every fragment key
        id[k] = -1;
    }
    int wmax_bits = __float_as_int(2.0f);   // bound on the strip's K-th keys (they only decrease)
    int gap_max = 0x3fffffff;               // soft-only triangles farther (pixels) than this are culled
    if (HYB) {
        sslot[p] = RS_EMPTY;
        if (p < 4) scost[p >> 1][p & 1] = 0;
    }

    for (int walk = 0; walk < (SM ? 3 : 1); walk++) {   // hard only: covering triangles
        for (int c0 = 0; c0 < nbin; c0 += RL_BATCH) {
            const int n = min(RL_BATCH, nbin - c0);
            const int par = (c0 / RL_BATCH) & 1;
            bool use_tp = false;
            if (walk == 0 || nbin > RL_BATCH) {   // a single batch stays staged
                __syncthreads();
                // the other parity's costs were read before this barrier
                if (HYB && p < 2) scost[par ^ 1][p] = 0;
                int tp_pix = 0, pp_steps = 0;
                bool stage = p < n;
                if (BAND == 1 && stage) {
                    // the first banded pass takes covering triangles only: one
                    // whose vertex box misses this tile is marked far away
                    // (never wanted by the covering walk) without loading
                    // the rest of its record
                    const int2 hb = *reinterpret_cast<const int2 *>(&sv[c0 == 0 ? t_first : bin[c0 + p]].hbox0);
                    const int ty0 = ty * DRESSI_TILE, ty1 = ty0 + DRESSI_TILE - 1;
                    if (hi16(hb.x) < wx0 || lo16(hb.x) > wx1 || hi16(hb.y) < ty0 || lo16(hb.y) > ty1) {
                        shb[p] = make_int2((int)0x80008000u, (int)0x80008000u);
                        sbox[p] = make_int2(0, 0);
                        szlb[p] = 0;
                        stage = false;
                    }
                }
                if (stage) {
                    const int t = c0 == 0 ? t_first : bin[c0 + p];
                    const TriSetup s = sv[t];
                    // 32-bit integer path: every pixel-to-vertex difference over the
                    // tile and every edge vector below 2^15 in magnitude
                    const int lim15 = 1 << 15, span = DRESSI_SUBPIX * (DRESSI_TILE - 1);
                    bool small = true;
#pragma unroll
                    for (int i = 0; i < 3; i++) {
                        small = small && abs(px0 - s.X[i]) < lim15 && abs(px0 + span - s.X[i]) < lim15 &&
                                abs(py0 - s.Y[i]) < lim15 && abs(py0 + span - s.Y[i]) < lim15;
                        const int a = (i + 1) % 3, c = (i + 2) % 3;
                        const int ex = s.X[c] - s.X[a], ey = s.Y[c] - s.Y[a];
                        small = small && abs(ex) < lim15 && abs(ey) < lim15;
                    }
                    sel[p] = make_float4(s.elen[0], s.elen[1], s.elen[2], 0.0f);
                    sfi[p] = make_int2((s.meta & 0xffff) | (small ? 0x10000 : 0), t);
                    sbox[p] = make_int2(s.box0, s.box1);
                    shb[p] = make_int2(s.hbox0, s.hbox1);
                    szlb[p] = s.zlb;
                    sxy0[p] = make_int4(s.X[0], s.X[1], s.X[2], s.Y[0]);
                    sxy1[p] = make_int2(s.Y[1], s.Y[2]);
                    sz[p] = make_float4(s.zn[0], s.zn[1], s.zn[2], s.Af);
                    if (HYB && (s.meta & 1)) {
                        const int bx0 = max(s.box0 & 0xffff, wx0), bx1 = min(s.box0 >> 16, wx1);
                        const int by0 = max(s.box1 & 0xffff, ty * DRESSI_TILE);
                        const int by1 = min(s.box1 >> 16, ty * DRESSI_TILE + DRESSI_TILE - 1);
                        if (bx0 <= bx1 && by0 <= by1) {
                            tp_pix = (bx1 - bx0 + 1) * (by1 - by0 + 1);
                            const int strip = 64 / DRESSI_TILE;   // rows per wavefront
                            pp_steps = (by1 - ty * DRESSI_TILE) / strip - (by0 - ty * DRESSI_TILE) / strip + 1;
                        }
                    }
                }
                if (HYB) {
                    tp_pix = wave_max_i(tp_pix);
                    pp_steps = wave_sum_i(pp_steps);
                    if (lane == 0) {
                        atomicAdd(&scost[par][0], tp_pix);
                        atomicAdd(&scost[par][1], pp_steps);
                    }
                }
                __syncthreads();
            }
            if (HYB) use_tp = 16 * scost[par][0] < hyb_w * scost[par][1];
            if (HYB && use_tp) {
                if (p < n) rl_tri_in_tile(p, sfi, sbox, sxy0, sxy1, sz, tx, ty, sslot);
                continue;
            }
            for (int c = 0; c < n; c += 64) {
                // 64 triangles tested at once, one per lane
                const int e = c + lane;
                bool want = false;
                if (e < n) {
                    const int2 bx = sbox[e];
                    const bool hit = !(hi16(bx.x) < wx0 || (bx.x & 0xffff) > wx1 || hi16(bx.y) < wy0 ||
                                       (bx.y & 0xffff) > wy1);
                    const int2 hb = shb[e];
                    const int gx = max(max(lo16(hb.x) - wx1, wx0 - hi16(hb.x)), 0);
                    const int gy = max(max(lo16(hb.y) - wy1, wy0 - hi16(hb.y)), 0);
                    const int g = max(gx, gy);
                    if (walk == 0) want = hit && g == 0 && szlb[e] <= wmax_bits;
                    else if (walk == 1) want = waveE && hit && g > 0 && g <= RL_NEAR && g <= gap_max;
                    else want = waveE && hit && g > RL_NEAR && g <= gap_max;
                }
                unsigned long long todo = __ballot(want);
                while (todo) {
                    const int j = c + __ffsll((long long)todo) - 1;
                    todo &= todo - 1ull;
                    const int2 fi = sfi[j];
                    const int fl = fi.x, t = fi.y;
                    const float4 e4 = sel[j];
                    const int4 q0 = sxy0[j];
                    const int2 q1 = sxy1[j];
                    const float4 z4 = sz[j];
                    TriSetup s;
                    s.X[0] = q0.x; s.X[1] = q0.y; s.X[2] = q0.z;
                    s.Y[0] = q0.w; s.Y[1] = q1.x; s.Y[2] = q1.y;
                    s.zn[0] = z4.x; s.zn[1] = z4.y; s.zn[2] = z4.z;
                    s.Af = z4.w;
                    s.meta = fl & 0xffff;
                    const float el[3] = {e4.x, e4.y, e4.z};
                    if (BAND == 2 && !inE) continue;
                    if (fl >> 16) {
                        // exact in 32-bit integers (see the staging test)
                        int ex[3], ey[3], len2[3];
                        rl_edges(s, ex, ey);
#pragma unroll
                        for (int i = 0; i < 3; i++) len2[i] = __mul24(ex[i], ex[i]) + __mul24(ey[i], ey[i]);
                        int qx[3], qy[3], E[3];
#pragma unroll
                        for (int v = 0; v < 3; v++) {
                            qx[v] = px - s.X[v];
                            qy[v] = py - s.Y[v];
                        }
#pragma unroll
                        for (int i = 0; i < 3; i++) {
                            const int a = (i + 1) % 3;
                            E[i] = __mul24(ex[i], qy[a]) - __mul24(ey[i], qx[a]);
                        }
                        if (walk == 0)
                            rl_merge<KL, true, int, SM>(s, E, el, t, px, py, dscale, r, reach, key, id, qx, qy, ex,
                                                        ey, len2);
                        else
                            rl_merge<KL, false, int, SM>(s, E, el, t, px, py, dscale, r, reach, key, id, qx, qy, ex,
                                                         ey, len2);
                    } else {
                        double E[3];
#pragma unroll
                        for (int i = 0; i < 3; i++) E[i] = dr_edge(s.X, s.Y, i, px, py);
                        if (walk == 0) rl_merge<KL, true, double, SM>(s, E, el, t, px, py, dscale, r, reach, key, id);
                        else rl_merge<KL, false, double, SM>(s, E, el, t, px, py, dscale, r, reach, key, id);
                    }
                }
                // keys only decrease: refresh the strip's bounds
                const float wm = wave_max(BAND == 2 && !inE ? 0.0f : key[KL - 1]);
                wmax_bits = __float_as_int(wm);
                // a soft candidate needs dn <= 2 (wmax - 0.5) + one key rounding;
                // a pixel gap g (L-infinity, whole pixels) gives dn > (g - 1) / W
                const float dp = (2.0f * (wm - 0.5f) + 1e-7f) * (float)W * 1.001f;
                gap_max = (int)floorf(fminf(dp, 1.0e9f)) + 1;
            }
        }
    }
    __syncthreads();
    if (HYB) {
        const unsigned long long v = sslot[p];
        if (v != RS_EMPTY) {
            const float k2 = __uint_as_float((unsigned)(v >> 32));
            const int t2 = (int)(v & 0xffffffffu);
            if (k2 < key[0] || (k2 == key[0] && t2 < id[0])) {
                key[0] = k2;
                id[0] = t2;
            }
        }
    }
    if (p == 0 && !keep_counts) counts[bt] = 0;   // every lane has read it before the first barrier
    if (BAND == 2 && !inE) return;
    if constexpr (KL == K) {
        resolve_store<K, SOFT>(sv, key, id, b, x, y, px, py, H, W, dscale, tri_id, bary, dist);
    } else {
        float kk[K];
        int ii[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            kk[k] = k < KL ? key[k] : 2.0f;
            ii[k] = k < KL ? id[k] : -1;
        }
        resolve_store<K, SOFT>(sv, kk, ii, b, x, y, px, py, H, W, dscale, tri_id, bary, dist);
    }
}

// Hard single-layer rasterization without bins (strategy 3, K = 1): one lane
// per (view, triangle) sets the triangle up as k_setup_bin does and merges
// its key (depth bits << 32 | id, as k_raster) into every covered pixel of its
// box with a 64-bit global atomicMax of the key's complement, on a per-pixel
// array kept at zero between calls (zero: no fragment); a second kernel
// resolves each pixel from the surviving key, recomputing the winner's setup,
// and sets the entry back to zero.  The smallest key and the smallest id at
// it, whatever the order of the atomics: the layer the other strategies
// select.  A lane's work is its triangle's box, so this suits small
// triangles; the autotuner times it against the others.
__device__ __forceinline__ bool direct_setup(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris,
                                             const Viewports &vp, int b, int V, int t, int H, int W, int cull,
                                             TriSetup &s) {
    const int32_t *tv = tris + 3 * (int64_t)t;
    const int v0 = tv[0], v1 = tv[1], v2 = tv[2];
    if (v0 < 0 || v0 >= V || v1 < 0 || v1 >= V || v2 < 0 || v2 >= V) return false;
    const int4 q = dr_viewport(vp, t, H, W);
    s = dr_setup(pos_clip + (int64_t)b * V, v0, v1, v2, q.w, q.z, q.x, q.y, cull, 0);
    return (s.meta & 1) != 0;
}

__global__ void k_raster_direct(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris, Viewports vp,
                                int B, int V, int T, int H, int W, int cull, unsigned long long *__restrict__ zbuf) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)B * T) return;
    const int b = (int)(gid / T), t = (int)(gid - (int64_t)b * T);
    TriSetup s;
    if (!direct_setup(pos_clip, tris, vp, b, V, t, H, W, cull, s)) return;
    dr_direct_merge(s, t, W, zbuf + (int64_t)b * H * W);
}

__global__ void k_raster_direct_resolve(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris,
                                        Viewports vp, int B, int V, int T, int H, int W, int cull,
                                        unsigned long long *__restrict__ zbuf, int32_t *__restrict__ tri_id,
                                        float2 *__restrict__ bary) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npix = (int64_t)H * W;
    if (i >= (int64_t)B * npix) return;
    const unsigned long long c = zbuf[i];
    if (c == 0ull) {   // no fragment
        tri_id[i] = -1;
        bary[i] = make_float2(0.0f, 0.0f);
        return;
    }
    zbuf[i] = 0ull;
    const unsigned long long v = ~c;
    const int t = (int)(v & 0xffffffffu);
    const int b = (int)(i / npix);
    const int64_t pix = i - (int64_t)b * npix;
    const int y = (int)(pix / W), x = (int)(pix - (int64_t)y * W);
    TriSetup s;
    direct_setup(pos_clip, tris, vp, b, V, t, H, W, cull, s);   // valid: it produced the key
    resolve_frag<false>(s, t, DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2, DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2,
                        __uint_as_float((unsigned)(v >> 32)), 0.0f, i, tri_id, bary, nullptr);
}

// Hard rasterization has two strategies with identical results (the layer
// selection does not depend on visiting order): triangle-parallel per tile
// with LDS atomics (small triangles) or pixel-parallel with register lists
// (large triangles); dressi_tune picks one per context.
template <int K>
static void launch_raster_k(bool soft, int hard_pix, int hyb_w, dim3 g, hipStream_t st, const TriSetup *setup,
                            int32_t *counts, const int32_t *bins, int cap, int T, int H, int W, int ntx, int nt,
                            float r, int32_t *tid, float2 *bary, float *dist) {
    if (soft)
        DR_LAUNCH("k_raster_list", (k_raster_list<K, true>), g, DRESSI_TILE_PIX, 0, st, setup, counts, bins, cap,
                  T, H, W, ntx, nt, r, tid, bary, dist, 0, nullptr, 0);
    else if (hard_pix == 2 && K == 1)
        DR_LAUNCH("k_raster_list", (k_raster_list<1, false, true>), g, DRESSI_TILE_PIX, 0, st, setup, counts,
                  bins, cap, T, H, W, ntx, nt, r, tid, bary, dist, hyb_w, nullptr, 0);
    else if (hard_pix == 1 || hard_pix == 2)
        DR_LAUNCH("k_raster_list", (k_raster_list<K, false>), g, DRESSI_TILE_PIX, 0, st, setup, counts, bins,
                  cap, T, H, W, ntx, nt, r, tid, bary, dist, 0, nullptr, 0);
    else
        DR_LAUNCH("k_raster", (k_raster<K, false>), g, DRESSI_TILE_PIX, 0, st, setup, counts, bins, cap, T, H,
                  W, ntx, nt, r, tid, bary, dist);
}

static int soft_margin(float r, int W) {
    if (!(r > 0.0f)) return 0;
    return (int)ceilf(r * (float)W) + 1;
}

// triangles per tile bin: 8x the mean load of a covered tile, at least 2048
static int default_tile_capacity(int B, int T, int nt, int margin) {
    double side = 1.0 + (2.0 * margin + 2.0) / DRESSI_TILE;
    double mean = (double)T * side * side / (nt > 0 ? nt : 1);
    int cap = 2048;
    while (cap < 8.0 * mean && cap < (1 << 24)) cap <<= 1;
    return cap;
}

static int tile_capacity(const dressi_ctx *ctx, int B, int T, int nt, int margin) {
    int cap = default_tile_capacity(B, T, nt, margin);
    if (ctx && ctx->bin_capacity > cap) cap = (int)std::min<int64_t>(ctx->bin_capacity, 1 << 26);
    return cap;
}

static size_t raster_scratch(int B, int T, int nt, int cap, Carver &c, size_t *o) {
    o[0] = c.take(sizeof(TriSetup) * (size_t)B * T);            // setup
    o[1] = c.take(sizeof(int32_t) * (size_t)B * nt * cap);      // bins
    return c.off;
}

static int check_raster_args(dressi_ctx *ctx, const void *pos, const void *tris, int B, int V,
                             int T, int H, int W, int K, float r) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || V < 0 || T < 0 || H <= 0 || W <= 0 || H > 32767 || W > 32767)
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: bad dimensions");
    if (K < 1 || K > DRESSI_MAX_K) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: K must be 1..5");
    if (!(r >= 0.0f && r <= 1.0f)) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: r must be in [0,1]");
    if (T >= 0x7fffffff) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: T must be < 2^31-1");
    if ((B * (int64_t)T > 0) && (!pos || !tris))
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: null pos_clip or tris");
    return DRESSI_OK;
}

// band: -2 = the full form; otherwise the edge-band form of a blend whose
// edge mask is empty (-1) or the boundary of S^H dilated by band >= 0 pixels.
static int rasterize_impl(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, Viewports vp, int B,
                          int V, int T, int H, int W, int K, float r, int cull, int32_t *tri_id, float *bary,
                          float *dist, void *stream, int band = -2) {
    int rc = check_raster_args(ctx, pos_clip, tris, B, V, T, H, W, K, r);
    if (rc) return rc;
    if (!tri_id || !bary) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: null tri_id or bary");
    bool soft = r > 0.0f;
    if (soft && !dist) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: dist is required when r > 0");
    if (B == 0) return DRESSI_OK;
    hipStream_t st = (hipStream_t)stream;
    if (!soft && K == 1 && ctx->hard_raster == 3) {
        // binless (strategy 3): a per-pixel key array in the zeroed counters
        const int64_t npx = (int64_t)B * H * W;
        rc = dressi_counters(ctx, (size_t)(2 * npx), st);
        if (rc) return rc;
        unsigned long long *zbuf = reinterpret_cast<unsigned long long *>(ctx->counters);
        const float4 *pc4 = reinterpret_cast<const float4 *>(pos_clip);
        const int64_t ntri = (int64_t)B * T;
        if (ntri > 0)
            DR_LAUNCH("k_raster_direct", (k_raster_direct), (int)((ntri + 255) / 256), 256, 0, st, pc4, tris, vp, B,
                      V, T, H, W, cull, zbuf);
        DR_LAUNCH("k_raster_direct_resolve", (k_raster_direct_resolve), (int)((npx + 255) / 256), 256, 0, st, pc4,
                  tris, vp, B, V, T, H, W, cull, zbuf, tri_id, reinterpret_cast<float2 *>(bary));
        return dressi_launch_check(ctx, "rasterize");
    }
    int ntx = tiles_x(W), nty = tiles_y(H), nt = ntx * nty;
    int margin = soft_margin(r, W);
    int cap = tile_capacity(ctx, B, T, nt, margin);
    const bool banded = soft && band >= -1;
    Carver c;
    size_t o[2];
    raster_scratch(B, T, nt, cap, c, o);
    const size_t o_band = banded ? c.take(3 * (size_t)B * H * W) : 0;   // boundary, rows, edge mask
    rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    rc = dressi_counters(ctx, (size_t)B * nt, st);
    if (rc) return rc;
    void *S = ctx->scratch;
    TriSetup *setup = at<TriSetup>(S, o[0]);
    int32_t *bins = at<int32_t>(S, o[1]);
    int32_t *counts = ctx->counters;
    int64_t ntri = (int64_t)B * T;
    if (ntri > 0)
        DR_LAUNCH("k_setup_bin", (k_setup_bin), (int)((ntri + 255) / 256), 256, 0, st,
                  reinterpret_cast<const float4 *>(pos_clip), tris, vp, B, V, T, H, W, cull, margin, ntx,
                  nt, cap, setup, counts, bins, reinterpret_cast<unsigned long long *>(ctx->status));
    dim3 g((unsigned)(B * nt));
    float2 *b2 = reinterpret_cast<float2 *>(bary);
    if (banded) {
        // first pass: the front hard fragment of every pixel (the bins are
        // read again by the second pass, so their counts are kept)
        uint8_t *bnd = at<uint8_t>(S, o_band);
        uint8_t *rows = bnd + (size_t)B * H * W, *edge = rows + (size_t)B * H * W;
        const int keep = band >= 0 ? 1 : 0;
        switch (K) {
#define DR_BAND1(KK)                                                                                       \
    case KK:                                                                                               \
        DR_LAUNCH("k_raster_list_band1", (k_raster_list<KK, true, false, 1>), g, DRESSI_TILE_PIX, 0, st, setup, \
                  counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist, 0, nullptr, keep);            \
        break;
            DR_BAND1(1) DR_BAND1(2) DR_BAND1(3) DR_BAND1(4) DR_BAND1(5)
#undef DR_BAND1
        }
        if (band >= 0) {
            dressi_edge_mask(tri_id, dist, B, K, H, W, band, bnd, rows, edge, st);
            switch (K) {
#define DR_BAND2(KK)                                                                                       \
    case KK:                                                                                               \
        DR_LAUNCH("k_raster_list", (k_raster_list<KK, true, false, 2>), g, DRESSI_TILE_PIX, 0, st, setup,    \
                  counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist, 0, edge, 0);                  \
        break;
                DR_BAND2(1) DR_BAND2(2) DR_BAND2(3) DR_BAND2(4) DR_BAND2(5)
#undef DR_BAND2
            }
        }
        return dressi_launch_check(ctx, "rasterize_banded");
    }
    const int hp = ctx->hard_raster, hw = ctx->hybrid_weight;
    switch (K) {
    case 1: launch_raster_k<1>(soft, hp, hw, g, st, setup, counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    case 2: launch_raster_k<2>(soft, hp, hw, g, st, setup, counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    case 3: launch_raster_k<3>(soft, hp, hw, g, st, setup, counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    case 4: launch_raster_k<4>(soft, hp, hw, g, st, setup, counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    default: launch_raster_k<5>(soft, hp, hw, g, st, setup, counts, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    }
    return dressi_launch_check(ctx, "rasterize");
}

extern "C" int dressi_rasterize(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B,
                                int V, int T, int H, int W, int K, float r, int cull,
                                int32_t *tri_id, float *bary, float *dist, void *stream) {
    return rasterize_impl(ctx, pos_clip, tris, Viewports{nullptr, nullptr}, B, V, T, H, W, K, r, cull, tri_id,
                          bary, dist, stream);
}

extern "C" int dressi_rasterize_banded(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B,
                                       int V, int T, int H, int W, int K, float r, int cull, float delta,
                                       int blend_mode, int32_t *tri_id, float *bary, float *dist, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (!(r > 0.0f)) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize_banded: needs a soft reach r > 0");
    int band;
    switch (blend_mode) {
    case DRESSI_BLEND_HSR: band = std::max((int)ceilf(delta * (float)W) - 1, -1); break;
    case DRESSI_BLEND_AA: band = 0; break;
    case DRESSI_BLEND_SOFTRAS: band = -2; break;   // the edge mask is everything: the full form
    case DRESSI_BLEND_HARD: band = -1; break;
    default: return dressi_fail(ctx, DRESSI_EINVAL, "rasterize_banded: bad blend mode");
    }
    return rasterize_impl(ctx, pos_clip, tris, Viewports{nullptr, nullptr}, B, V, T, H, W, K, r, cull, tri_id,
                          bary, dist, stream, band);
}

static int check_views(dressi_ctx *ctx, const int32_t *tri_view, const void *views, int n, int T) {
    if (n < 1) return dressi_fail(ctx, DRESSI_EINVAL, "batched: need at least one view");
    if (T > 0 && (!tri_view || !views)) return dressi_fail(ctx, DRESSI_EINVAL, "batched: null tri_view or views");
    return DRESSI_OK;
}

extern "C" int dressi_rasterize_batched(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                                        const int32_t *tri_view, const int32_t *views, int n, int V, int T,
                                        int H, int W, int K, int cull, int32_t *tri_id, float *bary,
                                        void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    int rc = check_views(ctx, tri_view, views, n, T);
    if (rc) return rc;
    return rasterize_impl(ctx, pos_clip, tris, Viewports{tri_view, reinterpret_cast<const int4 *>(views)}, 1, V,
                          T, H, W, K, 0.0f, cull, tri_id, bary, nullptr, stream);
}

// ---------------------------------------------------------------------------
// per-tile fragment lists sorted by triangle id
// ---------------------------------------------------------------------------
// Sort keys are (triangle id << EB | local fragment k*256 + pixel), EB = 8
// for one layer and 11 for up to five; an empty slot gets the sentinel bits
// (all ones above EB) | local, above every fragment key.  The keys are 32-bit
// when the triangle count leaves room (T < 2^(32 - EB) - 1), else 64-bit:
// the same order either way.  All keys of a tile are distinct, so a key's
// rank is its sorted position.  A triangle id >= T (never written by the
// rasterizer) is recorded as T, which every consumer skips.
template <typename KT>
__device__ __forceinline__ KT shfl_xor_key(KT v, int m) {
    if constexpr (sizeof(KT) == 4) {
        return (KT)__shfl_xor((unsigned)v, m, 64);
    } else {
        const unsigned lo = __shfl_xor((unsigned)(v & 0xffffffffu), m, 64);
        const unsigned hi = __shfl_xor((unsigned)(v >> 32), m, 64);
        return ((KT)hi << 32) | lo;
    }
}

// bitonic sort of one key per lane across a wavefront, ascending in lane order
template <typename KT>
__device__ __forceinline__ KT wave_sort_key(KT v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const KT o = shfl_xor_key(v, j);
            const bool up = (lane & k) == 0;   // this lane's block sorts ascending
            const bool low = (lane & j) == 0;
            const KT mn = v < o ? v : o, mx = v < o ? o : v;
            v = (low == up) ? mn : mx;
        }
    }
    return v;
}

// number of keys below v in a sorted run of 64
template <typename KT>
__device__ __forceinline__ int run_rank(const KT *run, KT v) {
    int lo = 0;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        if (run[lo + s - 1] < v) lo += s;
    if (run[lo] < v) lo++;
    return lo;
}

// One workgroup per tile: the tile's K*256 keys are sorted in runs of 64 (one
// wavefront each, in registers), every key is placed at its rank (its index in
// its run plus its rank in each other run), and the sorted list is cut into
// per-triangle records.  tv: this lane's pixel's triangle id in each layer
// (-1: none); the whole workgroup calls it.
template <typename KT, int EB>
__device__ __forceinline__ void fragsort_tile(int bt, int b, const int *tv, int K, int T,
                                              int32_t *__restrict__ n_frag, int32_t *__restrict__ n_rec,
                                              uint16_t *__restrict__ frag, int32_t *__restrict__ rec_tri,
                                              int32_t *__restrict__ rec_start, int32_t *__restrict__ tri_counts) {
    constexpr KT SENT = (KT)(~(KT)0) << EB;
    constexpr unsigned EMASK = (1u << EB) - 1u;
    constexpr int KMAX = EB == 8 ? 1 : DRESSI_MAX_K;
    __shared__ KT runs[KMAX * DRESSI_TILE_PIX];
    __shared__ KT keys[KMAX * DRESSI_TILE_PIX];
    __shared__ int wsum[DRESSI_TILE_PIX / 64];
    const int p = threadIdx.x;
    const int np = K * DRESSI_TILE_PIX, nruns = np / 64;
    int any = 0;
    KT kv[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; k++) {
        const int e = k * DRESSI_TILE_PIX + p;
        kv[k] = SENT | (KT)e;
        const int t = k < K ? tv[k] : -1;
        if (t >= 0) {
            kv[k] = ((KT)(t < T ? t : T) << EB) | (KT)e;
            any = 1;
        }
    }
    if (!__syncthreads_or(any)) {
        if (p == 0) {
            n_frag[bt] = 0;
            n_rec[bt] = 0;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < KMAX; k++)
        if (k < K) runs[k * DRESSI_TILE_PIX + p] = wave_sort_key(kv[k]);   // run = this wavefront's layer-k keys
    __syncthreads();
    for (int k = 0; k < K; k++) {
        const int e = k * DRESSI_TILE_PIX + p;
        const int run = e >> 6;
        const KT v = runs[e];
        int pos = e & 63;
        for (int r2 = 0; r2 < nruns; r2++)
            if (r2 != run) pos += run_rank(runs + r2 * 64, v);
        keys[pos] = v;
    }
    __syncthreads();
    // each thread owns a contiguous run of K sorted keys
    const int per = K;
    const int i0 = p * per;
    int heads = 0, valid = 0;
    for (int j = 0; j < per; j++) {
        const KT kv = keys[i0 + j];
        if (kv >= SENT) break;
        valid++;
        if (i0 + j == 0 || (keys[i0 + j - 1] >> EB) != (kv >> EB)) heads++;
    }
    int total_heads;
    int rbase;
    {
        // block exclusive scan of heads (64-lane waves)
        const int lane = p & 63, wid = p >> 6;
        int xs = heads;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int yv = __shfl_up(xs, o, 64);
            if (lane >= o) xs += yv;
        }
        if (lane == 63) wsum[wid] = xs;
        __syncthreads();
        int base = 0;
        for (int w = 0; w < wid; w++) base += wsum[w];
        total_heads = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        rbase = base + xs - heads;
    }
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX * K;
    int r = rbase;
    for (int j = 0; j < per; j++) {
        int i = i0 + j;
        const KT kv = keys[i];
        if (kv >= SENT) break;
        frag[base + i] = (uint16_t)(kv & EMASK);
        if (i == 0 || (keys[i - 1] >> EB) != (kv >> EB)) {
            int t = (int)(kv >> EB);
            rec_tri[base + r] = t;
            rec_start[base + r] = i;
            if (t < T) atomicAdd(&tri_counts[(int64_t)b * T + t], 1);
            r++;
        }
    }
    // number of valid keys = position of the first sentinel (keys are sorted)
    if (valid < per) {
        int i = i0 + valid;
        if (i == 0 || keys[i - 1] < SENT) n_frag[bt] = i;
    } else if (p == DRESSI_TILE_PIX - 1) {
        n_frag[bt] = np;
    }
    if (p == 0) n_rec[bt] = total_heads;
}

template <typename KT, int EB>
__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    k_fragsort(const int32_t *__restrict__ tri_id, int K, int H, int W, int ntx, int nt, int T,
               int32_t *__restrict__ n_frag, int32_t *__restrict__ n_rec, uint16_t *__restrict__ frag,
               int32_t *__restrict__ rec_tri, int32_t *__restrict__ rec_start,
               int32_t *__restrict__ tri_counts, int32_t *__restrict__ nlong) {
    // the long-list queue of k_tt_fill starts empty (read after this launch)
    if (blockIdx.x == 0 && threadIdx.x == 0) *nlong = 0;
    constexpr int KMAX = EB == 8 ? 1 : DRESSI_MAX_K;
    // several views: XCD-aware order (each XCD whole views); one view keeps the
    // default interleave, which balances uneven work over the image
    const int bt = (int)gridDim.x > nt ? (int)xcd_block() : (int)blockIdx.x;
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + p / DRESSI_TILE;
    int tv[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; k++)
        tv[k] = (k < K && x < W && y < H) ? tri_id[(((int64_t)b * K + k) * H + y) * W + x] : -1;
    fragsort_tile<KT, EB>(bt, b, tv, K, T, n_frag, n_rec, frag, rec_tri, rec_start, tri_counts);
}

// The binless resolve of one tile (K = 1, as k_raster_direct_resolve)
// followed by the tile's fragment sort (as k_fragsort): the pixels' triangle
// ids go to the sort in registers.
template <typename KT, int EB>
__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    k_raster_direct_resolve_sort(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris,
                                 Viewports vp, int B, int V, int T, int H, int W, int cull, int ntx, int nt,
                                 unsigned long long *__restrict__ zbuf, int32_t *__restrict__ tri_id,
                                 float2 *__restrict__ bary, FragLists fl, int32_t *__restrict__ tri_counts,
                                 int32_t *__restrict__ nlong) {
    // the long-list queue of k_tt_fill starts empty (read after this launch)
    if (blockIdx.x == 0 && threadIdx.x == 0) *nlong = 0;
    const int bt = (int)gridDim.x > nt ? (int)xcd_block() : (int)blockIdx.x;
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + p / DRESSI_TILE;
    int t = -1;
    if (x < W && y < H) {
        const int64_t i = ((int64_t)b * H + y) * W + x;
        const unsigned long long c = zbuf[i];
        if (c == 0ull) {   // no fragment
            tri_id[i] = -1;
            bary[i] = make_float2(0.0f, 0.0f);
        } else {
            zbuf[i] = 0ull;
            const unsigned long long v = ~c;
            t = (int)(v & 0xffffffffu);
            TriSetup s;
            direct_setup(pos_clip, tris, vp, b, V, t, H, W, cull, s);   // valid: it produced the key
            resolve_frag<false>(s, t, DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2, DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2,
                                __uint_as_float((unsigned)(v >> 32)), 0.0f, i, tri_id, bary, nullptr);
        }
    }
    fragsort_tile<KT, EB>(bt, b, &t, 1, T, fl.n_frag, fl.n_rec, fl.frag, fl.rec_tri, fl.rec_start, tri_counts);
}

static void fragindex_layout(int B, int K, int H, int W, int T, Carver &c, size_t *o) {
    int64_t nt = (int64_t)tiles_x(W) * tiles_y(H);
    int64_t n = (int64_t)B * nt * DRESSI_TILE_PIX * K;
    o[0] = c.take(sizeof(int32_t) * B * nt);                 // n_frag
    o[1] = c.take(sizeof(int32_t) * B * nt);                 // n_rec
    o[2] = c.take(sizeof(uint16_t) * n);                     // frag
    o[3] = c.take(sizeof(int32_t) * n);                      // rec_tri
    o[4] = c.take(sizeof(int32_t) * n);                      // rec_start
    o[5] = c.take(sizeof(int32_t) * ((int64_t)B * T + 1));   // triangle -> tiles offsets
    o[6] = c.take(sizeof(int2) * n);                         // triangle -> tiles entries
}

size_t dressi_fragindex_bytes(int B, int K, int H, int W, int T) {
    Carver c;
    size_t o[7];
    fragindex_layout(B, K, H, W, T, c, o);
    return c.off;
}

void dressi_fragindex_view(void *base, int B, int K, int H, int W, int T, FragLists &fl, TriTiles &tt) {
    Carver c;
    size_t o[7];
    fragindex_layout(B, K, H, W, T, c, o);
    fl.n_frag = at<int32_t>(base, o[0]);
    fl.n_rec = at<int32_t>(base, o[1]);
    fl.frag = at<uint16_t>(base, o[2]);
    fl.rec_tri = at<int32_t>(base, o[3]);
    fl.rec_start = at<int32_t>(base, o[4]);
    tt.offsets = at<int32_t>(base, o[5]);
    tt.entries = at<int2>(base, o[6]);
}

// ---------------------------------------------------------------------------
// triangle -> tiles transpose of the per-tile records
// ---------------------------------------------------------------------------
// Lists longer than TT_SHORT entries (a triangle over many tiles) are ordered
// by a workgroup-wide merge sort instead of per-entry counting (quadratic in
// the list length); k_tt_fill queues them, at most n / (TT_SHORT + 1).  The
// workgroup bodies are in dressi_internal.h.
__global__ void k_tt_fill(FragLists fl, int K, int T, int nt, const int32_t *__restrict__ offsets,
                          int32_t *__restrict__ counts, int2 *__restrict__ entries, int32_t *__restrict__ nlong,
                          int64_t *__restrict__ longk, int cap) {
    tt_fill_block(fl, K, T, nt, offsets, counts, entries, nlong, longk, cap, (int)blockIdx.x, (int)gridDim.x);
}

__global__ void k_tt_rank(FragLists fl, int K, int T, int nt, const int32_t *__restrict__ offsets,
                          const int2 *__restrict__ unsorted, int2 *__restrict__ entries, int2 *__restrict__ sbuf,
                          int64_t nkeys, const int32_t *__restrict__ nlong, const int64_t *__restrict__ longk,
                          int cap) {
    tt_rank_block(fl, K, T, nt, offsets, unsorted, entries, sbuf, nkeys, nlong, longk, cap, (int)blockIdx.x,
                  (int)gridDim.x);
}

__global__ void __launch_bounds__(256) k_list_job(ListJob j) { list_job_block(j, (int)blockIdx.x); }

void dr_flush_list_jobs(dressi_ctx *ctx, hipStream_t st) {
    while (ctx->n_list_jobs > 0) {
        const ListJob j = dr_take_list_job(ctx);
        if (j.nb > 0) DR_LAUNCH("k_list_job", (k_list_job), j.nb, 256, 0, st, j);
    }
}

// scan temporary, then the unsorted triangle -> tiles entries, then the
// long-list queue (its count, then the (view, triangle) keys), then the
// long lists' sort buffer
static size_t tt_long_cap(int64_t ne) { return (size_t)(ne / (TT_SHORT + 1)) + 1; }

size_t dressi_fragindex_tmp_bytes(int B, int K, int H, int W, int T) {
    const int64_t n = (int64_t)B * tiles_x(W) * tiles_y(H) * DRESSI_TILE_PIX * K;
    return (dressi_scan_tmp_bytes((int64_t)B * T) + 255) / 256 * 256 + sizeof(int2) * (size_t)n + 8 +
           sizeof(int64_t) * tt_long_cap(n) + sizeof(int2) * (size_t)n;
}

static void fragindex_lists(int B, int K, int H, int W, int T, const FragLists &fl, const TriTiles &tt, void *tmp,
                            int32_t *counts, hipStream_t s);

// the long-list queue's count in a fragment index's temporary
static int32_t *fragindex_qcount(void *tmp, int B, int K, int H, int W, int T) {
    const int64_t nb = (int64_t)B * T;
    const int64_t ne = (int64_t)B * tiles_x(W) * tiles_y(H) * DRESSI_TILE_PIX * K;
    return reinterpret_cast<int32_t *>(static_cast<char *>(tmp) + (dressi_scan_tmp_bytes(nb) + 255) / 256 * 256 +
                                       sizeof(int2) * (size_t)ne);
}

// counts: B*T zero counters (left at zero)
void dressi_build_fragindex(const int32_t *tri_id, int B, int K, int H, int W, int T, void *base,
                            void *tmp, int32_t *counts, hipStream_t s) {
    FragLists fl;
    TriTiles tt;
    dressi_fragindex_view(base, B, K, H, W, T, fl, tt);
    int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    int32_t *qcount = fragindex_qcount(tmp, B, K, H, W, T);
    if (B * nt > 0) {
        // 32-bit keys while the triangle ids leave room above the local index
        if (K == 1 && T < (1 << 24) - 1)
            DR_LAUNCH("k_fragsort", (k_fragsort<uint32_t, 8>), B * nt, DRESSI_TILE_PIX, 0, s, tri_id, K, H, W, ntx,
                      nt, T, fl.n_frag, fl.n_rec, fl.frag, fl.rec_tri, fl.rec_start, counts, qcount);
        else if (T < (1 << 21) - 1)
            DR_LAUNCH("k_fragsort", (k_fragsort<uint32_t, 11>), B * nt, DRESSI_TILE_PIX, 0, s, tri_id, K, H, W, ntx,
                      nt, T, fl.n_frag, fl.n_rec, fl.frag, fl.rec_tri, fl.rec_start, counts, qcount);
        else
            DR_LAUNCH("k_fragsort", (k_fragsort<unsigned long long, 11>), B * nt, DRESSI_TILE_PIX, 0, s, tri_id, K,
                      H, W, ntx, nt, T, fl.n_frag, fl.n_rec, fl.frag, fl.rec_tri, fl.rec_start, counts, qcount);
    }
    fragindex_lists(B, K, H, W, T, fl, tt, tmp, counts, s);
}

// The triangle -> tile lists of a fragment index whose tiles are sorted
// (counts: the per-(view, triangle) record counts the sort left, set back to
// zero here).
static void fragindex_lists(int B, int K, int H, int W, int T, const FragLists &fl, const TriTiles &tt, void *tmp,
                            int32_t *counts, hipStream_t s) {
    const int nt = tiles_x(W) * tiles_y(H);
    int64_t n = (int64_t)B * T;
    dressi_exclusive_scan(counts, tt.offsets, n, tmp, s);
    int2 *unsorted = reinterpret_cast<int2 *>(static_cast<char *>(tmp) +
                                              (dressi_scan_tmp_bytes(n) + 255) / 256 * 256);
    const int64_t ne = (int64_t)B * nt * DRESSI_TILE_PIX * K;   // entry capacity (at least the entries)
    int32_t *nlong = reinterpret_cast<int32_t *>(unsorted + ne);
    int64_t *longk = reinterpret_cast<int64_t *>(nlong + 2);
    int2 *sbuf = reinterpret_cast<int2 *>(longk + tt_long_cap(ne));
    const int cap = (int)std::min<size_t>(tt_long_cap(ne), 0x7fffffff);
    if (B * nt > 0) {
        DR_LAUNCH("k_tt_fill", (k_tt_fill), B * nt, 256, 0, s, fl, K, T, nt, tt.offsets, counts, unsorted, nlong,
                  longk, cap);
        DR_LAUNCH("k_tt_rank", (k_tt_rank), (int)std::min<int64_t>((ne + 255) / 256, 4096), 256, 0, s, fl, K, T,
                  nt, tt.offsets, unsorted, tt.entries, sbuf, n, nlong, longk, cap);
    }
}

extern "C" size_t dressi_fragment_index_bytes(int B, int K, int H, int W, int T) {
    if (B < 0 || K < 1 || K > DRESSI_MAX_K || H < 0 || W < 0 || T < 0) return 0;
    return dressi_fragindex_bytes(B, K, H, W, T);
}

extern "C" int dressi_fragment_index(dressi_ctx *ctx, const int32_t *tri_id, int B, int K, int H, int W,
                                     int T, void *index, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || K < 1 || K > DRESSI_MAX_K || H < 0 || W < 0 || T < 0)
        return dressi_fail(ctx, DRESSI_EINVAL, "fragment_index: bad dimensions");
    if (!index || ((int64_t)B * H * W > 0 && !tri_id))
        return dressi_fail(ctx, DRESSI_EINVAL, "fragment_index: null pointer");
    hipStream_t st = (hipStream_t)stream;
    int rc = dressi_scratch(ctx, dressi_fragindex_tmp_bytes(B, K, H, W, T), st);
    if (rc) return rc;
    rc = dressi_counters(ctx, (size_t)B * T, st);
    if (rc) return rc;
    dressi_build_fragindex(tri_id, B, K, H, W, T, index, ctx->scratch, ctx->counters, st);
    return dressi_launch_check(ctx, "fragment_index");
}

struct VertexStageArgs;
static int direct_indexed(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B, int V, int T, int H,
                          int W, int cull, int32_t *tri_id, float *bary, void *index, hipStream_t st,
                          const VertexStageArgs *vs, void *tmp = nullptr, bool lists = true);

extern "C" int dressi_rasterize_indexed(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B, int V,
                                        int T, int H, int W, int cull, int32_t *tri_id, float *bary,
                                        void *index, void *stream) {
    int rc = check_raster_args(ctx, pos_clip, tris, B, V, T, H, W, 1, 0.0f);
    if (rc) return rc;
    if (!tri_id || !bary || !index)
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize_indexed: null tri_id, bary or index");
    if (B == 0) return DRESSI_OK;
    hipStream_t st = (hipStream_t)stream;
    if (ctx->hard_raster != 3) {
        // a binned strategy: the two calls in sequence
        rc = rasterize_impl(ctx, pos_clip, tris, Viewports{nullptr, nullptr}, B, V, T, H, W, 1, 0.0f, cull, tri_id,
                            bary, nullptr, stream);
        if (rc) return rc;
        return dressi_fragment_index(ctx, tri_id, B, 1, H, W, T, index, stream);
    }
    return direct_indexed(ctx, pos_clip, tris, B, V, T, H, W, cull, tri_id, bary, index, st, nullptr);
}

// The binless path of dressi_rasterize_indexed; with `vs`, the merge runs in
// the vertex stage's launch (dr_vertex_raster_direct) instead of after it.
struct VertexStageArgs {
    const float *pos, *extra, *mvp;
    const int32_t *adj;
    int C;
    float *vattr;
};
static int direct_indexed(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B, int V, int T, int H,
                          int W, int cull, int32_t *tri_id, float *bary, void *index, hipStream_t st,
                          const VertexStageArgs *vs, void *tmp, bool lists) {
    // the per-pixel keys after the record counters, both kept at zero
    const size_t nc = ((size_t)B * T + 1) / 2 * 2;
    const int64_t npx = (int64_t)B * H * W;
    int rc = tmp ? DRESSI_OK : dressi_scratch(ctx, dressi_fragindex_tmp_bytes(B, 1, H, W, T), st);
    if (rc) return rc;
    if (!tmp) tmp = ctx->scratch;
    rc = dressi_counters(ctx, nc + 2 * (size_t)npx, st);
    if (rc) return rc;
    int32_t *counts = ctx->counters;
    unsigned long long *zbuf = reinterpret_cast<unsigned long long *>(ctx->counters + nc);
    const float4 *pc4 = reinterpret_cast<const float4 *>(pos_clip);
    const Viewports vp{nullptr, nullptr};
    const int64_t ntri = (int64_t)B * T;
    if (vs)
        dr_vertex_raster_direct(vs->pos, tris, vs->extra, vs->adj, V, vs->C, vs->vattr, vs->mvp, B,
                                const_cast<float *>(pos_clip), T, H, W, cull, zbuf, st);
    else if (ntri > 0)
        DR_LAUNCH("k_raster_direct", (k_raster_direct), (int)((ntri + 255) / 256), 256, 0, st, pc4, tris, vp, B, V,
                  T, H, W, cull, zbuf);
    FragLists fl;
    TriTiles tt;
    dressi_fragindex_view(index, B, 1, H, W, T, fl, tt);
    const int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    int32_t *qcount = fragindex_qcount(tmp, B, 1, H, W, T);
    float2 *b2 = reinterpret_cast<float2 *>(bary);
    if (T < (1 << 24) - 1)
        DR_LAUNCH("k_raster_direct_resolve_sort", (k_raster_direct_resolve_sort<uint32_t, 8>), B * nt,
                  DRESSI_TILE_PIX, 0, st, pc4, tris, vp, B, V, T, H, W, cull, ntx, nt, zbuf, tri_id, b2, fl, counts,
                  qcount);
    else
        DR_LAUNCH("k_raster_direct_resolve_sort", (k_raster_direct_resolve_sort<unsigned long long, 11>), B * nt,
                  DRESSI_TILE_PIX, 0, st, pc4, tris, vp, B, V, T, H, W, cull, ntx, nt, zbuf, tri_id, b2, fl, counts,
                  qcount);
    if (lists) fragindex_lists(B, 1, H, W, T, fl, tt, tmp, counts, st);
    return dressi_launch_check(ctx, vs ? "geometry_fwd" : "rasterize_indexed");
}

extern "C" int dressi_geometry_fwd(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                                   const float *extra, const int32_t *adj, const float *mvp, int B, float *vattr,
                                   float *pos_clip, int H, int W, int cull, int32_t *tri_id, float *bary,
                                   void *index, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    int rc = check_raster_args(ctx, pos_clip, tris, B, V, T, H, W, 1, 0.0f);
    if (rc) return rc;
    if (B < 1) return dressi_fail(ctx, DRESSI_EINVAL, "geometry_fwd: B must be >= 1");
    if (!pos || !mvp || !vattr || !pos_clip || !tri_id || !bary || !index)
        return dressi_fail(ctx, DRESSI_EINVAL, "geometry_fwd: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (ctx->hard_raster != 3 || !adj || V == 0) {
        // the two calls in sequence
        rc = dressi_vertex_stage(ctx, pos, tris, V, T, extra, adj, mvp, nullptr, B, vattr, pos_clip, stream);
        if (rc) return rc;
        return dressi_rasterize_indexed(ctx, pos_clip, tris, B, V, T, H, W, cull, tri_id, bary, index, stream);
    }
    const VertexStageArgs vs{pos, extra, mvp, adj, extra ? 9 : 6, vattr};
    return direct_indexed(ctx, pos_clip, tris, B, V, T, H, W, cull, tri_id, bary, index, st, &vs);
}

// binary search of triangle t among the sorted records of one tile; returns
// the fragment range [j0, j1) or an empty range
__device__ __forceinline__ void frag_range(const FragLists &fl, int64_t bt, int64_t base, int t,
                                           int &j0, int &j1) {
    int lo = 0, hi = fl.n_rec[bt];
    const int32_t *rt = fl.rec_tri + base;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rt[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    j0 = j1 = 0;
    if (lo < fl.n_rec[bt] && rt[lo] == t) {
        j0 = fl.rec_start[base + lo];
        j1 = (lo + 1 < fl.n_rec[bt]) ? fl.rec_start[base + lo + 1] : fl.n_frag[bt];
    }
}

// ---------------------------------------------------------------------------
// rasterization backward
//
// 1. per tile: every fragment's gradient w.r.t. the screen positions (and the
//    direct w term) of its triangle's three corners, kept in LDS; the tile's
//    fragments are already sorted by triangle, so each triangle's fragments are
//    summed in that order into one record (a segmented sum);
// 2. per (view, vertex): each corner's records summed in tile order and mapped
//    from screen to clip space, the corners combined in a fixed order.
// ---------------------------------------------------------------------------

// gradient of one fragment: out[corner*3 + {0,1,2}] = d/dx_screen, d/dy_screen,
// d/dw (direct) of that corner, original corner order.  Every array index is a
// compile-time constant (selects, not indexing by the corner order), so the
// whole record stays in registers.
__device__ __forceinline__ void rast_frag_grad(const TriSetup &s, int x, int y, float2 g2, float gdist,
                                               bool want_dist, int W, float *out) {
    const int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2, py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
    double E[3];
    bool in = true;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        E[i] = dr_edge(s.X, s.Y, i, px, py);
        bool own = (s.meta >> (1 + i)) & 1;
        in = in && (E[i] > 0 || (E[i] == 0 && own));
    }
    const bool swapped = dr_corner(s.meta, 1) == 2;
    // the barycentric chain runs in double (see the forward); reciprocals are
    // taken once per fragment
    const double iA2 = 1.0 / (double)s.Af;
    // d(edge)/d(screen) scale: 1/256 per sub-pixel unit over the area in pixels
    const double sA = 256.0 * iA2;
    double l[3], q[3], iw[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        iw[i] = 1.0 / (double)s.w[i];
        l[i] = E[i] * iA2;
        q[i] = l[i] * iw[i];
    }
    const double iQ = 1.0 / (q[0] + q[1] + q[2]);
    // gradient on the normalised-order barycentrics (original corner 2 has none)
    double gb[3] = {g2.x, swapped ? 0.0 : (double)g2.y, swapped ? (double)g2.y : 0.0};
    double sb = (gb[0] * q[0] + gb[1] * q[1] + gb[2] * q[2]) * iQ;
    double Gx = 0.0, Gy = 0.0, gw[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        int a = (i + 1) % 3, c = (i + 2) % 3;
        double gq = (gb[i] - sb) * iQ;
        double gl = gq * iw[i];
        gw[i] = -gq * l[i] * iw[i] * iw[i];
        Gx -= gl * ((double)s.Y[c] - (double)s.Y[a]) * sA;
        Gy += gl * ((double)s.X[c] - (double)s.X[a]) * sA;
    }
    float gsx[3], gsy[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        gsx[i] = (float)(-l[i] * Gx);
        gsy[i] = (float)(-l[i] * Gy);
    }
    if (want_dist && gdist != 0.0f) {
        int ne;
        dr_distnorm(s.X, s.Y, px, py, E, (float)W * 256.0f, ne);
        // the nearest edge runs from corner a = ne+1 to corner c = ne+2 (mod 3)
        const int Xa = ne == 0 ? s.X[1] : (ne == 1 ? s.X[2] : s.X[0]);
        const int Ya = ne == 0 ? s.Y[1] : (ne == 1 ? s.Y[2] : s.Y[0]);
        const int Xc = ne == 0 ? s.X[2] : (ne == 1 ? s.X[0] : s.X[1]);
        const int Yc = ne == 0 ? s.Y[2] : (ne == 1 ? s.Y[0] : s.Y[1]);
        // The vector from the closest point of the segment to the pixel, from
        // exact fixed-point quantities (a difference of nearby float screen
        // coordinates would lose it near the edge, where the weights are
        // largest): q = p - a, e = c - a; inside the segment it is the part of
        // q perpendicular to e, (E / |e|^2) (-e_y, e_x) with E = e x q the
        // exact edge function; past an end it is p minus that end.
        const double ex = (double)(Xc - Xa), ey = (double)(Yc - Ya);
        const double qx = (double)(px - Xa), qy = (double)(py - Ya);
        const double len2 = ex * ex + ey * ey;
        double tt = (qx * ex + qy * ey) / len2, dx, dy;
        if (tt <= 0.0) {
            tt = 0.0;
            dx = qx;
            dy = qy;
        } else if (tt >= 1.0) {
            tt = 1.0;
            dx = (double)(px - Xc);
            dy = (double)(py - Yc);
        } else {
            const double En = ne == 0 ? E[0] : (ne == 1 ? E[1] : E[2]);
            dx = -En * ey / len2;
            dy = En * ex / len2;
        }
        const double d = sqrt(dx * dx + dy * dy);   // fixed-point units: the ratio dx / d is what matters
        if (d > 0.0) {
            const double sg = (double)(in ? gdist : -gdist) / ((double)W * d);
            const double ga = sg * (1.0 - tt), gc = sg * tt;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                const bool is_a = i == (ne + 1) % 3, is_c = i == (ne + 2) % 3;
                gsx[i] -= (float)(is_a ? ga * dx : (is_c ? gc * dx : 0.0));
                gsy[i] -= (float)(is_a ? ga * dy : (is_c ? gc * dy : 0.0));
            }
        }
    }
    // normalised order is (0, 1, 2), or (0, 2, 1) when the winding was flipped
    out[0] = gsx[0];
    out[1] = gsy[0];
    out[2] = (float)gw[0];
    out[3] = swapped ? gsx[2] : gsx[1];
    out[4] = swapped ? gsy[2] : gsy[1];
    out[5] = (float)(swapped ? gw[2] : gw[1]);
    out[6] = swapped ? gsx[1] : gsx[2];
    out[7] = swapped ? gsy[1] : gsy[2];
    out[8] = (float)(swapped ? gw[1] : gw[2]);
}

__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    __attribute__((amdgpu_waves_per_eu(5))) k_rast_bwd_tile(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris, Viewports vp, int V,
                    int T, int H, int W, int K, int cull, int margin, const int32_t *__restrict__ tri_id,
                    FragLists fl, int ntx, int nt, const float2 *__restrict__ grad_bary,
                    const float *__restrict__ grad_dist, float *__restrict__ partial) {
    extern __shared__ float vals[];   // [K*256][9]
    __shared__ uint16_t sfrag[DRESSI_MAX_K * DRESSI_TILE_PIX];   // the tile's sorted fragment list
    // several views: XCD-aware order (each XCD whole views); one view keeps the
    // default interleave, which balances uneven work over the image
    const int bt = (int)gridDim.x > nt ? (int)xcd_block() : (int)blockIdx.x;
    const int nf = fl.n_frag[bt];
    if (nf == 0) return;
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    // the tile's sorted list is read before the fragments' gradients, not
    // after the barrier (in bounds whatever the count: K*256 slots)
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX * K;
    const int nr = fl.n_rec[bt];
    const int np = K * DRESSI_TILE_PIX;
    for (int i = p; i < np; i += DRESSI_TILE_PIX) sfrag[i] = fl.frag[base + i];
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + p / DRESSI_TILE;
    const float4 *pc = pos_clip + (int64_t)b * V;
    if (x < W && y < H) {
        for (int k = 0; k < K; k++) {
            int64_t o = (((int64_t)b * K + k) * H + y) * W + x;
            int t = tri_id[o];
            if (t < 0 || t >= T) continue;
            const int32_t *tv = tris + 3 * (int64_t)t;
            const int4 q = dr_viewport(vp, t, H, W);
            TriSetup s = dr_setup_tri(pc, tv, V, q.w, q.z, q.x, q.y, cull, margin);
            float *dst = vals + (k * DRESSI_TILE_PIX + p) * 9;
            if (!(s.meta & 1)) {
#pragma unroll
                for (int c = 0; c < 9; c++) dst[c] = 0.0f;
                continue;
            }
            float gd = grad_dist ? grad_dist[o] : 0.0f;
            float g9[9];
            rast_frag_grad(s, x, y, grad_bary[o], gd, grad_dist != nullptr, W, g9);
#pragma unroll
            for (int c = 0; c < 9; c++) dst[c] = g9[c];
        }
    }
    __syncthreads();
    for (int r = p; r < nr; r += DRESSI_TILE_PIX) {
        const int j0 = fl.rec_start[base + r];
        const int j1 = (r + 1 < nr) ? fl.rec_start[base + r + 1] : nf;
        float acc[9];
#pragma unroll
        for (int c = 0; c < 9; c++) acc[c] = 0.0f;
        for (int j = j0; j < j1; j++) {
            const float *v = vals + (int)sfrag[j] * 9;
#pragma unroll
            for (int c = 0; c < 9; c++) acc[c] += v[c];
        }
        float *dst = partial + (base + r) * 9;
#pragma unroll
        for (int c = 0; c < 9; c++) dst[c] = acc[c];
    }
}

// Eight lanes per (view, vertex); lane j takes the vertex's corners j, j+8,
// ... in ascending order.  Each corner's tile records are summed in tile
// order (double) and mapped from screen to clip space at the vertex
// (x_s = (x/w + 1) W/2, y_s = (1 - y/w) H/2, with the triangle's view size),
// rounded to float and added to the lane's sum; the eight lane sums are then
// combined in a fixed butterfly order.
#define RBV_LANES 8
__global__ void k_rast_bwd_vertex(const float4 *__restrict__ pos_clip, Viewports vp, int B, int V, int T, int H,
                                  int W, int K, TriTiles tt, const float *__restrict__ partial, Adjacency adj,
                                  float4 *__restrict__ grad_pos) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t vid = gid / RBV_LANES;
    const int slot = (int)(gid - vid * RBV_LANES);
    const bool live = vid < (int64_t)B * V;
    float gx = 0.0f, gy = 0.0f, gw = 0.0f;
    if (live) {
        const int b = (int)(vid / V), v = (int)(vid - (int64_t)b * V);
        const float4 p = pos_clip[vid];
        const double iw = 1.0 / (double)p.w, xn = (double)(p.x / p.w), yn = (double)(p.y / p.w);
        for (int j = adj.offsets[v] + slot; j < adj.offsets[v + 1]; j += RBV_LANES) {
            const int c = adj.corners[j];
            const int t = c / 3, i = c - 3 * t;
            const int64_t key = (int64_t)b * T + t;
            // a triangle without fragments adds nothing; it may be one that
            // setup dropped for this vertex's w <= 0 or non-finite position,
            // whose clip map below would not be finite
            if (tt.offsets[key] == tt.offsets[key + 1]) continue;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            for (int e = tt.offsets[key]; e < tt.offsets[key + 1]; e++) {
                const int2 ent = tt.entries[e];
                const float *r = partial + ((int64_t)ent.x * DRESSI_TILE_PIX * K + ent.y) * 9 + 3 * i;
                a0 += (double)r[0];
                a1 += (double)r[1];
                a2 += (double)r[2];
            }
            const int4 q = dr_viewport(vp, t, H, W);
            const double hw = 0.5 * (double)q.z, hh = 0.5 * (double)q.w;
            gx += (float)(a0 * hw * iw);
            gy += (float)(-a1 * hh * iw);
            gw += (float)((-a0 * hw * xn + a1 * hh * yn) * iw + a2);
        }
    }
#pragma unroll
    for (int m = 1; m < RBV_LANES; m <<= 1) {
        gx += __shfl_xor(gx, m, 64);
        gy += __shfl_xor(gy, m, 64);
        gw += __shfl_xor(gw, m, 64);
    }
    if (live && slot == 0) grad_pos[vid] = make_float4(gx, gy, 0.0f, gw);
}

static size_t partial_floats(int B, int K, int H, int W, int per) {
    return (size_t)B * tiles_x(W) * tiles_y(H) * DRESSI_TILE_PIX * K * per;
}

static int rasterize_bwd_impl(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, Viewports vp,
                              int B, int V, int T, int H, int W, int K, float r, int cull,
                              const int32_t *tri_id, const float *grad_bary, const float *grad_dist,
                              const void *frag_index, const int32_t *adj, float *grad_pos_clip,
                              void *stream) {
    int rc = check_raster_args(ctx, pos_clip, tris, B, V, T, H, W, K, r);
    if (rc) return rc;
    if (!tri_id || !grad_bary || (!grad_pos_clip && B * (int64_t)V > 0))
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize_bwd: null tri_id, grad_bary or grad_pos_clip");
    if (B == 0 || V == 0) return DRESSI_OK;
    hipStream_t st = (hipStream_t)stream;
    int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    int margin = soft_margin(r, W);
    Carver c;
    size_t o_fi = frag_index ? 0 : c.take(dressi_fragindex_bytes(B, K, H, W, T));
    size_t o_adj = adj ? 0 : c.take(adjacency_buf_bytes(V, T));
    size_t o_tmp = c.take(std::max(frag_index ? (size_t)0 : dressi_fragindex_tmp_bytes(B, K, H, W, T),
                                   adj ? (size_t)0 : dressi_adjacency_tmp_bytes(V, T)));
    size_t o_part = c.take(sizeof(float) * partial_floats(B, K, H, W, 9));
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
        dressi_build_adjacency_into(tris, T, V, buf, at<void>(S, o_tmp), st);
        ab = buf;
    }
    Adjacency A = adjacency_view(ab, V);
    float *part = at<float>(S, o_part);
    if ((int64_t)B * nt > 0)
        DR_LAUNCH("k_rast_bwd_tile", (k_rast_bwd_tile), B * nt, DRESSI_TILE_PIX,
                  sizeof(float) * 9 * DRESSI_TILE_PIX * K, st, reinterpret_cast<const float4 *>(pos_clip), tris,
                  vp, V, T, H, W, K, cull, margin, tri_id, fl, ntx, nt,
                  reinterpret_cast<const float2 *>(grad_bary), grad_dist, part);
    int64_t nv = (int64_t)B * V;
    DR_LAUNCH("k_rast_bwd_vertex", (k_rast_bwd_vertex), (int)((nv * RBV_LANES + 255) / 256), 256, 0, st,
              reinterpret_cast<const float4 *>(pos_clip), vp, B, V, T, H, W, K, tt, part, A,
              reinterpret_cast<float4 *>(grad_pos_clip));
    return dressi_launch_check(ctx, "rasterize_bwd");
}

extern "C" int dressi_rasterize_bwd(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                                    int B, int V, int T, int H, int W, int K, float r, int cull,
                                    const int32_t *tri_id, const float *grad_bary,
                                    const float *grad_dist, const void *frag_index,
                                    const int32_t *adj, float *grad_pos_clip, void *stream) {
    return rasterize_bwd_impl(ctx, pos_clip, tris, Viewports{nullptr, nullptr}, B, V, T, H, W, K, r, cull, tri_id,
                              grad_bary, grad_dist, frag_index, adj, grad_pos_clip, stream);
}

extern "C" int dressi_rasterize_batched_bwd(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                                            const int32_t *tri_view, const int32_t *views, int n, int V, int T,
                                            int H, int W, int K, int cull, const int32_t *tri_id,
                                            const float *grad_bary, const void *frag_index, const int32_t *adj,
                                            float *grad_pos_clip, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    int rc = check_views(ctx, tri_view, views, n, T);
    if (rc) return rc;
    return rasterize_bwd_impl(ctx, pos_clip, tris, Viewports{tri_view, reinterpret_cast<const int4 *>(views)}, 1,
                              V, T, H, W, K, 0.0f, cull, tri_id, grad_bary, nullptr, frag_index, adj,
                              grad_pos_clip, stream);
}

// ---------------------------------------------------------------------------
// worst-case scratch of one call of each kind, for dressi_reserve
// ---------------------------------------------------------------------------
int64_t dr_tile_capacity(const dressi_limits &l) {
    const int nt = tiles_x(l.W) * tiles_y(l.H);
    const int64_t cap = default_tile_capacity(l.B, l.T, nt, soft_margin(l.r, l.W));
    return std::min<int64_t>(std::max<int64_t>(cap, l.bin_entries), 1 << 26);
}

// rasterize (full, banded or batched), rasterize_bwd and fragment_index
// ---------------------------------------------------------------------------
// geometry adjoint of one image (B = 1, K = 1, hard): interpolation,
// rasterization, transform and vertex-normal adjoints in three launches
// ---------------------------------------------------------------------------
// Per tile (B = K = 1): the interpolation adjoint of every fragment (its
// barycentric gradient and staged row, as k_interp_bwd_tile), then, from that
// barycentric gradient, the rasterization adjoint of the same fragment (as
// k_rast_bwd_tile); after one barrier each triangle record sums both in the
// tile's sorted order.  The same values as the two kernels in sequence.
template <int CC>
__global__ void __launch_bounds__(DRESSI_TILE_PIX) __attribute__((amdgpu_waves_per_eu(5)))
    k_geo_tile(const float *__restrict__ attr, int Va, const int32_t *__restrict__ tris, int T,
               const float4 *__restrict__ pos_clip, Viewports vp, int H, int W, int cull,
               const int32_t *__restrict__ tri_id, const float2 *__restrict__ bary, int ntx, FragLists fl,
               const float *__restrict__ grad_out, const float2 *__restrict__ gb_in, float2 *__restrict__ grad_bary,
               float *__restrict__ ipart, float *__restrict__ rpart, int skip_empty, ListJob lj, int nmain) {
    extern __shared__ float vals[];   // [256][ib_stride(CC)] interpolation rows, then [256][9]
    // workgroups past the tiles run a list-building job of the step
    if ((int)blockIdx.x >= nmain) {
        list_job_block(lj, (int)blockIdx.x - nmain);
        return;
    }
    constexpr int S = (CC + 2) | 1;
    float *rvals = vals + DRESSI_TILE_PIX * S;
    __shared__ uint16_t sfrag[DRESSI_TILE_PIX];   // the tile's sorted fragment list
    const int bt = (int)blockIdx.x;
    const int tx = bt % ntx, ty = bt / ntx;
    const int p = threadIdx.x;
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + p / DRESSI_TILE;
    // the tile's lists are read before the fragments' adjoints, not after
    // the barrier (in bounds whatever the counts: a tile has 256 slots of
    // each; entries past the counts are never used)
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX;
    const int nf = fl.n_frag[bt];
    const int nr = fl.n_rec[bt];
    const uint16_t fr = fl.frag[base + p];   // into LDS before the barrier (its load overlaps the fragment's)
    const int rs0 = fl.rec_start[base + p];
    const int rs1 = p + 1 < DRESSI_TILE_PIX ? fl.rec_start[base + p + 1] : 0;
    if (x < W && y < H) {
        // The fragment's loads in two rounds: its corners and viewport beside
        // its barycentrics, output gradient and incoming barycentric gradient;
        // then the corners' attribute rows beside their clip-space positions
        // (row 0 for an invalid corner, then unused).  The arithmetic is that
        // of ib_fragment and dr_setup.
        const int64_t o = (int64_t)y * W + x;
        const int t = tri_id[o];
        const bool tri = t >= 0 && t < T;
        int v0 = -1, v1 = -1, v2 = -1;
        int4 q = make_int4(0, 0, W, H);
        if (tri) {
            v0 = tris[3 * (int64_t)t];
            v1 = tris[3 * (int64_t)t + 1];
            v2 = tris[3 * (int64_t)t + 2];
            q = dr_viewport(vp, t, H, W);
        }
        const bool live = !(skip_empty && t < 0);
        // set only where live (and read only there), so that no copy at the
        // branch's end waits for the loads
        float2 w, acc;
        float gv[CC];
        if (live) {
            w = bary[o];
            ld_row<CC>(grad_out + o * CC, gv, CC);
            acc = gb_in ? gb_in[o] : make_float2(0.0f, 0.0f);
        }
        const bool ok = v0 >= 0 && v0 < Va && v1 >= 0 && v1 < Va && v2 >= 0 && v2 < Va;
        float r0[CC], r1[CC], r2[CC];
        float4 P[3];
        if (Va > 0) {
            const int c0 = ok ? v0 : 0, c1 = ok ? v1 : 0, c2 = ok ? v2 : 0;
            ld_row<CC>(attr + (int64_t)c0 * CC, r0, CC);
            ld_row<CC>(attr + (int64_t)c1 * CC, r1, CC);
            ld_row<CC>(attr + (int64_t)c2 * CC, r2, CC);
            P[0] = pos_clip[c0];
            P[1] = pos_clip[c1];
            P[2] = pos_clip[c2];
        }
        if (live) {
            ib_fragment_math<CC>(ok, t, w, gv, r0, r1, r2, vals + p * S, acc);
            if (grad_bary) grad_bary[o] = acc;
        }
        if (tri) {
            TriSetup s;
            if (ok) {
                s = dr_setup_pts(P, q.w, q.z, q.x, q.y, cull, 0);
            } else {
                s.meta = 0;
                s.box0 = s.box1 = 1;
                s.hbox0 = s.hbox1 = 1;
            }
            float *dst = rvals + p * 9;
            if (!(s.meta & 1)) {
#pragma unroll
                for (int c = 0; c < 9; c++) dst[c] = 0.0f;
            } else {
                float g9[9];
                rast_frag_grad(s, x, y, acc, 0.0f, false, W, g9);
#pragma unroll
                for (int c = 0; c < 9; c++) dst[c] = g9[c];
            }
        }
    }
    sfrag[p] = fr;
    __syncthreads();
    // one record per lane (a tile has at most 256)
    if (p < nr) {
        const int r = p;
        const int j0 = rs0;
        const int j1 = (r + 1 < nr) ? rs1 : nf;
        ib_record(vals, S, CC, sfrag, j0, j1, ipart + (base + r) * 3 * CC);
        float acc9[9];
#pragma unroll
        for (int c = 0; c < 9; c++) acc9[c] = 0.0f;
        for (int j = j0; j < j1; j++) {
            const float *v = rvals + (int)sfrag[j] * 9;
#pragma unroll
            for (int c = 0; c < 9; c++) acc9[c] += v[c];
        }
        float *dst = rpart + (base + r) * 9;
#pragma unroll
        for (int c = 0; c < 9; c++) dst[c] = acc9[c];
    }
}

static size_t geometry_scratch(int H, int W, int V, int Cv, Carver &c, size_t *o) {
    const size_t n = (size_t)tiles_x(W) * tiles_y(H) * DRESSI_TILE_PIX;
    o[0] = c.take(sizeof(float) * n * 3 * Cv);   // per-tile interpolation records
    o[1] = c.take(sizeof(float) * n * 9);        // per-tile rasterization records
    o[2] = c.take(sizeof(float) * 3 * (size_t)V);   // transform adjoint
    o[3] = c.take(sizeof(float) * 3 * (size_t)V);   // normal-sum adjoint
    return c.off;
}

extern "C" int dressi_geometry_bwd(dressi_ctx *ctx, const float *pos, const float *vattr, int V, int Cv,
                                   const int32_t *tris, int T,
                                   const float *pos_clip, const float *mvp, const int32_t *vert_view,
                                   const int32_t *tri_view, const int32_t *views, int n_views, int H, int W,
                                   int cull, const int32_t *tri_id, const float *bary, const float *grad_gbuf,
                                   const float *grad_bary_in, const void *frag_index, const int32_t *adj,
                                   float *grad_vattr, float *grad_bary, float *grad_pos_clip, float *grad_pos,
                                   void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (V < 0 || T < 0 || H < 0 || W < 0 || (cull != 0 && cull != 1))
        return dressi_fail(ctx, DRESSI_EINVAL, "geometry_bwd: bad dimensions");
    if (Cv != 6 && Cv != 9) return dressi_fail(ctx, DRESSI_EINVAL, "geometry_bwd: Cv must be 6 or 9");
    if ((tri_view == nullptr) != (views == nullptr) || (tri_view && !vert_view))
        return dressi_fail(ctx, DRESSI_EINVAL, "geometry_bwd: tri_view, views and vert_view go together");
    if (tri_view) {
        const int rc = check_views(ctx, tri_view, views, n_views, T);
        if (rc) return rc;
    }
    if (V == 0) return DRESSI_OK;
    if (!pos || !vattr || !tris || !pos_clip || !mvp || !tri_id || !bary || !grad_gbuf || !frag_index || !adj ||
        !grad_vattr || !grad_bary || !grad_pos_clip || !grad_pos)
        return dressi_fail(ctx, DRESSI_EINVAL, "geometry_bwd: null pointer");
    hipStream_t st = (hipStream_t)stream;
    Carver c;
    size_t o[4];
    geometry_scratch(H, W, V, Cv, c, o);
    int rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    float *ipart = at<float>(ctx->scratch, o[0]), *rpart = at<float>(ctx->scratch, o[1]);
    float *gpos_t = at<float>(ctx->scratch, o[2]), *gacc = at<float>(ctx->scratch, o[3]);
    FragLists fl;
    TriTiles tt;
    dressi_fragindex_view(const_cast<void *>(frag_index), 1, 1, H, W, T, fl, tt);
    const Viewports vp{tri_view, reinterpret_cast<const int4 *>(views)};
    const int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    // both per-tile adjoints in one kernel (6-channel rows are read in pairs:
    // 8-byte aligned bases), else one after the other
    const bool al8 = (((uintptr_t)vattr | (uintptr_t)grad_gbuf) & 7u) == 0;
    const float4 *pc4 = reinterpret_cast<const float4 *>(pos_clip);
    const float2 *b2 = reinterpret_cast<const float2 *>(bary);
    const float2 *gbi = reinterpret_cast<const float2 *>(grad_bary_in);
    float2 *gbo = reinterpret_cast<float2 *>(grad_bary);
    if (nt > 0 && (Cv == 9 || al8)) {
        const size_t lds = sizeof(float) * DRESSI_TILE_PIX * (((Cv + 2) | 1) + 9);
        const ListJob lj = dr_take_list_job(ctx);
        if (Cv == 6)
            DR_LAUNCH("k_geo_tile", (k_geo_tile<6>), nt + lj.nb, DRESSI_TILE_PIX, lds, st, vattr, V, tris, T, pc4, vp,
                      H, W, cull, tri_id, b2, ntx, fl, grad_gbuf, gbi, gbo, ipart, rpart, ctx->skip_empty, lj, nt);
        else
            DR_LAUNCH("k_geo_tile", (k_geo_tile<9>), nt + lj.nb, DRESSI_TILE_PIX, lds, st, vattr, V, tris, T, pc4, vp,
                      H, W, cull, tri_id, b2, ntx, fl, grad_gbuf, gbi, gbo, ipart, rpart, ctx->skip_empty, lj, nt);
    } else {
        dr_interp_bwd_tiles(vattr, 1, V, Cv, tris, T, tri_id, bary, 1, 1, H, W, fl, grad_gbuf, grad_bary_in,
                            grad_bary, ipart, ctx->skip_empty, st);
        if (nt > 0)
            DR_LAUNCH("k_rast_bwd_tile", (k_rast_bwd_tile), nt, DRESSI_TILE_PIX, sizeof(float) * 9 * DRESSI_TILE_PIX,
                      st, pc4, tris, vp, V, T, H, W, 1, cull, 0, tri_id, fl, ntx, nt, gbo, nullptr, rpart);
    }
    // a whole step's list jobs not run yet: the per-vertex pass reads the lists
    dr_flush_list_jobs(ctx, st);
    dr_geo_vertex(Cv, pos, tris, pos_clip, vp, V, H, W, tt, ipart, rpart, adjacency_view(adj, V), mvp, vert_view,
                  grad_vattr, grad_pos_clip, gpos_t, gacc, grad_pos, st);
    return dressi_launch_check(ctx, "geometry_bwd");
}

size_t dr_need_raster(const dressi_limits &l, int64_t cap) {
    const int B = l.B, T = l.T, H = l.H, W = l.W, K = std::max(l.K, 1);
    if (B <= 0 || H <= 0 || W <= 0) return 0;
    const int nt = tiles_x(W) * tiles_y(H);
    size_t need = 0;
    {
        Carver c;
        size_t o[2];
        raster_scratch(B, T, nt, (int)cap, c, o);
        if (l.r > 0.0f) c.take(3 * (size_t)B * H * W);
        need = std::max(need, c.off);
    }
    {
        Carver c;
        c.take(dressi_fragindex_bytes(B, K, H, W, T));
        c.take(adjacency_buf_bytes(l.V, T));
        c.take(std::max(dressi_fragindex_tmp_bytes(B, K, H, W, T), dressi_adjacency_tmp_bytes(l.V, T)));
        c.take(sizeof(float) * partial_floats(B, K, H, W, 9));
        need = std::max(need, c.off);
    }
    {
        // dressi_geometry_bwd (one image, single layer; attribute rows of up
        // to max(C, 9) channels)
        Carver c;
        size_t o[4];
        geometry_scratch(H, W, l.V, std::max(l.C, 9), c, o);
        need = std::max(need, c.off);
    }
    return std::max(need, dressi_fragindex_tmp_bytes(B, K, H, W, T));
}

extern "C" size_t dressi_limits_scratch_bytes(const dressi_limits *l) {
    if (!l || l->B < 0 || l->V < 0 || l->T < 0 || l->H < 0 || l->W < 0 || l->K < 0) return 0;
    size_t need = dr_need_raster(*l, dr_tile_capacity(*l));
    need = std::max(need, dr_need_interp(*l));
    need = std::max(need, dr_need_texture(*l));
    need = std::max(need, dr_need_shade(*l));
    need = std::max(need, dr_need_optim(*l));
    need = std::max(need, dr_need_pbs(*l));
    need = std::max(need, 2 * (size_t)std::max(l->B, 0) * std::max(l->H, 0) * std::max(l->W, 0));  // softras
    // the whole packed step of one image: the packed backward's and the
    // geometry adjoints' scratch, then the fragment index's temporary
    if (l->K <= 1 && l->H > 0 && l->W > 0) {
        Carver cg;
        size_t og[4];
        geometry_scratch(l->H, l->W, l->V, 9, cg, og);
        const size_t off = (std::max(cg.off, dr_need_shade(*l)) + 255) / 256 * 256;
        need = std::max(need, off + dressi_fragindex_tmp_bytes(1, 1, l->H, l->W, l->T));
    }
    return need;
}

extern "C" int dressi_reserve_limits(dressi_ctx *ctx, const dressi_limits *l) {
    if (!ctx) return DRESSI_EINVAL;
    if (!l) return dressi_fail(ctx, DRESSI_EINVAL, "reserve_limits: null limits");
    const size_t bytes = dressi_limits_scratch_bytes(l);
    const int64_t cap = dr_tile_capacity(*l);
    int rc = dressi_reserve(ctx, bytes, cap);
    if (rc) return rc;
    const size_t nt = (size_t)tiles_x(l->W) * tiles_y(l->H);
    size_t nc = std::max((size_t)std::max(l->B, 1) * nt, (size_t)std::max(l->B, 1) * std::max(l->T, 0));
    // one layer: the binless hard rasterizer's per-pixel keys (two counters a
    // pixel; after the record counters when it builds the fragment index too)
    if (l->K <= 1)
        nc = std::max(nc, ((size_t)std::max(l->B, 1) * std::max(l->T, 0) + 1) / 2 * 2 +
                              2 * (size_t)std::max(l->B, 1) * std::max(l->H, 0) * std::max(l->W, 0));
    return dressi_counters(ctx, nc, nullptr);
}

extern "C" size_t dressi_scratch_bytes(int B, int V, int T, int H, int W, int K, float r, int Va,
                                       int C, int64_t tex_cells, int tex_slices) {
    if (B < 0 || V < 0 || T < 0 || H < 0 || W < 0 || K < 1) return 0;
    int nt = tiles_x(W) * tiles_y(H);
    int margin = soft_margin(r, W);
    int Vm = Va > V ? Va : V;
    size_t need = 0;
    auto upd = [&](size_t v) { need = v > need ? v : need; };
    {
        Carver c;
        size_t o[2];
        raster_scratch(B, T, nt, default_tile_capacity(B, T, nt, margin), c, o);
        upd(c.off);
    }
    {   // a backward call that builds its own fragment index and adjacency
        Carver c;
        c.take(dressi_fragindex_bytes(B, K, H, W, T));
        c.take(adjacency_buf_bytes(Vm, T));
        c.take(std::max(dressi_fragindex_tmp_bytes(B, K, H, W, T), dressi_adjacency_tmp_bytes(Vm, T)));
        c.take(sizeof(float) * 3 * (size_t)(C > 9 ? C : 9) * B * T);
        c.take(sizeof(float) * partial_floats(B, K, H, W, 3 * (C > 3 ? C : 3)));
        upd(c.off);
    }
    {
        Carver c;
        c.take(sizeof(int32_t) * (size_t)tex_cells * (tex_slices > 0 ? tex_slices : 1));
        c.take(dressi_invuv_part_bytes(tex_cells, 16, tex_slices));
        upd(c.off);
    }
    {
        Carver c;
        c.take((size_t)B * H * W);
        c.take((size_t)B * H * W);
        upd(c.off);
    }
    return need;
}

extern "C" int dressi_packed_step(dressi_ctx *ctx, const dressi_packed_scene *sc, const dressi_packed_step_bufs *b,
                                  void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (!sc || !b) return dressi_fail(ctx, DRESSI_EINVAL, "packed_step: null scene or buffers");
    if (sc->vattr != b->vattr) return dressi_fail(ctx, DRESSI_EINVAL, "packed_step: scene->vattr must be b->vattr");
    const bool tex = sc->mode == DRESSI_SHADE_PHONG;
    if (tex && (!b->inv || !b->inv_rec || !b->grad_tex))
        return dressi_fail(ctx, DRESSI_EINVAL, "packed_step: the textured step needs inv, inv_rec and grad_tex");
    const int V = sc->V, T = sc->T, H = b->H, W = b->W, Cv = sc->Cv;
    hipStream_t st = (hipStream_t)stream;
    // With the binless rasterizer and a two-pass scan of the record counts,
    // the triangle -> tile lists are built by four jobs run in the launches
    // of the packed forward (the counts' chunk sums), the packed backward
    // (the scan), the texel gather (the fill) and the per-tile geometry
    // adjoint (the ranking); jobs without such a launch run on their own
    // before the per-vertex adjoint.  Otherwise the calls in sequence.
    const int64_t nchunk = ((int64_t)T + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const bool jobs = ctx->hard_raster == 3 && b->adj && V > 0 && T > 16384 && nchunk <= SCAN_DIRECT_MAX &&
                      b->pos_clip && b->tri_id && b->bary && b->index && b->pos && b->mvp && b->vattr &&
                      H > 0 && W > 0 && H <= 32767 && W <= 32767 && T < 0x7fffffff;
    int rc;
    ListJob j[4];   // taken by the calls below (so it lives until the function's end)
    if (!jobs) {
        rc = dressi_geometry_fwd(ctx, b->pos, sc->tris, V, T, b->extra, b->adj, b->mvp, 1, b->vattr, b->pos_clip, H,
                                 W, 0, b->tri_id, b->bary, b->index, stream);
    } else {
        // scratch: what the packed backward and the geometry adjoints take
        // (from the arena's start), then the fragment index's temporary, which
        // lives until the last job
        Carver cg;
        size_t og[4];
        geometry_scratch(H, W, V, Cv, cg, og);
        const size_t off = (std::max(cg.off, dr_packed_bwd_scratch(sc, 1, H, W, tex)) + 255) / 256 * 256;
        if ((rc = dressi_scratch(ctx, off + dressi_fragindex_tmp_bytes(1, 1, H, W, T), st))) return rc;
        void *tmp = static_cast<char *>(ctx->scratch) + off;
        const VertexStageArgs vs{b->pos, b->extra, b->mvp, b->adj, b->extra ? 9 : 6, b->vattr};
        rc = direct_indexed(ctx, b->pos_clip, sc->tris, 1, V, T, H, W, 0, b->tri_id, b->bary, b->index, st, &vs, tmp,
                            false);
        if (rc) return rc;
        FragLists fl;
        TriTiles tt;
        dressi_fragindex_view(b->index, 1, 1, H, W, T, fl, tt);
        const int nt = tiles_x(W) * tiles_y(H);
        const int64_t ne = (int64_t)nt * DRESSI_TILE_PIX;
        int2 *unsorted = reinterpret_cast<int2 *>(static_cast<char *>(tmp) +
                                                  (dressi_scan_tmp_bytes(T) + 255) / 256 * 256);
        int32_t *nlong = reinterpret_cast<int32_t *>(unsorted + ne);
        int64_t *longk = reinterpret_cast<int64_t *>(nlong + 2);
        int2 *sbuf = reinterpret_cast<int2 *>(longk + tt_long_cap(ne));
        for (int k = 0; k < 4; k++) {
            j[k].in = ctx->counters;
            j[k].out = tt.offsets;
            j[k].n = T;
            j[k].sums = static_cast<int32_t *>(tmp);
            j[k].fl = fl;
            j[k].K = 1;
            j[k].T = T;
            j[k].nt = nt;
            j[k].cap = (int)std::min<size_t>(tt_long_cap(ne), 0x7fffffff);
            j[k].counts = ctx->counters;
            j[k].nlong = nlong;
            j[k].unsorted = unsorted;
            j[k].entries = tt.entries;
            j[k].sbuf = sbuf;
            j[k].longk = longk;
        }
        j[0].kind = LJ_SCAN_REDUCE, j[0].nb = (int)nchunk;
        j[1].kind = LJ_SCAN_APPLY, j[1].nb = (int)nchunk;
        j[2].kind = LJ_TT_FILL, j[2].nb = nt;
        j[3].kind = LJ_TT_RANK, j[3].nb = (int)std::min<int64_t>((ne + 255) / 256, 4096);
        ctx->list_job = j;
        ctx->n_list_jobs = 4;
    }
    if (!rc)
        rc = dressi_packed_forward(ctx, sc, b->tri_id, b->bary, 1, H, W, b->gbuf, b->uvbuf, b->samp, b->color,
                                   b->sil, b->edge, b->inv, stream);
    if (!rc)
        rc = dressi_packed_backward(ctx, sc, b->tri_id, 1, H, W, b->gbuf, b->uvbuf, b->samp, b->color, b->sil,
                                    b->target, nullptr, b->loss, nullptr, nullptr, b->grad_gbuf, b->grad_samp,
                                    b->grad_bary_uv, b->inv, b->inv_rec, b->grad_tex, stream);
    if (!rc)
        rc = dressi_geometry_bwd(ctx, b->pos, b->vattr, V, Cv, sc->tris, T, b->pos_clip, b->mvp, nullptr, nullptr,
                                 nullptr, 0, H, W, 0, b->tri_id, b->bary, b->grad_gbuf,
                                 tex ? b->grad_bary_uv : nullptr, b->index, b->adj, b->grad_vattr, b->grad_bary,
                                 b->grad_pos_clip, b->grad_pos, stream);
    // jobs left by a call that stopped early run here (they keep the
    // counters' zero); none are left for later calls
    if (ctx->n_list_jobs > 0) dr_flush_list_jobs(ctx, st);
    ctx->list_job = nullptr;
    ctx->n_list_jobs = 0;
    return rc;
}
