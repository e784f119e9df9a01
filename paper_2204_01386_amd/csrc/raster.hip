// Rasterization forward and backward for gfx950.
//
// Forward (Algorithm 2 and the Shift equation of §3.4.2, depth peeling with K
// buffers): triangle setup -> per-tile counts -> scan -> bin fill -> tile
// rasterizer.  A 16x16 tile is one 256-lane workgroup, one lane per pixel.
// Triangle records of the tile's bin are staged through LDS 256 at a time and
// every lane keeps its K best (distinct key, smallest id) fragments in
// registers, which is what K passes of depth peeling with a LESS depth test
// select; the list is order independent, so bin order does not matter.
//
// Backward: the fragments of every tile are sorted by triangle id in LDS
// (bitonic sort); one thread per triangle then walks its fragments in the
// tiles its box covers (binary search in each tile's sorted record list),
// accumulating vertex gradients in registers, and one thread per vertex sums
// its corners in ascending order.  No float atomics: results are bitwise
// reproducible.
#include "dressi_internal.h"

#include <cfloat>

// ---------------------------------------------------------------------------
// setup, counting and bin fill
// ---------------------------------------------------------------------------
__global__ void k_setup_count(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris,
                              int B, int V, int T, int H, int W, int cull, int margin, int ntx,
                              int nt, TriSetup *__restrict__ setup, int32_t *__restrict__ tile_count) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)B * T) return;
    int b = (int)(gid / T), t = (int)(gid - (int64_t)b * T);
    const int32_t *tv = tris + 3 * (int64_t)t;
    int v0 = tv[0], v1 = tv[1], v2 = tv[2];
    TriSetup s;
    if (v0 < 0 || v0 >= V || v1 < 0 || v1 >= V || v2 < 0 || v2 >= V) {
        s.meta = 0;
        s.box0 = s.box1 = 1;
    } else {
        s = dr_setup(pos_clip + (int64_t)b * V, v0, v1, v2, H, W, cull, margin);
    }
    setup[gid] = s;
    if (!(s.meta & 1)) return;
    int tx0 = (s.box0 & 0xffff) / DRESSI_TILE, tx1 = (s.box0 >> 16) / DRESSI_TILE;
    int ty0 = (s.box1 & 0xffff) / DRESSI_TILE, ty1 = (s.box1 >> 16) / DRESSI_TILE;
    int32_t *tc = tile_count + (int64_t)b * nt;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) atomicAdd(&tc[ty * ntx + tx], 1);
}

__global__ void k_fill_bins(const TriSetup *__restrict__ setup, int B, int T, int ntx, int nt,
                            const int32_t *__restrict__ tile_off, int32_t *__restrict__ cursor,
                            int32_t *__restrict__ bins, int64_t cap,
                            unsigned long long *__restrict__ status) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) {
        int64_t total = tile_off[(int64_t)B * nt];
        if (total > cap) {
            atomicMax(&status[0], 1ull);
            atomicMax(&status[1], (unsigned long long)total);
        }
    }
    if (gid >= (int64_t)B * T) return;
    TriSetup s = setup[gid];
    if (!(s.meta & 1)) return;
    int b = (int)(gid / T), t = (int)(gid - (int64_t)b * T);
    int tx0 = (s.box0 & 0xffff) / DRESSI_TILE, tx1 = (s.box0 >> 16) / DRESSI_TILE;
    int ty0 = (s.box1 & 0xffff) / DRESSI_TILE, ty1 = (s.box1 >> 16) / DRESSI_TILE;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            int64_t bt = (int64_t)b * nt + ty * ntx + tx;
            int64_t slot = (int64_t)tile_off[bt] + atomicAdd(&cursor[bt], 1);
            if (slot < cap) bins[slot] = t;
        }
}

// ---------------------------------------------------------------------------
// tile rasterizer
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void klist_insert(float (&key)[K], int (&id)[K], float k, int t) {
    bool dup = false;
#pragma unroll
    for (int j = 0; j < K; j++)
        if (key[j] == k) {
            dup = true;
            id[j] = min(id[j], t);
        }
    if (dup || !(k < key[K - 1])) return;
    float ck = k;
    int ct = t;
#pragma unroll
    for (int j = 0; j < K; j++) {
        if (ck < key[j]) {
            float tk = key[j];
            int ti = id[j];
            key[j] = ck;
            id[j] = ct;
            ck = tk;
            ct = ti;
        }
    }
}

template <int K, bool SOFT>
__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    k_raster(const TriSetup *__restrict__ setup, const int32_t *__restrict__ tile_off,
             const int32_t *__restrict__ bins, int64_t cap, int T, int H, int W, int ntx, int nt,
             float r, int32_t *__restrict__ tri_id, float2 *__restrict__ bary,
             float *__restrict__ dist) {
    __shared__ TriSetup sh[DRESSI_TILE_PIX];
    __shared__ int shid[DRESSI_TILE_PIX];
    const int bt = blockIdx.x;
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int x = tx * DRESSI_TILE + (threadIdx.x & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + (threadIdx.x / DRESSI_TILE);
    const int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2;
    const int py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
    const float dscale = (float)W * 256.0f;
    const TriSetup *sv = setup + (int64_t)b * T;

    float key[K];
    int id[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        key[k] = FLT_MAX;
        id[k] = -1;
    }
    int64_t beg = tile_off[bt];
    int64_t end = tile_off[bt + 1];
    if (end > cap) end = cap;
    for (int64_t c0 = beg; c0 < end; c0 += DRESSI_TILE_PIX) {
        int n = (end - c0 < DRESSI_TILE_PIX) ? (int)(end - c0) : DRESSI_TILE_PIX;
        __syncthreads();
        if ((int)threadIdx.x < n) {
            int t = bins[c0 + threadIdx.x];
            shid[threadIdx.x] = t;
            sh[threadIdx.x] = sv[t];
        }
        __syncthreads();
        for (int j = 0; j < n; j++) {
            const TriSetup &s = sh[j];
            int bx0 = s.box0 & 0xffff, bx1 = s.box0 >> 16;
            int by0 = s.box1 & 0xffff, by1 = s.box1 >> 16;
            if (x < bx0 || x > bx1 || y < by0 || y > by1) continue;
            int64_t E[3];
            bool in = true;
#pragma unroll
            for (int i = 0; i < 3; i++) {
                E[i] = dr_edge(s.X, s.Y, i, px, py);
                bool own = (s.meta >> (1 + i)) & 1;
                in = in && (E[i] > 0 || (E[i] == 0 && own));
            }
            if (in) {
                float z = dr_depth(s, E);
                if (z > 0.0f && z < 1.0f) klist_insert<K>(key, id, 0.5f * z, shid[j]);
            } else if (SOFT) {
                int ne;
                float dn = dr_distnorm(s.X, s.Y, px, py, E, dscale, ne);
                if (dn <= r) {
                    float h = 0.5f * dn;
                    klist_insert<K>(key, id, h + 0.5f, shid[j]);
                }
            }
        }
    }
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
        TriSetup s = sv[t];
        int64_t E[3];
#pragma unroll
        for (int i = 0; i < 3; i++) E[i] = dr_edge(s.X, s.Y, i, px, py);
        // perspective division in double: soft fragments extrapolate and the
        // sum of l_i/w_i can come close to zero for grazing triangles
        const double A2 = (double)s.Af;
        double q0 = ((double)E[0] / A2) / (double)s.w[0];
        double q1 = ((double)E[1] / A2) / (double)s.w[1];
        double q2 = ((double)E[2] / A2) / (double)s.w[2];
        double Q = q0 + q1 + q2;
        double b0 = q0 / Q, b1 = q1 / Q, b2 = q2 / Q;
        bool swapped = dr_corner(s.meta, 1) == 2;
        tri_id[o] = t;
        bary[o] = make_float2((float)b0, (float)(swapped ? b2 : b1));
        if (SOFT) {
            int ne;
            float dn = dr_distnorm(s.X, s.Y, px, py, E, dscale, ne);
            dist[o] = key[k] < 0.5f ? dn : -dn;
        }
    }
}

template <int K>
static void launch_raster_k(bool soft, dim3 g, hipStream_t st, const TriSetup *setup,
                            const int32_t *off, const int32_t *bins, int64_t cap, int T, int H,
                            int W, int ntx, int nt, float r, int32_t *tid, float2 *bary,
                            float *dist) {
    if (soft)
        DR_LAUNCH("k_raster", (k_raster<K, true>), g, DRESSI_TILE_PIX, 0, st, setup, off, bins, cap, T, H, W, ntx, nt, r,
                                                         tid, bary, dist);
    else
        DR_LAUNCH("k_raster", (k_raster<K, false>), g, DRESSI_TILE_PIX, 0, st, setup, off, bins, cap, T, H, W, ntx, nt,
                                                          r, tid, bary, dist);
}

static int soft_margin(float r, int W) {
    if (!(r > 0.0f)) return 0;
    return (int)ceilf(r * (float)W) + 1;
}

static int64_t default_bin_capacity(int B, int T, int nt, int margin) {
    int64_t per = 4 + 2 * (int64_t)((margin + DRESSI_TILE - 1) / DRESSI_TILE);
    int64_t cap = (int64_t)B * T * per * per / 4 + (int64_t)B * nt + 4096;
    return cap;
}

static size_t raster_scratch(int B, int T, int nt, int64_t cap, Carver &c, size_t *o) {
    o[0] = c.take(sizeof(TriSetup) * (size_t)B * T);            // setup
    o[1] = c.take(sizeof(int32_t) * (size_t)B * nt);            // counts
    o[2] = c.take(sizeof(int32_t) * ((size_t)B * nt + 1));      // offsets
    o[3] = c.take(sizeof(int32_t) * (size_t)B * nt);            // cursor
    o[4] = c.take(dressi_scan_tmp_bytes((int64_t)B * nt));      // scan tmp
    o[5] = c.take(sizeof(int32_t) * (size_t)cap);               // bins
    return c.off;
}

static int check_raster_args(dressi_ctx *ctx, const void *pos, const void *tris, int B, int V,
                             int T, int H, int W, int K, float r) {
    if (!ctx) return DRESSI_EINVAL;
    if (B < 0 || V < 0 || T < 0 || H <= 0 || W <= 0 || H > 32767 || W > 32767)
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: bad dimensions");
    if (K < 1 || K > DRESSI_MAX_K) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: K must be 1..5");
    if (!(r >= 0.0f && r <= 1.0f)) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: r must be in [0,1]");
    if (T >= (1 << 21) - 1) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: T must be < 2^21-1");
    if ((B * (int64_t)T > 0) && (!pos || !tris))
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: null pos_clip or tris");
    return DRESSI_OK;
}

extern "C" int dressi_rasterize(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B,
                                int V, int T, int H, int W, int K, float r, int cull,
                                int32_t *tri_id, float *bary, float *dist, void *stream) {
    int rc = check_raster_args(ctx, pos_clip, tris, B, V, T, H, W, K, r);
    if (rc) return rc;
    if (!tri_id || !bary) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: null tri_id or bary");
    bool soft = r > 0.0f;
    if (soft && !dist) return dressi_fail(ctx, DRESSI_EINVAL, "rasterize: dist is required when r > 0");
    if (B == 0) return DRESSI_OK;
    hipStream_t st = (hipStream_t)stream;
    int ntx = tiles_x(W), nty = tiles_y(H), nt = ntx * nty;
    int margin = soft_margin(r, W);
    int64_t cap = ctx->bin_capacity;
    int64_t dflt = default_bin_capacity(B, T, nt, margin);
    if (cap < dflt) cap = dflt;
    Carver c;
    size_t o[6];
    raster_scratch(B, T, nt, cap, c, o);
    rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    void *S = ctx->scratch;
    TriSetup *setup = at<TriSetup>(S, o[0]);
    int32_t *counts = at<int32_t>(S, o[1]);
    int32_t *offs = at<int32_t>(S, o[2]);
    int32_t *cursor = at<int32_t>(S, o[3]);
    int32_t *bins = at<int32_t>(S, o[5]);
    int64_t ntri = (int64_t)B * T;
    dressi_fill_i32(counts, 0, (int64_t)B * nt, st);
    dressi_fill_i32(cursor, 0, (int64_t)B * nt, st);
    if (ntri > 0)
        DR_LAUNCH("k_setup_count", (k_setup_count), (int)((ntri + 255) / 256), 256, 0, st, 
            reinterpret_cast<const float4 *>(pos_clip), tris, B, V, T, H, W, cull, margin, ntx, nt,
            setup, counts);
    dressi_exclusive_scan(counts, offs, (int64_t)B * nt, at<void>(S, o[4]), st);
    DR_LAUNCH("k_fill_bins", (k_fill_bins), (int)((ntri + 255) / 256 + 1), 256, 0, st, 
        setup, B, T, ntx, nt, offs, cursor, bins, cap,
        reinterpret_cast<unsigned long long *>(ctx->status));
    dim3 g((unsigned)(B * nt));
    float2 *b2 = reinterpret_cast<float2 *>(bary);
    switch (K) {
    case 1: launch_raster_k<1>(soft, g, st, setup, offs, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    case 2: launch_raster_k<2>(soft, g, st, setup, offs, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    case 3: launch_raster_k<3>(soft, g, st, setup, offs, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    case 4: launch_raster_k<4>(soft, g, st, setup, offs, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    default: launch_raster_k<5>(soft, g, st, setup, offs, bins, cap, T, H, W, ntx, nt, r, tri_id, b2, dist); break;
    }
    return dressi_launch_check(ctx, "rasterize");
}

// ---------------------------------------------------------------------------
// per-tile fragment lists sorted by triangle id
// ---------------------------------------------------------------------------
#define FS_MAXN 2048
#define FS_SENT 0xffffffffu

__global__ void __launch_bounds__(DRESSI_TILE_PIX)
    k_fragsort(const int32_t *__restrict__ tri_id, int K, int H, int W, int ntx, int nt, int np,
               int32_t *__restrict__ n_frag, int32_t *__restrict__ n_rec, uint16_t *__restrict__ frag,
               int32_t *__restrict__ rec_tri, int32_t *__restrict__ rec_start) {
    __shared__ uint32_t keys[FS_MAXN];
    __shared__ int wsum[DRESSI_TILE_PIX / 64];
    const int bt = blockIdx.x;
    const int b = bt / nt, tile = bt - b * nt;
    const int tx = tile % ntx, ty = tile / ntx;
    const int p = threadIdx.x;
    const int x = tx * DRESSI_TILE + (p & (DRESSI_TILE - 1));
    const int y = ty * DRESSI_TILE + p / DRESSI_TILE;
    for (int i = p; i < np; i += DRESSI_TILE_PIX) keys[i] = FS_SENT;
    __syncthreads();
    int any = 0;
    if (x < W && y < H) {
        for (int k = 0; k < K; k++) {
            int t = tri_id[(((int64_t)b * K + k) * H + y) * W + x];
            if (t >= 0) {
                keys[k * DRESSI_TILE_PIX + p] = ((uint32_t)t << 11) | (uint32_t)(k * DRESSI_TILE_PIX + p);
                any = 1;
            }
        }
    }
    if (!__syncthreads_or(any)) {
        if (p == 0) {
            n_frag[bt] = 0;
            n_rec[bt] = 0;
        }
        return;
    }
    // bitonic sort of np keys (np a power of two)
    for (int size = 2; size <= np; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = p; i < (np >> 1); i += DRESSI_TILE_PIX) {
                int lo = 2 * i - (i & (stride - 1));
                int hi = lo + stride;
                bool asc = (lo & size) == 0;
                uint32_t a = keys[lo], c = keys[hi];
                if ((a > c) == asc) {
                    keys[lo] = c;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    // each thread owns a contiguous run of `per` sorted keys
    const int per = np / DRESSI_TILE_PIX;
    const int i0 = p * per;
    int heads = 0, valid = 0;
    for (int j = 0; j < per; j++) {
        uint32_t kv = keys[i0 + j];
        if (kv == FS_SENT) break;
        valid++;
        if (i0 + j == 0 || (keys[i0 + j - 1] >> 11) != (kv >> 11)) heads++;
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
        uint32_t kv = keys[i];
        if (kv == FS_SENT) break;
        frag[base + i] = (uint16_t)(kv & 2047u);
        if (i == 0 || (keys[i - 1] >> 11) != (kv >> 11)) {
            rec_tri[base + r] = (int32_t)(kv >> 11);
            rec_start[base + r] = i;
            r++;
        }
    }
    // number of valid keys = position of the first sentinel (keys are sorted)
    if (valid < per) {
        int i = i0 + valid;
        if (i == 0 || keys[i - 1] != FS_SENT) n_frag[bt] = i;
    } else if (p == DRESSI_TILE_PIX - 1) {
        n_frag[bt] = np;
    }
    if (p == 0) n_rec[bt] = total_heads;
}

size_t dressi_fraglists_bytes(int B, int H, int W, int K) {
    int64_t nt = (int64_t)tiles_x(W) * tiles_y(H);
    int64_t n = (int64_t)B * nt * DRESSI_TILE_PIX * K;
    Carver c;
    c.take(sizeof(int32_t) * B * nt);
    c.take(sizeof(int32_t) * B * nt);
    c.take(sizeof(uint16_t) * n);
    c.take(sizeof(int32_t) * n);
    c.take(sizeof(int32_t) * n);
    return c.off;
}

void dressi_build_fraglists(const int32_t *tri_id, int B, int K, int H, int W, void *scratch,
                            FragLists &fl, hipStream_t s) {
    int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    int64_t n = (int64_t)B * nt * DRESSI_TILE_PIX * K;
    Carver c;
    fl.n_frag = at<int32_t>(scratch, c.take(sizeof(int32_t) * B * nt));
    fl.n_rec = at<int32_t>(scratch, c.take(sizeof(int32_t) * B * nt));
    fl.frag = at<uint16_t>(scratch, c.take(sizeof(uint16_t) * n));
    fl.rec_tri = at<int32_t>(scratch, c.take(sizeof(int32_t) * n));
    fl.rec_start = at<int32_t>(scratch, c.take(sizeof(int32_t) * n));
    int np = 256;
    while (np < DRESSI_TILE_PIX * K) np <<= 1;
    if (B * nt > 0)
        DR_LAUNCH("k_fragsort", (k_fragsort), B * nt, DRESSI_TILE_PIX, 0, s, tri_id, K, H, W, ntx, nt, np, fl.n_frag,
                                                       fl.n_rec, fl.frag, fl.rec_tri, fl.rec_start);
}

// ---------------------------------------------------------------------------
// triangle -> tiles transpose of the per-tile records
// ---------------------------------------------------------------------------
__global__ void k_tt_count(FragLists fl, int K, int T, int nt, int32_t *__restrict__ counts) {
    const int bt = blockIdx.x;
    const int b = bt / nt;
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX * K;
    const int n = fl.n_rec[bt];
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        int t = fl.rec_tri[base + r];
        if (t >= 0 && t < T) atomicAdd(&counts[(int64_t)b * T + t], 1);
    }
}

__global__ void k_tt_fill(FragLists fl, int K, int T, int nt, const int32_t *__restrict__ offsets,
                          int32_t *__restrict__ cursor, int2 *__restrict__ entries) {
    const int bt = blockIdx.x;
    const int b = bt / nt;
    const int64_t base = (int64_t)bt * DRESSI_TILE_PIX * K;
    const int n = fl.n_rec[bt];
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        int t = fl.rec_tri[base + r];
        if (t < 0 || t >= T) continue;
        int64_t bt_t = (int64_t)b * T + t;
        int slot = offsets[bt_t] + atomicAdd(&cursor[bt_t], 1);
        entries[slot] = make_int2(bt, r);
    }
}

__global__ void k_tt_sort(const int32_t *__restrict__ offsets, int2 *__restrict__ entries,
                          int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = offsets[i], e = offsets[i + 1];
    for (int j = a + 1; j < e; j++) {
        int2 v = entries[j];
        int m = j - 1;
        while (m >= a && entries[m].x > v.x) {
            entries[m + 1] = entries[m];
            m--;
        }
        entries[m + 1] = v;
    }
}

size_t dressi_tritiles_bytes(int B, int T, int H, int W, int K) {
    int64_t nt = (int64_t)tiles_x(W) * tiles_y(H);
    int64_t n = (int64_t)B * T;
    Carver c;
    c.take(sizeof(int32_t) * (n + 1));
    c.take(sizeof(int2) * (size_t)B * nt * DRESSI_TILE_PIX * K);
    c.take(sizeof(int32_t) * n);
    c.take(sizeof(int32_t) * n);
    c.take(dressi_scan_tmp_bytes(n));
    return c.off;
}

void dressi_build_tritiles(const FragLists &fl, int B, int T, int K, int H, int W, void *scratch,
                           TriTiles &tt, hipStream_t s) {
    int nt = tiles_x(W) * tiles_y(H);
    int64_t n = (int64_t)B * T;
    Carver c;
    tt.offsets = at<int32_t>(scratch, c.take(sizeof(int32_t) * (n + 1)));
    tt.entries = at<int2>(scratch, c.take(sizeof(int2) * (size_t)B * nt * DRESSI_TILE_PIX * K));
    int32_t *counts = at<int32_t>(scratch, c.take(sizeof(int32_t) * n));
    int32_t *cursor = at<int32_t>(scratch, c.take(sizeof(int32_t) * n));
    void *tmp = at<void>(scratch, c.take(dressi_scan_tmp_bytes(n)));
    dressi_fill_i32(counts, 0, n, s);
    dressi_fill_i32(cursor, 0, n, s);
    if (B * nt > 0) DR_LAUNCH("k_tt_count", (k_tt_count), B * nt, 256, 0, s, fl, K, T, nt, counts);
    dressi_exclusive_scan(counts, tt.offsets, n, tmp, s);
    if (B * nt > 0) DR_LAUNCH("k_tt_fill", (k_tt_fill), B * nt, 256, 0, s, fl, K, T, nt, tt.offsets, cursor, tt.entries);
    if (n > 0) DR_LAUNCH("k_tt_sort", (k_tt_sort), (int)((n + 255) / 256), 256, 0, s, tt.offsets, tt.entries, n);
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
// ---------------------------------------------------------------------------
__global__ void k_rast_bwd_tri(const float4 *__restrict__ pos_clip, const int32_t *__restrict__ tris,
                               int B, int V, int T, int H, int W, int K, int cull, int margin,
                               int ntx, int nt, FragLists fl, const float2 *__restrict__ grad_bary,
                               const float *__restrict__ grad_dist, float *__restrict__ corner_grad) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)B * T) return;
    int b = (int)(gid / T), t = (int)(gid - (int64_t)b * T);
    float *cg = corner_grad + gid * 9;
    const int32_t *tv = tris + 3 * (int64_t)t;
    int vid[3] = {tv[0], tv[1], tv[2]};
    bool ok = vid[0] >= 0 && vid[0] < V && vid[1] >= 0 && vid[1] < V && vid[2] >= 0 && vid[2] < V;
    TriSetup s;
    if (ok) s = dr_setup(pos_clip + (int64_t)b * V, vid[0], vid[1], vid[2], H, W, cull, margin);
    if (!ok || !(s.meta & 1)) {
#pragma unroll
        for (int i = 0; i < 9; i++) cg[i] = 0.0f;
        return;
    }
    float sx[3], sy[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        sx[i] = (float)s.X[i] * (1.0f / 256.0f);
        sy[i] = (float)s.Y[i] * (1.0f / 256.0f);
    }
    const double A2d = (double)s.Af;
    const double A = A2d * (1.0 / 65536.0);
    // grad_p lambda_i (pixel units), edge i from a = i+1 to c = i+2
    double glx[3], gly[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        int a = (i + 1) % 3, c = (i + 2) % 3;
        glx[i] = -((double)s.Y[c] - (double)s.Y[a]) * (1.0 / 256.0) / A;
        gly[i] = ((double)s.X[c] - (double)s.X[a]) * (1.0 / 256.0) / A;
    }
    const bool swapped = dr_corner(s.meta, 1) == 2;
    const float dscale = (float)W * 256.0f;
    const float invW = 1.0f / (float)W;
    double gsx[3] = {0, 0, 0}, gsy[3] = {0, 0, 0}, gw[3] = {0, 0, 0};
    int tx0 = (s.box0 & 0xffff) / DRESSI_TILE, tx1 = (s.box0 >> 16) / DRESSI_TILE;
    int ty0 = (s.box1 & 0xffff) / DRESSI_TILE, ty1 = (s.box1 >> 16) / DRESSI_TILE;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            int64_t bt = (int64_t)b * nt + ty * ntx + tx;
            int64_t base = bt * DRESSI_TILE_PIX * K;
            int j0, j1;
            frag_range(fl, bt, base, t, j0, j1);
            for (int j = j0; j < j1; j++) {
                int f = fl.frag[base + j];
                int k = f >> 8, pl = f & 255;
                int x = tx * DRESSI_TILE + (pl & 15), y = ty * DRESSI_TILE + (pl >> 4);
                int64_t o = (((int64_t)b * K + k) * H + y) * W + x;
                int px = DRESSI_SUBPIX * x + DRESSI_SUBPIX / 2, py = DRESSI_SUBPIX * y + DRESSI_SUBPIX / 2;
                int64_t E[3];
                bool in = true;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    E[i] = dr_edge(s.X, s.Y, i, px, py);
                    bool own = (s.meta >> (1 + i)) & 1;
                    in = in && (E[i] > 0 || (E[i] == 0 && own));
                }
                // the barycentric chain runs in double (see the forward)
                double l[3], q[3];
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    l[i] = (double)E[i] / A2d;
                    q[i] = l[i] / (double)s.w[i];
                }
                double Q = q[0] + q[1] + q[2];
                float2 g2 = grad_bary[o];
                // gradient on the normalised-order barycentrics (original corner 2 has none)
                double gb[3] = {g2.x, swapped ? 0.0 : (double)g2.y, swapped ? (double)g2.y : 0.0};
                double sb = (gb[0] * q[0] + gb[1] * q[1] + gb[2] * q[2]) / Q;
                double Gx = 0.0, Gy = 0.0;
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    double wi = (double)s.w[i];
                    double gq = (gb[i] - sb) / Q;
                    double gl = gq / wi;
                    gw[i] -= gq * l[i] / (wi * wi);
                    Gx += gl * glx[i];
                    Gy += gl * gly[i];
                }
#pragma unroll
                for (int i = 0; i < 3; i++) {
                    gsx[i] -= l[i] * Gx;
                    gsy[i] -= l[i] * Gy;
                }
                if (grad_dist) {
                    float g = grad_dist[o];
                    int ne;
                    dr_distnorm(s.X, s.Y, px, py, E, dscale, ne);
                    int a = (ne + 1) % 3, c = (ne + 2) % 3;
                    float Px = (float)x + 0.5f, Py = (float)y + 0.5f;
                    float ex = sx[c] - sx[a], ey = sy[c] - sy[a];
                    float tt = ((Px - sx[a]) * ex + (Py - sy[a]) * ey) / (ex * ex + ey * ey);
                    tt = fminf(fmaxf(tt, 0.0f), 1.0f);
                    float cx = sx[a] + tt * ex, cy = sy[a] + tt * ey;
                    float dx = Px - cx, dy = Py - cy;
                    float d = sqrtf(dx * dx + dy * dy);
                    if (d > 0.0f && g != 0.0f) {
                        float sg = (in ? g : -g) * invW / d;
                        gsx[a] -= sg * (1.0f - tt) * dx;
                        gsy[a] -= sg * (1.0f - tt) * dy;
                        gsx[c] -= sg * tt * dx;
                        gsy[c] -= sg * tt * dy;
                    }
                }
            }
        }
    // screen -> clip: x_s = (x/w + 1) W/2, y_s = (1 - y/w) H/2
    const float hw = 0.5f * (float)W, hh = 0.5f * (float)H;
    const float4 *pc = pos_clip + (int64_t)b * V;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        int corner = dr_corner(s.meta, i);
        float4 p = pc[vid[corner]];
        float xn = p.x / p.w, yn = p.y / p.w;
        double w = p.w;
        double gx = gsx[i] * hw / w;
        double gy = -gsy[i] * hh / w;
        double gww = (-gsx[i] * hw * xn + gsy[i] * hh * yn) / w + gw[i];
        cg[corner * 3 + 0] = (float)gx;
        cg[corner * 3 + 1] = (float)gy;
        cg[corner * 3 + 2] = (float)gww;
    }
}

// one thread per (view, vertex): sum the corner gradients of its triangles in
// ascending corner order
__global__ void k_vertex_gather_pos(const float *__restrict__ corner_grad, Adjacency adj, int B,
                                    int V, int T, float4 *__restrict__ grad_pos) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)B * V) return;
    int b = (int)(gid / V), v = (int)(gid - (int64_t)b * V);
    float gx = 0.0f, gy = 0.0f, gw = 0.0f;
    const float *cgb = corner_grad + (int64_t)b * T * 9;
    for (int j = adj.offsets[v]; j < adj.offsets[v + 1]; j++) {
        int c = adj.corners[j];
        const float *g = cgb + (int64_t)(c / 3) * 9 + (c % 3) * 3;
        gx += g[0];
        gy += g[1];
        gw += g[2];
    }
    grad_pos[gid] = make_float4(gx, gy, 0.0f, gw);
}

extern "C" int dressi_rasterize_bwd(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                                    int B, int V, int T, int H, int W, int K, float r, int cull,
                                    const int32_t *tri_id, const float *grad_bary,
                                    const float *grad_dist, float *grad_pos_clip, void *stream) {
    int rc = check_raster_args(ctx, pos_clip, tris, B, V, T, H, W, K, r);
    if (rc) return rc;
    if (!tri_id || !grad_bary || (!grad_pos_clip && B * (int64_t)V > 0))
        return dressi_fail(ctx, DRESSI_EINVAL, "rasterize_bwd: null tri_id, grad_bary or grad_pos_clip");
    if (B == 0 || V == 0) return DRESSI_OK;
    hipStream_t st = (hipStream_t)stream;
    int ntx = tiles_x(W), nt = ntx * tiles_y(H);
    int margin = soft_margin(r, W);
    Carver c;
    size_t o_fl = c.take(dressi_fraglists_bytes(B, H, W, K));
    size_t o_adj = c.take(dressi_adjacency_bytes(V, T));
    size_t o_cg = c.take(sizeof(float) * 9 * (size_t)B * T);
    rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    void *S = ctx->scratch;
    FragLists fl;
    dressi_build_fraglists(tri_id, B, K, H, W, at<void>(S, o_fl), fl, st);
    Adjacency adj;
    dressi_build_adjacency(tris, T, V, at<void>(S, o_adj), adj, st);
    float *cg = at<float>(S, o_cg);
    int64_t ntri = (int64_t)B * T;
    if (ntri > 0)
        DR_LAUNCH("k_rast_bwd_tri", (k_rast_bwd_tri), (int)((ntri + 127) / 128), 128, 0, st, 
            reinterpret_cast<const float4 *>(pos_clip), tris, B, V, T, H, W, K, cull, margin, ntx,
            nt, fl, reinterpret_cast<const float2 *>(grad_bary), grad_dist, cg);
    int64_t nv = (int64_t)B * V;
    DR_LAUNCH("k_vertex_gather_pos", (k_vertex_gather_pos), (int)((nv + 255) / 256), 256, 0, st, 
        cg, adj, B, V, T, reinterpret_cast<float4 *>(grad_pos_clip));
    return dressi_launch_check(ctx, "rasterize_bwd");
}

// ---------------------------------------------------------------------------
// worst-case scratch of one call of each kind, for dressi_reserve
// ---------------------------------------------------------------------------
extern "C" size_t dressi_scratch_bytes(int B, int V, int T, int H, int W, int K, float r, int Va,
                                       int C, int64_t tex_cells, int tex_slices) {
    if (B < 0 || V < 0 || T < 0 || H < 0 || W < 0 || K < 1) return 0;
    int nt = tiles_x(W) * tiles_y(H);
    int margin = soft_margin(r, W);
    size_t need = 0;
    {
        Carver c;
        size_t o[6];
        raster_scratch(B, T, nt, default_bin_capacity(B, T, nt, margin), c, o);
        need = c.off > need ? c.off : need;
    }
    {
        Carver c;
        c.take(dressi_fraglists_bytes(B, H, W, K));
        c.take(dressi_adjacency_bytes(V, T));
        c.take(sizeof(float) * 9 * (size_t)B * T);
        need = c.off > need ? c.off : need;
    }
    {
        Carver c;
        c.take(dressi_fraglists_bytes(B, H, W, K));
        c.take(dressi_tritiles_bytes(B, T, H, W, K));
        c.take(dressi_adjacency_bytes(Va > V ? Va : V, T));
        c.take(sizeof(float) * 3 * (size_t)(C > 0 ? C : 1) * B * T);
        need = c.off > need ? c.off : need;
    }
    {
        Carver c;
        c.take(sizeof(int32_t) * (size_t)tex_cells * (tex_slices > 0 ? tex_slices : 1));
        need = c.off > need ? c.off : need;
    }
    {
        Carver c;
        c.take((size_t)B * H * W);
        c.take((size_t)B * H * W);
        need = c.off > need ? c.off : need;
    }
    return need;
}
