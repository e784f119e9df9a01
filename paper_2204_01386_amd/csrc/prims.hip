// Small device primitives of libdressi: fills, a multi-block exclusive scan,
// and the vertex -> corner adjacency used by the deterministic gathers.
#include "dressi_internal.h"

// ---------------------------------------------------------------------------
// fills (used instead of hipMemsetAsync so every call stays graph-safe)
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static int fill_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    return g < 1 ? 1 : (int)g;
}

void dressi_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    DR_LAUNCH("k_fill_i32", (k_fill_i32), fill_grid(n), 256, 0, s, p, v, n);
}

void dressi_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    DR_LAUNCH("k_fill_f32", (k_fill_f32), fill_grid(n), 256, 0, s, p, v, n);
}

// ---------------------------------------------------------------------------
// multi-block exclusive scan (block_exclusive_scan and the chunk bodies are
// in dressi_internal.h, shared with the whole step's co-launched jobs)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(SCAN_BS) k_scan_reduce(const int32_t *in, int64_t n,
                                                         int32_t *block_sums) {
    scan_reduce_block(in, n, block_sums, (int)blockIdx.x);
}

// single block: exclusive scan of the block sums in place
__global__ void __launch_bounds__(1024) k_scan_blocks(int32_t *sums, int nb) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int start = 0; start < nb; start += 1024) {
        int i = start + threadIdx.x;
        int v = i < nb ? sums[i] : 0;
        int total;
        int ex = block_exclusive_scan<1024>(v, total, wsum);
        if (i < nb) sums[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(SCAN_BS) k_scan_apply(const int32_t *in, int32_t *out, int64_t n,
                                                        const int32_t *block_offsets) {
    __shared__ int wsum[SCAN_BS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
    int v[SCAN_PER];
    int s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        s += v[j];
    }
    int total;
    int ex = block_exclusive_scan<SCAN_BS>(s, total, wsum) + block_offsets[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_PER; j++) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BS - 1) out[n] = ex;
}

// The same, where each block first adds up the totals of the blocks before
// it (at most SCAN_DIRECT_MAX of them, from L2) instead of reading a scanned
// copy: one launch fewer than reduce, scan of the totals, apply.
__global__ void __launch_bounds__(SCAN_BS) k_scan_apply_direct(const int32_t *in, int32_t *out, int64_t n,
                                                               const int32_t *block_sums) {
    scan_apply_direct_block(in, out, n, block_sums, (int)blockIdx.x, (int)gridDim.x);
}

// whole scan in one workgroup (small n): chunks of 4096 with a running carry
__global__ void __launch_bounds__(1024) k_scan_single(const int32_t *in, int32_t *out, int64_t n) {
    __shared__ int wsum[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += 4096) {
        int64_t i0 = c0 + 4 * (int64_t)threadIdx.x;
        int v[4];
        int sum = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            v[j] = i0 + j < n ? in[i0 + j] : 0;
            sum += v[j];
        }
        int total;
        int ex = block_exclusive_scan<1024>(sum, total, wsum) + carry;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (i0 + j < n) out[i0 + j] = ex;
            ex += v[j];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

size_t dressi_scan_tmp_bytes(int64_t n) {
    int64_t nb = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    return (size_t)(nb + 1) * sizeof(int32_t);
}

void dressi_exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *tmp, hipStream_t s) {
    if (n <= 0) {
        dressi_fill_i32(out, 0, 1, s);
        return;
    }
    if (n <= 16384) {
        DR_LAUNCH("k_scan_single", (k_scan_single), 1, 1024, 0, s, in, out, n);
        return;
    }
    int nb = (int)((n + SCAN_CHUNK - 1) / SCAN_CHUNK);
    int32_t *sums = static_cast<int32_t *>(tmp);
    DR_LAUNCH("k_scan_reduce", (k_scan_reduce), nb, SCAN_BS, 0, s, in, n, sums);
    if (nb <= SCAN_DIRECT_MAX) {
        DR_LAUNCH("k_scan_apply", (k_scan_apply_direct), nb, SCAN_BS, 0, s, in, out, n, sums);
        return;
    }
    DR_LAUNCH("k_scan_blocks", (k_scan_blocks), 1, 1024, 0, s, sums, nb);
    DR_LAUNCH("k_scan_apply", (k_scan_apply), nb, SCAN_BS, 0, s, in, out, n, sums);
}

// ---------------------------------------------------------------------------
// vertex -> corner adjacency (CSR), each vertex's corners in ascending order
// ---------------------------------------------------------------------------
__global__ void k_count_corners(const int32_t *tris, int64_t n3, int V, int32_t *counts, int32_t *nlong) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) *nlong = 0;   // the long-list queue of k_sort_corners, read after this launch
    if (c >= n3) return;
    int v = tris[c];
    if (v >= 0 && v < V) atomicAdd(&counts[v], 1);
}

__global__ void k_place_corners(const int32_t *tris, int64_t n3, int V, const int32_t *offsets,
                                int32_t *cursor, int32_t *corners) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n3) return;
    int v = tris[c];
    if (v < 0 || v >= V) return;
    int slot = offsets[v] + atomicAdd(&cursor[v], 1);
    corners[slot] = (int32_t)c;
}

// The atomics above place corners in arbitrary order: every list is sorted so
// that gathers sum in a fixed order.  Lists of up to ADJ_SHORT corners are
// insertion-sorted by one thread; longer ones (a vertex of high valence) are
// queued for k_sort_corners_long, at most n3 / (ADJ_SHORT + 1) of them.
#define ADJ_SHORT 64
__global__ void k_sort_corners(const int32_t *offsets, int32_t *corners, int V, int32_t *nlong,
                               int32_t *longv, int cap) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    int a = offsets[v], b = offsets[v + 1];
    if (b - a > ADJ_SHORT) {
        const int q = atomicAdd(nlong, 1);
        if (q < cap) longv[q] = v;
        return;
    }
    for (int i = a + 1; i < b; i++) {
        int x = corners[i];
        int j = i - 1;
        while (j >= a && corners[j] > x) {
            corners[j + 1] = corners[j];
            j--;
        }
        corners[j + 1] = x;
    }
}

// One workgroup per queued list: a bottom-up merge sort between the list and
// its stretch of `tmp`, runs of width 1, 2, 4, ...  The corner indices of a
// list are distinct, so each corner's place in its merged pair of runs is its
// rank in its own run plus the number of smaller corners in the other run,
// found by binary search.
__global__ void __launch_bounds__(1024) k_sort_corners_long(const int32_t *offsets, int32_t *corners, int32_t *tmp,
                                                           const int32_t *nlong, const int32_t *longv, int cap) {
    const int nq = min(*nlong, cap);
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int v = longv[q];
        const int a = offsets[v], n = offsets[v + 1] - a;
        int32_t *src = corners + a, *dst = tmp + a;
        for (int w = 1; w < n; w <<= 1) {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                const int x = src[i];
                const int r = i / w;
                const int own = r * w, base = (r & ~1) * w;
                const int ps = (r ^ 1) * w, pe = min(ps + w, n);
                int lo = ps, hi = max(ps, pe);
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (src[mid] < x) lo = mid + 1;
                    else hi = mid;
                }
                dst[base + (i - own) + (lo - ps)] = x;
            }
            __syncthreads();
            int32_t *t = src;
            src = dst;
            dst = t;
        }
        if (src != corners + a)
            for (int i = threadIdx.x; i < n; i += blockDim.x) corners[a + i] = src[i];
        __syncthreads();
    }
}

static size_t adj_long_cap(int T) { return 3 * (size_t)T / (ADJ_SHORT + 1) + 1; }

size_t dressi_adjacency_tmp_bytes(int V, int T) {
    Carver c;
    c.take(sizeof(int32_t) * (size_t)V);                     // counts
    c.take(sizeof(int32_t) * (size_t)V);                     // cursor
    c.take(dressi_scan_tmp_bytes(V));
    c.take(sizeof(int32_t) * (1 + adj_long_cap(T)));         // long-list queue: count, vertices
    c.take(sizeof(int32_t) * 3 * (size_t)T);                 // merge-sort buffer
    return c.off;
}

void dressi_build_adjacency_into(const int32_t *tris, int T, int V, int32_t *buf, void *tmp,
                                 hipStream_t s) {
    Adjacency adj = adjacency_view(buf, V);
    Carver c;
    int32_t *counts = at<int32_t>(tmp, c.take(sizeof(int32_t) * (size_t)V));
    int32_t *cursor = at<int32_t>(tmp, c.take(sizeof(int32_t) * (size_t)V));
    void *stmp = at<void>(tmp, c.take(dressi_scan_tmp_bytes(V)));
    const int cap = (int)adj_long_cap(T);
    int32_t *nlong = at<int32_t>(tmp, c.take(sizeof(int32_t) * (1 + (size_t)cap)));
    int32_t *longv = nlong + 1;
    int32_t *sbuf = at<int32_t>(tmp, c.take(sizeof(int32_t) * 3 * (size_t)T));
    int64_t n3 = 3 * (int64_t)T;
    dressi_fill_i32(counts, 0, 2 * (int64_t)((sizeof(int32_t) * (size_t)V + 255) / 256 * 64), s);
    if (n3 > 0)
        DR_LAUNCH("k_count_corners", (k_count_corners), (int)((n3 + 255) / 256), 256, 0, s, tris, n3, V, counts,
                  nlong);
    dressi_exclusive_scan(counts, adj.offsets, V, stmp, s);
    if (n3 > 0)
        DR_LAUNCH("k_place_corners", (k_place_corners), (int)((n3 + 255) / 256), 256, 0, s, tris, n3, V, adj.offsets, cursor,
                                                               adj.corners);
    if (V > 0 && n3 > 0) {
        DR_LAUNCH("k_sort_corners", (k_sort_corners), (V + 255) / 256, 256, 0, s, adj.offsets, adj.corners, V, nlong,
                  longv, cap);
        DR_LAUNCH("k_sort_corners", (k_sort_corners_long), 64, 1024, 0, s, adj.offsets, adj.corners, sbuf, nlong,
                  longv, cap);
    }
}

extern "C" int dressi_adjacency(dressi_ctx *ctx, const int32_t *tris, int T, int V, int32_t *adj,
                                void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (T < 0 || V < 0) return dressi_fail(ctx, DRESSI_EINVAL, "adjacency: bad dimensions");
    if (!adj || (T > 0 && !tris)) return dressi_fail(ctx, DRESSI_EINVAL, "adjacency: null pointer");
    hipStream_t st = (hipStream_t)stream;
    int rc = dressi_scratch(ctx, dressi_adjacency_tmp_bytes(V, T), st);
    if (rc) return rc;
    dressi_build_adjacency_into(tris, T, V, adj, ctx->scratch, st);
    return dressi_launch_check(ctx, "adjacency");
}
