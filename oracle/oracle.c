/*
 * CPU oracle for the Dressi rasterization hot path (test infrastructure).
 *
 * This file is the plain, slow reference that the GPU library is checked
 * against.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it; the product path never does.  It shares no source, header
 * or helper with the HIP library.
 *
 * Precision: every value is computed in double precision.  Where a floating
 * point quantity decides an integer result (vertex snapping, the depth key, the
 * soft-distance test and key, texel and cell selection, the edge-mask radius),
 * the decision is taken in single precision with the operation order written
 * out below, because the method's visibility is defined by those discrete
 * choices and both implementations must take them identically.
 *
 * Paper references (Dressi, Eurographics 2022):
 *   - rendering decomposition and loss: §3.4.1;
 *   - HardSoftRas rasterization: Algorithm 2, §3.4.2 (Enlarge, SignedDist,
 *     the Shift depth equation, depth peeling with K buffers);
 *   - shading and blending: §3.4.3 (probability D_k = sigmoid(dist_k/sigma),
 *     the edge/non-edge blend, colour and silhouette equations);
 *   - inverse UV texture: §3.3.2, Algorithm 1;
 *   - the listings of the appendix (BuildRasterize, BuildBlend, PeelDepth)
 *     for the order of operations.
 * Readings of passages the paper leaves open are stated where they are used.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

#define SUBPIX 256 /* 8 sub-pixel bits */

/* ------------------------------------------------------------------------ */
/* Triangle setup                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ok;           /* rasterizable */
    int v[3];         /* vertex ids, reordered so that the area is positive */
    int corner[3];    /* corner[i] = corner of tris[t] that vertex i came from */
    int64_t X[3], Y[3]; /* snapped fixed-point screen coords (1/256 px)       */
    int64_t A2;       /* twice the (positive) area in fixed point^2           */
    float zn[3];      /* z/w in single precision (depth-key input)            */
    double w[3];      /* clip w                                               */
    double xn[3], yn[3]; /* x/w, y/w in double (used for the unsnapped mode)  */
} otri;

/* Viewport snap: x_px = (x/w + 1) * W/2 and y_px = (1 - y/w) * H/2 in float,
 * then round-to-nearest-even of x_px * 256.  Rejects coordinates outside the
 * +-2^22 guard band (also catches NaN). */
static int snap_f32(float c, float w, float half, int is_y, int64_t *out)
{
    float n = c / w;
    float p = is_y ? (1.0f - n) * half : (n + 1.0f) * half;
    float f = p * 256.0f;
    if (!(fabsf(f) < 4194304.0f)) return 0;
    *out = (int64_t)nearbyintf(f);
    return 1;
}

static otri setup_tri(const float *pc, const int32_t *tri, int H, int W, int cull)
{
    otri s;
    memset(&s, 0, sizeof s);
    float hw = 0.5f * (float)W, hh = 0.5f * (float)H;
    int64_t X[3], Y[3];
    float zn[3];
    for (int i = 0; i < 3; i++) {
        const float *p = pc + 4 * (int64_t)tri[i];
        if (!(p[3] > 0.0f)) return s;            /* behind the eye: dropped */
        if (!snap_f32(p[0], p[3], hw, 0, &X[i])) return s;
        if (!snap_f32(p[1], p[3], hh, 1, &Y[i])) return s;
        zn[i] = p[2] / p[3];
    }
    int64_t A2 = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
    if (A2 == 0) return s;                       /* degenerate: dropped */
    /* Screen y points down, so a positive A2 is clockwise in NDC (y up), i.e.
     * a back face for counter-clockwise front faces. */
    if (cull && A2 > 0) return s;
    int order[3] = {0, 1, 2};
    if (A2 < 0) { order[1] = 2; order[2] = 1; A2 = -A2; }
    for (int i = 0; i < 3; i++) {
        int c = order[i];
        const float *p = pc + 4 * (int64_t)tri[c];
        s.v[i] = tri[c];
        s.corner[i] = c;
        s.X[i] = X[c];
        s.Y[i] = Y[c];
        s.zn[i] = zn[c];
        s.w[i] = (double)p[3];
        s.xn[i] = (double)p[0] / (double)p[3];
        s.yn[i] = (double)p[1] / (double)p[3];
    }
    s.A2 = A2;
    s.ok = 1;
    return s;
}

/* Edge function of the edge opposite vertex i (from vertex i+1 to i+2),
 * evaluated at fixed-point point (px, py).  E_i(v_i) = A2 > 0. */
static int64_t edge_fn(const otri *s, int i, int64_t px, int64_t py)
{
    int a = (i + 1) % 3, b = (i + 2) % 3;
    return (s->X[b] - s->X[a]) * (py - s->Y[a]) - (s->Y[b] - s->Y[a]) * (px - s->X[a]);
}

/* Fill convention (the paper relies on the hardware's): a sample exactly on an
 * edge belongs to the triangle that contains the sample nudged by an
 * infinitesimal (eps, eps^2) to the right and down.  For E = dx*(py-ya) -
 * dy*(px-xa) this owns E == 0 iff dy < 0, or dy == 0 and dx > 0 (the usual
 * top-left rule).  Every point is thus covered exactly once by a tiling. */
static int edge_owns_zero(const otri *s, int i)
{
    int a = (i + 1) % 3, b = (i + 2) % 3;
    int64_t dx = s->X[b] - s->X[a], dy = s->Y[b] - s->Y[a];
    return dy < 0 || (dy == 0 && dx > 0);
}

static int covers(const otri *s, int64_t px, int64_t py, int64_t E[3])
{
    int in = 1;
    for (int i = 0; i < 3; i++) {
        E[i] = edge_fn(s, i, px, py);
        if (!(E[i] > 0 || (E[i] == 0 && edge_owns_zero(s, i)))) in = 0;
    }
    return in;
}

/* Depth key input: z = z0 + l1*(z1-z0) + l2*(z2-z0) with l_i = E_i/A2, all in
 * float (int64 -> float rounds to nearest), summed left to right. */
static float depth_f32(const otri *s, const int64_t E[3])
{
    float A = (float)s->A2;
    float l1 = (float)E[1] / A;
    float l2 = (float)E[2] / A;
    float d1 = s->zn[1] - s->zn[0];
    float d2 = s->zn[2] - s->zn[0];
    float t1 = l1 * d1;
    float t2 = l2 * d2;
    float z = s->zn[0] + t1;
    return z + t2;
}

/* Distance (fixed-point units) from (px,py) to the closed segment of edge i,
 * evaluated in float from exact integer dot products. */
static float seg_dist_f32(const otri *s, int i, int64_t px, int64_t py, int64_t E)
{
    int a = (i + 1) % 3, b = (i + 2) % 3;
    int64_t ex = s->X[b] - s->X[a], ey = s->Y[b] - s->Y[a];
    int64_t qx = px - s->X[a], qy = py - s->Y[a];
    int64_t dot = qx * ex + qy * ey;
    int64_t len2 = ex * ex + ey * ey;
    if (dot <= 0) return sqrtf((float)(qx * qx + qy * qy));
    if (dot >= len2) {
        int64_t rx = px - s->X[b], ry = py - s->Y[b];
        return sqrtf((float)(rx * rx + ry * ry));
    }
    int64_t ae = E < 0 ? -E : E;
    return (float)ae / sqrtf((float)len2);
}

/* SignedDist magnitude decision (§3.4.2): the pixel's distance to the triangle
 * boundary, i.e. the minimum over the three edge segments, in [0,1] screen
 * units (pixels / W).  Returns the nearest edge (lowest index on ties). */
static float dist_norm_f32(const otri *s, int64_t px, int64_t py, const int64_t E[3],
                           int W, int *nearest)
{
    float best = 0.0f;
    int bi = 0;
    for (int i = 0; i < 3; i++) {
        float d = seg_dist_f32(s, i, px, py, E[i]);
        if (i == 0 || d < best) { best = d; bi = i; }
    }
    if (nearest) *nearest = bi;
    return best / ((float)W * 256.0f);
}

/* ------------------------------------------------------------------------ */
/* Rasterization with K layers (Algorithm 2, Shift, PeelDepth)              */
/* ------------------------------------------------------------------------ */

typedef struct { float key; int32_t id; } frag;

/* Layer k of a pixel is the k-th smallest *distinct* key among all of the
 * pixel's fragments, carried by the smallest triangle id at that key.  This is
 * what K passes of depth peeling give: PeelDepth discards keys <= the previous
 * layer's key, and a LESS depth test keeps the first (lowest-id) primitive
 * among equal keys.  The running list below is insertion into a sorted list of
 * at most K distinct keys, which yields the same set in any visiting order. */
static void klist_insert(frag *L, int *n, int K, float key, int32_t id)
{
    for (int j = 0; j < *n; j++) {
        if (L[j].key == key) { if (id < L[j].id) L[j].id = id; return; }
    }
    int pos = *n;
    while (pos > 0 && key < L[pos - 1].key) pos--;
    if (pos >= K) return;
    int last = (*n < K) ? *n : K - 1;
    for (int j = last; j > pos; j--) L[j] = L[j - 1];
    L[pos].key = key;
    L[pos].id = id;
    if (*n < K) (*n)++;
}

static void resolve_one(const otri *s, int px_i, int py_i, int hard, int snap,
                        int H, int W, double *b0, double *b1, double *dist);

/* The K layers of the pixels of the window [wx0, wx0 + ww) x [wy0, wy0 + wh)
 * of an H x W image; every triangle is considered, only the window's pixels
 * are visited and stored ([B,K,wh,ww] outputs).  The full image is the window
 * (0, 0, W, H). */
int orc_rasterize_window(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                         int H, int W, int K, float r, int cull, int wx0, int wy0, int ww, int wh,
                         int32_t *tri_id, uint8_t *hard, double *bary, double *dist)
{
    if (B < 0 || V < 0 || T < 0 || H <= 0 || W <= 0 || K < 1 || K > 5) return -1;
    if (!(r >= 0.0f && r <= 1.0f)) return -1;
    if (wx0 < 0 || wy0 < 0 || ww <= 0 || wh <= 0 || wx0 + ww > W || wy0 + wh > H) return -1;
    int64_t N = (int64_t)wh * ww;
    frag *lists = (frag *)malloc(sizeof(frag) * (size_t)(N * K));
    int *cnt = (int *)malloc(sizeof(int) * (size_t)N);
    if (!lists || !cnt) { free(lists); free(cnt); return -2; }
    /* pixels within r of a triangle lie at most ceil(r*W) + 2 pixels from its bbox */
    int margin = (r > 0.0f) ? (int)ceil((double)r * W) + 2 : 0;
    for (int b = 0; b < B; b++) {
        const float *pc = pos_clip + (int64_t)b * V * 4;
        memset(cnt, 0, sizeof(int) * (size_t)N);
        for (int t = 0; t < T; t++) {
            otri s = setup_tri(pc, tris + 3 * (int64_t)t, H, W, cull);
            if (!s.ok) continue;
            int64_t xmin = s.X[0], xmax = s.X[0], ymin = s.Y[0], ymax = s.Y[0];
            for (int i = 1; i < 3; i++) {
                if (s.X[i] < xmin) xmin = s.X[i];
                if (s.X[i] > xmax) xmax = s.X[i];
                if (s.Y[i] < ymin) ymin = s.Y[i];
                if (s.Y[i] > ymax) ymax = s.Y[i];
            }
            int64_t x0 = (int64_t)floor(xmin / 256.0) - 1 - margin;
            int64_t x1 = (int64_t)ceil(xmax / 256.0) + 1 + margin;
            int64_t y0 = (int64_t)floor(ymin / 256.0) - 1 - margin;
            int64_t y1 = (int64_t)ceil(ymax / 256.0) + 1 + margin;
            if (x0 < wx0) x0 = wx0;
            if (y0 < wy0) y0 = wy0;
            if (x1 > wx0 + ww - 1) x1 = wx0 + ww - 1;
            if (y1 > wy0 + wh - 1) y1 = wy0 + wh - 1;
            for (int64_t y = y0; y <= y1; y++) {
                for (int64_t x = x0; x <= x1; x++) {
                    int64_t px = SUBPIX * x + SUBPIX / 2, py = SUBPIX * y + SUBPIX / 2;
                    int64_t E[3];
                    float key;
                    if (covers(&s, px, py, E)) {
                        /* hard fragment: Shift gives 0.5 * depth */
                        float z = depth_f32(&s, E);
                        if (!(z > 0.0f && z < 1.0f)) continue;
                        key = 0.5f * z;
                    } else {
                        if (!(r > 0.0f)) continue;
                        /* soft fragment: Shift gives 0.5 * |dist| + 0.5 */
                        float dn = dist_norm_f32(&s, px, py, E, W, NULL);
                        if (!(dn <= r)) continue;
                        float h = 0.5f * dn;
                        key = h + 0.5f;
                    }
                    int64_t p = (y - wy0) * ww + (x - wx0);
                    klist_insert(lists + p * K, &cnt[p], K, key, t);
                }
            }
        }
        for (int64_t p = 0; p < N; p++) {
            int y = wy0 + (int)(p / ww), x = wx0 + (int)(p % ww);
            for (int k = 0; k < K; k++) {
                int64_t o = ((int64_t)b * K + k) * N + p;
                if (k < cnt[p]) {
                    int32_t t = lists[p * K + k].id;
                    tri_id[o] = t;
                    /* hard keys are < 0.5, soft keys >= 0.5 */
                    int hd = lists[p * K + k].key < 0.5f;
                    if (hard) hard[o] = (uint8_t)hd;
                    otri s = setup_tri(pc, tris + 3 * (int64_t)t, H, W, cull);
                    double b0, b1, d;
                    resolve_one(&s, x, y, hd, 1, H, W, &b0, &b1, &d);
                    if (bary) { bary[2 * o] = b0; bary[2 * o + 1] = b1; }
                    if (dist) dist[o] = d;
                } else {
                    tri_id[o] = -1;
                    if (hard) hard[o] = 0;
                    if (bary) { bary[2 * o] = 0.0; bary[2 * o + 1] = 0.0; }
                    if (dist) dist[o] = 0.0;
                }
            }
        }
    }
    free(lists);
    free(cnt);
    return 0;
}

int orc_rasterize(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                  int H, int W, int K, float r, int cull,
                  int32_t *tri_id, uint8_t *hard, double *bary, double *dist)
{
    return orc_rasterize_window(pos_clip, tris, B, V, T, H, W, K, r, cull, 0, 0, W, H,
                                tri_id, hard, bary, dist);
}

/* ------------------------------------------------------------------------ */
/* Resolve: barycentrics and signed distance for a frozen fragment          */
/* ------------------------------------------------------------------------ */

/* Screen-space vertex positions in pixels: the snapped ones (X/256) when
 * snap != 0, otherwise the exact ones computed in double (used for finite
 * differences, where snapping would make the values piecewise constant). */
static void screen_xy(const otri *s, int snap, int H, int W, double sx[3], double sy[3])
{
    for (int i = 0; i < 3; i++) {
        if (snap) {
            sx[i] = (double)s->X[i] / SUBPIX;
            sy[i] = (double)s->Y[i] / SUBPIX;
        } else {
            sx[i] = (s->xn[i] + 1.0) * 0.5 * W;
            sy[i] = (1.0 - s->yn[i]) * 0.5 * H;
        }
    }
}

/* Screen-linear barycentrics lambda_i = E_i / A2 (double), E_i for the edge
 * opposite vertex i.  Soft fragments extrapolate (no clamping). */
static void lambdas(const double sx[3], const double sy[3], double px, double py, double l[3])
{
    double A = (sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]);
    for (int i = 0; i < 3; i++) {
        int a = (i + 1) % 3, b = (i + 2) % 3;
        double E = (sx[b] - sx[a]) * (py - sy[a]) - (sy[b] - sy[a]) * (px - sx[a]);
        l[i] = E / A;
    }
}

/* Closest point parameter on the segment of edge i and the distance to it. */
static double seg_dist_d(const double sx[3], const double sy[3], int i, double px, double py,
                         double *t_out)
{
    int a = (i + 1) % 3, b = (i + 2) % 3;
    double ex = sx[b] - sx[a], ey = sy[b] - sy[a];
    double t = ((px - sx[a]) * ex + (py - sy[a]) * ey) / (ex * ex + ey * ey);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double cx = sx[a] + t * ex, cy = sy[a] + t * ey;
    if (t_out) *t_out = t;
    return hypot(px - cx, py - cy);
}

/* Nearest edge: in snapped mode the single-precision decision of the
 * rasterizer; otherwise the double-precision minimum. */
static int nearest_edge(const otri *s, int snap, const double sx[3], const double sy[3],
                        int x, int y, int W)
{
    if (snap) {
        int64_t px = SUBPIX * (int64_t)x + SUBPIX / 2, py = SUBPIX * (int64_t)y + SUBPIX / 2;
        int64_t E[3];
        for (int i = 0; i < 3; i++) E[i] = edge_fn(s, i, px, py);
        int ne;
        dist_norm_f32(s, px, py, E, W, &ne);
        return ne;
    }
    double best = 0.0;
    int bi = 0;
    for (int i = 0; i < 3; i++) {
        double d = seg_dist_d(sx, sy, i, x + 0.5, y + 0.5, NULL);
        if (i == 0 || d < best) { best = d; bi = i; }
    }
    return bi;
}

static void resolve_one(const otri *s, int x, int y, int hard, int snap,
                        int H, int W, double *b0, double *b1, double *dist)
{
    double sx[3], sy[3], l[3], q[3], bn[3], bo[3];
    screen_xy(s, snap, H, W, sx, sy);
    double px = x + 0.5, py = y + 0.5;
    lambdas(sx, sy, px, py, l);
    /* perspective-correct barycentrics: b_i = (l_i/w_i) / sum_j (l_j/w_j) */
    double Q = 0.0;
    for (int i = 0; i < 3; i++) { q[i] = l[i] / s->w[i]; Q += q[i]; }
    for (int i = 0; i < 3; i++) bn[i] = q[i] / Q;
    for (int i = 0; i < 3; i++) bo[s->corner[i]] = bn[i];
    *b0 = bo[0];
    *b1 = bo[1];
    int ne = nearest_edge(s, snap, sx, sy, x, y, W);
    double d = seg_dist_d(sx, sy, ne, px, py, NULL) / W;
    /* sign: + for hard (inside) fragments, - for soft ones; the sign bit
     * carries the flag even at distance 0 */
    *dist = hard ? d : -d;
}

int orc_resolve(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                int H, int W, int K, int cull, int snap,
                const int32_t *tri_id, const uint8_t *hard, double *bary, double *dist)
{
    for (int b = 0; b < B; b++) {
        const float *pc = pos_clip + (int64_t)b * V * 4;
        for (int k = 0; k < K; k++)
            for (int y = 0; y < H; y++)
                for (int x = 0; x < W; x++) {
                    int64_t o = (((int64_t)b * K + k) * H + y) * W + x;
                    int32_t t = tri_id[o];
                    if (t < 0 || t >= T) {
                        if (bary) { bary[2 * o] = 0.0; bary[2 * o + 1] = 0.0; }
                        if (dist) dist[o] = 0.0;
                        continue;
                    }
                    otri s = setup_tri(pc, tris + 3 * (int64_t)t, H, W, cull);
                    if (!s.ok) return -3;
                    double b0, b1, d;
                    resolve_one(&s, x, y, hard[o], snap, H, W, &b0, &b1, &d);
                    if (bary) { bary[2 * o] = b0; bary[2 * o + 1] = b1; }
                    if (dist) dist[o] = d;
                }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rasterization backward: d(bary, dist)/d(pos_clip) with frozen visibility */
/* ------------------------------------------------------------------------ */

/* Rasterize and PeelDepth have no backward in the paper; gradients reach the
 * vertices only through the barycentrics and the signed distance, which are
 * differentiable functions of the projected vertices.  Snapping is treated as
 * the identity (straight-through), with values taken at the snapped point. */
/* The pixels of window (wx0, wy0, ww, wh) of an H x W image: tri_id, hard,
 * grad_bary and grad_dist are [B,K,wh,ww]; the whole image is the window
 * (0, 0, W, H). */
int orc_rasterize_bwd_window(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                             int H, int W, int K, int cull, int snap, int wx0, int wy0, int ww, int wh,
                             const int32_t *tri_id, const uint8_t *hard,
                             const double *grad_bary, const double *grad_dist, double *grad_pos)
{
    if (wx0 < 0 || wy0 < 0 || ww <= 0 || wh <= 0 || wx0 + ww > W || wy0 + wh > H) return -1;
    memset(grad_pos, 0, sizeof(double) * (size_t)B * V * 4);
    for (int b = 0; b < B; b++) {
        const float *pc = pos_clip + (int64_t)b * V * 4;
        double *gp = grad_pos + (int64_t)b * V * 4;
        for (int k = 0; k < K; k++)
            for (int y = wy0; y < wy0 + wh; y++)
                for (int x = wx0; x < wx0 + ww; x++) {
                    int64_t o = (((int64_t)b * K + k) * wh + (y - wy0)) * ww + (x - wx0);
                    int32_t t = tri_id[o];
                    if (t < 0 || t >= T) continue;
                    otri s = setup_tri(pc, tris + 3 * (int64_t)t, H, W, cull);
                    if (!s.ok) return -3;
                    double sx[3], sy[3], l[3], q[3], bn[3];
                    screen_xy(&s, snap, H, W, sx, sy);
                    double px = x + 0.5, py = y + 0.5;
                    lambdas(sx, sy, px, py, l);
                    double Q = 0.0;
                    for (int i = 0; i < 3; i++) { q[i] = l[i] / s.w[i]; Q += q[i]; }
                    for (int i = 0; i < 3; i++) bn[i] = q[i] / Q;
                    /* gradient w.r.t. the normalized-order barycentrics; b2 of
                     * the original order is 1 - b0 - b1 and carries none */
                    double go[3] = {grad_bary[2 * o], grad_bary[2 * o + 1], 0.0};
                    double gb[3], gsx[3] = {0, 0, 0}, gsy[3] = {0, 0, 0}, gw[3];
                    for (int i = 0; i < 3; i++) gb[i] = go[s.corner[i]];
                    double sb = gb[0] * bn[0] + gb[1] * bn[1] + gb[2] * bn[2];
                    double gl[3];
                    for (int i = 0; i < 3; i++) {
                        double gq = (gb[i] - sb) / Q;
                        gl[i] = gq / s.w[i];
                        gw[i] = -gq * l[i] / (s.w[i] * s.w[i]);
                    }
                    /* d lambda_i / d v_j = -lambda_j * grad_p lambda_i */
                    double A = (sx[1] - sx[0]) * (sy[2] - sy[0]) - (sx[2] - sx[0]) * (sy[1] - sy[0]);
                    double Gx = 0.0, Gy = 0.0;
                    for (int i = 0; i < 3; i++) {
                        int a = (i + 1) % 3, c = (i + 2) % 3;
                        Gx += gl[i] * (-(sy[c] - sy[a]) / A);
                        Gy += gl[i] * ((sx[c] - sx[a]) / A);
                    }
                    for (int j = 0; j < 3; j++) { gsx[j] -= l[j] * Gx; gsy[j] -= l[j] * Gy; }
                    /* signed distance: d(dist)/d(endpoints) of the nearest segment */
                    if (grad_dist) {
                        double g = grad_dist[o];
                        int ne = nearest_edge(&s, snap, sx, sy, x, y, W);
                        double tt;
                        double d = seg_dist_d(sx, sy, ne, px, py, &tt);
                        if (d > 0.0 && g != 0.0) {
                            int a = (ne + 1) % 3, c = (ne + 2) % 3;
                            double cx = sx[a] + tt * (sx[c] - sx[a]);
                            double cy = sy[a] + tt * (sy[c] - sy[a]);
                            double ux = (px - cx) / d, uy = (py - cy) / d;
                            double sg = (hard[o] ? 1.0 : -1.0) * g / W;
                            gsx[a] += sg * (-(1.0 - tt) * ux);
                            gsy[a] += sg * (-(1.0 - tt) * uy);
                            gsx[c] += sg * (-tt * ux);
                            gsy[c] += sg * (-tt * uy);
                        }
                    }
                    /* screen -> clip: x_s = (x/w + 1) W/2, y_s = (1 - y/w) H/2 */
                    for (int j = 0; j < 3; j++) {
                        double w = s.w[j];
                        double *g = gp + 4 * (int64_t)s.v[j];
                        g[0] += gsx[j] * (0.5 * W) / w;
                        g[1] += gsy[j] * (-0.5 * H) / w;
                        g[3] += gsx[j] * (-0.5 * W) * s.xn[j] / w
                              + gsy[j] * (0.5 * H) * s.yn[j] / w + gw[j];
                    }
                }
    }
    return 0;
}

int orc_rasterize_bwd(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                      int H, int W, int K, int cull, int snap,
                      const int32_t *tri_id, const uint8_t *hard,
                      const double *grad_bary, const double *grad_dist, double *grad_pos)
{
    return orc_rasterize_bwd_window(pos_clip, tris, B, V, T, H, W, K, cull, snap, 0, 0, W, H,
                                    tri_id, hard, grad_bary, grad_dist, grad_pos);
}

/* ------------------------------------------------------------------------ */
/* Attribute interpolation (BuildInterpolate)                                */
/* ------------------------------------------------------------------------ */

int orc_interpolate(const double *attr, int Ba, int Va, int C, const int32_t *attr_tris, int T,
                    const int32_t *tri_id, const double *bary, int B, int K, int H, int W,
                    double *out)
{
    int64_t N = (int64_t)K * H * W;
    for (int b = 0; b < B; b++) {
        const double *a = attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
        for (int64_t p = 0; p < N; p++) {
            int64_t o = (int64_t)b * N + p;
            int32_t t = tri_id[o];
            double *y = out + o * C;
            if (t < 0 || t >= T) { for (int c = 0; c < C; c++) y[c] = 0.0; continue; }
            double w0 = bary[2 * o], w1 = bary[2 * o + 1], w2 = 1.0 - w0 - w1;
            const int32_t *tv = attr_tris + 3 * (int64_t)t;
            for (int c = 0; c < C; c++)
                y[c] = w0 * a[(int64_t)tv[0] * C + c] + w1 * a[(int64_t)tv[1] * C + c]
                     + w2 * a[(int64_t)tv[2] * C + c];
        }
    }
    return 0;
}

int orc_interpolate_bwd(const double *attr, int Ba, int Va, int C, const int32_t *attr_tris,
                        int T, const int32_t *tri_id, const double *bary, int B, int K, int H,
                        int W, const double *grad_out, double *grad_attr, double *grad_bary)
{
    int64_t N = (int64_t)K * H * W;
    memset(grad_attr, 0, sizeof(double) * (size_t)Ba * Va * C);
    for (int b = 0; b < B; b++) {
        const double *a = attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
        double *ga = grad_attr + (Ba == 1 ? 0 : (int64_t)b * Va * C);
        for (int64_t p = 0; p < N; p++) {
            int64_t o = (int64_t)b * N + p;
            int32_t t = tri_id[o];
            if (t < 0 || t >= T) { grad_bary[2 * o] = 0.0; grad_bary[2 * o + 1] = 0.0; continue; }
            double w[3] = {bary[2 * o], bary[2 * o + 1], 0.0};
            w[2] = 1.0 - w[0] - w[1];
            const int32_t *tv = attr_tris + 3 * (int64_t)t;
            const double *g = grad_out + o * C;
            double g0 = 0.0, g1 = 0.0;
            for (int c = 0; c < C; c++) {
                double a0 = a[(int64_t)tv[0] * C + c], a1 = a[(int64_t)tv[1] * C + c];
                double a2 = a[(int64_t)tv[2] * C + c];
                g0 += g[c] * (a0 - a2);
                g1 += g[c] * (a1 - a2);
                for (int i = 0; i < 3; i++) ga[(int64_t)tv[i] * C + c] += w[i] * g[c];
            }
            grad_bary[2 * o] = g0;
            grad_bary[2 * o + 1] = g1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bilinear texture sampling (the sampler behind GLSL texture())             */
/* ------------------------------------------------------------------------ */

/* Taps along one axis: s = u*n - 1/2 in float, i0 = floor(s), f = s - i0.
 * Wrap: repeat (mod n) or clamp (index clamped).  Returns the wrapped taps. */
static void taps_1d(float u, int n, int wrap, int *i0, int *i1, double *f)
{
    float s = u * (float)n;
    s = s - 0.5f;
    float fl = floorf(s);
    float fr = s - fl;
    int a = (int)fl, b = a + 1;
    if (wrap == ORC_WRAP_REPEAT) {
        a %= n; if (a < 0) a += n;
        b %= n; if (b < 0) b += n;
    } else {
        if (a < 0) a = 0;
        if (a > n - 1) a = n - 1;
        if (b < 0) b = 0;
        if (b > n - 1) b = n - 1;
    }
    *i0 = a;
    *i1 = b;
    *f = (double)fr;
}

/* The cell of Algorithm 1 ("normalize UV, store at p_tex"): floor(u * n),
 * wrapped or clamped like the taps. */
static int cell_1d(float u, int n, int wrap)
{
    float p = u * (float)n;
    int c = (int)floorf(p);
    if (wrap == ORC_WRAP_REPEAT) { c %= n; if (c < 0) c += n; }
    else { if (c < 0) c = 0; if (c > n - 1) c = n - 1; }
    return c;
}

/* Cube-map face and face coordinates (standard major-axis mapping, faces
 * +X,-X,+Y,-Y,+Z,-Z; ties prefer x, then y).  Float, in this order. */
static int cube_face(const float d[3], float *u, float *v)
{
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    int f;
    float sc, tc, ma;
    if (ax >= ay && ax >= az) {
        ma = ax;
        if (d[0] >= 0.0f) { f = 0; sc = -d[2]; tc = -d[1]; }
        else { f = 1; sc = d[2]; tc = -d[1]; }
    } else if (ay >= az) {
        ma = ay;
        if (d[1] >= 0.0f) { f = 2; sc = d[0]; tc = d[2]; }
        else { f = 3; sc = d[0]; tc = -d[2]; }
    } else {
        ma = az;
        if (d[2] >= 0.0f) { f = 4; sc = d[0]; tc = -d[1]; }
        else { f = 5; sc = -d[0]; tc = -d[1]; }
    }
    if (!(ma > 0.0f)) return -1;
    float us = sc / ma, vs = tc / ma;
    *u = (us + 1.0f) * 0.5f;
    *v = (vs + 1.0f) * 0.5f;
    return f;
}

/* d(u,v)/d(direction) of the cube mapping for face f (double). */
static void cube_face_jac(const float d[3], int f, double J[2][3])
{
    double x = d[0], y = d[1], z = d[2];
    double sc, tc, ma;
    int si, ti, mi;
    double ss, ts, ms;
    switch (f) {
    case 0: sc = -z; tc = -y; ma = x; si = 2; ss = -1; ti = 1; ts = -1; mi = 0; ms = 1; break;
    case 1: sc = z; tc = -y; ma = -x; si = 2; ss = 1; ti = 1; ts = -1; mi = 0; ms = -1; break;
    case 2: sc = x; tc = z; ma = y; si = 0; ss = 1; ti = 2; ts = 1; mi = 1; ms = 1; break;
    case 3: sc = x; tc = -z; ma = -y; si = 0; ss = 1; ti = 2; ts = -1; mi = 1; ms = -1; break;
    case 4: sc = x; tc = -y; ma = z; si = 0; ss = 1; ti = 1; ts = -1; mi = 2; ms = 1; break;
    default: sc = -x; tc = -y; ma = -z; si = 0; ss = -1; ti = 1; ts = -1; mi = 2; ms = -1; break;
    }
    memset(J, 0, sizeof(double) * 6);
    /* u = (sc/ma + 1)/2 with ma = |major component| > 0 */
    J[0][si] += 0.5 * ss / ma;
    J[0][mi] += -0.5 * sc / (ma * ma) * ms;
    J[1][ti] += 0.5 * ts / ma;
    J[1][mi] += -0.5 * tc / (ma * ma) * ms;
}

typedef struct {
    int ok;
    int face;         /* 0 for 2D */
    int x[2], y[2];   /* tap indices */
    double fx, fy;
    float u, v;       /* face / texture coordinates */
} otap;

static otap tex_taps(const orc_tex_desc *td, const float *coord)
{
    otap t;
    memset(&t, 0, sizeof t);
    float u, v;
    int face = 0;
    if (td->kind == ORC_TEX_CUBE) {
        face = cube_face(coord, &u, &v);
        if (face < 0) return t;
        taps_1d(u, td->Wt, ORC_WRAP_CLAMP, &t.x[0], &t.x[1], &t.fx);
        taps_1d(v, td->Ht, ORC_WRAP_CLAMP, &t.y[0], &t.y[1], &t.fy);
    } else {
        u = coord[0];
        v = coord[1];
        taps_1d(u, td->Wt, td->wrap_u, &t.x[0], &t.x[1], &t.fx);
        taps_1d(v, td->Ht, td->wrap_v, &t.y[0], &t.y[1], &t.fy);
    }
    t.face = face;
    t.u = u;
    t.v = v;
    t.ok = 1;
    return t;
}

static const double *texel(const orc_tex_desc *td, const double *tex, int f, int y, int x)
{
    return tex + ((((int64_t)f * td->Ht + y) * td->Wt) + x) * td->Ct;
}

int orc_texture(const double *tex, const orc_tex_desc *td, const float *coord,
                const int32_t *tri_id, int64_t N, double *out)
{
    int cd = td->kind == ORC_TEX_CUBE ? 3 : 2;
    int Ct = td->Ct;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double *y = out + i * Ct;
        for (int c = 0; c < Ct; c++) y[c] = 0.0;
        if (tri_id && tri_id[i] < 0) continue;
        otap t = tex_taps(td, coord + i * cd);
        if (!t.ok) continue;
        double wx[2] = {1.0 - t.fx, t.fx}, wy[2] = {1.0 - t.fy, t.fy};
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                const double *tx = texel(td, tex, t.face, t.y[a], t.x[b]);
                for (int c = 0; c < Ct; c++) y[c] += wy[a] * wx[b] * tx[c];
            }
    }
    return 0;
}

/* d out / d coord: derivative of the bilinear weights (piecewise; at f == 0
 * the derivative of the cell starting at the tap, i.e. the upper cell). */
int orc_texture_bwd_coord(const double *tex, const orc_tex_desc *td, const float *coord,
                          const int32_t *tri_id, int64_t N, const double *grad_out,
                          double *grad_coord)
{
    int cd = td->kind == ORC_TEX_CUBE ? 3 : 2;
    int Ct = td->Ct;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double *gc = grad_coord + i * cd;
        for (int j = 0; j < cd; j++) gc[j] = 0.0;
        if (tri_id && tri_id[i] < 0) continue;
        otap t = tex_taps(td, coord + i * cd);
        if (!t.ok) continue;
        const double *g = grad_out + i * Ct;
        double du = 0.0, dv = 0.0;
        for (int c = 0; c < Ct; c++) {
            double t00 = texel(td, tex, t.face, t.y[0], t.x[0])[c];
            double t01 = texel(td, tex, t.face, t.y[0], t.x[1])[c];
            double t10 = texel(td, tex, t.face, t.y[1], t.x[0])[c];
            double t11 = texel(td, tex, t.face, t.y[1], t.x[1])[c];
            du += g[c] * ((1.0 - t.fy) * (t01 - t00) + t.fy * (t11 - t10));
            dv += g[c] * ((1.0 - t.fx) * (t10 - t00) + t.fx * (t11 - t01));
        }
        du *= td->Wt;
        dv *= td->Ht;
        if (td->kind == ORC_TEX_CUBE) {
            double J[2][3];
            cube_face_jac(coord + i * cd, t.face, J);
            for (int j = 0; j < 3; j++) gc[j] = du * J[0][j] + dv * J[1][j];
        } else {
            gc[0] = du;
            gc[1] = dv;
        }
    }
    return 0;
}

/* Inverse UV (Algorithm 1): for every covered pixel i in increasing order,
 * store i at the texture cell its UV falls into.  A later pixel overwrites an
 * earlier one, so each cell ends up holding the largest such pixel index (the
 * paper's "last updated value").  One slice per (view, layer). */
int orc_invuv_build(const orc_tex_desc *td, const float *coord, const int32_t *tri_id,
                    int S, int64_t Npix, int32_t *inv)
{
    int cd = td->kind == ORC_TEX_CUBE ? 3 : 2;
    int F = td->kind == ORC_TEX_CUBE ? 6 : 1;
    int64_t cells = (int64_t)F * td->Ht * td->Wt;
    for (int s = 0; s < S; s++) {
        int32_t *iv = inv + (int64_t)s * cells;
        for (int64_t c = 0; c < cells; c++) iv[c] = -1;
        for (int64_t i = 0; i < Npix; i++) {
            int64_t o = (int64_t)s * Npix + i;
            if (tri_id[o] < 0) continue;
            const float *q = coord + o * cd;
            int f = 0, cx, cy;
            if (td->kind == ORC_TEX_CUBE) {
                float u, v;
                f = cube_face(q, &u, &v);
                if (f < 0) continue;
                cx = cell_1d(u, td->Wt, ORC_WRAP_CLAMP);
                cy = cell_1d(v, td->Ht, ORC_WRAP_CLAMP);
            } else {
                cx = cell_1d(q[0], td->Wt, td->wrap_u);
                cy = cell_1d(q[1], td->Ht, td->wrap_v);
            }
            iv[((int64_t)f * td->Ht + cy) * td->Wt + cx] = (int32_t)i;
        }
    }
    return 0;
}

/* Weight with which texel (ty,tx) is a tap of sample t (taps can coincide
 * under clamping, their weights then add). */
static double tap_weight(const otap *t, int ty, int tx)
{
    double wx[2] = {1.0 - t->fx, t->fx}, wy[2] = {1.0 - t->fy, t->fy};
    double w = 0.0;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            if (t->y[a] == ty && t->x[b] == tx) w += wy[a] * wx[b];
    return w;
}

/* Texture gradient through the inverse UV: every texel looks at the distinct
 * in-range cells of the 3x3 block around it in every slice, and takes the
 * recorded pixel's gradient times its bilinear weight on this texel.  Every
 * recorded pixel thus feeds all four of its taps; pixels that lost their cell
 * deliver nothing (the method's approximation).  Summation order: slice, then
 * cells row-major. */
int orc_texture_bwd_tex(const orc_tex_desc *td, const float *coord, const int32_t *tri_id,
                        int S, int64_t Npix, const double *grad_out, const int32_t *inv,
                        double *grad_tex)
{
    int cd = td->kind == ORC_TEX_CUBE ? 3 : 2;
    int F = td->kind == ORC_TEX_CUBE ? 6 : 1;
    int Ht = td->Ht, Wt = td->Wt, Ct = td->Ct;
    int wu = td->kind == ORC_TEX_CUBE ? ORC_WRAP_CLAMP : td->wrap_u;
    int wv = td->kind == ORC_TEX_CUBE ? ORC_WRAP_CLAMP : td->wrap_v;
    int64_t cells = (int64_t)F * Ht * Wt;
    memset(grad_tex, 0, sizeof(double) * (size_t)cells * Ct);
#pragma omp parallel for collapse(2) schedule(static)
    for (int f = 0; f < F; f++)
        for (int ty = 0; ty < Ht; ty++)
            for (int tx = 0; tx < Wt; tx++) {
                double *gt = grad_tex + (((int64_t)f * Ht + ty) * Wt + tx) * Ct;
                for (int s = 0; s < S; s++) {
                    const int32_t *iv = inv + (int64_t)s * cells;
                    for (int dy = -1; dy <= 1; dy++) {
                        int cy = ty + dy;
                        if (wv == ORC_WRAP_REPEAT) cy = (cy % Ht + Ht) % Ht;
                        else if (cy < 0 || cy >= Ht) continue;
                        for (int dx = -1; dx <= 1; dx++) {
                            int cx = tx + dx;
                            if (wu == ORC_WRAP_REPEAT) cx = (cx % Wt + Wt) % Wt;
                            else if (cx < 0 || cx >= Wt) continue;
                            int32_t i = iv[((int64_t)f * Ht + cy) * Wt + cx];
                            if (i < 0) continue;
                            int64_t o = (int64_t)s * Npix + i;
                            otap t = tex_taps(td, coord + o * cd);
                            if (!t.ok || t.face != f) continue;
                            double w = tap_weight(&t, ty, tx);
                            if (w == 0.0) continue;
                            const double *g = grad_out + o * Ct;
                            for (int c = 0; c < Ct; c++) gt[c] += w * g[c];
                        }
                    }
                }
            }
    return 0;
}

/* Exact adjoint of the bilinear sampler (S^T g, every pixel counted), used as
 * a diagnostic and as the special case the inverse UV must equal when no two
 * pixels share a cell. */
int orc_texture_adjoint(const orc_tex_desc *td, const float *coord, const int32_t *tri_id,
                        int64_t N, const double *grad_out, double *grad_tex)
{
    int cd = td->kind == ORC_TEX_CUBE ? 3 : 2;
    int F = td->kind == ORC_TEX_CUBE ? 6 : 1;
    int Ct = td->Ct;
    memset(grad_tex, 0, sizeof(double) * (size_t)F * td->Ht * td->Wt * Ct);
    for (int64_t i = 0; i < N; i++) {
        if (tri_id && tri_id[i] < 0) continue;
        otap t = tex_taps(td, coord + i * cd);
        if (!t.ok) continue;
        double wx[2] = {1.0 - t.fx, t.fx}, wy[2] = {1.0 - t.fy, t.fy};
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double *gt = grad_tex + ((((int64_t)t.face * td->Ht + t.y[a]) * td->Wt) + t.x[b]) * Ct;
                for (int c = 0; c < Ct; c++) gt[c] += wy[a] * wx[b] * grad_out[i * Ct + c];
            }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* HardSoftRas blending (§3.4.3, BuildBlend)                                 */
/* ------------------------------------------------------------------------ */

/* S^H: the front layer is present and hard.  Hardness travels in the sign bit
 * of dist (+0 hard, -0 soft); without dist every fragment is hard. */
static int front_hard(const int32_t *tri_id, const double *dist, int64_t o)
{
    if (tri_id[o] < 0) return 0;
    if (!dist) return 1;
    return !signbit(dist[o]);
}

/* Edge mask E: pixels of S^H that differ from an in-image 4-neighbour are
 * boundary pixels (both sides of the silhouette); E dilates them by an
 * L-infinity square of radius rho, with rho the largest integer below
 * delta * W pixels (so delta*W = 1 pixel gives E = boundary, the AA mode). */
int orc_edge_mask(const int32_t *tri_id, const double *dist, int B, int K, int H, int W,
                  float delta, int mode, uint8_t *E)
{
    int64_t N = (int64_t)H * W;
    uint8_t *sh = (uint8_t *)malloc((size_t)N);
    uint8_t *bd = (uint8_t *)malloc((size_t)N);
    if (!sh || !bd) { free(sh); free(bd); return -2; }
    int rho;
    if (mode == ORC_BLEND_AA) rho = 0;
    else {
        float dw = delta * (float)W;
        rho = (int)ceilf(dw) - 1;
    }
    for (int b = 0; b < B; b++) {
        for (int64_t p = 0; p < N; p++) sh[p] = (uint8_t)front_hard(tri_id, dist, (int64_t)b * K * N + p);
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                int64_t p = (int64_t)y * W + x;
                int e = 0;
                if (x > 0 && sh[p - 1] != sh[p]) e = 1;
                if (x < W - 1 && sh[p + 1] != sh[p]) e = 1;
                if (y > 0 && sh[p - W] != sh[p]) e = 1;
                if (y < H - 1 && sh[p + W] != sh[p]) e = 1;
                bd[p] = (uint8_t)e;
            }
        for (int y = 0; y < H; y++)
            for (int x = 0; x < W; x++) {
                uint8_t e = 0;
                if (mode == ORC_BLEND_SOFTRAS) e = 1;
                else if (mode == ORC_BLEND_HARD) e = 0;
                else if (rho >= 0) {
                    for (int qy = y - rho; qy <= y + rho && !e; qy++) {
                        if (qy < 0 || qy >= H) continue;
                        for (int qx = x - rho; qx <= x + rho; qx++) {
                            if (qx < 0 || qx >= W) continue;
                            if (bd[(int64_t)qy * W + qx]) { e = 1; break; }
                        }
                    }
                }
                E[(int64_t)b * N + (int64_t)y * W + x] = e;
            }
    }
    free(sh);
    free(bd);
    return 0;
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* I = E I^e + (1-E) I^ne with
 *   D_k = sigmoid(dist_k / sigma), w_k = D_k S_k,
 *   I_c^e = sum w_k C_k / sum w_k   (background 0 when no layer is present),
 *   I_c^ne = S^H C_1,  I_s^e = 1 - prod_k (1 - w_k),  I_s^ne = S^H.
 * The listing's normalisation by the stencil count does not match the colour
 * equation; the equation is followed. */
int orc_softras(const double *color, const double *dist, const int32_t *tri_id,
                int B, int K, int H, int W, int Cc, double sigma, float delta, int mode,
                double *out_color, double *out_sil, uint8_t *E)
{
    int rc = orc_edge_mask(tri_id, dist, B, K, H, W, delta, mode, E);
    if (rc) return rc;
    int64_t N = (int64_t)H * W;
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int64_t p = 0; p < N; p++) {
            int64_t q = (int64_t)b * N + p;
            double *oc = out_color + q * Cc;
            int64_t o1 = (int64_t)b * K * N + p;
            int sH = front_hard(tri_id, dist, o1);
            if (!E[q]) {
                for (int c = 0; c < Cc; c++) oc[c] = sH ? color[o1 * Cc + c] : 0.0;
                out_sil[q] = sH ? 1.0 : 0.0;
                continue;
            }
            double Wsum = 0.0, prod = 1.0;
            int nS = 0;
            for (int c = 0; c < Cc; c++) oc[c] = 0.0;
            for (int k = 0; k < K; k++) {
                int64_t o = ((int64_t)b * K + k) * N + p;
                if (tri_id[o] < 0) continue;
                double d = dist ? dist[o] : 0.0;
                double w = sigmoid(d / sigma);
                nS++;
                Wsum += w;
                prod *= (1.0 - w);
                for (int c = 0; c < Cc; c++) oc[c] += w * color[o * Cc + c];
            }
            for (int c = 0; c < Cc; c++) oc[c] = nS > 0 ? oc[c] / Wsum : 0.0;
            out_sil[q] = 1.0 - prod;
        }
    return 0;
}

int orc_softras_bwd(const double *color, const double *dist, const int32_t *tri_id,
                    int B, int K, int H, int W, int Cc, double sigma, const uint8_t *E,
                    const double *grad_color, const double *grad_sil,
                    double *grad_layer_color, double *grad_dist)
{
    int64_t N = (int64_t)H * W;
    memset(grad_layer_color, 0, sizeof(double) * (size_t)B * K * N * Cc);
    if (grad_dist) memset(grad_dist, 0, sizeof(double) * (size_t)B * K * N);
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int64_t p = 0; p < N; p++) {
            int64_t q = (int64_t)b * N + p;
            int64_t o1 = (int64_t)b * K * N + p;
            const double *gc = grad_color + q * Cc;
            double gs = grad_sil ? grad_sil[q] : 0.0;
            if (!E[q]) {
                if (front_hard(tri_id, dist, o1))
                    for (int c = 0; c < Cc; c++) grad_layer_color[o1 * Cc + c] = gc[c];
                continue;
            }
            double w[5] = {0}, D[5] = {0}, Wsum = 0.0;
            int S[5] = {0}, nS = 0;
            for (int k = 0; k < K; k++) {
                int64_t o = ((int64_t)b * K + k) * N + p;
                if (tri_id[o] < 0) continue;
                S[k] = 1;
                nS++;
                D[k] = sigmoid((dist ? dist[o] : 0.0) / sigma);
                w[k] = D[k];
                Wsum += w[k];
            }
            if (nS == 0) continue;
            double Ic[16];
            for (int c = 0; c < Cc; c++) {
                Ic[c] = 0.0;
                for (int k = 0; k < K; k++)
                    if (S[k]) Ic[c] += w[k] * color[(((int64_t)b * K + k) * N + p) * Cc + c];
                Ic[c] /= Wsum;
            }
            for (int k = 0; k < K; k++) {
                if (!S[k]) continue;
                int64_t o = ((int64_t)b * K + k) * N + p;
                double gw = 0.0;
                for (int c = 0; c < Cc; c++) {
                    grad_layer_color[o * Cc + c] = gc[c] * w[k] / Wsum;
                    gw += gc[c] * (color[o * Cc + c] - Ic[c]) / Wsum;
                }
                double others = 1.0;
                for (int j = 0; j < K; j++)
                    if (j != k && S[j]) others *= (1.0 - w[j]);
                gw += gs * others;
                if (grad_dist) grad_dist[o] = gw * D[k] * (1.0 - D[k]) / sigma;
            }
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Vertex transform, vertex normals, shading and loss (§3.4.1 decomposition */
/* I = f_pp(f_shade(f_rasterize(...))); the listing's BuildRasterize and    */
/* BuildNormalCompute; deferred shading per layer, §3.4.3)                  */
/* ------------------------------------------------------------------------ */

/* pos_clip[b,v] = M_b [p_v, 1] (column vector), M_b = projection x view. */
int orc_transform(const double *pos, const double *mvp, int B, int V, double *out)
{
    for (int b = 0; b < B; b++) {
        const double *M = mvp + 16 * (int64_t)b;
        for (int v = 0; v < V; v++) {
            const double *p = pos + 3 * (int64_t)v;
            double *o = out + 4 * ((int64_t)b * V + v);
            for (int r = 0; r < 4; r++)
                o[r] = M[4 * r] * p[0] + M[4 * r + 1] * p[1] + M[4 * r + 2] * p[2] + M[4 * r + 3];
        }
    }
    return 0;
}

int orc_transform_bwd(const double *mvp, int B, int V, const double *grad_clip, double *grad_pos)
{
    memset(grad_pos, 0, sizeof(double) * 3 * (size_t)V);
    for (int b = 0; b < B; b++) {
        const double *M = mvp + 16 * (int64_t)b;
        for (int v = 0; v < V; v++) {
            const double *g = grad_clip + 4 * ((int64_t)b * V + v);
            for (int c = 0; c < 3; c++)
                grad_pos[3 * (int64_t)v + c] += M[c] * g[0] + M[4 + c] * g[1] + M[8 + c] * g[2] + M[12 + c] * g[3];
        }
    }
    return 0;
}

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Vertex normal = normalize(sum over incident faces of (p1-p0) x (p2-p0)),
 * i.e. face normals weighted by twice their area. */
int orc_vertex_normals(const double *pos, const int32_t *tris, int V, int T, double *out)
{
    double *acc = (double *)calloc((size_t)V * 3, sizeof(double));
    if (!acc) return -2;
    for (int t = 0; t < T; t++) {
        const int32_t *f = tris + 3 * (int64_t)t;
        double e1[3], e2[3], n[3];
        for (int c = 0; c < 3; c++) {
            e1[c] = pos[3 * f[1] + c] - pos[3 * f[0] + c];
            e2[c] = pos[3 * f[2] + c] - pos[3 * f[0] + c];
        }
        cross3(e1, e2, n);
        for (int i = 0; i < 3; i++)
            for (int c = 0; c < 3; c++) acc[3 * f[i] + c] += n[c];
    }
    for (int v = 0; v < V; v++) {
        double *a = acc + 3 * v;
        double l = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        for (int c = 0; c < 3; c++) out[3 * v + c] = l > 0 ? a[c] / l : 0.0;
    }
    free(acc);
    return 0;
}

/* gradient of normalize(a): (g - (g.n) n) / |a| */
static void normalize_bwd(const double *a, const double *g, double *ga)
{
    double l = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (!(l > 0)) { ga[0] = ga[1] = ga[2] = 0.0; return; }
    double n[3] = {a[0] / l, a[1] / l, a[2] / l};
    double d = g[0] * n[0] + g[1] * n[1] + g[2] * n[2];
    for (int c = 0; c < 3; c++) ga[c] = (g[c] - d * n[c]) / l;
}

int orc_vertex_normals_bwd(const double *pos, const int32_t *tris, int V, int T,
                           const double *grad_n, double *grad_pos)
{
    double *acc = (double *)calloc((size_t)V * 3, sizeof(double));
    double *gacc = (double *)calloc((size_t)V * 3, sizeof(double));
    if (!acc || !gacc) { free(acc); free(gacc); return -2; }
    for (int t = 0; t < T; t++) {
        const int32_t *f = tris + 3 * (int64_t)t;
        double e1[3], e2[3], n[3];
        for (int c = 0; c < 3; c++) {
            e1[c] = pos[3 * f[1] + c] - pos[3 * f[0] + c];
            e2[c] = pos[3 * f[2] + c] - pos[3 * f[0] + c];
        }
        cross3(e1, e2, n);
        for (int i = 0; i < 3; i++)
            for (int c = 0; c < 3; c++) acc[3 * f[i] + c] += n[c];
    }
    for (int v = 0; v < V; v++) normalize_bwd(acc + 3 * v, grad_n + 3 * v, gacc + 3 * v);
    memset(grad_pos, 0, sizeof(double) * 3 * (size_t)V);
    for (int t = 0; t < T; t++) {
        const int32_t *f = tris + 3 * (int64_t)t;
        double gn[3] = {0, 0, 0}, e1[3], e2[3], g1[3], g2[3];
        for (int i = 0; i < 3; i++)
            for (int c = 0; c < 3; c++) gn[c] += gacc[3 * f[i] + c];
        for (int c = 0; c < 3; c++) {
            e1[c] = pos[3 * f[1] + c] - pos[3 * f[0] + c];
            e2[c] = pos[3 * f[2] + c] - pos[3 * f[0] + c];
        }
        /* n = e1 x e2: dn.gn = gn.(de1 x e2) + gn.(e1 x de2) -> ge1 = e2 x gn, ge2 = gn x e1 */
        cross3(e2, gn, g1);
        cross3(gn, e1, g2);
        for (int c = 0; c < 3; c++) {
            grad_pos[3 * f[1] + c] += g1[c];
            grad_pos[3 * f[2] + c] += g2[c];
            grad_pos[3 * f[0] + c] -= g1[c] + g2[c];
        }
    }
    free(acc);
    free(gacc);
    return 0;
}

/* Tangent-space normal mapping: n^ = normalize(n), t^ = normalize(t - (t.n^) n^),
 * b^ = n^ x t^, out = normalize(m_x t^ + m_y b^ + m_z n^). */
static void nmap_fwd(const double *n, const double *t, const double *m, double *out,
                     double *nh, double *tp, double *th, double *bh, double *u)
{
    double ln = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int c = 0; c < 3; c++) nh[c] = n[c] / ln;
    double d = t[0] * nh[0] + t[1] * nh[1] + t[2] * nh[2];
    for (int c = 0; c < 3; c++) tp[c] = t[c] - d * nh[c];
    double lt = sqrt(tp[0] * tp[0] + tp[1] * tp[1] + tp[2] * tp[2]);
    for (int c = 0; c < 3; c++) th[c] = tp[c] / lt;
    cross3(nh, th, bh);
    for (int c = 0; c < 3; c++) u[c] = m[0] * th[c] + m[1] * bh[c] + m[2] * nh[c];
    double lu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int c = 0; c < 3; c++) out[c] = u[c] / lu;
}

int orc_normal_map(const double *n, const double *t, const double *m, const int32_t *tri_id,
                   int64_t N, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double nh[3], tp[3], th[3], bh[3], u[3];
        if (tri_id[i] < 0) { out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = 0.0; continue; }
        nmap_fwd(n + 3 * i, t + 3 * i, m + 3 * i, out + 3 * i, nh, tp, th, bh, u);
    }
    return 0;
}

int orc_normal_map_bwd(const double *n, const double *t, const double *m, const int32_t *tri_id,
                       int64_t N, const double *g, double *gn, double *gt, double *gm)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        const double *ni = n + 3 * i, *ti = t + 3 * i, *mi = m + 3 * i;
        double *gni = gn + 3 * i, *gti = gt + 3 * i, *gmi = gm + 3 * i;
        for (int c = 0; c < 3; c++) gni[c] = gti[c] = gmi[c] = 0.0;
        if (tri_id[i] < 0) continue;
        double nh[3], tp[3], th[3], bh[3], u[3], o[3];
        nmap_fwd(ni, ti, mi, o, nh, tp, th, bh, u);
        double gu[3];
        normalize_bwd(u, g + 3 * i, gu);
        gmi[0] = gu[0] * th[0] + gu[1] * th[1] + gu[2] * th[2];
        gmi[1] = gu[0] * bh[0] + gu[1] * bh[1] + gu[2] * bh[2];
        gmi[2] = gu[0] * nh[0] + gu[1] * nh[1] + gu[2] * nh[2];
        double gth[3], gbh[3], gnh[3];
        for (int c = 0; c < 3; c++) {
            gth[c] = mi[0] * gu[c];
            gbh[c] = mi[1] * gu[c];
            gnh[c] = mi[2] * gu[c];
        }
        /* b = nh x th: gnh += th x gbh, gth += gbh x nh */
        double tmp[3];
        cross3(th, gbh, tmp);
        for (int c = 0; c < 3; c++) gnh[c] += tmp[c];
        cross3(gbh, nh, tmp);
        for (int c = 0; c < 3; c++) gth[c] += tmp[c];
        double gtp[3];
        normalize_bwd(tp, gth, gtp);
        /* tp = t - (t.nh) nh */
        double d = ti[0] * nh[0] + ti[1] * nh[1] + ti[2] * nh[2];
        double gd = -(gtp[0] * nh[0] + gtp[1] * nh[1] + gtp[2] * nh[2]);
        for (int c = 0; c < 3; c++) {
            gti[c] = gtp[c] + gd * nh[c];
            gnh[c] += -d * gtp[c] + gd * ti[c];
        }
        normalize_bwd(ni, gnh, gni);
    }
    return 0;
}

static const double LIGHT[3] = {0.40824829046386302, 0.40824829046386302, 0.81649658092772603};

/* Reflection direction of the view ray for the environment lookup:
 * d = reflect(-v^, n^) = 2 (n^.v^) n^ - v^, v^ = normalize(eye_b - pos). */
int orc_reflect(const double *n, const double *pos, const double *eye, const int32_t *tri_id,
                int B, int64_t Npv, double *out)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int64_t j = 0; j < Npv; j++) {
            int64_t i = (int64_t)b * Npv + j;
            double *o = out + 3 * i;
            if (tri_id[i] < 0) { o[0] = o[1] = o[2] = 0.0; continue; }
            double nh[3], vv[3], vh[3];
            double ln = sqrt(n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2]);
            for (int c = 0; c < 3; c++) { nh[c] = n[3 * i + c] / ln; vv[c] = eye[3 * b + c] - pos[3 * i + c]; }
            double lv = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
            for (int c = 0; c < 3; c++) vh[c] = vv[c] / lv;
            double d = nh[0] * vh[0] + nh[1] * vh[1] + nh[2] * vh[2];
            for (int c = 0; c < 3; c++) o[c] = 2.0 * d * nh[c] - vh[c];
        }
    return 0;
}

int orc_reflect_bwd(const double *n, const double *pos, const double *eye, const int32_t *tri_id,
                    int B, int64_t Npv, const double *g, double *gn, double *gpos)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int64_t j = 0; j < Npv; j++) {
            int64_t i = (int64_t)b * Npv + j;
            double *gni = gn + 3 * i, *gpi = gpos + 3 * i;
            for (int c = 0; c < 3; c++) gni[c] = gpi[c] = 0.0;
            if (tri_id[i] < 0) continue;
            double nh[3], vv[3], vh[3];
            double ln = sqrt(n[3 * i] * n[3 * i] + n[3 * i + 1] * n[3 * i + 1] + n[3 * i + 2] * n[3 * i + 2]);
            for (int c = 0; c < 3; c++) { nh[c] = n[3 * i + c] / ln; vv[c] = eye[3 * b + c] - pos[3 * i + c]; }
            double lv = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
            for (int c = 0; c < 3; c++) vh[c] = vv[c] / lv;
            double d = nh[0] * vh[0] + nh[1] * vh[1] + nh[2] * vh[2];
            const double *go = g + 3 * i;
            double gdn = go[0] * nh[0] + go[1] * nh[1] + go[2] * nh[2];
            double gnh[3], gvh[3];
            for (int c = 0; c < 3; c++) {
                gnh[c] = 2.0 * d * go[c] + 2.0 * gdn * vh[c];
                gvh[c] = 2.0 * gdn * nh[c] - go[c];
            }
            double gvv[3];
            normalize_bwd(n + 3 * i, gnh, gni);
            normalize_bwd(vv, gvh, gvv);
            for (int c = 0; c < 3; c++) gpi[c] = -gvv[c];
        }
    return 0;
}

/* Deferred shading of one fragment, white directional light l = (1,1,2)/|.|:
 *   Lambert: c = a_rgb (0.1 + 0.9 max(0, n^.l))
 *   Phong:   c = a_rgb (0.1 + 0.8 max(0, n^.l)) + 0.2 a_a max(0, r.v^)^32,
 *            r = 2 (n^.l) n^ - l, v^ = normalize(eye_b - pos)
 *   + env:   c += 0.5 a_a e  (e = environment sample in the reflection direction)
 * The derivative of max(0, x) at 0 is taken as 0. */
static void shade_one(int mode, const double *n, const double *p, const double *a, int Ca,
                      const double *e, const double *eye, double *c, double *grad_n,
                      double *grad_p, double *grad_a, double *grad_e, const double *g)
{
    double ln = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double nh[3] = {n[0] / ln, n[1] / ln, n[2] / ln};
    double ndl = nh[0] * LIGHT[0] + nh[1] * LIGHT[1] + nh[2] * LIGHT[2];
    double dif = ndl > 0 ? ndl : 0.0;
    double kd = mode == ORC_SHADE_LAMBERT ? 0.9 : 0.8;
    double base = 0.1 + kd * dif;
    double alpha = Ca > 3 ? a[3] : 0.0;
    double spec = 0.0, rv = 0.0, vv[3] = {0, 0, 0}, vh[3] = {0, 0, 0}, r[3] = {0, 0, 0}, lv = 1.0;
    if (mode != ORC_SHADE_LAMBERT) {
        for (int k = 0; k < 3; k++) vv[k] = eye[k] - p[k];
        lv = sqrt(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
        for (int k = 0; k < 3; k++) { vh[k] = vv[k] / lv; r[k] = 2.0 * ndl * nh[k] - LIGHT[k]; }
        rv = r[0] * vh[0] + r[1] * vh[1] + r[2] * vh[2];
        spec = rv > 0 ? pow(rv, 32.0) : 0.0;
    }
    if (c) {
        for (int k = 0; k < 3; k++) {
            c[k] = a[k] * base;
            if (mode != ORC_SHADE_LAMBERT) c[k] += 0.2 * alpha * spec;
            if (mode == ORC_SHADE_PHONG_ENV) c[k] += 0.5 * alpha * e[k];
        }
    }
    if (!g) return;
    double gsum = g[0] + g[1] + g[2];
    double ga_dot = g[0] * a[0] + g[1] * a[1] + g[2] * a[2];
    for (int k = 0; k < 3; k++) grad_a[k] = g[k] * base;
    if (Ca > 3) {
        grad_a[3] = 0.0;
        if (mode != ORC_SHADE_LAMBERT) grad_a[3] += 0.2 * spec * gsum;
        if (mode == ORC_SHADE_PHONG_ENV) grad_a[3] += 0.5 * (g[0] * e[0] + g[1] * e[1] + g[2] * e[2]);
    }
    if (grad_e) for (int k = 0; k < 3; k++) grad_e[k] = mode == ORC_SHADE_PHONG_ENV ? 0.5 * alpha * g[k] : 0.0;
    /* d/d ndl of the diffuse term */
    double g_ndl = ndl > 0 ? kd * ga_dot : 0.0;
    double gnh[3] = {g_ndl * LIGHT[0], g_ndl * LIGHT[1], g_ndl * LIGHT[2]};
    double gvh[3] = {0, 0, 0};
    if (mode != ORC_SHADE_LAMBERT && rv > 0) {
        double g_rv = 0.2 * alpha * gsum * 32.0 * pow(rv, 31.0);
        /* rv = r.vh, r = 2 ndl nh - l */
        double g_r[3], r_dot_dummy;
        (void)r_dot_dummy;
        for (int k = 0; k < 3; k++) { g_r[k] = g_rv * vh[k]; gvh[k] = g_rv * r[k]; }
        double g_ndl2 = 2.0 * (g_r[0] * nh[0] + g_r[1] * nh[1] + g_r[2] * nh[2]);
        for (int k = 0; k < 3; k++) gnh[k] += 2.0 * ndl * g_r[k] + g_ndl2 * LIGHT[k];
    }
    normalize_bwd(n, gnh, grad_n);
    if (grad_p) {
        double gvv[3];
        if (mode != ORC_SHADE_LAMBERT) normalize_bwd(vv, gvh, gvv);
        else gvv[0] = gvv[1] = gvv[2] = 0.0;
        for (int k = 0; k < 3; k++) grad_p[k] = -gvv[k];
    }
}

int orc_shade(int mode, const double *n, const double *pos, const double *albedo, int Ca,
              const double *env, const double *eye, const int32_t *tri_id, int B, int64_t Npv,
              double *out)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int64_t j = 0; j < Npv; j++) {
            int64_t i = (int64_t)b * Npv + j;
            double *o = out + 3 * i;
            if (tri_id[i] < 0) { o[0] = o[1] = o[2] = 0.0; continue; }
            shade_one(mode, n + 3 * i, pos ? pos + 3 * i : NULL, albedo + (int64_t)Ca * i, Ca,
                      env ? env + 3 * i : NULL, eye + 3 * b, o, NULL, NULL, NULL, NULL, NULL);
        }
    return 0;
}

int orc_shade_bwd(int mode, const double *n, const double *pos, const double *albedo, int Ca,
                  const double *env, const double *eye, const int32_t *tri_id, int B, int64_t Npv,
                  const double *g, double *gn, double *gpos, double *galb, double *genv)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; b++)
        for (int64_t j = 0; j < Npv; j++) {
            int64_t i = (int64_t)b * Npv + j;
            double dn[3], dp[3], da[4], de[3];
            if (tri_id[i] < 0) {
                memset(dn, 0, sizeof dn); memset(dp, 0, sizeof dp);
                memset(da, 0, sizeof da); memset(de, 0, sizeof de);
            } else {
                shade_one(mode, n + 3 * i, pos ? pos + 3 * i : NULL, albedo + (int64_t)Ca * i, Ca,
                          env ? env + 3 * i : NULL, eye + 3 * b, NULL, dn, dp, da, de, g + 3 * i);
            }
            for (int k = 0; k < 3; k++) {
                gn[3 * i + k] = dn[k];
                if (gpos) gpos[3 * i + k] = dp[k];
                if (genv) genv[3 * i + k] = de[k];
            }
            for (int k = 0; k < Ca; k++) galb[(int64_t)Ca * i + k] = da[k];
        }
    return 0;
}

/* L = mean over B*H*W*4 of (RGBA - target)^2 with RGBA = (colour, silhouette). */
int orc_loss_l2(const double *color, const double *sil, const double *target, int64_t Npix,
                double *loss, double *grad_color, double *grad_sil)
{
    double s = 0.0, inv = 1.0 / (4.0 * (double)Npix);
    for (int64_t i = 0; i < Npix; i++) {
        for (int c = 0; c < 3; c++) {
            double d = color[3 * i + c] - target[4 * i + c];
            s += d * d;
            if (grad_color) grad_color[3 * i + c] = 2.0 * d * inv;
        }
        double d = sil[i] - target[4 * i + 3];
        s += d * d;
        if (grad_sil) grad_sil[i] = 2.0 * d * inv;
    }
    *loss = s * inv;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-precision versions of the two value computations that feed        */
/* discrete decisions downstream: clip coordinates (snapping) and texture   */
/* coordinates (texel and inverse-UV cell selection).  Both sides compute   */
/* them in float with this operation order, so the decisions coincide.      */
/* ------------------------------------------------------------------------ */

/* o_r = ((M_r0 x + M_r1 y) + M_r2 z) + M_r3, no fused multiply-add */
int orc_transform_f32(const float *pos, const float *mvp, int B, int V, float *out)
{
    for (int b = 0; b < B; b++) {
        const float *M = mvp + 16 * (int64_t)b;
        for (int v = 0; v < V; v++) {
            const float *p = pos + 3 * (int64_t)v;
            float *o = out + 4 * ((int64_t)b * V + v);
            for (int r = 0; r < 4; r++) {
                float t0 = M[4 * r] * p[0];
                float t1 = M[4 * r + 1] * p[1];
                float t2 = M[4 * r + 2] * p[2];
                float s = t0 + t1;
                s = s + t2;
                o[r] = s + M[4 * r + 3];
            }
        }
    }
    return 0;
}

/* out = (b0 a0 + b1 a1) + b2 a2 with b2 = (1 - b0) - b1, all float */
int orc_interpolate_f32(const float *attr, int Va, int C, const int32_t *attr_tris, int T,
                        const int32_t *tri_id, const float *bary, int64_t N, float *out)
{
    for (int64_t o = 0; o < N; o++) {
        float *y = out + o * C;
        int32_t t = tri_id[o];
        if (t < 0 || t >= T) { for (int c = 0; c < C; c++) y[c] = 0.0f; continue; }
        const int32_t *tv = attr_tris + 3 * (int64_t)t;
        float w0 = bary[2 * o], w1 = bary[2 * o + 1];
        float w2 = 1.0f - w0;
        w2 = w2 - w1;
        for (int c = 0; c < C; c++) {
            float a = w0 * attr[(int64_t)tv[0] * C + c];
            float b = w1 * attr[(int64_t)tv[1] * C + c];
            float d = w2 * attr[(int64_t)tv[2] * C + c];
            float s = a + b;
            y[c] = s + d;
        }
    }
    (void)Va;
    return 0;
}

/* Bilinear sample (2-D or cube) in float: the taps and fractions of
 * tex_taps, weights w00 = (1-fy)(1-fx), w01 = (1-fy)fx, w10 = fy(1-fx),
 * w11 = fy fx, and out = ((w00 t00 + w01 t01) + w10 t10) + w11 t11.  A
 * tangent-space normal-map sample feeds the shading normal, whose direction
 * selects cube texels and the side of the max(0, .) kinks, so it is taken
 * in this order on both sides. */
int orc_texture_f32(const float *tex, const orc_tex_desc *td, const float *coord,
                    const int32_t *tri_id, int64_t N, float *out)
{
    int cd = td->kind == ORC_TEX_CUBE ? 3 : 2;
    int Ct = td->Ct;
    for (int64_t i = 0; i < N; i++) {
        float *y = out + i * Ct;
        for (int c = 0; c < Ct; c++) y[c] = 0.0f;
        if (tri_id && tri_id[i] < 0) continue;
        otap t = tex_taps(td, coord + i * cd);
        if (!t.ok) continue;
        const float fx = (float)t.fx, fy = (float)t.fy;
        const float gx = 1.0f - fx, gy = 1.0f - fy;
        const float w00 = gy * gx, w01 = gy * fx, w10 = fy * gx, w11 = fy * fx;
        const int64_t face = (int64_t)t.face * td->Ht * td->Wt;
        const float *t00 = tex + (face + (int64_t)t.y[0] * td->Wt + t.x[0]) * Ct;
        const float *t01 = tex + (face + (int64_t)t.y[0] * td->Wt + t.x[1]) * Ct;
        const float *t10 = tex + (face + (int64_t)t.y[1] * td->Wt + t.x[0]) * Ct;
        const float *t11 = tex + (face + (int64_t)t.y[1] * td->Wt + t.x[1]) * Ct;
        for (int c = 0; c < Ct; c++) {
            float s = w00 * t00[c];
            s = s + w01 * t01[c];
            s = s + w10 * t10[c];
            y[c] = s + w11 * t11[c];
        }
    }
    return 0;
}

/* Threads of the per-pixel and per-texel loops (OpenMP; each output element
 * is computed by one thread in a fixed order, so results do not depend on
 * the count).  Test runs keep one; the CPU baseline times all host cores. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
    return n > 0 ? n : 1;
#else
    (void)n;
    return 1;
#endif
}
