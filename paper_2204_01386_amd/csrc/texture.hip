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
#include "texcore.h"


// Large textures (4 Mi cells a face and more): the per-pixel kernels give
// each XCD one contiguous range of pixels, whose texels are then fetched
// into one L2; smaller textures keep the default interleave.
#define IV_LARGE_CELLS (1 << 22)
__device__ __forceinline__ int64_t tex_block(const dressi_tex_desc &td) {
    return (int64_t)td.Ht * td.Wt >= IV_LARGE_CELLS ? xcd_block() : (int64_t)blockIdx.x;
}

template <int CT>
__global__ void __launch_bounds__(256)
    k_tex_fwd(const float *__restrict__ tex, dressi_tex_desc td, const float *__restrict__ coord,
              const int32_t *__restrict__ tri_id, int64_t n, float *__restrict__ out, int skip_empty) {
    int64_t i = tex_block(td) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (skip_empty && tri_id && tri_id[i] < 0) return;
    const int Ct = CT > 0 ? CT : td.Ct;
    const int cd = td.kind == DRESSI_TEX_CUBE ? 3 : 2;
    float *y = out + i * Ct;
    float r[TEX_NC(CT)];
    Taps t;
    t.ok = 0;
    if (!tri_id || tri_id[i] >= 0) t = make_taps(td, coord + i * cd, tex_layer(td, tri_id, i));
    if (!t.ok) {
#pragma unroll
        for (int c = 0; c < TEX_NC(CT); c++) r[c] = 0.0f;
        stv<CT>(y, r, Ct);
        return;
    }
    tex_bilinear<CT>(tex, td, t, r, Ct);
    stv<CT>(y, r, Ct);
}

// Per pixel: d out / d coord and, when `inv` is given, the inverse-UV record
// (the pixel index written into its cell with atomicMax).
template <int CT>
__global__ void __launch_bounds__(256)
    k_tex_bwd_pixel(const float *__restrict__ tex, dressi_tex_desc td,
                                const float *__restrict__ coord, const int32_t *__restrict__ tri_id,
                                int64_t npix, int S, const float *__restrict__ grad_out,
                                float *__restrict__ grad_coord, int32_t *__restrict__ inv, int skip_empty) {
    int64_t i = tex_block(td) * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * npix) return;
    const int Ct = CT > 0 ? CT : td.Ct;
    const bool cube = td.kind == DRESSI_TEX_CUBE;
    const int cd = cube ? 3 : 2;
    const float *q = coord + i * cd;
    Taps t;
    t.ok = 0;
    bool covered = !tri_id || tri_id[i] >= 0;
    if (covered) t = make_taps(td, q, tex_layer(td, tri_id, i));
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
        int64_t cells = (int64_t)tex_faces(td) * td.Ht * td.Wt;
        atomicMax(&inv[(int64_t)s * cells + ((int64_t)t.face * td.Ht + cy) * td.Wt + cx], pix);
    }
    if (!grad_coord || (skip_empty && !covered)) return;
    float *gc = grad_coord + i * cd;
    if (!t.ok) {
        for (int j = 0; j < cd; j++) gc[j] = 0.0f;
        return;
    }
    float g[TEX_NC(CT)];
    ldv<CT>(grad_out + i * Ct, g, Ct);
    float du, dv;
    tex_dcoord<CT>(tex, td, t, g, Ct, du, dv);
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

// Sobol jitter of the inverse UV (§3.3.2: the sampling positions move by a
// quasi-random offset every frame, so the pixel kept by a texel cell changes
// from frame to frame).  Frame f moves every pixel centre by o_f = Sobol(f) -
// 1/2 in both axes; the taps of the moved point are the pixels (x + dx, y +
// dy) + {0,1}^2 with the fixed weights w of the fractions (fx, fy).  A covered
// pixel whose four taps are covered pixels of the image registers the
// coordinate and the gradient sampled there, ((w00 v00 + w01 v01) + w10 v10)
// + w11 v11 in float; the others do not register.  The moved samples are
// written to jc [S,H,W,cd] and jg [S,H,W,Ct] at the pixel's index, so the
// gather reads them exactly where it reads the unmoved ones.
struct Jitter {
    int dx, dy;                  // tap offsets (floor of the offset), -1 or 0
    float w00, w01, w10, w11;    // bilinear weights of the fractions
};

template <int CT>
__global__ void __launch_bounds__(256)
    k_invuv_jitter(dressi_tex_desc td, const float *__restrict__ coord, const int32_t *__restrict__ tri_id,
                   int H, int W, int S, const float *__restrict__ grad_out, Jitter j, float *__restrict__ jc,
                   float *__restrict__ jg, int32_t *__restrict__ inv) {
    const int64_t npix = (int64_t)H * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * npix || tri_id[i] < 0) return;
    const int s = (int)(i / npix);
    const int pix = (int)(i - (int64_t)s * npix);
    const int y = pix / W, x = pix - y * W;
    const int x0 = x + j.dx, y0 = y + j.dy;
    if (x0 < 0 || y0 < 0 || x0 + 1 >= W || y0 + 1 >= H) return;
    const int64_t o00 = (int64_t)s * npix + (int64_t)y0 * W + x0, o01 = o00 + 1, o10 = o00 + W, o11 = o10 + 1;
    if (tri_id[o00] < 0 || tri_id[o01] < 0 || tri_id[o10] < 0 || tri_id[o11] < 0) return;
    const bool cube = td.kind == DRESSI_TEX_CUBE;
    const int cd = cube ? 3 : 2;
    const int Ct = CT > 0 ? CT : td.Ct;
    float c[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (k >= cd) break;
        float v = j.w00 * coord[o00 * cd + k];
        v = v + j.w01 * coord[o01 * cd + k];
        v = v + j.w10 * coord[o10 * cd + k];
        c[k] = v + j.w11 * coord[o11 * cd + k];
        jc[i * cd + k] = c[k];
    }
#pragma unroll
    for (int k = 0; k < TEX_NC(CT); k++) {
        if (CT == 0 && k >= Ct) break;
        float v = j.w00 * grad_out[o00 * Ct + k];
        v = v + j.w01 * grad_out[o01 * Ct + k];
        v = v + j.w10 * grad_out[o10 * Ct + k];
        jg[i * Ct + k] = v + j.w11 * grad_out[o11 * Ct + k];
    }
    int f = 0, cx, cy;
    if (cube) {
        float u, v, sc, tc, ma;
        f = cube_face(c[0], c[1], c[2], u, v, sc, tc, ma);
        if (f < 0) return;
        cx = cell1d(u, td.Wt, DRESSI_WRAP_CLAMP);
        cy = cell1d(v, td.Ht, DRESSI_WRAP_CLAMP);
    } else {
        cx = cell1d(c[0], td.Wt, td.wrap_u);
        cy = cell1d(c[1], td.Ht, td.wrap_v);
    }
    const int64_t cells = (int64_t)tex_faces(td) * td.Ht * td.Wt;
    atomicMax(&inv[(int64_t)s * cells + ((int64_t)f * td.Ht + cy) * td.Wt + cx], pix);
}

// The 2-D Sobol point of index f (f = 0, 1, 2, ...) to 24 bits: the first
// coordinate is the base-2 radical inverse of f, the second uses the
// direction numbers m_1 = 1, m_k = 2 m_{k-1} xor m_{k-1} (the primitive
// polynomial x + 1); each coordinate is the xor, over the set bits k of f,
// of m_(k+1) / 2^(k+1), truncated to 24 fraction bits (exact in float).
static void sobol2(uint32_t f, float *u, float *v) {
    uint32_t a = 0, b = 0, m = 1;
    for (int k = 0; k < 32; k++) {
        if ((f >> k) & 1u) {
            a ^= 1u << (31 - k);
            b ^= m << (31 - k);
        }
        m = (m << 1) ^ m;
    }
    *u = (float)(a >> 8) * (1.0f / 16777216.0f);
    *v = (float)(b >> 8) * (1.0f / 16777216.0f);
}

static Jitter jitter_of_frame(uint32_t frame) {
    float u, v;
    sobol2(frame, &u, &v);
    const float ox = u - 0.5f, oy = v - 0.5f;   // exact: 24-bit fractions
    const float flx = floorf(ox), fly = floorf(oy);
    const float fx = ox - flx, fy = oy - fly;    // exact
    Jitter j;
    j.dx = (int)flx;
    j.dy = (int)fly;
    const float gx = 1.0f - fx, gy = 1.0f - fy;
    j.w00 = gy * gx;
    j.w01 = gy * fx;
    j.w10 = fy * gx;
    j.w11 = fy * fx;
    return j;
}

// Texture gradient through the inverse UV.  A workgroup of 256 lanes (16
// columns x 16 rows) owns a block of 16 x 16R texels, R texels per lane (rows
// ly, ly + 16, ...).  Per slice the cells around the block (a one-cell halo)
// are staged in LDS (wrapped, or empty outside a clamped texture), each with
// its winner's taps, bilinear fractions and gradient; blocks whose cells are
// all empty skip the slice.  Each texel then visits its 3x3 cells in
// row-major order and adds the kept pixel's gradient times that pixel's
// bilinear weight on the texel.
#define IV_T 16
// Per texel: the sum over slices [s0, s1), in ascending order, of the distinct
// in-range cells of its 3x3 block, row-major, of the winner pixel's bilinear
// weight on this texel times its gradient.  A block of texels loads the
// haloed cells of SG slices at once (all loads in flight) and the next group's
// while it works on the current one, skips a group when every cell is empty,
// then gathers.  With nsplit > 1 the slice range is split over grid.z and each
// part writes its own partial sum.  A winner found in a cell of face or layer
// f has its taps on f, so they are recomputed from its coordinate alone.
// More rows per lane (R) means fewer, larger blocks: more loads in flight per
// lane and fewer halo cells per texel, against more LDS per block.
// c modulo n in [0, n): one addition or subtraction for the halo's usual
// range, a division only for blocks that reach past a small texture
__device__ __forceinline__ int wrap_repeat(int c, int n) {
    if (c >= 0 && c < n) return c;
    if (c < 0 && c >= -n) return c + n;
    if (c >= n && c < 2 * n) return c - n;
    return ((c % n) + n) % n;
}

template <int SG, int R>
struct IvGeom {
    static constexpr int NT = 256;                 // lanes: 16 columns x 16 rows
    static constexpr int TY = 16 * R;              // texel rows per block
    static constexpr int HW = IV_T + 2, HH = TY + 2, HN = HW * HH;   // halo
    static constexpr int PT = (HN + NT - 1) / NT;  // halo cells per lane
};

// With REC (RGBA, 2-D or array textures) each kept pixel's taps, fractions
// and gradient come from its record (invrec_put) in one 32-byte read, in
// place of its coordinate and gradient: the same values.
template <int CT, int SG, int R, bool REC = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(((R == 1 && CT == 8) || (R == 2 && CT > 0 && CT <= 4)) ? 8 : 1)))
    k_invuv_gather(dressi_tex_desc td, const float *__restrict__ coord, const int32_t *__restrict__ tri_id,
                   int64_t npix, int S, int nsplit, const int32_t *__restrict__ inv,
                   const float *__restrict__ grad_out, float *__restrict__ out, int xcd,
                   const int4 *__restrict__ rec, LossJob lj, ListJob job, int jcols) {
    static_assert(!REC || CT == 4, "records hold an RGBA gradient");
    // per halo cell of each slice of the group: the winner's four tap
    // coordinates, bilinear fractions (fx < 0: no winner, or one on another
    // cube face) and pixel gradient
    using G = IvGeom<SG, R>;
    constexpr int NC = TEX_NC(CT);
    __shared__ int2 ctap[SG][G::HN];   // x0 | x1 << 16, y0 | y1 << 16
    __shared__ float2 cfr[SG][G::HN];  // fx, fy (also the loss job's 256 floats)
    static_assert(2 * SG * G::HN >= 256, "the loss job reuses cfr");
    __shared__ float cg[SG][G::HN * NC];
    const int Ht = td.Ht, Wt = td.Wt, Ct = CT > 0 ? CT : td.Ct;
    const bool cube = td.kind == DRESSI_TEX_CUBE;
    const int F = tex_faces(td);
    const int wu = cube ? DRESSI_WRAP_CLAMP : td.wrap_u;
    const int wv = cube ? DRESSI_WRAP_CLAMP : td.wrap_v;
    const int cd = cube ? 3 : 2;
    // workgroups of neighbouring texel blocks share inverse-UV cells and their
    // winners' pixel rows: with `xcd`, each XCD takes one contiguous range of
    // the grid (rows of blocks), so they are fetched into one L2
    // with a loss job, the grid's last column of workgroups is the job's (its
    // first workgroup runs it, the others exit)
    // and with a list-building job of the step, the columns after it are the
    // job's workgroups
    const int lc = lj.loss ? 1 : 0;
    const int gxb = (int)gridDim.x - lc - jcols;
    if ((int)blockIdx.x >= gxb) {
        if (lj.loss && (int)blockIdx.x == gxb) {
            if (blockIdx.y == 0 && blockIdx.z == 0) loss_sum_block(lj, reinterpret_cast<float *>(&cfr[0][0]));
            return;
        }
        list_job_block(job, (((int)blockIdx.x - gxb - lc) * (int)gridDim.y + (int)blockIdx.y) * (int)gridDim.z +
                                (int)blockIdx.z);
        return;
    }
    // (the divisions stay off the common path: with many short workgroups
    // the scalar unit's division sequences cost more than their loads)
    int bxi = blockIdx.x, byi = blockIdx.y, bz = blockIdx.z;
    if (xcd) {
        const int64_t gxy = (int64_t)gxb * gridDim.y;
        const int64_t lin = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gxb + blockIdx.x;
        const int64_t lb = xcd_block(lin, gxy * gridDim.z);
        bz = (int)(lb / gxy);
        byi = (int)((lb - bz * gxy) / gxb);
        bxi = (int)(lb - bz * gxy - (int64_t)byi * gxb);
    }
    int f = bz, part = 0, s0 = 0, s1 = S;
    if (nsplit > 1) {
        f = bz / nsplit;
        part = bz - f * nsplit;
        const int per = (S + nsplit - 1) / nsplit;
        s0 = part * per;
        s1 = min(S, s0 + per);
    }
    const int bx0 = bxi * IV_T, by0 = byi * G::TY;
    const int lx = threadIdx.x % IV_T, ly = threadIdx.x / IV_T;
    const int tx = bx0 + lx;
    const int64_t face_cells = (int64_t)Ht * Wt;
    const int64_t cells_all = (int64_t)F * face_cells;
    // this lane's halo entries (row-major over the halo) and their cell offsets
    int hoff[G::PT];
#pragma unroll
    for (int k = 0; k < G::PT; k++) {
        const int h = threadIdx.x + k * G::NT;
        hoff[k] = -1;
        if (h < G::HN) {
            int cy = by0 - 1 + h / G::HW, cx = bx0 - 1 + h % G::HW;
            bool ok = true;
            if (wv == DRESSI_WRAP_REPEAT) cy = wrap_repeat(cy, Ht);
            else ok = cy >= 0 && cy < Ht;
            if (wu == DRESSI_WRAP_REPEAT) cx = wrap_repeat(cx, Wt);
            else ok = ok && cx >= 0 && cx < Wt;
            if (ok) hoff[k] = cy * Wt + cx;
        }
    }
    float acc[R][NC];
#pragma unroll
    for (int r = 0; r < R; r++)
#pragma unroll
        for (int c = 0; c < NC; c++) acc[r][c] = 0.0f;
    // winners of a group's halo cells; the next group's are loaded while the
    // current one is processed
    auto load_group = [&](int g0, int (*w)[G::PT]) {
        const int ng = min(SG, s1 - g0);
#pragma unroll
        for (int q = 0; q < SG; q++) {
            const int32_t *iv = inv + (int64_t)(g0 + q) * cells_all + (int64_t)f * face_cells;
#pragma unroll
            for (int k = 0; k < G::PT; k++) w[q][k] = (q < ng && hoff[k] >= 0) ? iv[hoff[k]] : -1;
        }
    };
    int wnext[SG][G::PT];
    if (s0 < s1) load_group(s0, wnext);
    for (int g0 = s0; g0 < s1; g0 += SG) {
        const int ng = min(SG, s1 - g0);
        int wpix[SG][G::PT];
#pragma unroll
        for (int q = 0; q < SG; q++)
#pragma unroll
            for (int k = 0; k < G::PT; k++) wpix[q][k] = wnext[q][k];
        if (g0 + SG < s1) load_group(g0 + SG, wnext);
        int found = 0;
        // records: the first HK halo entries' loads are all in flight before
        // the first is stored (all of them with one row per lane, two with
        // more rows, where holding a third would spill registers)
        constexpr int HK = REC ? (R == 1 ? G::PT : (G::PT < 2 ? G::PT : 2)) : 0;
        int4 ra[SG][HK > 0 ? HK : 1], rb[SG][HK > 0 ? HK : 1];
#pragma unroll
        for (int q = 0; q < SG; q++)
#pragma unroll
            for (int k = 0; k < HK; k++) {
                const int i = wpix[q][k];
                ra[q][k] = make_int4(0, 0, -1, 0);
                rb[q][k] = make_int4(0, 0, 0, 0);
                if (i >= 0) {
                    const int4 *rp = rec + 2 * ((int64_t)(g0 + q) * npix + i);
                    ra[q][k] = rp[0];
                    rb[q][k] = rp[1];
                }
            }
        // each winner's taps, computed once for the up to 9 texels that visit it
#pragma unroll
        for (int q = 0; q < SG; q++) {
#pragma unroll
            for (int k = 0; k < G::PT; k++) {
                const int h = threadIdx.x + k * G::NT;
                if (h >= G::HN) continue;
                const int i = wpix[q][k];
                int2 tp = make_int2(0, 0);
                float2 fr = make_float2(-1.0f, 0.0f);
                if (REC && i >= 0) {
                    // a kept pixel's taps are on the face or layer of its cell
                    int4 a, b;
                    if (k < HK) {
                        a = ra[q][k < HK ? k : 0];
                        b = rb[q][k < HK ? k : 0];
                    } else {
                        const int4 *rp = rec + 2 * ((int64_t)(g0 + q) * npix + i);
                        a = rp[0];
                        b = rp[1];
                    }
                    tp = make_int2(a.x, a.y);
                    fr = make_float2(__int_as_float(a.z), __int_as_float(a.w));
                    found = 1;
                    cg[q][h * NC] = __int_as_float(b.x);
                    cg[q][h * NC + 1] = __int_as_float(b.y);
                    cg[q][h * NC + 2] = __int_as_float(b.z);
                    cg[q][h * NC + 3] = __int_as_float(b.w);
                } else if (!REC && i >= 0) {
                    const int64_t o = (int64_t)(g0 + q) * npix + i;
                    // the winner's gradient is read alongside its coordinate
                    float g[NC];
                    ldv<CT>(grad_out + o * Ct, g, Ct);
                    const Taps t = make_taps(td, coord + o * cd, f);
                    if (t.ok && t.face == f) {
                        tp = make_int2(t.x0 | (t.x1 << 16), t.y0 | (t.y1 << 16));
                        fr = make_float2(t.fx, t.fy);
                        found = 1;
#pragma unroll
                        for (int c = 0; c < NC; c++)
                            if (CT > 0 || c < Ct) cg[q][h * NC + c] = g[c];
                    }
                }
                ctap[q][h] = tp;
                cfr[q][h] = fr;
            }
        }
        if (!__syncthreads_or(found)) continue;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int ry = ly + 16 * r, ty = by0 + ry;
            if (tx >= Wt || ty >= Ht) continue;
            for (int q = 0; q < ng; q++) {
#pragma unroll
                for (int dy = 0; dy < 3; dy++) {
#pragma unroll
                    for (int dx = 0; dx < 3; dx++) {
                        const int h = (ry + dy) * G::HW + lx + dx;
                        const float2 fr = cfr[q][h];
                        if (fr.x < 0.0f) continue;
                        const int2 tp = ctap[q][h];
                        const int x0 = tp.x & 0xffff, x1 = tp.x >> 16, y0 = tp.y & 0xffff, y1 = tp.y >> 16;
                        float w = 0.0f;
                        if (y0 == ty && x0 == tx) w += (1.0f - fr.y) * (1.0f - fr.x);
                        if (y0 == ty && x1 == tx) w += (1.0f - fr.y) * fr.x;
                        if (y1 == ty && x0 == tx) w += fr.y * (1.0f - fr.x);
                        if (y1 == ty && x1 == tx) w += fr.y * fr.x;
                        if (w == 0.0f) continue;
                        float g[NC];
#pragma unroll
                        for (int c = 0; c < NC; c++)
                            if (CT > 0 || c < Ct) g[c] = cg[q][h * NC + c];
#pragma unroll
                        for (int c = 0; c < NC; c++)
                            if (CT > 0 || c < Ct) acc[r][c] += w * g[c];
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int ty = by0 + ly + 16 * r;
        if (tx >= Wt || ty >= Ht) continue;
        float *gt = out + ((int64_t)part * cells_all + (int64_t)f * face_cells + (int64_t)ty * Wt + tx) * Ct;
        stv<CT>(gt, acc[r], Ct);
    }
}

// Sums the per-part partial texture gradients in part order.
__global__ void k_invuv_reduce(const float *__restrict__ part, int nsplit, int64_t n, float *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float a = part[i];
    for (int k = 1; k < nsplit; k++) a += part[(int64_t)k * n + i];
    out[i] = a;
}

template <int SG, int R>
static void launch_gather_r(int ct, dim3 g, hipStream_t st, const dressi_tex_desc &td, const float *coord,
                            const int32_t *tri_id, int64_t npix, int S, int nsplit, const int32_t *inv,
                            const float *grad_out, float *dst, int xcd, const int4 *rec, LossJob lj,
                            const ListJob &job, int jcols) {
    constexpr int nt = IvGeom<SG, R>::NT;
    if (rec)
        DR_LAUNCH("k_invuv_gather", (k_invuv_gather<4, SG, R, true>), g, nt, 0, st, td, coord, tri_id, npix, S,
                  nsplit, inv, grad_out, dst, xcd, rec, lj, job, jcols);
    else if (ct == 4)
        DR_LAUNCH("k_invuv_gather", (k_invuv_gather<4, SG, R>), g, nt, 0, st, td, coord, tri_id, npix, S,
                  nsplit, inv, grad_out, dst, xcd, rec, lj, job, jcols);
    else if (ct == 3)
        DR_LAUNCH("k_invuv_gather", (k_invuv_gather<3, SG, R>), g, nt, 0, st, td, coord, tri_id, npix, S,
                  nsplit, inv, grad_out, dst, xcd, rec, lj, job, jcols);
    else if (ct == 8)
        DR_LAUNCH("k_invuv_gather", (k_invuv_gather<8, SG, R>), g, nt, 0, st, td, coord, tri_id, npix, S,
                  nsplit, inv, grad_out, dst, xcd, rec, lj, job, jcols);
    else
        DR_LAUNCH("k_invuv_gather", (k_invuv_gather<0, SG, 1>), g, nt, 0, st, td, coord, tri_id, npix, S,
                  nsplit, inv, grad_out, dst, xcd, rec, lj, job, jcols);
}

// Large textures take the XCD-contiguous block order and two texel rows per
// lane in the gather as well.

// Texel rows per lane of the gather: `rows` (1, 2 or 4) or, for 0, 2 rows
// for a single slice or a large texture and 1 otherwise (measured: with one
// slice the larger blocks are faster; with many slices of a 1024^2 texture
// the loop over slices prefers more, smaller blocks in flight; a 4096^2
// texture prefers the larger blocks again).  Any choice gives the same sums
// in the same order.
static int gather_rows(int rows, int ct, int S, const dressi_tex_desc &td, bool rec) {
    if (ct != 3 && ct != 4 && ct != 8) return 1;
    if (rows == 1 || rows == 2 || rows == 4) return rows;
    if ((int64_t)td.Ht * td.Wt >= IV_LARGE_CELLS) return 2;
    return (S == 1 && !rec) ? 2 : 1;
}

static void launch_gather(int rows, int ct, int64_t gx, int64_t ty_cells, int gz, hipStream_t st,
                          const dressi_tex_desc &td, const float *coord, const int32_t *tri_id, int64_t npix,
                          int S, int nsplit, const int32_t *inv, const float *grad_out, float *dst,
                          const int4 *rec, LossJob lj, const ListJob &job) {
    const int R = gather_rows(rows, ct, S, td, rec != nullptr);
    const int xcd = (int64_t)td.Ht * td.Wt >= IV_LARGE_CELLS;
    const int64_t gy = (ty_cells + 16 * R - 1) / (16 * R);
    const int jcols = job.nb > 0 ? (int)((job.nb + gy * gz - 1) / (gy * gz)) : 0;
    dim3 g((unsigned)(gx + (lj.loss ? 1 : 0) + jcols), (unsigned)gy, (unsigned)gz);
    if (R == 4)
        launch_gather_r<DRESSI_IV_SG, 4>(ct, g, st, td, coord, tri_id, npix, S, nsplit, inv, grad_out, dst, xcd,
                                          rec, lj, job, jcols);
    else if (R == 2)
        launch_gather_r<DRESSI_IV_SG, 2>(ct, g, st, td, coord, tri_id, npix, S, nsplit, inv, grad_out, dst, xcd,
                                          rec, lj, job, jcols);
    else
        launch_gather_r<DRESSI_IV_SG, 1>(ct, g, st, td, coord, tri_id, npix, S, nsplit, inv, grad_out, dst, xcd,
                                          rec, lj, job, jcols);
}

// float4 rows need 16-byte aligned bases
static bool aligned16(const void *a, const void *b) {
    return (((uintptr_t)a | (uintptr_t)b) & 15u) == 0;
}

static int check_tex(dressi_ctx *ctx, const void *tex, const dressi_tex_desc *td, const void *coord,
                     const void *tid, int S, int H, int W) {
    if (!ctx) return DRESSI_EINVAL;
    if (!td) return dressi_fail(ctx, DRESSI_EINVAL, "texture: null descriptor");
    if (td->kind != DRESSI_TEX_2D && td->kind != DRESSI_TEX_CUBE && td->kind != DRESSI_TEX_2D_ARRAY)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: bad kind");
    if (td->kind == DRESSI_TEX_2D_ARRAY && (td->layers < 1 || !td->tri_layer || !tid))
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: an array needs layers >= 1, tri_layer and tri_id");
    if (td->Ht < 1 || td->Wt < 1 || td->Ct < 1 || td->Ct > 16 || td->Ht > 32767 || td->Wt > 32767)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: bad texture shape (Ht, Wt 1..32767, Ct 1..16)");
    if (td->kind == DRESSI_TEX_CUBE && td->Ht != td->Wt)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture: cube faces must be square");
    if (td->kind != DRESSI_TEX_CUBE) {
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
    const int g = (int)((n + 255) / 256);
    switch (aligned16(tex, out) ? td->Ct : 0) {
    case 3: DR_LAUNCH("k_tex_fwd", (k_tex_fwd<3>), g, 256, 0, st, tex, *td, coord, tri_id, n, out, ctx->skip_empty); break;
    case 4: DR_LAUNCH("k_tex_fwd", (k_tex_fwd<4>), g, 256, 0, st, tex, *td, coord, tri_id, n, out, ctx->skip_empty); break;
    case 8: DR_LAUNCH("k_tex_fwd", (k_tex_fwd<8>), g, 256, 0, st, tex, *td, coord, tri_id, n, out, ctx->skip_empty); break;
    default: DR_LAUNCH("k_tex_fwd", (k_tex_fwd<0>), g, 256, 0, st, tex, *td, coord, tri_id, n, out, ctx->skip_empty); break;
    }
    return dressi_launch_check(ctx, "texture");
}

// Records every covered pixel of the S slices in its cell of the inverse-UV
// map (cleared to -1 first) and, when grad_coord is given, writes d out / d coord.
static void tex_bwd_pixels(const float *tex, const dressi_tex_desc &td, const float *coord,
                           const int32_t *tri_id, int64_t npix, int S, const float *grad_out,
                           float *grad_coord, int32_t *inv, hipStream_t st, int skip_empty = 0) {
    const int64_t n = (int64_t)S * npix;
    // cleared for every slice, also when slices are empty: the gather reads them all
    if (inv && S > 0) dressi_fill_i32(inv, -1, (int64_t)tex_faces(td) * td.Ht * td.Wt * S, st);
    if (n == 0 || (!grad_coord && !inv)) return;
    const int g = (int)((n + 255) / 256);
    switch (grad_coord && aligned16(tex, grad_out) ? td.Ct : 0) {
    case 3: DR_LAUNCH("k_tex_bwd_pixel", (k_tex_bwd_pixel<3>), g, 256, 0, st, tex, td, coord, tri_id, npix, S,
                      grad_out, grad_coord, inv, skip_empty); break;
    case 4: DR_LAUNCH("k_tex_bwd_pixel", (k_tex_bwd_pixel<4>), g, 256, 0, st, tex, td, coord, tri_id, npix, S,
                      grad_out, grad_coord, inv, skip_empty); break;
    case 8: DR_LAUNCH("k_tex_bwd_pixel", (k_tex_bwd_pixel<8>), g, 256, 0, st, tex, td, coord, tri_id, npix, S,
                      grad_out, grad_coord, inv, skip_empty); break;
    default: DR_LAUNCH("k_tex_bwd_pixel", (k_tex_bwd_pixel<0>), g, 256, 0, st, tex, td, coord, tri_id, npix,
                       S, grad_out, grad_coord, inv, skip_empty); break;
    }
}

// The texture gradient gathered from a built inverse-UV map.  Small textures
// (an environment map) have few texel blocks: their slices are split over the
// grid as well and the parts summed afterwards in `part`.
static void tex_gather(const dressi_tex_desc &td, const float *coord, const int32_t *tri_id, int64_t npix,
                       int S, const int32_t *inv, const float *grad_out, float *part, float *grad_tex,
                       hipStream_t st, int rows, const int4 *rec = nullptr, LossJob lj = LossJob{},
                       const ListJob &job = ListJob{}) {
    const int64_t cells = (int64_t)tex_faces(td) * td.Ht * td.Wt;
    const int nsplit = dressi_invuv_nsplit(cells, S);
    float *dst = nsplit > 1 ? part : grad_tex;
    const int ct = rec ? 4 : (aligned16(grad_out, dst) ? td.Ct : 0);
    launch_gather(rows, ct, (td.Wt + IV_T - 1) / IV_T, td.Ht, tex_faces(td) * nsplit, st, td, coord, tri_id,
                  npix, S, nsplit, inv, grad_out, dst, rec, lj, job);
    if (nsplit > 1) {
        int64_t ne = cells * td.Ct;
        DR_LAUNCH("k_invuv_reduce", (k_invuv_reduce), (int)((ne + 255) / 256), 256, 0, st, part, nsplit, ne,
                  grad_tex);
    }
}

static int check_grad_tex(dressi_ctx *ctx, const dressi_tex_desc *td, const int32_t *tri_id, const char *what) {
    if (!tri_id) return dressi_fail(ctx, DRESSI_EINVAL, what);
    if (td->kind != DRESSI_TEX_CUBE &&
        ((td->wrap_u == DRESSI_WRAP_REPEAT && td->Wt < 3) || (td->wrap_v == DRESSI_WRAP_REPEAT && td->Ht < 3)))
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_bwd: repeat wrap needs at least 3 texels");
    return DRESSI_OK;
}

extern "C" int dressi_texture_bwd(dressi_ctx *ctx, const float *tex, const dressi_tex_desc *td,
                                  const float *coord, const int32_t *tri_id, int S, int H, int W,
                                  const float *grad_out, uint32_t frame, float *grad_tex, float *grad_coord,
                                  void *stream) {
    int rc = check_tex(ctx, tex, td, coord, tri_id, S, H, W);
    if (rc) return rc;
    int64_t npix = (int64_t)H * W, n = (int64_t)S * npix;
    if (n > 0 && !grad_out) return dressi_fail(ctx, DRESSI_EINVAL, "texture_bwd: null grad_out");
    if (grad_tex && (rc = check_grad_tex(ctx, td, tri_id, "texture_bwd: the texture gradient needs tri_id")))
        return rc;
    const bool jit = grad_tex && frame > 0;
    if (jit && td->kind == DRESSI_TEX_2D_ARRAY)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_bwd: jitter (frame > 0) is for 2-D and cube textures");
    hipStream_t st = (hipStream_t)stream;
    int32_t *inv = nullptr;
    float *part = nullptr, *jc = nullptr, *jg = nullptr;
    const int cd = td->kind == DRESSI_TEX_CUBE ? 3 : 2;
    int64_t cells = (int64_t)tex_faces(*td) * td->Ht * td->Wt;
    if (grad_tex) {
        Carver c;
        size_t o_inv = c.take(sizeof(int32_t) * (size_t)cells * (S > 0 ? S : 1));
        size_t o_part = c.take(dressi_invuv_part_bytes(cells, td->Ct, S));
        size_t o_jc = jit ? c.take(sizeof(float) * (size_t)n * cd) : 0;
        size_t o_jg = jit ? c.take(sizeof(float) * (size_t)n * td->Ct) : 0;
        rc = dressi_scratch(ctx, c.off, st);
        if (rc) return rc;
        inv = at<int32_t>(ctx->scratch, o_inv);
        part = at<float>(ctx->scratch, o_part);
        if (jit) {
            jc = at<float>(ctx->scratch, o_jc);
            jg = at<float>(ctx->scratch, o_jg);
        }
    }
    if (!jit) {
        tex_bwd_pixels(tex, *td, coord, tri_id, npix, S, grad_out, grad_coord, inv, st, ctx->skip_empty);
        if (grad_tex) tex_gather(*td, coord, tri_id, npix, S, inv, grad_out, part, grad_tex, st, ctx->iv_rows);
        return dressi_launch_check(ctx, "texture_bwd");
    }
    // jittered registration beside the unmoved coordinate gradient
    tex_bwd_pixels(tex, *td, coord, tri_id, npix, S, grad_out, grad_coord, nullptr, st, ctx->skip_empty);
    if (S > 0) dressi_fill_i32(inv, -1, cells * S, st);
    if (n > 0) {
        const Jitter j = jitter_of_frame(frame);
        const int g = (int)((n + 255) / 256);
        switch (td->Ct) {
        case 3: DR_LAUNCH("k_invuv_jitter", (k_invuv_jitter<3>), g, 256, 0, st, *td, coord, tri_id, H, W, S,
                          grad_out, j, jc, jg, inv); break;
        case 4: DR_LAUNCH("k_invuv_jitter", (k_invuv_jitter<4>), g, 256, 0, st, *td, coord, tri_id, H, W, S,
                          grad_out, j, jc, jg, inv); break;
        case 8: DR_LAUNCH("k_invuv_jitter", (k_invuv_jitter<8>), g, 256, 0, st, *td, coord, tri_id, H, W, S,
                          grad_out, j, jc, jg, inv); break;
        default: DR_LAUNCH("k_invuv_jitter", (k_invuv_jitter<0>), g, 256, 0, st, *td, coord, tri_id, H, W, S,
                           grad_out, j, jc, jg, inv); break;
        }
    }
    tex_gather(*td, jc, tri_id, npix, S, inv, jg, part, grad_tex, st, ctx->iv_rows);
    return dressi_launch_check(ctx, "texture_bwd");
}

extern "C" size_t dressi_invuv_bytes(const dressi_tex_desc *td, int S) {
    if (!td || S < 0 || td->Ht < 1 || td->Wt < 1) return 0;
    if (td->kind == DRESSI_TEX_2D_ARRAY && td->layers < 1) return 0;
    return sizeof(int32_t) * (size_t)tex_faces(*td) * td->Ht * td->Wt * (size_t)S;
}

extern "C" int dressi_invuv_build(dressi_ctx *ctx, const dressi_tex_desc *td, const float *coord,
                                  const int32_t *tri_id, int S, int H, int W, int32_t *inv, void *stream) {
    // the texels themselves are not read: any non-null pointer passes the shared check
    int rc = check_tex(ctx, coord, td, coord, tri_id, S, H, W);
    if (rc) return rc;
    if ((rc = check_grad_tex(ctx, td, tri_id, "invuv_build: needs tri_id"))) return rc;
    if (S > 0 && !inv) return dressi_fail(ctx, DRESSI_EINVAL, "invuv_build: null inv");
    tex_bwd_pixels(nullptr, *td, coord, tri_id, (int64_t)H * W, S, nullptr, nullptr, inv, (hipStream_t)stream);
    return dressi_launch_check(ctx, "invuv_build");
}

extern "C" int dressi_texture_grad_invuv(dressi_ctx *ctx, const dressi_tex_desc *td, const float *coord,
                                         const int32_t *tri_id, int S, int H, int W, const int32_t *inv,
                                         const float *grad_out, float *grad_tex, void *stream) {
    int rc = check_tex(ctx, coord, td, coord, tri_id, S, H, W);
    if (rc) return rc;
    if ((rc = check_grad_tex(ctx, td, tri_id, "texture_grad_invuv: needs tri_id"))) return rc;
    if (!grad_tex) return dressi_fail(ctx, DRESSI_EINVAL, "texture_grad_invuv: null grad_tex");
    if (S > 0 && (!inv || (H * W > 0 && !grad_out)))
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_grad_invuv: null inv or grad_out");
    hipStream_t st = (hipStream_t)stream;
    const int64_t cells = (int64_t)tex_faces(*td) * td->Ht * td->Wt;
    float *part = nullptr;
    const size_t pb = dressi_invuv_part_bytes(cells, td->Ct, S);
    if (pb) {
        if ((rc = dressi_scratch(ctx, pb, st))) return rc;
        part = at<float>(ctx->scratch, 0);
    }
    tex_gather(*td, coord, tri_id, (int64_t)H * W, S, inv, grad_out, part, grad_tex, st, ctx->iv_rows);
    return dressi_launch_check(ctx, "texture_grad_invuv");
}

void dr_gather_invrec(const dressi_tex_desc &td, int S, int64_t npix, const int32_t *inv, const int4 *rec,
                      float *part, float *grad_tex, hipStream_t st, int rows, LossJob lj, const ListJob &job) {
    tex_gather(td, nullptr, nullptr, npix, S, inv, nullptr, part, grad_tex, st, rows, rec, lj, job);
}

extern "C" int dressi_texture_grad_invrec(dressi_ctx *ctx, const dressi_tex_desc *td, int S, int H, int W,
                                          const int32_t *inv, const void *rec, float *grad_tex, void *stream) {
    // the records stand in for the texels, coordinates and triangle ids in the shared checks
    int rc = check_tex(ctx, rec, td, rec, rec, S, H, W);
    if (rc) return rc;
    if ((rc = check_grad_tex(ctx, td, inv, "texture_grad_invrec: null inv"))) return rc;
    if (td->kind == DRESSI_TEX_CUBE || td->Ct != 4)
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_grad_invrec: records are for 2-D RGBA textures and arrays");
    if (!grad_tex || !aligned16(rec, grad_tex))
        return dressi_fail(ctx, DRESSI_EINVAL, "texture_grad_invrec: rec and grad_tex must be 16-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int64_t cells = (int64_t)tex_faces(*td) * td->Ht * td->Wt;
    float *part = nullptr;
    const size_t pb = dressi_invuv_part_bytes(cells, td->Ct, S);
    if (pb) {
        if ((rc = dressi_scratch(ctx, pb, st))) return rc;
        part = at<float>(ctx->scratch, 0);
    }
    tex_gather(*td, nullptr, nullptr, (int64_t)H * W, S, inv, nullptr, part, grad_tex, st, ctx->iv_rows,
               static_cast<const int4 *>(rec));
    return dressi_launch_check(ctx, "texture_grad_invrec");
}

// texture_bwd (with jitter when asked), texture_grad_invuv and _invrec
size_t dr_need_texture(const dressi_limits &l) {
    if (l.tex_cells <= 0 || l.tex_channels <= 0) return 0;
    const int S = std::max(l.tex_slices, 1);
    Carver c;
    c.take(sizeof(int32_t) * (size_t)l.tex_cells * S);
    c.take(dressi_invuv_part_bytes(l.tex_cells, l.tex_channels, S));
    if (l.jitter) {
        const size_t n = (size_t)S * std::max(l.H, 0) * std::max(l.W, 0);
        c.take(sizeof(float) * n * 3);
        c.take(sizeof(float) * n * l.tex_channels);
    }
    return c.off;
}
