/*
 * dressi.h — C ABI of libdressi.so, the gfx950 (MI355X) implementation of the
 * rasterization hot path of the differentiable renderer "Dressi"
 * (Eurographics 2022): rasterization with HardSoftRas soft coverage,
 * perspective-correct attribute interpolation, bilinear texture sampling,
 * the HardSoftRas blend, and the backward of each.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer to caller-owned, contiguous,
 *   row-major memory of the dtype stated (float = IEEE binary32, int32_t,
 *   uint8_t).  The library never frees, keeps or reallocates caller memory.
 * - Per-pixel planes are laid out [B,K,H,W(,c)]: view b, layer k, row y (row 0
 *   at the top of the image), column x.  Pixel (x,y) is sampled at its centre
 *   (x + 1/2, y + 1/2).  Clip coordinates are (x,y,z,w) with x/w, y/w in [-1,1]
 *   across the viewport (y up) and z/w in [0,1] between near and far.
 * - Outputs and gradient outputs are fully OVERWRITTEN (never accumulated).
 * - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *   enqueues work on it and returns without waiting; it performs no host
 *   synchronisation and no allocation once the context holds enough scratch
 *   (dressi_reserve), so calls can be captured into a hipGraph.  Calls that
 *   share a context must be issued on one stream (they share its scratch).
 * - Return value: DRESSI_OK or a negative status; dressi_last_error() gives a
 *   message.  Errors are detected on the host (arguments, scratch) before any
 *   launch; a rejected call launches nothing (dressi_packed_step, which
 *   chains four calls, stops at the first that refuses: see there).
 *   Bin-capacity overflow can only
 *   be seen on the device: it is recorded there and reported by
 *   dressi_check_status(), and the affected outputs are then invalid.
 *
 * Paper references name sections, equations and algorithms of the paper.
 */
#ifndef DRESSI_H
#define DRESSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DRESSI_OK 0
#define DRESSI_EINVAL (-1)    /* bad argument (null pointer, shape, range)   */
#define DRESSI_ENOMEM (-2)    /* scratch too small while capturing / no mem  */
#define DRESSI_EHIP (-3)      /* a HIP runtime call or launch failed         */
#define DRESSI_EOVERFLOW (-4) /* device-side bin capacity exceeded           */

/* texture kinds and wrap modes */
#define DRESSI_TEX_2D 0   /* tex [Ht,Wt,Ct], coord (u,v); u along columns, v along rows */
#define DRESSI_TEX_CUBE 1 /* tex [6,S,S,Ct] faces +X,-X,+Y,-Y,+Z,-Z; coord = direction */
#define DRESSI_TEX_2D_ARRAY 2 /* tex [L,Ht,Wt,Ct]; coord (u,v); layer from the triangle */
#define DRESSI_WRAP_REPEAT 0
#define DRESSI_WRAP_CLAMP 1

/* blend modes of the HardSoftRas blend (§3.4.3) */
#define DRESSI_BLEND_HSR 0     /* edge mask from S^H, dilated to width delta       */
#define DRESSI_BLEND_AA 1      /* edge mask = silhouette boundary (delta = 1 pixel) */
#define DRESSI_BLEND_SOFTRAS 2 /* edge mask = 1 everywhere                         */
#define DRESSI_BLEND_HARD 3    /* edge mask = 0: I = S^H C_1, alpha = S^H           */

typedef struct dressi_ctx dressi_ctx;

typedef struct {
    int kind;           /* DRESSI_TEX_2D, DRESSI_TEX_CUBE (Ht == Wt == S) or DRESSI_TEX_2D_ARRAY */
    int Ht, Wt, Ct;     /* texels per column, per row (1..32767), channels (1..16) */
    int wrap_u, wrap_v; /* 2D and arrays; repeat needs Wt (Ht) >= 3               */
    int layers;         /* arrays: number of layers                              */
    const int32_t *tri_layer; /* arrays: device [T] layer of each triangle; a
                                 fragment samples its triangle's layer (tri_id
                                 is then required)                              */
} dressi_tex_desc;

/* ----------------------------------------------------------------------------
 * Context.  Owns only scratch memory (setup records, tile bins, per-tile
 * fragment lists, inverse-UV slices, adjacency lists) and a small device
 * status word.  One context per device and stream.
 * ------------------------------------------------------------------------- */
int dressi_create(dressi_ctx **ctx, int device);
int dressi_destroy(dressi_ctx *ctx);
const char *dressi_last_error(const dressi_ctx *ctx);
/* Grow scratch to at least `bytes` and the tile-bin capacity to at least
 * `bin_entries` (pass 0 to leave either unchanged).  Synchronises the device.
 * Scratch grows (here, or in an eager call that needs more) by allocating a
 * larger arena; the old one is retired, not freed, because a graph captured
 * before the growth still uses its addresses.  Retired arenas are freed by
 * dressi_destroy, so a captured graph stays valid until then; reserve the
 * largest shapes first to keep a single arena. */
int dressi_reserve(dressi_ctx *ctx, size_t bytes, int64_t bin_entries);
/* Bytes of scratch the given call shapes need (for dressi_reserve before a
 * graph capture).  Pass the largest shapes of the step. */
size_t dressi_scratch_bytes(int B, int V, int T, int H, int W, int K, float r,
                            int Va, int C, int64_t tex_cells, int tex_slices);
/* (dressi_scratch_bytes covers the four rendering stages; the limits below
 * cover every entry point.) */

/* The largest shapes a context will be called with, for sizing its scratch
 * once, before any graph capture.  Zero fields are unused stages. */
typedef struct {
    int B, V, T, H, W, K; /* views (or 1 for an uneven batch), vertices, triangles,
                             image, layers of rasterize(_banded, _batched)(_bwd),
                             fragment_index, adjacency and vertex_attrs(_bwd)   */
    float r;              /* soft reach (0 = hard only)                           */
    int Va, C;            /* attribute rows and channels of interpolate_bwd        */
    int64_t tex_cells;    /* faces (or layers) x Ht x Wt of the largest texture    */
    int tex_channels;     /* its channels Ct                                       */
    int tex_slices;       /* slices S of a texture_bwd call                        */
    int jitter;           /* 1 if texture_bwd is called with frame >= 1            */
    int ibl_S, ibl_Si, ibl_Sp, ibl_L; /* ibl_filter(_bwd) shapes (0 = none)        */
    int64_t pbs_fragments; /* N of shade_pbs_bwd with a material gradient          */
    int64_t bin_entries;  /* tile-bin capacity (0 = automatic for the shapes)      */
} dressi_limits;
/* Bytes of scratch that every entry point needs at these limits (the
 * largest single call, with every optional index built internally). */
size_t dressi_limits_scratch_bytes(const dressi_limits *l);
/* Grows the context's scratch arena, its zeroed counters and the tile-bin
 * capacity to the limits: afterwards no call within them allocates, so a
 * graph can be captured without an eager call first.  Synchronises the
 * device. */
int dressi_reserve_limits(dressi_ctx *ctx, const dressi_limits *l);
/* Waits for `stream`, then returns DRESSI_EOVERFLOW (and clears the flag) if a
 * rasterization since the last check overflowed the bin capacity; *needed
 * receives the capacity that call required (may be NULL). */
int dressi_check_status(dressi_ctx *ctx, int64_t *needed, void *stream);

/* Tuning knobs that change speed, never results (an autotuner times the
 * candidates on the real workload and keeps the fastest):
 * DRESSI_TUNE_BIN_CAPACITY: triangles per 16x16 tile bin (0 = automatic;
 *   too small a capacity is reported by dressi_check_status);
 * DRESSI_TUNE_HARD_RASTER: hard rasterization (r = 0) strategy, 0 =
 *   triangle-parallel per tile with LDS atomics (small triangles), 1 =
 *   pixel-parallel with per-pixel lists in registers (large triangles), 2 =
 *   chosen per tile and batch of 256 binned triangles from their on-tile
 *   extents (K = 1; with K > 1 it acts as 1), 3 = without bins: one lane per
 *   triangle merges its keys into a per-pixel array with global atomics,
 *   then each pixel is resolved (K = 1; with K > 1 it acts as 0; small
 *   triangles).  All select exactly the same layers;
 * DRESSI_TUNE_HYBRID_WEIGHT: for strategy 2, the cost of a pixel-parallel
 *   triangle step relative to a triangle-parallel pixel step, in sixteenths
 *   (1..1024, default 24).
 * DRESSI_TUNE_EMPTY_SLOTS: 0 (default) = per-fragment outputs are fully
 *   overwritten, with zeros at empty fragment slots (tri_id < 0); 1 = the
 *   entries of empty slots are left unwritten (undefined) by
 *   dressi_interpolate (out), dressi_texture (out), dressi_shade (color,
 *   dir), dressi_softras_bwd (grad_layer_color, grad_dist),
 *   dressi_shade_bwd (every member), dressi_texture_bwd (grad_coord) and
 *   dressi_interpolate_bwd (grad_bary).  Every entry point reads those
 *   outputs only at non-empty slots, so a pipeline built from them gets the
 *   same results either way and skips the zero stores (most slots of the
 *   deeper layers are empty).  Changes which bytes are written, never a
 *   value at a non-empty slot.
 * DRESSI_TUNE_IV_ROWS: texel rows per lane of the inverse-UV gather of
 *   dressi_texture_bwd and dressi_texture_grad_invuv: 1, 2 or 4 (0 =
 *   automatic).  Each workgroup covers 16 x 16*rows texels; every choice
 *   adds the same terms in the same order. */
#define DRESSI_TUNE_BIN_CAPACITY 1
#define DRESSI_TUNE_HARD_RASTER 2
#define DRESSI_TUNE_HYBRID_WEIGHT 3
#define DRESSI_TUNE_EMPTY_SLOTS 4
#define DRESSI_TUNE_IV_ROWS 5
int dressi_tune(dressi_ctx *ctx, int key, int64_t value);

/* Kernel timing for measurement: while on, every kernel launch of the library
 * gets a start/stop HIP event pair that the runtime stamps from the launch's
 * own dispatch (the kernel's execution time alone).  dressi_profile_start(n) turns it
 * on for up to n launches (0 turns it off); dressi_profile_read waits for the
 * recorded launches, returns their count and fills names[i] (static strings)
 * and ms[i], then starts a new window.  Process-wide; not for use while a
 * stream is being captured. */
int dressi_profile_start(int max_launches);
int dressi_profile_read(const char **names, float *ms, int max);

/* ----------------------------------------------------------------------------
 * Rasterization (Algorithm 2, §3.4.2; the Shift equation; PeelDepth).
 *
 * pos_clip [B,V,4] float: clip-space vertices of view b.  tris [T,3] int32:
 * vertex indices, shared by all views.  K in 1..5 layers, r in [0,1]: soft
 * reach in screen units (pixels / W); r = 0 rasterizes hard coverage only.
 * cull: 0 = none, 1 = drop faces that are clockwise in NDC.
 *
 * Triangles are snapped to 1/256 pixel.  A pixel is hard-covered under the
 * top-left fill rule with depth key 0.5*z/w (fragments with z/w outside (0,1)
 * are dropped); when r > 0 a pixel not hard-covered whose distance to the
 * triangle is <= r gets a soft fragment with key 0.5 + 0.5*distance.  Layer k
 * of a pixel holds the k-th smallest distinct key, and the smallest triangle
 * id at that key.  Outputs:
 *   tri_id [B,K,H,W] int32  triangle index, -1 for an empty layer;
 *   bary   [B,K,H,W,2] float perspective-correct barycentrics of corners 0,1
 *          (corner 2 = 1 - b0 - b1; soft fragments extrapolate), 0 if empty;
 *   dist   [B,K,H,W] float  signed distance to the triangle in screen units,
 *          + for hard and - for soft fragments (the sign bit carries the
 *          flag, also at 0), 0 if empty.  Required iff r > 0, else may be NULL.
 * Limits: T < 2^31 - 1, |vertex| within a +-16384-pixel guard band, w > 0
 * for all three vertices of a rasterized triangle (others are dropped).
 * ------------------------------------------------------------------------- */
int dressi_rasterize(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                     int B, int V, int T, int H, int W, int K, float r, int cull,
                     int32_t *tri_id, float *bary, float *dist, void *stream);

/* Edge-band form of dressi_rasterize for a HardSoftRas blend (§3.4.3): with
 * the blend's edge mask E (dressi_softras with the same delta and mode), the
 * image outside E is S^H C_1 and the silhouette S^H, so there only the front
 * hard fragment reaches the image or any gradient.  The banded outputs equal
 * dressi_rasterize's on every pixel of E; outside E, layer 0 is kept when it
 * is hard (else empty) and layers 1..K-1 are empty.  E is built here from
 * the front hard fragments (S^H does not depend on the soft layers), and the
 * soft candidates are searched only in tiles that meet E.  blend_mode:
 * DRESSI_BLEND_HSR (E = boundary of S^H dilated by ceil(delta W) - 1
 * pixels), _AA (the boundary itself), _HARD (E empty), _SOFTRAS (E is every
 * pixel: the full form).  Needs r > 0 and dist.  The blend's image, its
 * silhouette and the gradients of positions and vertex attributes are those
 * of the full form; texture gradients differ where the full form's pixels
 * outside E (whose gradient is zero) win inverse-UV cells. */
int dressi_rasterize_banded(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B, int V,
                            int T, int H, int W, int K, float r, int cull, float delta, int blend_mode,
                            int32_t *tri_id, float *bary, float *dist, void *stream);

/* Backward of dressi_rasterize with frozen visibility: the gradients of bary
 * and dist carried to the clip-space vertices (Rasterize and PeelDepth have no
 * backward of their own; snapping is treated as the identity).  grad_bary
 * [B,K,H,W,2], grad_dist [B,K,H,W] (NULL = zero), tri_id from the forward.
 * frag_index: a fragment index of tri_id (dressi_fragment_index) or NULL to
 * build one internally; adj: the vertex adjacency of tris (dressi_adjacency)
 * or NULL.  Output grad_pos_clip [B,V,4] (the z component is 0).
 * Deterministic: fragments are sorted by triangle id per tile, every triangle
 * sums its fragments in that order and every vertex its corners in order. */
int dressi_rasterize_bwd(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                         int B, int V, int T, int H, int W, int K, float r, int cull,
                         const int32_t *tri_id, const float *grad_bary, const float *grad_dist,
                         const void *frag_index, const int32_t *adj, float *grad_pos_clip,
                         void *stream);

/* Uneven batches, hard rasterization (r = 0): triangle t of the concatenated
 * meshes belongs to view tri_view[t], drawn in the rectangle
 * views[4*v .. 4*v+3] = (x0, y0, W_v, H_v) (device int32) of one H x W image.
 * Each triangle is snapped in its own view's frame (exactly as a standalone
 * W_v x H_v render) and then moved by the integer offset; it covers only
 * pixels of its rectangle.  Outputs as dressi_rasterize with B = 1:
 * tri_id [K,H,W] (global triangle ids), bary [K,H,W,2].  The backward gives
 * grad_pos_clip [V,4] of the concatenated vertices. */
int dressi_rasterize_batched(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                             const int32_t *tri_view, const int32_t *views, int n, int V, int T,
                             int H, int W, int K, int cull, int32_t *tri_id, float *bary,
                             void *stream);
int dressi_rasterize_batched_bwd(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris,
                                 const int32_t *tri_view, const int32_t *views, int n, int V, int T,
                                 int H, int W, int K, int cull, const int32_t *tri_id,
                                 const float *grad_bary, const void *frag_index, const int32_t *adj,
                                 float *grad_pos_clip, void *stream);

/* ----------------------------------------------------------------------------
 * Reusable index structures for the deterministic backward reductions.
 *
 * dressi_adjacency: for a mesh tris [T,3] over V vertices, writes adj
 * (V + 1 + 3T int32, caller-owned): offsets [V+1] then, per vertex, its
 * corners 3t+i in ascending order.  Depends only on the topology: build once
 * per mesh and pass it to the calls taking `adj`.
 *
 * dressi_fragment_index: from tri_id [B,K,H,W] (triangles < T), writes into
 * `index` (dressi_fragment_index_bytes(...) bytes, caller-owned, opaque) the
 * fragments of every 16x16 screen tile sorted by triangle id (per tile:
 * wavefront sorts of 64 keys merged by rank in LDS) and, per (view, triangle), the list of tiles holding its
 * fragments.  Build once per rasterization and pass it to rasterize_bwd and
 * interpolate_bwd.
 * ------------------------------------------------------------------------- */
int dressi_adjacency(dressi_ctx *ctx, const int32_t *tris, int T, int V, int32_t *adj, void *stream);
size_t dressi_fragment_index_bytes(int B, int K, int H, int W, int T);
int dressi_fragment_index(dressi_ctx *ctx, const int32_t *tri_id, int B, int K, int H, int W, int T,
                          void *index, void *stream);
/* Rasterization (Algorithm 2 for one hard layer) and the fragment index of
 * its result in one call: the outputs of dressi_rasterize with K = 1, r = 0
 * (tri_id [B,H,W], bary [B,H,W,2]) and of dressi_fragment_index of that
 * tri_id (index: dressi_fragment_index_bytes(B, 1, H, W, T) bytes).  With the
 * binless strategy (DRESSI_TUNE_HARD_RASTER = 3) each tile's resolve hands
 * its triangle ids to the tile's fragment sort in the same launch; with the
 * others the two calls run in sequence.  The caller owns every buffer; the
 * library's scratch and zero-kept counters serve the launches.  Errors:
 * DRESSI_EINVAL for a null pointer, B, V or T negative, T >= 2^31 - 1, or H
 * or W outside 1..32767, with nothing launched. */
int dressi_rasterize_indexed(dressi_ctx *ctx, const float *pos_clip, const int32_t *tris, int B, int V, int T,
                             int H, int W, int cull, int32_t *tri_id, float *bary, void *index, void *stream);

/* ----------------------------------------------------------------------------
 * Attribute interpolation (BuildInterpolate, appendix listing):
 *   out[b,k,y,x,:] = b0*attr[a0] + b1*attr[a1] + (1-b0-b1)*attr[a2],
 * (a0,a1,a2) = attr_tris[tri_id], 0 where tri_id < 0.  attr [Ba,Va,C] with
 * Ba = 1 (shared by all views) or Ba = B.  attr_tris [T,3] may differ from the
 * raster triangles (e.g. split UV seams).  C in 1..64.
 * ------------------------------------------------------------------------- */
int dressi_interpolate(dressi_ctx *ctx, const float *attr, int Ba, int Va, int C,
                       const int32_t *attr_tris, int T, const int32_t *tri_id,
                       const float *bary, int B, int K, int H, int W, float *out, void *stream);

/* grad_attr [Ba,Va,C] (summed over views when Ba = 1) and grad_bary
 * [B,K,H,W,2]; either may be NULL.  grad_bary_in (NULL = 0) is added to
 * grad_bary, so several interpolations of one rasterization can chain their
 * barycentric gradients.  frag_index / adj (of attr_tris over Va vertices):
 * as for dressi_rasterize_bwd, NULL = built internally.  Deterministic.
 * With grad_attr, ((C + 2) | 1) * K must be at most 160 (a tile's fragments are
 * staged in at most 160 KiB of LDS); larger requests return DRESSI_EINVAL. */
int dressi_interpolate_bwd(dressi_ctx *ctx, const float *attr, int Ba, int Va, int C,
                           const int32_t *attr_tris, int T, const int32_t *tri_id,
                           const float *bary, int B, int K, int H, int W,
                           const float *grad_out, const float *grad_bary_in,
                           const void *frag_index, const int32_t *adj, float *grad_attr,
                           float *grad_bary, void *stream);

/* ----------------------------------------------------------------------------
 * Bilinear texture sampling (the sampler behind GLSL texture(), §3.3.2).
 * coord [S,H,W,2] (u,v) for 2D or [S,H,W,3] directions for cube maps, one
 * slice per (view, layer); tri_id [S,H,W] masks empty pixels (output 0).
 * Texel coordinates s = u*Wt - 1/2, t = v*Ht - 1/2; taps floor(s)+{0,1},
 * floor(t)+{0,1} wrapped (repeat) or clamped.  out [S,H,W,Ct].
 * ------------------------------------------------------------------------- */
int dressi_texture(dressi_ctx *ctx, const float *tex, const dressi_tex_desc *td,
                   const float *coord, const int32_t *tri_id, int S, int H, int W,
                   float *out, void *stream);

/* Backward.  grad_coord [S,H,W,2|3]: analytic derivative of the bilinear
 * weights (and of the cube face mapping).  grad_tex [(6,)Ht,Wt,Ct]: the
 * paper's inverse-UV texture (Algorithm 1): per slice, each texel cell keeps
 * the largest covered pixel index whose coordinate falls in it; every texel
 * then gathers, from the distinct in-range cells of its 3x3 neighbourhood in
 * every slice, the kept pixel's gradient times that pixel's bilinear weight on
 * the texel.  Integer atomicMax on pixel indices only, no float atomics; the
 * sum runs over slices, then cells in row-major order.  Either output may be
 * NULL.  Needs Ht, Wt >= 3 for repeat wrap.
 * frame: 0 = no jitter (as above).  frame >= 1 moves the sampling positions
 * of the inverse UV by the frame's quasi-random offset (§3.3.2: a Sobol
 * sequence, so that the pixel a cell keeps changes from frame to frame):
 * o = Sobol(frame) - 1/2 in both axes (the 2-D Sobol point of index frame,
 * base-2 radical inverse and the direction numbers of x + 1, 24 bits).  A
 * covered pixel registers the coordinate and the gradient sampled
 * bilinearly from this slice's coord and grad_out planes at its centre plus
 * o (in float, ((w00 v00 + w01 v01) + w10 v10) + w11 v11), but only when
 * the four pixels sampled are covered pixels of the image; the gather then
 * uses those samples.  grad_coord does not depend on frame.  2-D and cube
 * textures (EINVAL for arrays). */
int dressi_texture_bwd(dressi_ctx *ctx, const float *tex, const dressi_tex_desc *td,
                       const float *coord, const int32_t *tri_id, int S, int H, int W,
                       const float *grad_out, uint32_t frame, float *grad_tex, float *grad_coord,
                       void *stream);

/* The two halves of the texture gradient of dressi_texture_bwd, for a scene
 * whose geometry is held fixed while only textures are optimised (the
 * paper's reactive cache, §3.3.3, skips the unchanged rasterization; its
 * cross-platform table times texture-only iterations): the inverse-UV map
 * depends only on coord and tri_id, so it is built once and every later
 * step only gathers.
 * dressi_invuv_bytes: size of the map, S * F * Ht * Wt int32 (F = 6 for a
 * cube map, the layer count of an array, else 1); 0 for a bad descriptor.
 * dressi_invuv_build: writes the map into caller-owned device memory `inv`
 * (every cell -1, then the largest covered pixel index of each slice whose
 * coordinate falls in it).  Texels are not read.
 * dressi_texture_grad_invuv: grad_tex from grad_out [S,H,W,Ct] through a map
 * built from the same coord and tri_id; bitwise what dressi_texture_bwd
 * gives.  Both need tri_id, and Ht, Wt >= 3 for repeat wrap (DRESSI_EINVAL
 * otherwise); inv is read, never written, by the gather. */
size_t dressi_invuv_bytes(const dressi_tex_desc *td, int S);
int dressi_invuv_build(dressi_ctx *ctx, const dressi_tex_desc *td, const float *coord,
                       const int32_t *tri_id, int S, int H, int W, int32_t *inv, void *stream);
int dressi_texture_grad_invuv(dressi_ctx *ctx, const dressi_tex_desc *td, const float *coord,
                              const int32_t *tri_id, int S, int H, int W, const int32_t *inv,
                              const float *grad_out, float *grad_tex, void *stream);
/* The same gather (Algorithm 1's gathering pass, §3.3.2) from per-pixel
 * records instead of coordinates and gradients: rec [S, H*W] of 32 bytes
 * each, 16-byte aligned, as dressi_packed_backward writes them beside its
 * registrations in inv (a registered pixel's bilinear taps, packed as
 * x0 | x1 << 16 and y0 | y1 << 16, its fractions fx, fy, then the gradient
 * of its RGBA sample).  A kept pixel costs one 32-byte read and no tap
 * arithmetic; the sums are bitwise those of dressi_texture_grad_invuv on the
 * same map.  2-D RGBA textures and texture arrays (Ct = 4), grad_tex 16-byte
 * aligned; repeat wrap needs Ht, Wt >= 3 (DRESSI_EINVAL otherwise).  Only the
 * records of pixels registered in inv are read. */
int dressi_texture_grad_invrec(dressi_ctx *ctx, const dressi_tex_desc *td, int S, int H, int W,
                               const int32_t *inv, const void *rec, float *grad_tex, void *stream);

/* ----------------------------------------------------------------------------
 * HardSoftRas blend (§3.4.3, BuildBlend):
 *   D_k = sigmoid(dist_k / sigma), w_k = D_k [tri_id_k >= 0],
 *   I_c^e = sum w_k C_k / sum w_k (0 if no layer), I_s^e = 1 - prod (1 - w_k),
 *   I_c = E I_c^e + (1 - E) S^H C_1,  I_s = E I_s^e + (1 - E) S^H,
 * S^H = front layer present and hard (sign bit of dist; all hard if dist is
 * NULL).  E: silhouette boundary of S^H (pixels with a differing in-image
 * 4-neighbour) dilated by an L-infinity square of radius ceil(delta*W) - 1.
 * color [B,K,H,W,Cc] (Cc 1..16) -> out_color [B,H,W,Cc], out_sil [B,H,W],
 * edge_mask [B,H,W] uint8 (kept for the backward).
 * ------------------------------------------------------------------------- */
int dressi_softras(dressi_ctx *ctx, const float *color, const float *dist, const int32_t *tri_id,
                   int B, int K, int H, int W, int Cc, float sigma, float delta, int mode,
                   float *out_color, float *out_sil, uint8_t *edge_mask, void *stream);

/* grad_layer_color [B,K,H,W,Cc], grad_dist [B,K,H,W] (NULL allowed);
 * grad_sil may be NULL (zero). */
int dressi_softras_bwd(dressi_ctx *ctx, const float *color, const float *dist,
                       const int32_t *tri_id, int B, int K, int H, int W, int Cc, float sigma,
                       const uint8_t *edge_mask, const float *grad_color, const float *grad_sil,
                       float *grad_layer_color, float *grad_dist, void *stream);


/* Allocation-free variant of dressi_softras, for callers that cannot
 * allocate device memory at all (code under hipGraph capture that must not
 * grow the context's arena, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as dressi_softras; the two
 * one-byte-per-pixel edge-mask planes (boundary and row dilation) live in a
 * fixed device array of the library, 2 * DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS
 * bytes (32 MiB) per device, held from the first dressi_create on that
 * device until the process ends.  It calls no allocator.  B*H*W above
 * DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS returns DRESSI_EINVAL (use
 * dressi_softras).  Every call on one device shares that device's array and
 * fully rewrites the part it reads, so calls that overlap in time on one
 * device (concurrent streams, or several host threads) race and must be
 * ordered by the caller; calls on one stream are ordered by it. */
#define DRESSI_SOFTRAS_NOALLOC_MAX_PIXELS (16 * 1024 * 1024)
int dressi_softras_noalloc(dressi_ctx *ctx, const float *color, const float *dist,
                           const int32_t *tri_id, int B, int K, int H, int W, int Cc, float sigma,
                           float delta, int mode, float *out_color, float *out_sil,
                           uint8_t *edge_mask, void *stream);

/* ----------------------------------------------------------------------------
 * The rest of one rendering step around the four stages above (the paper's
 * decomposition I = f_pp(f_shade(f_rasterize(...))), §3.4.1, and the
 * BuildRasterize listing): vertex transform, per-vertex attribute assembly
 * with vertex normals, deferred shading of every layer, and the image loss.
 * ------------------------------------------------------------------------- */

/* pos_clip[b,v,:] = mvp[b] (4x4 row-major) applied to the column (p_v, 1).
 * pos [V,3], mvp [B,4,4], pos_clip [B,V,4]. */
int dressi_transform(dressi_ctx *ctx, const float *pos, const float *mvp, int B, int V,
                     float *pos_clip, void *stream);
/* grad_pos [V,3] = sum over views of mvp[b][:, :3]^T grad_clip[b,v] (views summed
 * in order, deterministic). */
int dressi_transform_bwd(dressi_ctx *ctx, const float *mvp, int B, int V, const float *grad_clip,
                         float *grad_pos, void *stream);

/* Uneven batches (many meshes, each seen by its own camera at its own
 * resolution, drawn into rectangles of one image so that every stage runs as
 * one launch for the whole batch).  The meshes are concatenated: vertex v
 * belongs to view vert_view[v] and is transformed by mvp[vert_view[v]]
 * ([n,4,4] row-major); pos [V,3] -> pos_clip [V,4].  The backward gives
 * grad_pos [V,3] = M^T grad_clip per vertex with its own view's matrix. */
int dressi_transform_batched(dressi_ctx *ctx, const float *pos, const int32_t *vert_view,
                             const float *mvp, int V, float *pos_clip, void *stream);
int dressi_transform_batched_bwd(dressi_ctx *ctx, const float *mvp, const int32_t *vert_view, int V,
                                 const float *grad_clip, float *grad_pos, void *stream);

/* adj: the mesh adjacency (dressi_adjacency) or NULL to build it internally.
 * Per-vertex attribute rows out[v] = (n_v, p_v[, extra_v]) with C = 6 or 9,
 * n_v = normalize(sum of (p1-p0) x (p2-p0) over the faces of v) (the
 * listing's BuildNormalCompute; area-weighted, summed in corner order).
 * extra [V,3] (a tangent, a colour, ...) may be NULL (then C = 6). */
int dressi_vertex_attrs(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                        const float *extra, const int32_t *adj, float *out, void *stream);
/* grad_pos [V,3] from grad_out [V,C] through the normal and position columns,
 * plus grad_pos_in (NULL = 0).  The gradient of `extra` is grad_out[:, 6:9]
 * itself and is not written. */
int dressi_vertex_attrs_bwd(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                            int C, const int32_t *adj, const float *grad_out,
                            const float *grad_pos_in, float *grad_pos, void *stream);
/* The vertex stage of the render graph (§3.4.1: vertex normals and the
 * vertex transform): dressi_vertex_attrs (vattr [V,C]) and the vertex
 * transform in one launch, the same values: pos_clip [B,V,4] as dressi_transform with B views of mvp
 * [B,4,4], or, with vert_view (B = 1), [V,4] as dressi_transform_batched.
 * adj as for dressi_vertex_attrs.  DRESSI_EINVAL for B < 1, or B != 1 with
 * vert_view. */
int dressi_vertex_stage(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                        const float *extra, const int32_t *adj, const float *mvp, const int32_t *vert_view,
                        int B, float *vattr, float *pos_clip, void *stream);

#define DRESSI_SHADE_LAMBERT 0   /* c = a (0.1 + 0.9 max(0, n.l))                         */
#define DRESSI_SHADE_PHONG 1     /* c = a_rgb (0.1 + 0.8 max(0,n.l)) + 0.2 a_a max(0,r.v)^32 */
#define DRESSI_SHADE_PHONG_ENV 2 /* Phong + 0.5 a_a env(reflect(-v, n))                   */

/* Per-fragment shading inputs: each is a pointer to rows of `stride` floats
 * (so it can point into an interpolated attribute buffer) or NULL. */
typedef struct {
    const float *normal; int normal_stride;   /* interpolated normal (renormalised)    */
    const float *pos; int pos_stride;         /* world position (Phong modes)          */
    const float *tangent; int tangent_stride; /* tangent, for normal mapping           */
    const float *nmap; int nmap_stride;       /* tangent-space normal-map sample       */
    const float *albedo; int albedo_stride;   /* albedo rgb or rgba                    */
    int albedo_channels;                      /* 3 or 4 (Phong modes need 4)           */
    const float *env; int env_stride;         /* environment sample (PHONG_ENV)        */
    const int32_t *tri_eye;                   /* uneven batches: camera of each triangle
                                                 (index into eye), or NULL: eye[i / Npv] */
} dressi_frag_in;

typedef struct {
    float *normal; int normal_stride;
    float *pos; int pos_stride;
    float *tangent; int tangent_stride;
    float *nmap; int nmap_stride;
    float *albedo; int albedo_stride;
    float *env; int env_stride;
} dressi_frag_grad;

/* Deferred shading of N = B*Npv fragments (view b = i / Npv, eye[b] its camera
 * position, or eye[in->tri_eye[tri_id[i]]] in an uneven batch; light direction (1,1,2)/sqrt(6), white).  The shading normal is
 * normalize(normal), or, with tangent and nmap, normalize(m_x t^ + m_y b^ +
 * m_z n^) with t^ = normalize(t - (t.n^) n^), b^ = n^ x t^.  Writes, when
 * non-NULL: dir [N,3] = reflect(-v^, n') (the environment lookup direction)
 * and color [N,3] (PHONG_ENV then needs in->env).  Fragments with
 * tri_id < 0 give 0. */
int dressi_shade(dressi_ctx *ctx, int mode, const dressi_frag_in *in, const float *eye,
                 const int32_t *tri_id, int B, int64_t Npv, float *color, float *dir,
                 void *stream);
/* Backward of dressi_shade w.r.t. every non-NULL member of `grad` (rows of
 * `stride` floats; members may point into one packed buffer).  grad_dir
 * (NULL = 0) is the gradient of `dir`; the environment-sample gradient does
 * not depend on it, so it can be taken first (all other members NULL). */
int dressi_shade_bwd(dressi_ctx *ctx, int mode, const dressi_frag_in *in, const float *eye,
                     const int32_t *tri_id, int B, int64_t Npv, const float *grad_color,
                     const float *grad_dir, const dressi_frag_grad *grad, void *stream);

/* L = mean over B*H*W*4 of ((color, sil) - target)^2, or, with a per-pixel
 * weight [B,H,W] (NULL = uniform), L = sum over pixels of weight * sum over
 * the 4 channels of the squared difference (an uneven batch passes
 * 1 / (4 H_i W_i) for the pixels of view i and 0 elsewhere: the sum of the
 * per-view means).  color [B,H,W,3], sil [B,H,W], target [B,H,W,4]; writes
 * loss [1] (device, fixed-order reduction) and, when non-NULL, grad_color and
 * grad_sil of L. */
int dressi_loss_l2(dressi_ctx *ctx, const float *color, const float *sil, const float *target,
                   const float *weight, int B, int H, int W, float *loss, float *grad_color,
                   float *grad_sil, void *stream);

/* ----------------------------------------------------------------------------
 * Stage packing of a single-layer hard image (§3.3.3: the per-fragment
 * function objects of one image size packed into one pass, so that only the
 * values used beyond the pass are written).  K = 1, no blend edge (the hard
 * blend: the image is the front fragment's colour where one is present).
 * Shading: DRESSI_SHADE_LAMBERT with per-vertex normal, position and colour
 * (Cv = 9), or DRESSI_SHADE_PHONG with per-vertex normal and position (Cv = 6),
 * per-corner texture coordinates and a 2-D RGBA albedo texture (or a texture
 * array, layer td.tri_layer[t] for triangle t: uneven batches).
 * ------------------------------------------------------------------------- */
typedef struct {
    int mode;                 /* DRESSI_SHADE_LAMBERT or DRESSI_SHADE_PHONG */
    const float *vattr;       /* [V, Cv] per-vertex attributes (dressi_vertex_attrs) */
    int V, Cv;
    const int32_t *tris;      /* [T, 3] */
    int T;
    const float *uv;          /* Phong: [Vuv, 2] texture coordinates, indexed by uv_tris [T, 3] */
    const int32_t *uv_tris;
    int Vuv;
    const float *tex;         /* Phong: [Ht, Wt, 4] albedo (kind 2-D, Ct = 4) or [layers, Ht, Wt, 4]
                                 (kind 2-D array), 16-byte aligned */
    dressi_tex_desc td;
    const float *eye;         /* camera positions [B, 3], or [n, 3] with tri_eye */
    const int32_t *tri_eye;   /* uneven batches: camera of each triangle, or NULL: eye[view] */
} dressi_packed_scene;

/* Forward of the packed pass over B views of H x W (tri_id [B,H,W] and bary
 * [B,H,W,2] from dressi_rasterize with K = 1, r = 0).  Writes the same values
 * as dressi_interpolate (vattr -> gbuf [B,H,W,Cv]; Phong: uv -> uvbuf
 * [B,H,W,2]), dressi_texture (Phong: tex -> samp [B,H,W,4], 16-byte aligned),
 * dressi_shade and dressi_softras with BLEND_HARD (color [B,H,W,3], sil
 * [B,H,W], edge [B,H,W] = 0) in sequence; under DRESSI_TUNE_EMPTY_SLOTS = 1
 * the gbuf, uvbuf and samp entries of empty pixels are left unwritten.
 * inv (Phong, nullable): the inverse-UV map [B, Ht, Wt] int32 of the
 * backward, 16-byte aligned, set to -1 here. */
int dressi_packed_forward(dressi_ctx *ctx, const dressi_packed_scene *scene, const int32_t *tri_id,
                          const float *bary, int B, int H, int W, float *gbuf, float *uvbuf, float *samp,
                          float *color, float *sil, uint8_t *edge, int32_t *inv, void *stream);
/* Backward of the packed pass with the L2 loss of dressi_loss_l2 against
 * target [B,H,W,4] (weight [B,H,W] or NULL, as there): loss [1] (its partial sums grouped by 256
 * pixels, so it may differ from dressi_loss_l2's in the last bits);
 * grad_color, grad_sil (nullable) as dressi_loss_l2 writes them; grad_gbuf
 * [B,H,W,Cv] and, Phong, grad_samp [B,H,W,4] as dressi_softras_bwd and
 * dressi_shade_bwd give them (normal, position and, Lambert, colour at the
 * gbuf's offsets); Phong: grad_bary_uv [B,H,W,2], the barycentric gradient
 * through the texture coordinate (dressi_texture_bwd's coordinate gradient
 * fed to dressi_interpolate_bwd of uv), and, when inv is given (as set by
 * dressi_packed_forward), every covered pixel registered in it as
 * dressi_invuv_build does: dressi_texture_grad_invuv then gives the texture
 * gradient.  inv_rec (Phong, nullable; [B, H*W] records of 32 bytes,
 * 16-byte aligned): the record of every covered pixel that a map registers
 * (here in inv, or earlier by dressi_invuv_build on the same coordinates)
 * for dressi_texture_grad_invrec, the faster gather; other entries are
 * left as they were.  grad_tex (nullable; needs inv and inv_rec, 16-byte
 * aligned, Ht, Wt >= 3 for repeat wrap): the texture gradient as
 * dressi_texture_grad_invrec gives it from this call's map and records,
 * gathered in this call (the loss's last sum rides in the gather's launch).
 * Inputs are the forward's outputs.  Phong: grad_gbuf and grad_bary_uv may
 * be NULL (only the albedo sample's gradient, as a texture-only step needs). */
int dressi_packed_backward(dressi_ctx *ctx, const dressi_packed_scene *scene, const int32_t *tri_id, int B,
                           int H, int W, const float *gbuf, const float *uvbuf, const float *samp,
                           const float *color, const float *sil, const float *target, const float *weight,
                           float *loss, float *grad_color, float *grad_sil, float *grad_gbuf,
                           float *grad_samp, float *grad_bary_uv, int32_t *inv, void *inv_rec, float *grad_tex,
                           void *stream);

/* Geometry stages of the forward pass for one hard layer (§3.4.1's vertex
 * stage, then rasterization by Algorithm 2 with K = 1, r = 0, and the
 * fragment index of its result): the outputs of dressi_vertex_stage (vattr
 * [V,C] with C = 9 when extra is given, else 6; pos_clip [B,V,4] for the B
 * matrices mvp [B,4,4]; vert_view NULL) followed by those of
 * dressi_rasterize_indexed (tri_id [B,H,W], bary [B,H,W,2], index).  adj:
 * dressi_adjacency of tris.  With the binless strategy
 * (DRESSI_TUNE_HARD_RASTER = 3) and adj given, the rasterizer's merge runs in
 * the vertex stage's launch, each triangle transforming its corners with the
 * stage's own arithmetic (the same positions, bit for bit); otherwise the
 * two calls run in sequence.  The caller owns every buffer.  Errors:
 * DRESSI_EINVAL for B < 1, a null pointer other than extra and adj, or the
 * sizes dressi_rasterize refuses, with nothing launched. */
int dressi_geometry_fwd(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T, const float *extra,
                        const int32_t *adj, const float *mvp, int B, float *vattr, float *pos_clip, int H, int W,
                        int cull, int32_t *tri_id, float *bary, void *index, void *stream);

/* Geometry adjoints of one image (the reverse pass of §3.4's rasterization,
 * interpolation and vertex stages; B = 1, K = 1, hard: after the packed
 * pass), in three launches: the same values as dressi_interpolate_bwd of
 * vattr [V, Cv] (Cv = 6 or 9, indexed by tris, grad_out = grad_gbuf
 * [H,W,Cv], grad_bary_in nullable: the texture coordinates' barycentric
 * gradient), then dressi_rasterize_bwd (r = 0), then dressi_transform_bwd,
 * then dressi_vertex_attrs_bwd of the world positions pos [V,3] that vattr
 * was made from (dressi_vertex_attrs) with the transform's gradient as its
 * grad_pos_in.  Writes grad_vattr [V,Cv], grad_bary [H,W,2], grad_pos_clip
 * [V,4] and grad_pos [V,3], the gradient of the loss in pos.  An uneven
 * batch's packed image passes tri_view, views (n_views rectangles, as
 * dressi_rasterize_batched) and vert_view (the matrix of each vertex, as
 * dressi_transform_batched); otherwise all three are NULL and mvp is one
 * matrix.  frag_index: dressi_fragment_index of this tri_id (B = K = 1);
 * adj: dressi_adjacency of tris.  Kernels: both per-tile adjoints in one;
 * the per-vertex sums of both, the transform adjoint and the gradient of the
 * un-normalised normal sum in the second; the cross-product adjoint of the
 * vertex normals in the third. */
int dressi_geometry_bwd(dressi_ctx *ctx, const float *pos, const float *vattr, int V, int Cv,
                        const int32_t *tris, int T, const float *pos_clip, const float *mvp,
                        const int32_t *vert_view, const int32_t *tri_view, const int32_t *views, int n_views,
                        int H, int W, int cull, const int32_t *tri_id, const float *bary, const float *grad_gbuf,
                        const float *grad_bary_in, const void *frag_index, const int32_t *adj, float *grad_vattr,
                        float *grad_bary, float *grad_pos_clip, float *grad_pos, void *stream);

/* One whole packed step of one image (§3.3.4: the step as one recorded
 * sequence; B = 1, K = 1, hard blend, r = 0): dressi_geometry_fwd (mvp one
 * matrix, cull 0), dressi_packed_forward, dressi_packed_backward (weight
 * NULL, grad_color and grad_sil not written; Phong: the texel gradient from
 * the pixel records, inv_rec and grad_tex required) and dressi_geometry_bwd
 * (no viewports; grad_bary_in = grad_bary_uv when textured), the same values
 * as those calls in that order.  Because the library sees the whole step it
 * can launch independent kernels of different stages together: with the
 * binless rasterizer (DRESSI_TUNE_HARD_RASTER = 3), adj given and more than
 * 16,384 triangles, the fragment index's triangle -> tile lists are built in
 * the launches of the shading passes, the texel gather and the per-tile
 * geometry adjoint (otherwise the calls run in sequence).  The arena then
 * holds the index's temporary beside the later calls' scratch
 * (dressi_reserve_limits with K = 1 sizes it).  scene->vattr must be
 * b->vattr (written by the step).  Every buffer is the
 * caller's.  Errors: DRESSI_EINVAL, with nothing launched, for a null scene
 * or buffer set, a scene->vattr other than b->vattr or a textured step
 * without inv, inv_rec and grad_tex; otherwise the code of the first of the
 * four calls that refuses its arguments (the calls before it have run, and
 * the fragment index is complete). */
typedef struct {
    const float *pos;        /* [V,3] world positions */
    const float *extra;      /* [V,3] vertex colour (Lambert, Cv = 9) or NULL */
    const int32_t *adj;      /* dressi_adjacency of scene->tris */
    const float *mvp;        /* [4,4] */
    int H, W;
    const float *target;     /* [H,W,4] */
    /* forward values (written) */
    float *vattr, *pos_clip;
    int32_t *tri_id;
    float *bary;
    void *index;             /* dressi_fragment_index_bytes(1, 1, H, W, T) */
    float *gbuf, *uvbuf, *samp, *color, *sil;
    uint8_t *edge;
    int32_t *inv;
    void *inv_rec;
    /* gradients (written) */
    float *loss, *grad_gbuf, *grad_samp, *grad_bary_uv, *grad_tex;
    float *grad_vattr, *grad_bary, *grad_pos_clip, *grad_pos;
} dressi_packed_step_bufs;
int dressi_packed_step(dressi_ctx *ctx, const dressi_packed_scene *scene, const dressi_packed_step_bufs *b,
                       void *stream);

/* ----------------------------------------------------------------------------
 * The optimisation loop around the step (§4.1: vertex positions fitted to
 * silhouettes under a scheduled Laplacian regulariser, then the albedo
 * texture to colours, both with Adam).
 * ------------------------------------------------------------------------- */

/* One Adam step (Kingma & Ba, Algorithm 1) on n floats, in place:
 *   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
 *   param -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * with t the 1-based number of this step.  `state` is caller-owned device
 * memory of DRESSI_ADAM_STATE_BYTES, 16-byte aligned and zeroed before the
 * first step (one per parameter tensor); the call advances its step count
 * on the stream, so a captured step replays successive Adam steps.  m and v
 * (n floats each) start at zero.  betas in [0, 1), eps > 0, else EINVAL. */
#define DRESSI_ADAM_STATE_BYTES 16
int dressi_adam(dressi_ctx *ctx, float *param, const float *grad, float *m, float *v, int64_t n,
                float lr, float beta1, float beta2, float eps, void *state, void *stream);

/* Laplacian regulariser on vertex positions pos [V,3] of tris [T,3]:
 *   delta_v = p_v - (sum over the triangles t of v's fan of t's two other
 *             corners) / (2 |fan(v)|)   (0 for a vertex in no triangle),
 * the uniform (umbrella) Laplacian on closed manifold meshes;
 *   R = lam / V * sum_v |delta_v|^2,  lam = lam0 * gamma^i,
 * i = the step count in adam_state (the positions' Adam state; NULL: i = 0),
 * read before that step's dressi_adam.  Writes, when non-NULL,
 * grad_out [V,3] = grad_in (NULL = 0) + dR/dpos (grad_out may be grad_in)
 * and value [1] (device) = R.  adj: the mesh adjacency (dressi_adjacency) or
 * NULL to build it internally.  Sums in double, fixed order. */
int dressi_laplacian_reg(dressi_ctx *ctx, const float *pos, const int32_t *tris, int V, int T,
                         const int32_t *adj, float lam0, float gamma, const void *adam_state,
                         const float *grad_in, float *grad_out, float *value, void *stream);

/* ----------------------------------------------------------------------------
 * Physically-based shading with image-based lighting (the render graph of
 * appendix B: irradiance, prefiltered environment and BRDF integration maps
 * built from the environment image, then split-sum PBS; appendix C
 * optimises an environment map and the roughness with it).
 *
 * Cube maps are [6,S,S,3] float (faces +X,-X,+Y,-Y,+Z,-Z, the sampler's
 * convention).  Texel (f, row j, column i) has centre (a, b) =
 * (2(i+1/2)/S - 1, 2(j+1/2)/S - 1) on its face and its exact solid angle.
 * ------------------------------------------------------------------------- */
typedef struct {
    int S;    /* environment face size (1..1024)                       */
    int Si;   /* irradiance face size                                  */
    int Sp;   /* prefiltered face size                                 */
    int L;    /* prefiltered levels (2..16): roughness l/(L-1), GGX
                 alpha max(roughness^2, 1e-3)                          */
} dressi_ibl_desc;

/* dressi_ibl_filter: env [6,S,S,3] -> irr [6,Si,Si,3], the cosine
 * convolution sum_j env_j max(0, n.w_j) O_j / sum_j max(0, n.w_j) O_j over
 * every environment texel j (direction w_j, solid angle O_j); pref
 * [L,6,Sp,Sp,3], level l the GGX convolution with n = v = R:
 * sum_j env_j W_j / sum_j W_j, W_j = max(0, R.w_j) D(h_j) O_j.  norm (device,
 * dressi_ibl_norm_bytes) receives every output's denominator, for the
 * backward.  Sums in double.
 * dressi_ibl_filter_bwd: grad_env [6,S,S,3] = the exact adjoint, each
 * environment texel gathering sum_o grad_o K_oj / norm_o over every output
 * (no atomics, fixed order). */
size_t dressi_ibl_norm_bytes(const dressi_ibl_desc *d);
int dressi_ibl_filter(dressi_ctx *ctx, const float *env, const dressi_ibl_desc *d, float *irr,
                      float *pref, double *norm, void *stream);
int dressi_ibl_filter_bwd(dressi_ctx *ctx, const dressi_ibl_desc *d, const double *norm,
                          const float *grad_irr, const float *grad_pref, float *grad_env,
                          void *stream);

/* BRDF integration table lut [N,N,2] (rows: roughness (j+1/2)/N, columns:
 * n.v (i+1/2)/N) of the split sum's scale and bias (A, B): the mean over the
 * M-point Hammersley set (base-2 radical inverse) of GGX-sampled half
 * vectors, Smith G with k = alpha/2, Fresnel weight (1 - v.h)^5. */
int dressi_brdf_lut(dressi_ctx *ctx, int N, int M, float *lut, void *stream);

typedef struct {
    const float *normal; int normal_stride;   /* interpolated normal (renormalised) */
    const float *pos; int pos_stride;         /* world position                     */
    const float *albedo; int albedo_stride;   /* rgb                                */
    const float *irr; int irr_stride;         /* irradiance sampled along dir_n     */
    const float *pref; int pref_stride;       /* level l sampled along dir_r at     */
    int64_t pref_level_stride;                /*   pref + l * pref_level_stride     */
    const float *material;                    /* device [2]: metallic, roughness    */
    const float *lut; int lut_n;              /* dressi_brdf_lut table              */
    int levels;                               /* L of the prefiltered map           */
} dressi_pbs_in;

typedef struct {
    float *normal; int normal_stride;
    float *pos; int pos_stride;
    float *albedo; int albedo_stride;
    float *irr;       /* [N,3]                                                   */
    float *pref;      /* [L,N,3]: every level, 0 off the two the roughness uses  */
    float *material;  /* device [2], summed over the fragments in a fixed order  */
} dressi_pbs_grad;

/* Split-sum shading of N = B*Npv fragments (view b = i / Npv, eye[b]):
 *   n' = normalize(n), v = normalize(eye - p), c = max(n'.v, 1e-4),
 *   dir_n = n', dir_r = R = 2 (n'.v) n' - v,
 *   F0 = 0.04 (1 - m) + a m,  F = F0 + (max(1 - r, F0) - F0)(1 - c)^5,
 *   x = clamp(r, 0, 1) (L-1), l0 = min(floor x, L-2), f = x - l0,
 *   P = (1 - f) pref_l0 + f pref_l0+1,  (A, B) = lut bilinear (clamped) at (c, r),
 *   C = (1 - F)(1 - m) a irr + P (F0 A + B),  color = C / (1 + C).
 * Writes, when non-NULL: dir_n, dir_r [N,3] and level_tri_id [L,N] (tri_id
 * where level l is one of the two in use, else -1: the masks for sampling
 * and differentiating each prefiltered level); then color [N,3] (needs
 * the samples).  Fragments with tri_id < 0 give 0. */
int dressi_shade_pbs(dressi_ctx *ctx, const dressi_pbs_in *in, const float *eye,
                     const int32_t *tri_id, int B, int64_t Npv, float *color, float *dir_n,
                     float *dir_r, int32_t *level_tri_id, void *stream);
/* Backward of dressi_shade_pbs w.r.t. every non-NULL member of grad.  The
 * normal and position gradients include the lookups' direction gradients
 * grad_dir_n [N,3] and grad_dir_r [L,N,3] (summed over levels; NULL = 0);
 * the others do not depend on them, so they can be taken first. */
int dressi_shade_pbs_bwd(dressi_ctx *ctx, const dressi_pbs_in *in, const float *eye,
                         const int32_t *tri_id, int B, int64_t Npv, const float *grad_color,
                         const float *grad_dir_n, const float *grad_dir_r,
                         const dressi_pbs_grad *grad, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DRESSI_H */
