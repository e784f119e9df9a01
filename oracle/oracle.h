/*
 * CPU oracle for the Dressi rasterization hot path — test infrastructure only.
 * Layouts are row-major: per-pixel planes are [B,K,H,W(,c)], pixel (x,y) has
 * row y = 0 at the top and its centre at (x + 1/2, y + 1/2).  Values are
 * double precision; inputs that the GPU library receives as float32 are taken
 * as float where the method takes a discrete decision on them.
 */
#ifndef DRESSI_ORACLE_H
#define DRESSI_ORACLE_H
#include <stdint.h>

#define ORC_WRAP_REPEAT 0
#define ORC_WRAP_CLAMP 1
#define ORC_TEX_2D 0
#define ORC_TEX_CUBE 1
#define ORC_BLEND_HSR 0
#define ORC_BLEND_AA 1
#define ORC_BLEND_SOFTRAS 2
#define ORC_BLEND_HARD 3

typedef struct {
    int kind;   /* ORC_TEX_2D or ORC_TEX_CUBE ([6,Ht,Wt,Ct], Ht == Wt) */
    int Ht, Wt, Ct;
    int wrap_u, wrap_v;
} orc_tex_desc;

int orc_rasterize(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                  int H, int W, int K, float r, int cull,
                  int32_t *tri_id, uint8_t *hard, double *bary, double *dist);
int orc_rasterize_window(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                         int H, int W, int K, float r, int cull, int wx0, int wy0, int ww, int wh,
                         int32_t *tri_id, uint8_t *hard, double *bary, double *dist);
int orc_resolve(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                int H, int W, int K, int cull, int snap,
                const int32_t *tri_id, const uint8_t *hard, double *bary, double *dist);
int orc_rasterize_bwd_window(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                             int H, int W, int K, int cull, int snap, int wx0, int wy0, int ww, int wh,
                             const int32_t *tri_id, const uint8_t *hard,
                             const double *grad_bary, const double *grad_dist, double *grad_pos);
int orc_rasterize_bwd(const float *pos_clip, const int32_t *tris, int B, int V, int T,
                      int H, int W, int K, int cull, int snap,
                      const int32_t *tri_id, const uint8_t *hard,
                      const double *grad_bary, const double *grad_dist, double *grad_pos);
int orc_interpolate(const double *attr, int Ba, int Va, int C, const int32_t *attr_tris, int T,
                    const int32_t *tri_id, const double *bary, int B, int K, int H, int W,
                    double *out);
int orc_interpolate_bwd(const double *attr, int Ba, int Va, int C, const int32_t *attr_tris,
                        int T, const int32_t *tri_id, const double *bary, int B, int K, int H,
                        int W, const double *grad_out, double *grad_attr, double *grad_bary);
int orc_texture_f32(const float *tex, const orc_tex_desc *td, const float *coord,
                    const int32_t *tri_id, int64_t N, float *out);
int orc_texture(const double *tex, const orc_tex_desc *td, const float *coord,
                const int32_t *tri_id, int64_t N, double *out);
int orc_texture_bwd_coord(const double *tex, const orc_tex_desc *td, const float *coord,
                          const int32_t *tri_id, int64_t N, const double *grad_out,
                          double *grad_coord);
int orc_invuv_build(const orc_tex_desc *td, const float *coord, const int32_t *tri_id,
                    int S, int64_t Npix, int32_t *inv);
int orc_texture_bwd_tex(const orc_tex_desc *td, const float *coord, const int32_t *tri_id,
                        int S, int64_t Npix, const double *grad_out, const int32_t *inv,
                        double *grad_tex);
int orc_texture_adjoint(const orc_tex_desc *td, const float *coord, const int32_t *tri_id,
                        int64_t N, const double *grad_out, double *grad_tex);
int orc_edge_mask(const int32_t *tri_id, const double *dist, int B, int K, int H, int W,
                  float delta, int mode, uint8_t *E);
int orc_softras(const double *color, const double *dist, const int32_t *tri_id,
                int B, int K, int H, int W, int Cc, double sigma, float delta, int mode,
                double *out_color, double *out_sil, uint8_t *E);
int orc_softras_bwd(const double *color, const double *dist, const int32_t *tri_id,
                    int B, int K, int H, int W, int Cc, double sigma, const uint8_t *E,
                    const double *grad_color, const double *grad_sil,
                    double *grad_layer_color, double *grad_dist);
#define ORC_SHADE_LAMBERT 0
#define ORC_SHADE_PHONG 1
#define ORC_SHADE_PHONG_ENV 2
int orc_transform(const double *pos, const double *mvp, int B, int V, double *out);
int orc_transform_bwd(const double *mvp, int B, int V, const double *grad_clip, double *grad_pos);
int orc_vertex_normals(const double *pos, const int32_t *tris, int V, int T, double *out);
int orc_vertex_normals_bwd(const double *pos, const int32_t *tris, int V, int T,
                           const double *grad_n, double *grad_pos);
int orc_normal_map(const double *n, const double *t, const double *m, const int32_t *tri_id,
                   int64_t N, double *out);
int orc_normal_map_bwd(const double *n, const double *t, const double *m, const int32_t *tri_id,
                       int64_t N, const double *g, double *gn, double *gt, double *gm);
int orc_reflect(const double *n, const double *pos, const double *eye, const int32_t *tri_id,
                int B, int64_t Npv, double *out);
int orc_reflect_bwd(const double *n, const double *pos, const double *eye, const int32_t *tri_id,
                    int B, int64_t Npv, const double *g, double *gn, double *gpos);
int orc_shade(int mode, const double *n, const double *pos, const double *albedo, int Ca,
              const double *env, const double *eye, const int32_t *tri_id, int B, int64_t Npv,
              double *out);
int orc_shade_bwd(int mode, const double *n, const double *pos, const double *albedo, int Ca,
                  const double *env, const double *eye, const int32_t *tri_id, int B, int64_t Npv,
                  const double *g, double *gn, double *gpos, double *galb, double *genv);
int orc_loss_l2(const double *color, const double *sil, const double *target, int64_t Npix,
                double *loss, double *grad_color, double *grad_sil);
int orc_transform_f32(const float *pos, const float *mvp, int B, int V, float *out);
int orc_interpolate_f32(const float *attr, int Va, int C, const int32_t *attr_tris, int T,
                        const int32_t *tri_id, const float *bary, int64_t N, float *out);
#endif
