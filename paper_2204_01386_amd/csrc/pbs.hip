// Physically-based shading with image-based lighting, for gfx950: the
// irradiance and prefiltered environment maps built from the environment
// image, the BRDF integration table, and split-sum shading (the render
// graph of appendix B; appendix C optimises an environment map with it).
//
// The filters are dense sums over every environment texel, one workgroup per
// output texel, accumulated in double and reduced in a fixed tree.  Their
// adjoint is the transposed sum, one workgroup per environment texel, so the
// environment gradient is exact and needs no atomics.  Shading follows the
// split sum per fragment; its backward is analytic, with the material's
// scalar gradients reduced in a fixed order.
#include "dressi_internal.h"

#define PBS_BS 256

// ---------------------------------------------------------------------------
// cube texels: direction (the sampler's major-axis convention) and solid angle
// ---------------------------------------------------------------------------
__device__ __forceinline__ double3 cube_texel_dir(int S, int64_t idx) {
    const int f = (int)(idx / ((int64_t)S * S));
    const int rem = (int)(idx - (int64_t)f * S * S);
    const int j = rem / S, i = rem - j * S;
    const double a = 2.0 * (i + 0.5) / S - 1.0, b = 2.0 * (j + 0.5) / S - 1.0;
    double x, y, z;
    switch (f) {
    case 0: x = 1.0; y = -b; z = -a; break;
    case 1: x = -1.0; y = -b; z = a; break;
    case 2: x = a; y = 1.0; z = b; break;
    case 3: x = a; y = -1.0; z = -b; break;
    case 4: x = a; y = -b; z = 1.0; break;
    default: x = -a; y = -b; z = -1.0; break;
    }
    const double inv = 1.0 / sqrt(x * x + y * y + z * z);
    return make_double3(x * inv, y * inv, z * inv);
}

__device__ __forceinline__ double cube_texel_omega(int S, int64_t idx) {
    const int rem = (int)(idx % ((int64_t)S * S));
    const int j = rem / S, i = rem - j * S;
    const double a0 = 2.0 * i / S - 1.0, a1 = 2.0 * (i + 1) / S - 1.0;
    const double b0 = 2.0 * j / S - 1.0, b1 = 2.0 * (j + 1) / S - 1.0;
    auto F = [](double a, double b) { return atan2(a * b, sqrt(a * a + b * b + 1.0)); };
    return F(a1, b1) - F(a0, b1) - F(a1, b0) + F(a0, b0);
}

// (direction, solid angle) of every texel of an S x S cube
__global__ void k_cube_table(int S, double4 *__restrict__ tab) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 6ll * S * S) return;
    const double3 d = cube_texel_dir(S, idx);
    tab[idx] = make_double4(d.x, d.y, d.z, cube_texel_omega(S, idx));
}

__device__ __forceinline__ double level_alpha(int l, int L) {
    const double r = (double)l / (double)(L - 1);
    return fmax(r * r, 1e-3);
}

// Every output of the filters: o < 6 Si^2 is an irradiance texel, the rest
// the prefiltered levels, level by level.  (direction, alpha^2), alpha^2 < 0
// marking the irradiance.
__global__ void k_ibl_out_table(dressi_ibl_desc g, double4 *__restrict__ tab) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ni = 6ll * g.Si * g.Si, np = 6ll * g.Sp * g.Sp;
    if (o >= ni + (int64_t)g.L * np) return;
    double3 d;
    double a2 = -1.0;
    if (o < ni) {
        d = cube_texel_dir(g.Si, o);
    } else {
        const int l = (int)((o - ni) / np);
        d = cube_texel_dir(g.Sp, (o - ni) - (int64_t)l * np);
        const double a = level_alpha(l, g.L);
        a2 = a * a;
    }
    tab[o] = make_double4(d.x, d.y, d.z, a2);
}

// The filters' kernel between output q (direction, alpha^2) and environment
// texel e (direction, solid angle): max(0, q.w) O for the irradiance; for a
// prefiltered level max(0, R.w) D(h) O with (R.h)^2 = (1 + R.w) / 2 for unit
// vectors, D(h) = alpha^2 / (pi t^2), t = (R.h)^2 (alpha^2 - 1) + 1 =
// (1 - c) / 2 + (1 + c) alpha^2 / 2 (the form without cancellation: t is of
// order alpha^2 near the lobe's axis).  c and t in double; the quotient in
// float, where t's relative precision is kept.
__device__ __forceinline__ float filter_kernel(const double4 &q, const double4 &e) {
    const double c = q.x * e.x + q.y * e.y + q.z * e.z;
    if (!(c > 0.0)) return 0.0f;
    if (q.w < 0.0) return (float)(c * e.w);
    const float t = (float)(0.5 * (1.0 - c) + 0.5 * (1.0 + c) * q.w);
    return (float)(c * q.w * e.w) / (3.14159265358979f * t * t);
}

// one workgroup per output texel: out = sum_j env_j K_j / sum_j K_j
__global__ void __launch_bounds__(PBS_BS)
    k_ibl_filter(dressi_ibl_desc g, const double4 *__restrict__ tab, const double4 *__restrict__ otab,
                 const float *__restrict__ env, float *__restrict__ irr, float *__restrict__ pref,
                 double *__restrict__ norm) {
    __shared__ double red[4][PBS_BS];
    const int64_t o = blockIdx.x;
    const double4 q = otab[o];
    const int64_t ne = 6ll * g.S * g.S;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, sw = 0.0;
    for (int64_t j = threadIdx.x; j < ne; j += PBS_BS) {
        const float k = filter_kernel(q, tab[j]);
        if (k == 0.0f) continue;
        s0 += (double)(k * env[3 * j]);
        s1 += (double)(k * env[3 * j + 1]);
        s2 += (double)(k * env[3 * j + 2]);
        sw += (double)k;
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    red[3][threadIdx.x] = sw;
    __syncthreads();
    for (int s = PBS_BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 4; c++) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double inv = 1.0 / red[3][0];
    const int64_t ni = 6ll * g.Si * g.Si;
    float *dst = o < ni ? irr + 3 * o : pref + 3 * (o - ni);
    dst[0] = (float)(red[0][0] * inv);
    dst[1] = (float)(red[1][0] * inv);
    dst[2] = (float)(red[2][0] * inv);
    norm[o] = red[3][0];
}

// every output's gradient over its denominator, g_o / norm_o
__global__ void k_ibl_bwd_scale(dressi_ibl_desc g, const double *__restrict__ norm, const float *__restrict__ g_irr,
                                const float *__restrict__ g_pref, float4 *__restrict__ gs) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ni = 6ll * g.Si * g.Si, no = ni + (int64_t)g.L * 6 * g.Sp * g.Sp;
    if (o >= no) return;
    const float *go = o < ni ? g_irr + 3 * o : g_pref + 3 * (o - ni);
    const double inv = 1.0 / norm[o];
    gs[o] = make_float4((float)(go[0] * inv), (float)(go[1] * inv), (float)(go[2] * inv), 0.0f);
}

// one workgroup per environment texel j: g_env_j = sum_o K_oj g_o / norm_o
__global__ void __launch_bounds__(PBS_BS)
    k_ibl_filter_bwd(dressi_ibl_desc g, const double4 *__restrict__ tab, const double4 *__restrict__ otab,
                     const float4 *__restrict__ gs, float *__restrict__ g_env) {
    __shared__ double red[3][PBS_BS];
    const int64_t j = blockIdx.x;
    const double4 e = tab[j];
    const int64_t no = 6ll * g.Si * g.Si + (int64_t)g.L * 6 * g.Sp * g.Sp;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t o = threadIdx.x; o < no; o += PBS_BS) {
        const float k = filter_kernel(otab[o], e);
        if (k == 0.0f) continue;
        const float4 q = gs[o];
        s0 += (double)(k * q.x);
        s1 += (double)(k * q.y);
        s2 += (double)(k * q.z);
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int s = PBS_BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 3; c++) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    g_env[3 * j] = (float)red[0][0];
    g_env[3 * j + 1] = (float)red[1][0];
    g_env[3 * j + 2] = (float)red[2][0];
}

static int check_ibl(dressi_ctx *ctx, const dressi_ibl_desc *d) {
    if (!ctx) return DRESSI_EINVAL;
    if (!d || d->S < 1 || d->Si < 1 || d->Sp < 1 || d->L < 2 || d->S > 1024 || d->Si > 1024 || d->Sp > 1024 ||
        d->L > 16)
        return dressi_fail(ctx, DRESSI_EINVAL, "ibl: bad descriptor (S, Si, Sp in 1..1024, L in 2..16)");
    return DRESSI_OK;
}

// The environment texels' and the outputs' tables, in the context's scratch.
// (with gs, room for the backward's per-output gradient scale as well)
static int ibl_tables(dressi_ctx *ctx, const dressi_ibl_desc *d, hipStream_t st, double4 *&tab, double4 *&otab,
                      float4 **gs = nullptr) {
    const int64_t ne = 6ll * d->S * d->S;
    const int64_t no = 6ll * d->Si * d->Si + (int64_t)d->L * 6 * d->Sp * d->Sp;
    Carver c;
    const size_t o_t = c.take(sizeof(double4) * (size_t)ne), o_o = c.take(sizeof(double4) * (size_t)no);
    const size_t o_g = c.take(sizeof(float4) * (size_t)no);
    int rc = dressi_scratch(ctx, c.off, st);
    if (rc) return rc;
    tab = at<double4>(ctx->scratch, o_t);
    otab = at<double4>(ctx->scratch, o_o);
    if (gs) *gs = at<float4>(ctx->scratch, o_g);
    DR_LAUNCH("k_cube_table", (k_cube_table), (int)((ne + 255) / 256), 256, 0, st, d->S, tab);
    DR_LAUNCH("k_ibl_out_table", (k_ibl_out_table), (int)((no + 255) / 256), 256, 0, st, *d, otab);
    return DRESSI_OK;
}

extern "C" size_t dressi_ibl_norm_bytes(const dressi_ibl_desc *d) {
    if (!d || d->Si < 1 || d->Sp < 1 || d->L < 2) return 0;
    return sizeof(double) * (6ull * d->Si * d->Si + (size_t)d->L * 6ull * d->Sp * d->Sp);
}

extern "C" int dressi_ibl_filter(dressi_ctx *ctx, const float *env, const dressi_ibl_desc *d, float *irr,
                                 float *pref, double *norm, void *stream) {
    int rc = check_ibl(ctx, d);
    if (rc) return rc;
    if (!env || !irr || !pref || !norm) return dressi_fail(ctx, DRESSI_EINVAL, "ibl_filter: null pointer");
    hipStream_t st = (hipStream_t)stream;
    double4 *tab, *otab;
    if ((rc = ibl_tables(ctx, d, st, tab, otab))) return rc;
    const int64_t no = 6ll * d->Si * d->Si + (int64_t)d->L * 6 * d->Sp * d->Sp;
    DR_LAUNCH("k_ibl_filter", (k_ibl_filter), (int)no, PBS_BS, 0, st, *d, tab, otab, env, irr, pref, norm);
    return dressi_launch_check(ctx, "ibl_filter");
}

extern "C" int dressi_ibl_filter_bwd(dressi_ctx *ctx, const dressi_ibl_desc *d, const double *norm,
                                     const float *grad_irr, const float *grad_pref, float *grad_env,
                                     void *stream) {
    int rc = check_ibl(ctx, d);
    if (rc) return rc;
    if (!norm || !grad_irr || !grad_pref || !grad_env)
        return dressi_fail(ctx, DRESSI_EINVAL, "ibl_filter_bwd: null pointer");
    hipStream_t st = (hipStream_t)stream;
    double4 *tab, *otab;
    float4 *gs;
    if ((rc = ibl_tables(ctx, d, st, tab, otab, &gs))) return rc;
    const int64_t ne = 6ll * d->S * d->S;
    const int64_t no = 6ll * d->Si * d->Si + (int64_t)d->L * 6 * d->Sp * d->Sp;
    DR_LAUNCH("k_ibl_bwd_scale", (k_ibl_bwd_scale), (int)((no + 255) / 256), 256, 0, st, *d, norm, grad_irr,
              grad_pref, gs);
    DR_LAUNCH("k_ibl_filter_bwd", (k_ibl_filter_bwd), (int)ne, PBS_BS, 0, st, *d, tab, otab, gs, grad_env);
    return dressi_launch_check(ctx, "ibl_filter_bwd");
}

// ---------------------------------------------------------------------------
// BRDF integration table
// ---------------------------------------------------------------------------
__global__ void k_brdf_lut(int N, int M, float2 *__restrict__ lut) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * N) return;
    const int j = idx / N, i = idx - j * N;   // row: roughness, column: n.v
    const double r = (j + 0.5) / N, a = r * r, k = a / 2.0;
    const double c = (i + 0.5) / N;
    const double vx = sqrt(1.0 - c * c), vz = c;   // v in the xz plane, n = +z
    const double g1v = c / (c * (1.0 - k) + k);
    double A = 0.0, B = 0.0;
    for (int s = 0; s < M; s++) {
        const double x = (s + 0.5) / M;
        const double y = (double)__brev((unsigned)s) * (1.0 / 4294967296.0);   // radical inverse base 2
        const double ct = sqrt((1.0 - y) / (1.0 + (a * a - 1.0) * y));
        const double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double ph = 2.0 * 3.14159265358979323846 * x;
        const double hx = stt * cos(ph), hz = ct;
        const double vdh = vx * hx + vz * hz;
        const double ndl = 2.0 * vdh * hz - vz;
        if (!(ndl > 0.0)) continue;
        const double G = g1v * (ndl / (ndl * (1.0 - k) + k));
        const double gv = G * vdh / (hz * c);
        const double fc = pow(1.0 - vdh, 5.0);
        A += (1.0 - fc) * gv;
        B += fc * gv;
    }
    lut[idx] = make_float2((float)(A / M), (float)(B / M));
}

extern "C" int dressi_brdf_lut(dressi_ctx *ctx, int N, int M, float *lut, void *stream) {
    if (!ctx) return DRESSI_EINVAL;
    if (N < 1 || N > 1024 || M < 1 || !lut) return dressi_fail(ctx, DRESSI_EINVAL, "brdf_lut: bad arguments");
    DR_LAUNCH("k_brdf_lut", (k_brdf_lut), (N * N + 255) / 256, 256, 0, (hipStream_t)stream, N, M,
              reinterpret_cast<float2 *>(lut));
    return dressi_launch_check(ctx, "brdf_lut");
}

// ---------------------------------------------------------------------------
// split-sum shading
// ---------------------------------------------------------------------------
__device__ __forceinline__ double3 ld3f(const float *p) { return make_double3(p[0], p[1], p[2]); }

struct PbsFrag {
    double3 nn, v, R;   // shading normal, view direction, reflection
    double nlen, vlen, ndv, c;
    int l0;
    double f;
    bool rin;   // roughness inside [0, 1]: the level weight depends on it
};

__device__ __forceinline__ PbsFrag pbs_geometry(const dressi_pbs_in &in, const float *eye, int64_t i,
                                                double rough) {
    PbsFrag q;
    const double3 n = ld3f(in.normal + i * in.normal_stride), p = ld3f(in.pos + i * in.pos_stride);
    q.nlen = sqrt(n.x * n.x + n.y * n.y + n.z * n.z);
    q.nn = make_double3(n.x / q.nlen, n.y / q.nlen, n.z / q.nlen);
    double3 v = make_double3(eye[0] - p.x, eye[1] - p.y, eye[2] - p.z);
    q.vlen = sqrt(v.x * v.x + v.y * v.y + v.z * v.z);
    q.v = make_double3(v.x / q.vlen, v.y / q.vlen, v.z / q.vlen);
    q.ndv = q.nn.x * q.v.x + q.nn.y * q.v.y + q.nn.z * q.v.z;
    q.c = fmax(q.ndv, 1e-4);
    q.R = make_double3(2.0 * q.ndv * q.nn.x - q.v.x, 2.0 * q.ndv * q.nn.y - q.v.y, 2.0 * q.ndv * q.nn.z - q.v.z);
    // the level pair follows the roughness clamped to [0, 1] (also keeping
    // the level index in range for any roughness, NaN included)
    const double x = fmin(fmax(rough, 0.0), 1.0) * (in.levels - 1);
    q.l0 = min((int)floor(x), in.levels - 2);
    q.f = x - q.l0;
    q.rin = rough >= 0.0 && rough <= 1.0;
    return q;
}

// bilinear lookup of the (A, B) table at (c, r), clamped, with its derivatives
struct LutS {
    double A, B, dAc, dBc, dAr, dBr;
};
__device__ __forceinline__ LutS lut_sample(const float *lut, int N, double c, double r) {
    const double s = c * N - 0.5, t = r * N - 0.5;
    const double x0 = floor(s), y0 = floor(t);
    const double fx = s - x0, fy = t - y0;
    auto cl = [N](double q) { return (int)fmin(fmax(q, 0.0), (double)(N - 1)); };
    const int X0 = cl(x0), X1 = cl(x0 + 1.0), Y0 = cl(y0), Y1 = cl(y0 + 1.0);
    const float *T00 = lut + 2 * (Y0 * N + X0), *T01 = lut + 2 * (Y0 * N + X1);
    const float *T10 = lut + 2 * (Y1 * N + X0), *T11 = lut + 2 * (Y1 * N + X1);
    LutS o;
    o.A = (1 - fx) * (1 - fy) * T00[0] + fx * (1 - fy) * T01[0] + (1 - fx) * fy * T10[0] + fx * fy * T11[0];
    o.B = (1 - fx) * (1 - fy) * T00[1] + fx * (1 - fy) * T01[1] + (1 - fx) * fy * T10[1] + fx * fy * T11[1];
    o.dAc = N * ((1 - fy) * ((double)T01[0] - T00[0]) + fy * ((double)T11[0] - T10[0]));
    o.dBc = N * ((1 - fy) * ((double)T01[1] - T00[1]) + fy * ((double)T11[1] - T10[1]));
    o.dAr = N * ((1 - fx) * ((double)T10[0] - T00[0]) + fx * ((double)T11[0] - T01[0]));
    o.dBr = N * ((1 - fx) * ((double)T10[1] - T00[1]) + fx * ((double)T11[1] - T01[1]));
    return o;
}

// directions for the lookups and the per-level fragment masks
__global__ void k_pbs_dirs(dressi_pbs_in in, const float *__restrict__ eye, const int32_t *__restrict__ tri_id,
                           int64_t Npv, int64_t n, float *__restrict__ dir_n, float *__restrict__ dir_r,
                           int32_t *__restrict__ level_tid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = tri_id[i];
    const double rough = in.material[1];
    int l0 = -1;
    if (t >= 0) {
        const PbsFrag q = pbs_geometry(in, eye + 3 * (i / Npv), i, rough);
        l0 = q.l0;
        if (dir_n) {
            dir_n[3 * i] = (float)q.nn.x;
            dir_n[3 * i + 1] = (float)q.nn.y;
            dir_n[3 * i + 2] = (float)q.nn.z;
        }
        if (dir_r) {
            dir_r[3 * i] = (float)q.R.x;
            dir_r[3 * i + 1] = (float)q.R.y;
            dir_r[3 * i + 2] = (float)q.R.z;
        }
    } else {
        for (int c = 0; c < 3; c++) {
            if (dir_n) dir_n[3 * i + c] = 0.0f;
            if (dir_r) dir_r[3 * i + c] = 0.0f;
        }
    }
    if (level_tid)
        for (int l = 0; l < in.levels; l++)
            level_tid[(int64_t)l * n + i] = (t >= 0 && (l == l0 || l == l0 + 1)) ? t : -1;
}

__global__ void k_pbs_shade(dressi_pbs_in in, const float *__restrict__ eye, const int32_t *__restrict__ tri_id,
                            int64_t Npv, int64_t n, float *__restrict__ color) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *o = color + 3 * i;
    if (tri_id[i] < 0) {
        o[0] = o[1] = o[2] = 0.0f;
        return;
    }
    const double m = in.material[0], r = in.material[1];
    const PbsFrag q = pbs_geometry(in, eye + 3 * (i / Npv), i, r);
    const LutS ab = lut_sample(in.lut, in.lut_n, q.c, r);
    const double w5 = pow(1.0 - q.c, 5.0);
    const float *a = in.albedo + i * in.albedo_stride;
    const float *ir = in.irr + i * in.irr_stride;
    const float *p0 = in.pref + (int64_t)q.l0 * in.pref_level_stride + i * in.pref_stride;
    const float *p1 = p0 + in.pref_level_stride;
    for (int ch = 0; ch < 3; ch++) {
        const double F0 = 0.04 * (1.0 - m) + a[ch] * m;
        const double F = F0 + (fmax(1.0 - r, F0) - F0) * w5;
        const double P = (1.0 - q.f) * p0[ch] + q.f * p1[ch];
        const double C = (1.0 - F) * (1.0 - m) * a[ch] * ir[ch] + P * (F0 * ab.A + ab.B);
        o[ch] = (float)(C / (1.0 + C));
    }
}

// Backward per fragment.  Writes, when given: the albedo, irradiance-sample
// and prefiltered-sample gradients (every level, 0 off the two in use),
// normal and position gradients (with the lookups' direction gradients),
// and per-block partial sums of the material gradient.
__global__ void __launch_bounds__(PBS_BS)
    k_pbs_shade_bwd(dressi_pbs_in in, const float *__restrict__ eye, const int32_t *__restrict__ tri_id,
                    int64_t Npv, int64_t n, const float *__restrict__ grad_color,
                    const float *__restrict__ grad_dir_n, const float *__restrict__ grad_dir_r,
                    dressi_pbs_grad g, double *__restrict__ part) {
    __shared__ double red[2][PBS_BS];
    const int64_t i = (int64_t)blockIdx.x * PBS_BS + threadIdx.x;
    double gm = 0.0, gr = 0.0;
    if (i < n) {
        const bool cov = tri_id[i] >= 0;
        const int L = in.levels;
        if (!cov) {
            for (int ch = 0; ch < 3; ch++) {
                if (g.albedo) g.albedo[i * g.albedo_stride + ch] = 0.0f;
                if (g.irr) g.irr[3 * i + ch] = 0.0f;
                if (g.normal) g.normal[i * g.normal_stride + ch] = 0.0f;
                if (g.pos) g.pos[i * g.pos_stride + ch] = 0.0f;
                if (g.pref)
                    for (int l = 0; l < L; l++) g.pref[(int64_t)l * 3 * n + 3 * i + ch] = 0.0f;
            }
        } else {
            const double m = in.material[0], r = in.material[1];
            const float *e = eye + 3 * (i / Npv);
            const PbsFrag q = pbs_geometry(in, e, i, r);
            const LutS ab = lut_sample(in.lut, in.lut_n, q.c, r);
            const double w5 = pow(1.0 - q.c, 5.0);
            const float *a = in.albedo + i * in.albedo_stride;
            const float *ir = in.irr + i * in.irr_stride;
            const float *p0 = in.pref + (int64_t)q.l0 * in.pref_level_stride + i * in.pref_stride;
            const float *p1 = p0 + in.pref_level_stride;
            const float *go = grad_color + 3 * i;
            double gA = 0.0, gB = 0.0, gw5 = 0.0, gf = 0.0;
            for (int ch = 0; ch < 3; ch++) {
                const double ac = a[ch];
                const double F0 = 0.04 * (1.0 - m) + ac * m;
                const bool fr_f0 = F0 > 1.0 - r;     // max(1 - r, F0) takes F0
                const double Fr = fr_f0 ? F0 : 1.0 - r;
                const double F = F0 + (Fr - F0) * w5;
                const double P = (1.0 - q.f) * p0[ch] + q.f * p1[ch];
                const double kd = (1.0 - F) * (1.0 - m);
                const double C = kd * ac * ir[ch] + P * (F0 * ab.A + ab.B);
                const double gC = go[ch] / ((1.0 + C) * (1.0 + C));
                // diffuse: kd a irr
                const double gkd = gC * ac * ir[ch];
                double ga = gC * kd * ir[ch];
                const double girr = gC * kd * ac;
                double gF = -gkd * (1.0 - m);
                gm += -gkd * (1.0 - F);
                // specular: P (F0 A + B)
                const double gP = gC * (F0 * ab.A + ab.B);
                double gF0 = gC * P * ab.A;
                gA += gC * P * F0;
                gB += gC * P;
                // F = F0 + (Fr - F0) w5
                gF0 += gF * (1.0 - w5);
                if (fr_f0) gF0 += gF * w5;
                else gr += -gF * w5;
                gw5 += gF * (Fr - F0);
                // F0 = 0.04 (1 - m) + a m
                gm += gF0 * (ac - 0.04);
                ga += gF0 * m;
                // P = (1 - f) p0 + f p1
                gf += gP * ((double)p1[ch] - p0[ch]);
                if (g.albedo) g.albedo[i * g.albedo_stride + ch] = (float)ga;
                if (g.irr) g.irr[3 * i + ch] = (float)girr;
                if (g.pref)
                    for (int l = 0; l < L; l++)
                        g.pref[(int64_t)l * 3 * n + 3 * i + ch] =
                            l == q.l0 ? (float)(gP * (1.0 - q.f)) : (l == q.l0 + 1 ? (float)(gP * q.f) : 0.0f);
            }
            if (q.rin) gr += gf * (L - 1);
            double gc = gw5 * (-5.0 * pow(1.0 - q.c, 4.0)) + gA * ab.dAc + gB * ab.dBc;
            gr += gA * ab.dAr + gB * ab.dBr;
            if (g.normal || g.pos) {
                const double gndv = q.ndv >= 1e-4 ? gc : 0.0;
                double3 gnn = make_double3(gndv * q.v.x, gndv * q.v.y, gndv * q.v.z);
                double3 gv = make_double3(gndv * q.nn.x, gndv * q.nn.y, gndv * q.nn.z);
                if (grad_dir_n) {
                    gnn.x += grad_dir_n[3 * i];
                    gnn.y += grad_dir_n[3 * i + 1];
                    gnn.z += grad_dir_n[3 * i + 2];
                }
                if (grad_dir_r) {
                    double3 gR = make_double3(0.0, 0.0, 0.0);
                    for (int l = 0; l < L; l++) {
                        const float *gl = grad_dir_r + (int64_t)l * 3 * n + 3 * i;
                        gR.x += gl[0];
                        gR.y += gl[1];
                        gR.z += gl[2];
                    }
                    // R = 2 (n.v) n - v
                    const double gRn = gR.x * q.nn.x + gR.y * q.nn.y + gR.z * q.nn.z;
                    gnn.x += 2.0 * q.ndv * gR.x + 2.0 * gRn * q.v.x;
                    gnn.y += 2.0 * q.ndv * gR.y + 2.0 * gRn * q.v.y;
                    gnn.z += 2.0 * q.ndv * gR.z + 2.0 * gRn * q.v.z;
                    gv.x += 2.0 * gRn * q.nn.x - gR.x;
                    gv.y += 2.0 * gRn * q.nn.y - gR.y;
                    gv.z += 2.0 * gRn * q.nn.z - gR.z;
                }
                if (g.normal) {
                    const double d = gnn.x * q.nn.x + gnn.y * q.nn.y + gnn.z * q.nn.z;
                    float *gn = g.normal + i * g.normal_stride;
                    gn[0] = (float)((gnn.x - d * q.nn.x) / q.nlen);
                    gn[1] = (float)((gnn.y - d * q.nn.y) / q.nlen);
                    gn[2] = (float)((gnn.z - d * q.nn.z) / q.nlen);
                }
                if (g.pos) {
                    // v = (eye - p) / |eye - p|
                    const double d = gv.x * q.v.x + gv.y * q.v.y + gv.z * q.v.z;
                    float *gp = g.pos + i * g.pos_stride;
                    gp[0] = (float)(-(gv.x - d * q.v.x) / q.vlen);
                    gp[1] = (float)(-(gv.y - d * q.v.y) / q.vlen);
                    gp[2] = (float)(-(gv.z - d * q.v.z) / q.vlen);
                }
            }
        }
    }
    if (!g.material) return;   // uniform over the launch
    red[0][threadIdx.x] = gm;
    red[1][threadIdx.x] = gr;
    __syncthreads();
    for (int s = PBS_BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red[0][0];
        part[2 * blockIdx.x + 1] = red[1][0];
    }
}

__global__ void __launch_bounds__(PBS_BS) k_pbs_material_sum(const double *__restrict__ part, int nb,
                                                             float *__restrict__ out) {
    __shared__ double red[2][PBS_BS];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += PBS_BS) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = PBS_BS / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (float)red[0][0];
        out[1] = (float)red[1][0];
    }
}

static int check_pbs(dressi_ctx *ctx, const dressi_pbs_in *in, const float *eye, const int32_t *tri_id, int B,
                     int64_t Npv) {
    if (!ctx) return DRESSI_EINVAL;
    if (!in || B < 0 || Npv < 0) return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs: bad arguments");
    if ((int64_t)B * Npv == 0) return DRESSI_OK;
    if (!in->normal || !in->pos || !in->material || !eye || !tri_id)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs: null input");
    if (in->levels < 2 || in->levels > 16) return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs: levels in 2..16");
    if (in->normal_stride < 3 || in->pos_stride < 3)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs: strides below 3");
    return DRESSI_OK;
}

extern "C" int dressi_shade_pbs(dressi_ctx *ctx, const dressi_pbs_in *in, const float *eye,
                                const int32_t *tri_id, int B, int64_t Npv, float *color, float *dir_n,
                                float *dir_r, int32_t *level_tri_id, void *stream) {
    int rc = check_pbs(ctx, in, eye, tri_id, B, Npv);
    if (rc) return rc;
    const int64_t n = (int64_t)B * Npv;
    if (n == 0) return DRESSI_OK;
    if (color && (!in->albedo || !in->irr || !in->pref || !in->lut || in->lut_n < 1 || in->albedo_stride < 3 ||
                  in->irr_stride < 3 || in->pref_stride < 3))
        return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs: colour needs albedo, samples and the table");
    hipStream_t st = (hipStream_t)stream;
    const int g = (int)((n + 255) / 256);
    if (dir_n || dir_r || level_tri_id)
        DR_LAUNCH("k_pbs_dirs", (k_pbs_dirs), g, 256, 0, st, *in, eye, tri_id, Npv, n, dir_n, dir_r, level_tri_id);
    if (color) DR_LAUNCH("k_pbs_shade", (k_pbs_shade), g, 256, 0, st, *in, eye, tri_id, Npv, n, color);
    return dressi_launch_check(ctx, "shade_pbs");
}

extern "C" int dressi_shade_pbs_bwd(dressi_ctx *ctx, const dressi_pbs_in *in, const float *eye,
                                    const int32_t *tri_id, int B, int64_t Npv, const float *grad_color,
                                    const float *grad_dir_n, const float *grad_dir_r, const dressi_pbs_grad *grad,
                                    void *stream) {
    int rc = check_pbs(ctx, in, eye, tri_id, B, Npv);
    if (rc) return rc;
    if (!grad) return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs_bwd: null grad");
    const int64_t n = (int64_t)B * Npv;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        if (grad->material) dressi_fill_f32(grad->material, 0.0f, 2, st);
        return dressi_launch_check(ctx, "shade_pbs_bwd");
    }
    if (!grad_color || !in->albedo || !in->irr || !in->pref || !in->lut || in->lut_n < 1)
        return dressi_fail(ctx, DRESSI_EINVAL, "shade_pbs_bwd: null input");
    const int nb = (int)((n + PBS_BS - 1) / PBS_BS);
    double *part = nullptr;
    if (grad->material) {
        if ((rc = dressi_scratch(ctx, sizeof(double) * 2 * (size_t)nb, st))) return rc;
        part = at<double>(ctx->scratch, 0);
    }
    DR_LAUNCH("k_pbs_shade_bwd", (k_pbs_shade_bwd), nb, PBS_BS, 0, st, *in, eye, tri_id, Npv, n, grad_color,
              grad_dir_n, grad_dir_r, *grad, part);
    if (grad->material)
        DR_LAUNCH("k_pbs_material_sum", (k_pbs_material_sum), 1, PBS_BS, 0, st, part, nb, grad->material);
    return dressi_launch_check(ctx, "shade_pbs_bwd");
}

// ibl_filter(_bwd) tables and shade_pbs_bwd's material partials
size_t dr_need_pbs(const dressi_limits &l) {
    size_t need = 0;
    if (l.ibl_S > 0) {
        const int64_t ne = 6ll * l.ibl_S * l.ibl_S;
        const int64_t no = 6ll * l.ibl_Si * l.ibl_Si + (int64_t)l.ibl_L * 6 * l.ibl_Sp * l.ibl_Sp;
        Carver c;
        c.take(sizeof(double4) * (size_t)ne);
        c.take(sizeof(double4) * (size_t)no);
        c.take(sizeof(float4) * (size_t)no);
        need = c.off;
    }
    if (l.pbs_fragments > 0)
        need = std::max(need, sizeof(double) * 2 * (size_t)((l.pbs_fragments + PBS_BS - 1) / PBS_BS));
    return need;
}
