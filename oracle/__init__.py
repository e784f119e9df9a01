"""CPU oracle for the Dressi hot path — TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``liboracle.so`` (plain C, double precision,
compiled from ``oracle.c`` with gcc) behind numpy-in / numpy-out functions.
It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

WRAP_REPEAT, WRAP_CLAMP = 0, 1
TEX_2D, TEX_CUBE = 0, 1
BLEND_HSR, BLEND_AA, BLEND_SOFTRAS, BLEND_HARD = 0, 1, 2, 3


def build(openmp: bool = False) -> str:
    """Compile liboracle.so with gcc (no contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-o", LIB, SRC, "-lm"]
    subprocess.check_call(cmd)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_set_threads(1)
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's per-pixel and per-texel loops (1 unless a
    timing asks for more; results do not depend on it)."""
    return int(lib().orc_set_threads(int(n)))


class _TexDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("Ht", C.c_int), ("Wt", C.c_int), ("Ct", C.c_int),
                ("wrap_u", C.c_int), ("wrap_v", C.c_int)]


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


# ---------------------------------------------------------------------------
def rasterize(pos_clip, tris, H, W, K=1, r=0.0, cull=0):
    """Returns tri_id [B,K,H,W] i32, hard [B,K,H,W] u8, bary [..,2] f64, dist f64."""
    pc = _f32(pos_clip)
    if pc.ndim == 2:
        pc = pc[None]
    B, V, _ = pc.shape
    t = _i32(tris)
    T = t.shape[0]
    tri_id = np.empty((B, K, H, W), np.int32)
    hard = np.empty((B, K, H, W), np.uint8)
    bary = np.empty((B, K, H, W, 2), np.float64)
    dist = np.empty((B, K, H, W), np.float64)
    f = lib().orc_rasterize
    f.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int] * 6 + [C.c_float, C.c_int] + [C.c_void_p] * 4
    _check(f(_p(pc), _p(t), B, V, T, H, W, K, C.c_float(r), cull,
             _p(tri_id), _p(hard), _p(bary), _p(dist)), "rasterize")
    return tri_id, hard, bary, dist


def rasterize_window(pos_clip, tris, H, W, window, K=1, r=0.0, cull=0):
    """The layers of the pixels of window = (x0, y0, w, h) of an H x W image
    (every triangle considered): tri_id [B,K,h,w], hard, bary [..,2], dist."""
    pc = _f32(pos_clip)
    if pc.ndim == 2:
        pc = pc[None]
    B, V, _ = pc.shape
    t = _i32(tris)
    T = t.shape[0]
    x0, y0, w, h = (int(v) for v in window)
    tri_id = np.empty((B, K, h, w), np.int32)
    hard = np.empty((B, K, h, w), np.uint8)
    bary = np.empty((B, K, h, w, 2), np.float64)
    dist = np.empty((B, K, h, w), np.float64)
    f = lib().orc_rasterize_window
    f.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int] * 6 + [C.c_float, C.c_int] + [C.c_int] * 4 + \
        [C.c_void_p] * 4
    _check(f(_p(pc), _p(t), B, V, T, H, W, K, C.c_float(r), cull, x0, y0, w, h,
             _p(tri_id), _p(hard), _p(bary), _p(dist)), "rasterize_window")
    return tri_id, hard, bary, dist


def resolve(pos_clip, tris, tri_id, hard, snap=True, cull=0):
    pc = _f32(pos_clip)
    if pc.ndim == 2:
        pc = pc[None]
    B, V, _ = pc.shape
    t = _i32(tris)
    tid = _i32(tri_id)
    _, K, H, W = tid.shape
    bary = np.empty((B, K, H, W, 2), np.float64)
    dist = np.empty((B, K, H, W), np.float64)
    f = lib().orc_resolve
    f.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int] * 8 + [C.c_void_p] * 4
    _check(f(_p(pc), _p(t), B, V, t.shape[0], H, W, K, cull, int(snap),
             _p(tid), _p(_u8(hard)), _p(bary), _p(dist)), "resolve")
    return bary, dist


def rasterize_bwd(pos_clip, tris, tri_id, hard, grad_bary, grad_dist=None, snap=True, cull=0,
                  image=None, window=None):
    """Gradient of (bary, dist) w.r.t. pos_clip [B,V,4].  With `window` =
    (x0, y0, w, h) of an `image` = (H, W), the per-pixel arrays hold that
    window's pixels (as rasterize_window gives them)."""
    pc = _f32(pos_clip)
    if pc.ndim == 2:
        pc = pc[None]
    B, V, _ = pc.shape
    t = _i32(tris)
    tid = _i32(tri_id)
    _, K, h, w = tid.shape
    H, W = (h, w) if image is None else (int(image[0]), int(image[1]))
    x0, y0, ww, wh = (0, 0, w, h) if window is None else (int(v) for v in window)
    assert (ww, wh) == (w, h), "window size differs from the arrays"
    gp = np.empty((B, V, 4), np.float64)
    gd = _f64(grad_dist) if grad_dist is not None else None
    f = lib().orc_rasterize_bwd_window
    f.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int] * 12 + [C.c_void_p] * 5
    _check(f(_p(pc), _p(t), B, V, t.shape[0], H, W, K, cull, int(snap), x0, y0, ww, wh, _p(tid),
             _p(_u8(hard)), _p(_f64(grad_bary)), _p(gd), _p(gp)), "rasterize_bwd")
    return gp


def interpolate(attr, attr_tris, tri_id, bary):
    a = _f64(attr)
    if a.ndim == 2:
        a = a[None]
    Ba, Va, Cc = a.shape
    tid = _i32(tri_id)
    B, K, H, W = tid.shape
    at = _i32(attr_tris)
    out = np.empty((B, K, H, W, Cc), np.float64)
    f = lib().orc_interpolate
    f.argtypes = [C.c_void_p] + [C.c_int] * 3 + [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p] \
        + [C.c_int] * 4 + [C.c_void_p]
    _check(f(_p(a), Ba, Va, Cc, _p(at), at.shape[0], _p(tid), _p(_f64(bary)), B, K, H, W,
             _p(out)), "interpolate")
    return out


def interpolate_bwd(attr, attr_tris, tri_id, bary, grad_out):
    a = _f64(attr)
    squeeze = a.ndim == 2
    if squeeze:
        a = a[None]
    Ba, Va, Cc = a.shape
    tid = _i32(tri_id)
    B, K, H, W = tid.shape
    at = _i32(attr_tris)
    ga = np.empty((Ba, Va, Cc), np.float64)
    gb = np.empty((B, K, H, W, 2), np.float64)
    f = lib().orc_interpolate_bwd
    f.argtypes = [C.c_void_p] + [C.c_int] * 3 + [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p] \
        + [C.c_int] * 4 + [C.c_void_p] * 3
    _check(f(_p(a), Ba, Va, Cc, _p(at), at.shape[0], _p(tid), _p(_f64(bary)), B, K, H, W,
             _p(_f64(grad_out)), _p(ga), _p(gb)), "interpolate_bwd")
    return (ga[0] if squeeze else ga), gb


def _desc(tex, kind, wrap_u, wrap_v):
    if kind == TEX_CUBE:
        F, Ht, Wt, Ct = tex.shape
        assert F == 6
    else:
        Ht, Wt, Ct = tex.shape
    return _TexDesc(kind, Ht, Wt, Ct, wrap_u, wrap_v)


def texture(tex, coord, tri_id=None, kind=TEX_2D, wrap_u=WRAP_REPEAT, wrap_v=WRAP_CLAMP):
    tx = _f64(tex)
    d = _desc(tx, kind, wrap_u, wrap_v)
    cd = 3 if kind == TEX_CUBE else 2
    co = _f32(coord)
    N = co.size // cd
    out = np.empty(co.shape[:-1] + (d.Ct,), np.float64)
    tid = _i32(tri_id) if tri_id is not None else None
    f = lib().orc_texture
    f.argtypes = [C.c_void_p, C.POINTER(_TexDesc), C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    _check(f(_p(tx), C.byref(d), _p(co), _p(tid), N, _p(out)), "texture")
    return out


def texture_bwd_coord(tex, coord, grad_out, tri_id=None, kind=TEX_2D, wrap_u=WRAP_REPEAT,
                      wrap_v=WRAP_CLAMP):
    tx = _f64(tex)
    d = _desc(tx, kind, wrap_u, wrap_v)
    cd = 3 if kind == TEX_CUBE else 2
    co = _f32(coord)
    N = co.size // cd
    g = np.empty(co.shape, np.float64)
    tid = _i32(tri_id) if tri_id is not None else None
    f = lib().orc_texture_bwd_coord
    f.argtypes = [C.c_void_p, C.POINTER(_TexDesc), C.c_void_p, C.c_void_p, C.c_int64,
                  C.c_void_p, C.c_void_p]
    _check(f(_p(tx), C.byref(d), _p(co), _p(tid), N, _p(_f64(grad_out)), _p(g)), "texture_bwd_coord")
    return g


def invuv_build(tex_shape, coord, tri_id, kind=TEX_2D, wrap_u=WRAP_REPEAT, wrap_v=WRAP_CLAMP):
    """coord [S,H,W,cd], tri_id [S,H,W] -> inv [S,(6,)Ht,Wt] i32."""
    d = _desc(np.empty(tex_shape, np.float32), kind, wrap_u, wrap_v)
    co = _f32(coord)
    tid = _i32(tri_id)
    S = tid.shape[0]
    Npix = tid[0].size
    F = 6 if kind == TEX_CUBE else 1
    inv = np.empty((S, F, d.Ht, d.Wt), np.int32)
    f = lib().orc_invuv_build
    f.argtypes = [C.POINTER(_TexDesc), C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_void_p]
    _check(f(C.byref(d), _p(co), _p(tid), S, Npix, _p(inv)), "invuv_build")
    return inv if kind == TEX_CUBE else inv[:, 0]


def texture_bwd_tex(tex_shape, coord, tri_id, grad_out, inv=None, kind=TEX_2D,
                    wrap_u=WRAP_REPEAT, wrap_v=WRAP_CLAMP):
    """Texture gradient through the inverse UV; coord [S,H,W,cd], grad_out [S,H,W,Ct]."""
    d = _desc(np.empty(tex_shape, np.float32), kind, wrap_u, wrap_v)
    co = _f32(coord)
    tid = _i32(tri_id)
    S = tid.shape[0]
    Npix = tid[0].size
    if inv is None:
        inv = invuv_build(tex_shape, co, tid, kind, wrap_u, wrap_v)
    gt = np.empty(tex_shape, np.float64)
    f = lib().orc_texture_bwd_tex
    f.argtypes = [C.POINTER(_TexDesc), C.c_void_p, C.c_void_p, C.c_int, C.c_int64, C.c_void_p,
                  C.c_void_p, C.c_void_p]
    _check(f(C.byref(d), _p(co), _p(tid), S, Npix, _p(_f64(grad_out)), _p(_i32(inv)), _p(gt)),
           "texture_bwd_tex")
    return gt


def texture_adjoint(tex_shape, coord, tri_id, grad_out, kind=TEX_2D, wrap_u=WRAP_REPEAT,
                    wrap_v=WRAP_CLAMP):
    d = _desc(np.empty(tex_shape, np.float32), kind, wrap_u, wrap_v)
    co = _f32(coord)
    cd = 3 if kind == TEX_CUBE else 2
    N = co.size // cd
    gt = np.empty(tex_shape, np.float64)
    tid = _i32(tri_id) if tri_id is not None else None
    f = lib().orc_texture_adjoint
    f.argtypes = [C.POINTER(_TexDesc), C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    _check(f(C.byref(d), _p(co), _p(tid), N, _p(_f64(grad_out)), _p(gt)), "texture_adjoint")
    return gt


def edge_mask(tri_id, dist, delta, mode=BLEND_HSR):
    tid = _i32(tri_id)
    B, K, H, W = tid.shape
    E = np.empty((B, H, W), np.uint8)
    f = lib().orc_edge_mask
    f.argtypes = [C.c_void_p, C.c_void_p] + [C.c_int] * 4 + [C.c_float, C.c_int, C.c_void_p]
    dd = _f64(dist) if dist is not None else None
    _check(f(_p(tid), _p(dd), B, K, H, W, C.c_float(delta), mode, _p(E)), "edge_mask")
    return E


def softras(color, dist, tri_id, sigma, delta, mode=BLEND_HSR):
    tid = _i32(tri_id)
    B, K, H, W = tid.shape
    col = _f64(color)
    Cc = col.shape[-1]
    assert Cc <= 16
    oc = np.empty((B, H, W, Cc), np.float64)
    os_ = np.empty((B, H, W), np.float64)
    E = np.empty((B, H, W), np.uint8)
    dd = _f64(dist) if dist is not None else None
    f = lib().orc_softras
    f.argtypes = [C.c_void_p] * 3 + [C.c_int] * 5 + [C.c_double, C.c_float, C.c_int] + [C.c_void_p] * 3
    _check(f(_p(col), _p(dd), _p(tid), B, K, H, W, Cc, sigma, C.c_float(delta), mode,
             _p(oc), _p(os_), _p(E)), "softras")
    return oc, os_, E


def softras_bwd(color, dist, tri_id, sigma, E, grad_color, grad_sil):
    tid = _i32(tri_id)
    B, K, H, W = tid.shape
    col = _f64(color)
    Cc = col.shape[-1]
    gl = np.empty((B, K, H, W, Cc), np.float64)
    gd = np.empty((B, K, H, W), np.float64) if dist is not None else None
    dd = _f64(dist) if dist is not None else None
    gs = _f64(grad_sil) if grad_sil is not None else None
    f = lib().orc_softras_bwd
    f.argtypes = [C.c_void_p] * 3 + [C.c_int] * 5 + [C.c_double] + [C.c_void_p] * 5
    _check(f(_p(col), _p(dd), _p(tid), B, K, H, W, Cc, sigma, _p(_u8(E)), _p(_f64(grad_color)),
             _p(gs), _p(gl), _p(gd)), "softras_bwd")
    return gl, gd


# ---------------------------------------------------------------------------
# transform, normals, shading, loss
# ---------------------------------------------------------------------------
SHADE_LAMBERT, SHADE_PHONG, SHADE_PHONG_ENV = 0, 1, 2


def transform(pos, mvp):
    p = _f64(pos)
    m = _f64(mvp)
    if m.ndim == 2:
        m = m[None]
    B, V = m.shape[0], p.shape[0]
    out = np.empty((B, V, 4), np.float64)
    f = lib().orc_transform
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    _check(f(_p(p), _p(m), B, V, _p(out)), "transform")
    return out


def transform_bwd(mvp, grad_clip):
    m = _f64(mvp)
    if m.ndim == 2:
        m = m[None]
    g = _f64(grad_clip)
    B, V = g.shape[0], g.shape[1]
    out = np.empty((V, 3), np.float64)
    f = lib().orc_transform_bwd
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    _check(f(_p(m), B, V, _p(g), _p(out)), "transform_bwd")
    return out


def vertex_normals(pos, tris):
    p = _f64(pos)
    t = _i32(tris)
    out = np.empty_like(p)
    f = lib().orc_vertex_normals
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    _check(f(_p(p), _p(t), p.shape[0], t.shape[0], _p(out)), "vertex_normals")
    return out


def vertex_normals_bwd(pos, tris, grad_n):
    p = _f64(pos)
    t = _i32(tris)
    out = np.empty_like(p)
    f = lib().orc_vertex_normals_bwd
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    _check(f(_p(p), _p(t), p.shape[0], t.shape[0], _p(_f64(grad_n)), _p(out)), "vertex_normals_bwd")
    return out


def normal_map(n, t, m, tri_id):
    n_, t_, m_ = _f64(n), _f64(t), _f64(m)
    out = np.empty_like(n_)
    f = lib().orc_normal_map
    f.argtypes = [C.c_void_p] * 4 + [C.c_int64, C.c_void_p]
    _check(f(_p(n_), _p(t_), _p(m_), _p(_i32(tri_id)), n_.size // 3, _p(out)), "normal_map")
    return out


def normal_map_bwd(n, t, m, tri_id, g):
    n_, t_, m_ = _f64(n), _f64(t), _f64(m)
    gn, gt, gm = np.empty_like(n_), np.empty_like(n_), np.empty_like(n_)
    f = lib().orc_normal_map_bwd
    f.argtypes = [C.c_void_p] * 4 + [C.c_int64] + [C.c_void_p] * 4
    _check(f(_p(n_), _p(t_), _p(m_), _p(_i32(tri_id)), n_.size // 3, _p(_f64(g)), _p(gn), _p(gt),
             _p(gm)), "normal_map_bwd")
    return gn, gt, gm


def reflect(n, pos, eye, tri_id):
    n_, p_ = _f64(n), _f64(pos)
    tid = _i32(tri_id)
    B = tid.shape[0]
    out = np.empty_like(n_)
    f = lib().orc_reflect
    f.argtypes = [C.c_void_p] * 4 + [C.c_int, C.c_int64, C.c_void_p]
    _check(f(_p(n_), _p(p_), _p(_f64(eye)), _p(tid), B, tid.size // B, _p(out)), "reflect")
    return out


def reflect_bwd(n, pos, eye, tri_id, g):
    n_, p_ = _f64(n), _f64(pos)
    tid = _i32(tri_id)
    B = tid.shape[0]
    gn, gp = np.empty_like(n_), np.empty_like(n_)
    f = lib().orc_reflect_bwd
    f.argtypes = [C.c_void_p] * 4 + [C.c_int, C.c_int64] + [C.c_void_p] * 3
    _check(f(_p(n_), _p(p_), _p(_f64(eye)), _p(tid), B, tid.size // B, _p(_f64(g)), _p(gn), _p(gp)),
           "reflect_bwd")
    return gn, gp


def shade(mode, n, pos, albedo, env, eye, tri_id):
    n_ = _f64(n)
    a = _f64(albedo)
    Ca = a.shape[-1]
    tid = _i32(tri_id)
    B = tid.shape[0]
    out = np.empty(tid.shape + (3,), np.float64)
    f = lib().orc_shade
    f.argtypes = [C.c_int] + [C.c_void_p] * 3 + [C.c_int] + [C.c_void_p] * 3 + [C.c_int, C.c_int64,
                                                                                 C.c_void_p]
    _check(f(mode, _p(n_), _p(_f64(pos) if pos is not None else None), _p(a), Ca,
             _p(_f64(env) if env is not None else None), _p(_f64(eye)), _p(tid), B, tid.size // B,
             _p(out)), "shade")
    return out


def shade_bwd(mode, n, pos, albedo, env, eye, tri_id, g):
    n_ = _f64(n)
    a = _f64(albedo)
    Ca = a.shape[-1]
    tid = _i32(tri_id)
    B = tid.shape[0]
    gn = np.empty_like(n_)
    gp = np.empty_like(n_) if pos is not None else None
    ga = np.empty_like(a)
    ge = np.empty_like(n_) if env is not None else None
    f = lib().orc_shade_bwd
    f.argtypes = [C.c_int] + [C.c_void_p] * 3 + [C.c_int] + [C.c_void_p] * 3 + [C.c_int, C.c_int64] \
        + [C.c_void_p] * 5
    _check(f(mode, _p(n_), _p(_f64(pos) if pos is not None else None), _p(a), Ca,
             _p(_f64(env) if env is not None else None), _p(_f64(eye)), _p(tid), B, tid.size // B,
             _p(_f64(g)), _p(gn), _p(gp), _p(ga), _p(ge)), "shade_bwd")
    return gn, gp, ga, ge


def loss_l2(color, sil, target):
    c, s, t = _f64(color), _f64(sil), _f64(target)
    gc, gs = np.empty_like(c), np.empty_like(s)
    L = C.c_double(0.0)
    f = lib().orc_loss_l2
    f.argtypes = [C.c_void_p] * 3 + [C.c_int64] + [C.c_void_p] * 3
    _check(f(_p(c), _p(s), _p(t), s.size, C.byref(L), _p(gc), _p(gs)), "loss_l2")
    return L.value, gc, gs


def transform_f32(pos, mvp):
    p = _f32(pos)
    m = _f32(mvp)
    if m.ndim == 2:
        m = m[None]
    B, V = m.shape[0], p.shape[0]
    out = np.empty((B, V, 4), np.float32)
    f = lib().orc_transform_f32
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    _check(f(_p(p), _p(m), B, V, _p(out)), "transform_f32")
    return out


def interpolate_f32(attr, attr_tris, tri_id, bary):
    a = _f32(attr)
    Va, Cc = a.shape
    tid = _i32(tri_id)
    at = _i32(attr_tris)
    out = np.empty(tid.shape + (Cc,), np.float32)
    f = lib().orc_interpolate_f32
    f.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                  C.c_int64, C.c_void_p]
    _check(f(_p(a), Va, Cc, _p(at), at.shape[0], _p(tid), _p(_f32(bary)), tid.size, _p(out)),
           "interpolate_f32")
    return out


def texture_f32(tex, coord, tri_id=None, kind=TEX_2D, wrap_u=WRAP_REPEAT, wrap_v=WRAP_CLAMP):
    """Bilinear sample in float32 with a fixed operation order (for values
    that feed discrete decisions downstream)."""
    t = _f32(tex)
    d = _desc(t, kind, wrap_u, wrap_v)
    c = _f32(coord)
    cd = c.shape[-1]
    N = c.size // cd
    out = np.empty(c.shape[:-1] + (d.Ct,), np.float32)
    f = lib().orc_texture_f32
    f.argtypes = [C.c_void_p, C.POINTER(_TexDesc), C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    tid = _i32(tri_id) if tri_id is not None else None
    _check(f(_p(t), C.byref(d), _p(c), _p(tid), N, _p(out)), "texture_f32")
    return out


def band_layers(tri_id, hard, bary, dist, delta, mode=BLEND_HSR):
    """The edge-band form of rasterized layers for a blend of this delta and
    mode (§3.4.3: outside the blend's edge mask E the image is S^H C_1 and
    the silhouette S^H, so only the front hard fragment reaches them there).
    Inside E the layers are kept; outside E layer 0 is kept when it is hard
    and every other entry is emptied (tri_id -1, hard 0, bary 0, dist 0).
    E is the blend's own mask of these layers (edge_mask)."""
    tid = np.array(tri_id, np.int32)
    hd = np.array(hard, np.uint8)
    ba = np.array(bary, np.float64)
    di = np.array(dist, np.float64)
    E = edge_mask(tid, di, delta, mode).astype(bool)[:, None]          # [B,1,H,W]
    keep = np.broadcast_to(E, tid.shape).copy()
    keep[:, 0] |= hd[:, 0].astype(bool)
    tid[~keep] = -1
    hd[~keep] = 0
    ba[~keep] = 0.0
    di[~keep] = 0.0
    return tid, hd, ba, di


def sobol2(f):
    """The 2-D Sobol point of index f, to 24 fraction bits.  First
    coordinate: the base-2 radical inverse of f.  Second: the direction
    numbers of the primitive polynomial x + 1 (m_1 = 1, m_k = 2 m_(k-1) xor
    m_(k-1)).  Each coordinate is the xor over the set bits k of f of
    m_(k+1) / 2^(k+1)."""
    f = int(f)
    a = b = 0
    m = 1
    for k in range(32):
        if (f >> k) & 1:
            a ^= 1 << (31 - k)
            b ^= m << (31 - k)
        m = (m << 1) ^ m
    return (a >> 8) / 16777216.0, (b >> 8) / 16777216.0


def jitter_samples(coord, tri_id, grad, frame):
    """The inverse UV's jittered samples (§3.3.2: the sampling position of
    each pixel moves by a quasi-random offset per frame, o = Sobol(frame) -
    1/2 in both axes).  coord [S,H,W,cd] float32, tri_id [S,H,W], grad
    [S,H,W,Ct].  Every covered pixel whose four bilinear taps around its
    moved centre are covered pixels of the image registers the coordinate
    sampled there, ((w00 c00 + w01 c01) + w10 c10) + w11 c11 in float32 (it
    selects texture cells and taps), and the gradient sampled with the same
    weights (double).  Returns (coord', tri_id', grad'), tri_id' = -1 where a
    pixel does not register: the inputs of the unjittered inverse UV."""
    c = np.asarray(coord, np.float32)
    tid = np.asarray(tri_id, np.int32)
    g = np.asarray(grad, np.float64)
    S, H, W = tid.shape
    u, v = sobol2(frame)
    ox, oy = np.float32(u - 0.5), np.float32(v - 0.5)
    dx, dy = int(np.floor(ox)), int(np.floor(oy))
    fx, fy = ox - np.float32(dx), oy - np.float32(dy)
    one = np.float32(1.0)
    w = [(one - fy) * (one - fx), (one - fy) * fx, fy * (one - fx), fy * fx]
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    x0, y0 = xs + dx, ys + dy
    inside = (x0 >= 0) & (y0 >= 0) & (x0 + 1 < W) & (y0 + 1 < H)
    x0c, y0c = np.clip(x0, 0, W - 2), np.clip(y0, 0, H - 2)
    taps = [(y0c, x0c), (y0c, x0c + 1), (y0c + 1, x0c), (y0c + 1, x0c + 1)]
    ok = (tid >= 0) & inside[None]
    for ty, tx in taps:
        ok &= tid[:, ty, tx] >= 0
    jc = w[0] * c[:, taps[0][0], taps[0][1]]
    for k in range(1, 4):
        jc = jc + w[k] * c[:, taps[k][0], taps[k][1]]
    jg = sum(np.float64(w[k]) * g[:, taps[k][0], taps[k][1]] for k in range(4))
    return jc.astype(np.float32), np.where(ok, tid, -1).astype(np.int32), np.asarray(jg, np.float64)
