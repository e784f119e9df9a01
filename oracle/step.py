"""The oracle's end-to-end step (test infrastructure): the same decomposition
as the GPU step (§3.4.1: transform and vertex normals, rasterization,
interpolation, texture sampling, deferred shading, HardSoftRas blend, L2
loss, then the adjoints in reverse), composed from the oracle's own
functions in double precision.

Values that feed discrete decisions are taken in single precision with the
kernel's operation order, so that those decisions coincide: the clip
coordinates (snapped), the texture coordinates (texel and inverse-UV cell),
and the G-buffer rows the shading starts from (interpolated normal, position
and tangent, and the normal-map sample), whose shading normal selects the
environment map's cube face, texels and cell and the side of every
max(0, .) kink.  The shading itself is double precision on those values."""
from __future__ import annotations

import numpy as np

import oracle as O

MODES = {"lambert": O.SHADE_LAMBERT, "phong": O.SHADE_PHONG, "phong_env": O.SHADE_PHONG_ENV}


def _params(scene, target):
    pos = scene.target_pos if target and scene.target_pos is not None else scene.pos
    color = None
    tex = None
    if scene.shading == "lambert":
        color = scene.target_color if target and scene.target_color is not None else scene.color
    else:
        tex = scene.target_tex if target and scene.target_tex is not None else scene.tex
        if scene.nmap is not None:
            tex = np.concatenate([tex, scene.nmap], -1)
    return pos, color, tex


def banded(scene):
    """Whether the scene's layers take the edge-band form (the default for
    the HardSoftRas and anti-aliasing blends with a soft reach; a scene sets
    extra["band"] = False for the full form)."""
    blend = scene.extra.get("blend", "hsr" if scene.r > 0 else "hard")
    return scene.r > 0 and blend in ("hsr", "aa") and bool(scene.extra.get("band", True))


def _bands(y0, h, threads):
    """Row bands (y, rows) splitting rows y0 .. y0 + h - 1 into `threads` parts."""
    n = max(1, min(int(threads), h))
    cuts = [y0 + (h * i) // n for i in range(n + 1)]
    return [(a, b - a) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]


def _raster(pc, tris, H, W, K, r, window, threads):
    """The oracle's rasterization of the window (or image); with threads > 1,
    row bands of it in a thread pool (its C calls release the interpreter
    lock), concatenated: the same layers, for timing on all host cores."""
    x0, y0, w, h = window if window is not None else (0, 0, W, H)
    if threads <= 1:
        if window is None:
            return O.rasterize(pc, tris, H, W, K=K, r=r)
        return O.rasterize_window(pc, tris, H, W, window, K=K, r=r)
    from concurrent.futures import ThreadPoolExecutor
    bands = _bands(y0, h, threads)
    with ThreadPoolExecutor(len(bands)) as ex:
        parts = list(ex.map(lambda b: O.rasterize_window(pc, tris, H, W, (x0, b[0], w, b[1]), K=K, r=r), bands))
    return tuple(np.concatenate([p[i] for p in parts], axis=2) for i in range(4))


def _raster_bwd(pc, tris, tid, hard, g_bary, g_dist, image, window, threads):
    """The rasterization adjoint; with threads > 1, row bands in a thread
    pool whose window adjoints are summed (the adjoint is a sum over
    fragments)."""
    H, W = image
    x0, y0, w, h = window if window is not None else (0, 0, W, H)
    if threads <= 1:
        return O.rasterize_bwd(pc, tris, tid, hard, g_bary, g_dist, image=image, window=window)
    from concurrent.futures import ThreadPoolExecutor
    bands = _bands(y0, h, threads)

    def one(b):
        rows = slice(b[0] - y0, b[0] - y0 + b[1])
        cut = lambda a: None if a is None else np.ascontiguousarray(a[:, :, rows])
        return O.rasterize_bwd(pc, tris, cut(tid), cut(hard), cut(g_bary), cut(g_dist), image=image,
                               window=(x0, b[0], w, b[1]))
    with ThreadPoolExecutor(len(bands)) as ex:
        return sum(ex.map(one, bands))


def forward(scene, views=None, target=False, window=None, threads=1):
    """Forward of the scene's views.  window = (x0, y0, w, h): only the
    pixels of that rectangle of each H x W image (every triangle considered;
    the edge mask is exact where its boundary test and dilation stay inside
    the window)."""
    sl = slice(None) if views is None else views
    mvp = scene.mvp[sl].astype(np.float32)
    eye = scene.eyes[sl].astype(np.float64)
    mode = MODES[scene.shading]
    pos, color, tex = _params(scene, target)
    pos32 = np.ascontiguousarray(pos, np.float32)
    tris = scene.tris
    H, W, K, r = scene.H, scene.W, scene.K, float(scene.r)
    st = {"mode": mode, "mvp": mvp, "eye": eye, "pos": pos32.astype(np.float64), "tex": tex,
          "color_param": color}
    n = O.vertex_normals(st["pos"], tris)
    extra = None
    if mode == O.SHADE_LAMBERT:
        extra = np.asarray(color, np.float64)
    elif mode == O.SHADE_PHONG_ENV:
        extra = np.asarray(scene.extra["tangent"], np.float64)
    vattr = np.concatenate([n, st["pos"]] + ([extra] if extra is not None else []), 1)
    pc = O.transform_f32(pos32, mvp)
    tid, hard, bary, dist = _raster(pc, tris, H, W, K, r, window, threads)
    # the blend setting of §3.4.3: HardSoftRas with delta = r by default; a
    # scene may choose the anti-aliasing or SoftRas-like settings instead
    blend = {"hsr": O.BLEND_HSR, "aa": O.BLEND_AA, "softras": O.BLEND_SOFTRAS,
             "hard": O.BLEND_HARD}[scene.extra.get("blend", "hsr" if r > 0 else "hard")]
    # the dilation radius ceil(delta * width) - 1 is set by the image width
    delta = r if window is None else r * W / window[2]
    if banded(scene):
        tid, hard, bary, dist = O.band_layers(tid, hard, bary, dist, delta, blend)
    gb = O.interpolate(vattr, tris, tid, bary)
    # the shading's inputs: the per-vertex rows rounded once to float, then
    # interpolated in float (decision values, see the module docstring)
    b32 = bary.astype(np.float32)
    gs = O.interpolate_f32(vattr.astype(np.float32), tris, tid, b32).astype(np.float64)
    st.update(vattr=vattr, pc=pc, tid=tid, hard=hard, bary=bary, dist=dist if r > 0 else None, gbuf=gb,
              gshade=gs, image=(H, W), window=window, threads=threads)
    nrm = gs[..., 0:3]
    p = gs[..., 3:6]
    if mode == O.SHADE_LAMBERT:
        albedo = gs[..., 6:9]
        shade_n = nrm
    else:
        uv = O.interpolate_f32(scene.uv, scene.uv_tris, tid, b32)
        wu, wv = scene.extra.get("wrap", (O.WRAP_REPEAT, O.WRAP_CLAMP))
        samp = O.texture(tex, uv, tid, wrap_u=wu, wrap_v=wv)
        st.update(uv=uv, samp=samp)
        albedo = samp[..., 0:4]
        shade_n = nrm
    env_s = None
    if mode == O.SHADE_PHONG_ENV:
        m32 = O.texture_f32(tex, uv, tid, wrap_u=wu, wrap_v=wv)[..., 4:7].astype(np.float64)
        shade_n = O.normal_map(nrm, gs[..., 6:9], m32, tid)
        st.update(nmap_s=m32)
        d = O.reflect(shade_n, p, eye, tid)
        env_s = O.texture(scene.env, d.astype(np.float32), tid, kind=O.TEX_CUBE)
        st.update(shade_n=shade_n, dir=d, env_s=env_s)
    col = O.shade(mode, shade_n, p if mode != O.SHADE_LAMBERT else None, albedo, env_s, eye, tid)
    sigma = r / 7.0 if r > 0 else 1.0
    oc, os_, E = O.softras(col, st["dist"], tid, sigma, delta, blend)
    st.update(layer_color=col, albedo=albedo, color=oc, sil=os_, E=E, sigma=sigma)
    st["rgba"] = np.concatenate([oc, os_[..., None]], -1)
    return st


def backward(scene, st, target_rgba=None, grad_rgba=None):
    """Adjoint of the L2 loss against target_rgba, or, with grad_rgba, of a
    given image gradient [B,H,W,4] (colour, silhouette)."""
    mode = st["mode"]
    tid = st["tid"]
    tris = scene.tris
    if grad_rgba is None:
        L, g_c, g_s = O.loss_l2(st["color"], st["sil"], target_rgba)
    else:
        g = np.asarray(grad_rgba, np.float64)
        L, g_c, g_s = None, g[..., 0:3], g[..., 3]
    gl, gd = O.softras_bwd(st["layer_color"], st["dist"], tid, st["sigma"], st["E"], g_c, g_s)
    gb = st["gshade"]
    nrm, p = gb[..., 0:3], gb[..., 3:6]
    eye = st["eye"]
    g_gbuf = np.zeros_like(gb)
    out = {"loss": L}
    if mode == O.SHADE_LAMBERT:
        gn, _, ga, _ = O.shade_bwd(mode, nrm, None, st["albedo"], None, eye, tid, gl)
        g_gbuf[..., 0:3] = gn
        g_gbuf[..., 6:9] = ga
    elif mode == O.SHADE_PHONG:
        gn, gp, ga, _ = O.shade_bwd(mode, nrm, p, st["albedo"], None, eye, tid, gl)
        g_gbuf[..., 0:3] = gn
        g_gbuf[..., 3:6] = gp
        g_samp = ga
    else:
        gnp, gp, ga, ge = O.shade_bwd(mode, st["shade_n"], p, st["albedo"], st["env_s"], eye, tid, gl)
        d32 = st["dir"].astype(np.float32)
        gdir = O.texture_bwd_coord(scene.env, d32, ge, tid, kind=O.TEX_CUBE)
        out["env"] = O.texture_bwd_tex(scene.env.shape, d32.reshape((-1,) + d32.shape[2:]),
                                       tid.reshape((-1,) + tid.shape[2:]),
                                       ge.reshape((-1,) + ge.shape[2:]), kind=O.TEX_CUBE)
        gnp2, gp2 = O.reflect_bwd(st["shade_n"], p, eye, tid, gdir)
        gn, gt, gm = O.normal_map_bwd(nrm, gb[..., 6:9], st["nmap_s"], tid, gnp + gnp2)
        g_gbuf[..., 0:3] = gn
        g_gbuf[..., 3:6] = gp + gp2
        g_gbuf[..., 6:9] = gt
        g_samp = np.concatenate([ga, gm], -1)
    g_bary_uv = 0.0
    if mode != O.SHADE_LAMBERT:
        uv = st["uv"]
        S = tid.shape[0] * tid.shape[1]
        rs = lambda a: a.reshape((S,) + a.shape[2:])
        wu, wv = scene.extra.get("wrap", (O.WRAP_REPEAT, O.WRAP_CLAMP))
        g_uv = O.texture_bwd_coord(st["tex"], uv, g_samp, tid, wrap_u=wu, wrap_v=wv)
        out["tex"] = O.texture_bwd_tex(st["tex"].shape, rs(uv), rs(tid), rs(g_samp), wrap_u=wu, wrap_v=wv)
        _, g_bary_uv = O.interpolate_bwd(scene.uv, scene.uv_tris, tid, st["bary"], g_uv)
    g_vattr, g_bary = O.interpolate_bwd(st["vattr"], tris, tid, st["bary"], g_gbuf)
    g_bary = g_bary + g_bary_uv
    g_clip = _raster_bwd(st["pc"], tris, tid, st["hard"], g_bary, O_grad_dist(gd, st), st["image"],
                         st["window"], st["threads"])
    out["clip"] = g_clip
    g_pos = O.transform_bwd(st["mvp"], g_clip)
    g_pos += O.vertex_normals_bwd(st["pos"], tris, g_vattr[:, 0:3]) + g_vattr[:, 3:6]
    out["pos"] = g_pos
    if mode == O.SHADE_LAMBERT:
        out["color"] = g_vattr[:, 6:9]
    return out


def O_grad_dist(gd, st):
    return gd if st["dist"] is not None else None


def step(scene, views=None):
    """Forward of the target, forward of the current scene, loss and backward."""
    tgt = forward(scene, views, target=True)
    st = forward(scene, views)
    grads = backward(scene, st, tgt["rgba"])
    return st, tgt, grads
