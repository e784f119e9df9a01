"""One forward + backward step of the Dressi hot path on preallocated buffers.

The step follows the paper's decomposition (§3.4.1): vertex transform and
per-vertex attributes -> rasterization (Algorithm 2) -> attribute
interpolation -> texture sampling -> deferred shading of every layer ->
HardSoftRas blend (§3.4.3) -> L2 image loss, then every adjoint in reverse
order.  Each stage is one call into libdressi; all buffers are allocated once
here, so a step allocates nothing and can be captured into a hipGraph (the
analogue of the paper's single recorded command buffer, §3.3.4).

Textures sampled with the same UVs (albedo and normal map) are packed into
one 8-channel texture (RGBA, normal XYZ, zero) so that one sampler pass and
one inverse-UV gather serve both, with aligned float4 texel rows.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math

import numpy as np
import torch

from . import binding as Bd
from .scenes import Scene

_lib = Bd._lib

# per-tile hard rasterization: cost of a pixel-parallel triangle step over a
# triangle-parallel pixel step, in sixteenths; the autotuner tries these
HYBRID_WEIGHT_DEFAULT = 24
HYBRID_WEIGHTS = (6, 9, 12, 16, 24, 40)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _cp(t, off):
    return None if t is None else C.c_void_p(t.data_ptr() + 4 * off)


def pack_textures(albedo: np.ndarray, nmap: np.ndarray | None) -> np.ndarray:
    """Albedo [Ht,Wt,4] alone, or albedo + normal map [Ht,Wt,3] + one zero
    channel: 8 channels keep every texel row 32-byte aligned (two float4)."""
    if nmap is None:
        return albedo
    pad = np.zeros(albedo.shape[:2] + (1,), albedo.dtype)
    return np.concatenate([albedo, nmap, pad], -1)


class _TwoStreams:
    """With `concurrent` set, independent branches of a step run on a second
    stream (default priority) with a second library context, so that their
    scratch never meets the main stream's: the vertex attributes beside the
    rasterization ("attrs"), the fragment index beside the rest of the
    forward ("index") and the texel gradients beside the coordinate
    gradients ("texel").  `concurrent` is False (every call on the caller's
    stream), True (every branch), the name of one branch or a tuple of names.  Every fork makes
    the second stream wait for the main one and every join the reverse, so a
    step stays one ordered unit on the caller's stream, also when it is
    captured into a graph.  Which is faster depends on the workload
    (cross-stream dependencies cost more than they save on small steps):
    autotune_streams() times the schedules."""

    concurrent = False
    _forked = False
    # inverse-UV jitter of the texel gradients (dressi_texture_bwd's frame;
    # 0 = none).  A captured graph keeps the frame it was recorded with.
    frame = 0
    # every consumer in a step reads per-fragment buffers only at non-empty
    # slots, so the step's calls leave the entries of empty slots unwritten
    skip_empty = True
    # packed steps: the texel gather reads each kept pixel's record (taps,
    # fractions, gradient) written by the packed backward instead of its
    # coordinate and sample gradient; the sums are the same
    gather_rec = True
    inv_rec = None

    @contextlib.contextmanager
    def _sparse(self):
        """Sets DRESSI_TUNE_EMPTY_SLOTS on the step's contexts for the calls
        inside (a captured graph keeps the setting it was recorded with) and
        restores the default after."""
        ctxs = (self.ctx, self.ctx2) if self.skip_empty else ()
        for c in ctxs:
            c.tune(Bd.TUNE_EMPTY_SLOTS, 1)
        try:
            yield
        finally:
            for c in ctxs:
                c.tune(Bd.TUNE_EMPTY_SLOTS, 0)

    def _init_streams(self, dev):
        self._aux = None
        self.ctx2 = Bd.context_aux(dev.index)

    @property
    def aux(self):
        """The second stream, created on first use."""
        if self._aux is None:
            self._aux = torch.cuda.Stream(device=self.dev)
        return self._aux

    def _on(self, branch):
        c = self.concurrent
        return c is True or (isinstance(c, str) and c == branch) or (isinstance(c, tuple) and branch in c)

    def _fork(self, branch):
        if self._on(branch):
            self.aux.wait_stream(torch.cuda.current_stream())
            self._forked = True

    def _join(self):
        if self._forked:
            torch.cuda.current_stream().wait_stream(self.aux)
            self._forked = False

    def _h2(self, branch):
        return (self.ctx2 if self._on(branch) else self.ctx).handle

    def _sa(self, branch):
        return C.c_void_p((self.aux if self._on(branch) else torch.cuda.current_stream()).cuda_stream)

    def _chk2(self, rc, what, branch):
        if rc != 0:
            (self.ctx2 if self._on(branch) else self.ctx).check(rc, what)

    def _gather(self, handle, inv, rec, stream, branch=None):
        """Texel gradient of the albedo from the inverse-UV map `inv`: from the
        pixels' records `rec`, or from their coordinates and sample gradients
        when rec is None."""
        S, H, W = self.B * self.K, self.H, self.W
        if rec is not None:
            what = "texture_grad_invrec"
            rc = _lib.dressi_texture_grad_invrec(handle, C.byref(self.desc), S, H, W, _p(inv), _p(rec),
                                                 _p(self.g_tex), stream)
        else:
            what = "texture_grad_invuv"
            rc = _lib.dressi_texture_grad_invuv(handle, C.byref(self.desc), _p(self.uvbuf), _p(self.tri_id), S, H,
                                                W, _p(inv), _p(self.g_samp), _p(self.g_tex), stream)
        if branch is None:
            self._chk(rc, what)
        else:
            self._chk2(rc, what, branch)

    def _texture_bwd(self, tex, desc, coord, S, grad_out, grad_tex, grad_coord, what):
        """Texel gradient (inverse-UV gather) on the second stream and the
        coordinate gradient on the main one, or both in one call."""
        H, W = self.H, self.W
        if not self._on("texel"):
            self._chk(_lib.dressi_texture_bwd(self.ctx.handle, _p(tex), C.byref(desc), _p(coord), _p(self.tri_id),
                                              S, H, W, _p(grad_out), self.frame, _p(grad_tex), _p(grad_coord),
                                              self._s()), what)
            return
        self._fork("texel")
        self._chk2(_lib.dressi_texture_bwd(self._h2("texel"), _p(tex), C.byref(desc), _p(coord), _p(self.tri_id), S,
                                           H, W, _p(grad_out), self.frame, _p(grad_tex), None, self._sa("texel")),
                   what, "texel")
        self._chk(_lib.dressi_texture_bwd(self.ctx.handle, _p(tex), C.byref(desc), _p(coord), _p(self.tri_id), S,
                                          H, W, _p(grad_out), 0, None, _p(grad_coord), self._s()), what + " coord")


class Step(_TwoStreams):
    """Preallocated fwd+bwd of one scene (all views batched in every launch)."""

    def __init__(self, scene: Scene, device="cuda", views=None, target: "Step | None" = None,
                 params: dict | None = None):
        self.scene = scene
        dev = torch.device(device)
        self.dev = dev
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
        i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(dev)
        sl = slice(None) if views is None else views
        mvp = scene.mvp[sl]
        eyes = scene.eyes[sl]
        self.B = B = mvp.shape[0]
        self.H, self.W, self.K, self.r = scene.H, scene.W, scene.K, float(scene.r)
        H, W, K = self.H, self.W, self.K
        self.mvp = f32(mvp)
        self.eye = f32(eyes)
        self.tris = i32(scene.tris)
        self.V, self.T = scene.pos.shape[0], scene.tris.shape[0]
        p = params or {}
        self.pos = p.get("pos", None)
        if self.pos is None:
            self.pos = f32(scene.pos)
        self.mode = {"lambert": Bd.SHADE_LAMBERT, "phong": Bd.SHADE_PHONG,
                     "phong_env": Bd.SHADE_PHONG_ENV}[scene.shading]
        # HardSoftRas blend (§3.4.3): the paper's setting (edge band of width
        # delta = r, sigma = r / 7), or a scene's choice among its other
        # settings: "aa" (edge mask = the silhouette boundary, delta of one
        # pixel), "softras" (every pixel blended), "hard" (no blending)
        blend = scene.extra.get("blend", "hsr" if self.r > 0 else "hard")
        self.blend = {"hsr": Bd.BLEND_HSR, "aa": Bd.BLEND_AA, "softras": Bd.BLEND_SOFTRAS,
                      "hard": Bd.BLEND_HARD}[blend]
        if self.blend != Bd.BLEND_HARD and self.r <= 0:
            raise ValueError(f"blend {blend!r} needs a soft reach r > 0")
        self.sigma = self.r / 7.0 if self.r > 0 else 1.0
        self.delta = self.r
        # edge-band rasterization (the default for the HardSoftRas and
        # anti-aliasing blends): the soft layers only where the blend's edge
        # mask reaches; scene.extra["band"] = False keeps the full form
        self.band = (self.r > 0 and self.blend in (Bd.BLEND_HSR, Bd.BLEND_AA)
                     and bool(scene.extra.get("band", True)))
        # per-vertex attributes: normal, position, extra (colour or tangent)
        self.extra = None
        if self.mode == Bd.SHADE_LAMBERT:
            self.extra = p.get("color", None)
            if self.extra is None:
                self.extra = f32(scene.color)
        elif self.mode == Bd.SHADE_PHONG_ENV:
            self.extra = f32(scene.extra["tangent"])
        self.Cv = 9 if self.extra is not None else 6
        # textures: albedo (+ normal map) packed, environment cube map
        self.tex = None
        self.uv = self.uv_tris = None
        if self.mode != Bd.SHADE_LAMBERT:
            self.tex = p.get("tex", None)
            if self.tex is None:
                self.tex = f32(pack_textures(scene.tex, scene.nmap))
            self.uv = f32(scene.uv)
            self.uv_tris = i32(scene.uv_tris)
        self.Ct = 0 if self.tex is None else self.tex.shape[-1]
        self.env = None
        if self.mode == Bd.SHADE_PHONG_ENV:
            self.env = p.get("env", None)
            if self.env is None:
                self.env = f32(scene.env)
        self.desc = Bd.TexDesc(0, 0, 0, 0, 0, 0)
        if self.tex is not None:
            wu, wv = scene.extra.get("wrap", (Bd.WRAP_REPEAT, Bd.WRAP_CLAMP))
            self.desc = Bd.TexDesc(Bd.TEX_2D, self.tex.shape[0], self.tex.shape[1], self.Ct, wu, wv)
        if self.env is not None:
            self.env_desc = Bd.TexDesc(Bd.TEX_CUBE, self.env.shape[1], self.env.shape[2],
                                       self.env.shape[3], Bd.WRAP_CLAMP, Bd.WRAP_CLAMP)
        e = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device=dev)
        # forward buffers
        self.vattr = e(self.V, self.Cv)
        self.pos_clip = e(B, self.V, 4)
        self.tri_id = e(B, K, H, W, dt=torch.int32)
        self.bary = e(B, K, H, W, 2)
        self.dist = e(B, K, H, W) if self.r > 0 else None
        self.gbuf = e(B, K, H, W, self.Cv)
        self.uvbuf = e(B, K, H, W, 2) if self.uv is not None else None
        self.samp = e(B, K, H, W, self.Ct) if self.Ct else None
        self.dir = e(B, K, H, W, 3) if self.env is not None else None
        self.env_s = e(B, K, H, W, 3) if self.env is not None else None
        self.layer_color = e(B, K, H, W, 3)
        self.color = e(B, H, W, 3)
        self.sil = e(B, H, W)
        self.E = e(B, H, W, dt=torch.uint8)
        self.loss = e(1)
        self.target = e(B, H, W, 4) if target is None else target.rgba()
        # backward buffers
        self.g_color = e(B, H, W, 3)
        self.g_sil = e(B, H, W)
        self.g_layer = e(B, K, H, W, 3)
        self.g_dist = e(B, K, H, W) if self.r > 0 else None
        self.g_gbuf = e(B, K, H, W, self.Cv)
        # zeroed once: the padding channel of a packed texture is never written
        self.g_samp = torch.zeros((B, K, H, W, self.Ct), device=dev) if self.Ct else None
        self.g_env_s = e(B, K, H, W, 3) if self.env is not None else None
        self.g_dir = e(B, K, H, W, 3) if self.env is not None else None
        self.g_envtex = torch.empty_like(self.env) if self.env is not None else None
        self.g_tex = torch.empty_like(self.tex) if self.tex is not None else None
        self.g_uvbuf = e(B, K, H, W, 2) if self.uv is not None else None
        self.g_bary_uv = e(B, K, H, W, 2) if self.uv is not None else None
        self.g_bary = e(B, K, H, W, 2)
        self.g_vattr = e(self.V, self.Cv)
        self.g_clip = e(B, self.V, 4)
        self.g_pos_t = e(self.V, 3)
        self.g_pos = e(self.V, 3)
        self.ctx = Bd.context(dev.index)
        self._init_streams(dev)
        # topology-only structures: built once per mesh
        self.adj = Bd.dressi_adjacency(self.tris, self.V)
        self.uv_adj = Bd.dressi_adjacency(self.uv_tris, self.uv.shape[0]) if self.uv is not None else None
        nbytes = int(_lib.dressi_fragment_index_bytes(B, K, H, W, self.T))
        self.frag_index = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._fin = self._frag_in()
        self._fin_dir = self._frag_in(with_env=False)
        # stage packing (§3.3.3) of the single-layer hard image: interpolation,
        # texture, shading and blend as one forward pass, the loss and their
        # adjoints as one backward pass (same values; the loss is summed in
        # other groups); scene.extra["packed"] = False keeps the separate stages
        self.packed = (K == 1 and self.blend == Bd.BLEND_HARD and bool(scene.extra.get("packed", True))
                       and (self.mode == Bd.SHADE_LAMBERT
                            or (self.mode == Bd.SHADE_PHONG and self.Ct == 4 and self.desc.kind == Bd.TEX_2D)))
        self.inv = None
        if self.packed:
            ps = Bd.PackedScene()
            ps.mode, ps.vattr, ps.V, ps.Cv = self.mode, _p(self.vattr), self.V, self.Cv
            ps.tris, ps.T, ps.eye = _p(self.tris), self.T, _p(self.eye)
            if self.mode == Bd.SHADE_PHONG:
                ps.uv, ps.uv_tris, ps.Vuv = _p(self.uv), _p(self.uv_tris), self.uv.shape[0]
                ps.tex, ps.td = _p(self.tex), self.desc
                nb = int(_lib.dressi_invuv_bytes(C.byref(self.desc), B))
                self.inv = torch.empty(nb // 4, dtype=torch.int32, device=dev)
                # each covered pixel's gather record (taps, fractions, gradient)
                self.inv_rec = torch.empty((B, H * W, 8), dtype=torch.float32, device=dev)
            self._pscene = ps
        # one view: the geometry adjoints as one call (dressi_geometry_bwd)
        self.packed_geo = self.packed and B == 1
        self.hard_raster = None     # rasterization strategy chosen by autotune() (None: triangle-parallel)
        self.hybrid_weight = HYBRID_WEIGHT_DEFAULT
        # one hard layer: the fragment index built in the rasterization's call
        self.fuse_index = True
        # one view, packed: the whole step as one call (dressi_packed_step)
        self.whole_step = True
        self._step_bufs = None
        self._calibrate_bins()

    def _raster(self, attrs=False, index=False):
        """Transform and rasterization; with `attrs`, the vertex attributes
        in the transform's launch (dressi_vertex_stage); with `index` (one
        hard layer), the fragment index in the rasterization's call
        (dressi_rasterize_indexed); with both, all in one call
        (dressi_geometry_fwd)."""
        h, st = self.ctx.handle, self._s()
        self.ctx.tune(Bd.TUNE_HARD_RASTER, self.hard_raster or 0)
        self.ctx.tune(Bd.TUNE_HYBRID_WEIGHT, self.hybrid_weight)
        if attrs and index and not self.band:
            # the vertex stage, rasterization and fragment index in one call
            self._chk(_lib.dressi_geometry_fwd(h, _p(self.pos), _p(self.tris), self.V, self.T, _p(self.extra),
                                               _p(self.adj), _p(self.mvp), self.B, _p(self.vattr),
                                               _p(self.pos_clip), self.H, self.W, 0, _p(self.tri_id),
                                               _p(self.bary), _p(self.frag_index), st), "geometry_fwd")
            return
        if attrs:
            self._chk(_lib.dressi_vertex_stage(h, _p(self.pos), _p(self.tris), self.V, self.T, _p(self.extra),
                                               _p(self.adj), _p(self.mvp), None, self.B, _p(self.vattr),
                                               _p(self.pos_clip), st), "vertex_stage")
        else:
            self._chk(_lib.dressi_transform(h, _p(self.pos), _p(self.mvp), self.B, self.V, _p(self.pos_clip),
                                            st), "transform")
        if self.band:
            self._chk(_lib.dressi_rasterize_banded(h, _p(self.pos_clip), _p(self.tris), self.B, self.V, self.T,
                                                   self.H, self.W, self.K, self.r, 0, self.delta, self.blend,
                                                   _p(self.tri_id), _p(self.bary), _p(self.dist), st),
                      "rasterize_banded")
        elif index:
            self._chk(_lib.dressi_rasterize_indexed(h, _p(self.pos_clip), _p(self.tris), self.B, self.V, self.T,
                                                    self.H, self.W, 0, _p(self.tri_id), _p(self.bary),
                                                    _p(self.frag_index), st), "rasterize_indexed")
        else:
            self._chk(_lib.dressi_rasterize(h, _p(self.pos_clip), _p(self.tris), self.B, self.V, self.T, self.H,
                                            self.W, self.K, self.r, 0, _p(self.tri_id), _p(self.bary),
                                            _p(self.dist), st), "rasterize")

    def _calibrate_bins(self):
        """Rasterizes once and grows the tile-bin capacity until no tile
        overflows (dense or strongly overlapping geometry), so that later
        steps, captured or not, need no check."""
        for _ in range(4):
            self._raster()
            need = self.ctx.check_status()
            if need <= 0:
                return
            cap = 1
            while cap < need * 5 // 4:
                cap <<= 1
            self.ctx.reserve(0, cap)
        raise RuntimeError("tile bins still overflow after growing them")

    # ------------------------------------------------------------------
    def _frag_in(self, with_env=True):
        fi = Bd.FragIn()
        Cv = self.Cv
        fi.normal, fi.normal_stride = _cp(self.gbuf, 0), Cv
        if self.mode == Bd.SHADE_LAMBERT:
            fi.albedo, fi.albedo_stride, fi.albedo_channels = _cp(self.gbuf, 6), Cv, 3
        else:
            fi.pos, fi.pos_stride = _cp(self.gbuf, 3), Cv
            fi.albedo, fi.albedo_stride, fi.albedo_channels = _cp(self.samp, 0), self.Ct, 4
        if self.mode == Bd.SHADE_PHONG_ENV:
            fi.tangent, fi.tangent_stride = _cp(self.gbuf, 6), Cv
            fi.nmap, fi.nmap_stride = _cp(self.samp, 4), self.Ct
            if with_env:
                fi.env, fi.env_stride = _cp(self.env_s, 0), 3
        return fi

    def _chk(self, rc, what):
        if rc != 0:
            self.ctx.check(rc, what)

    def _s(self):
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def forward(self):
        with self._sparse():
            self._forward()

    def _forward(self):
        h, s = self.ctx.handle, self._s()
        B, V, T, H, W, K = self.B, self.V, self.T, self.H, self.W, self.K
        ck = self._chk
        # vertex attributes beside transform + rasterization, or in the
        # transform's launch
        if self._on("attrs"):
            self._fork("attrs")
            self._chk2(_lib.dressi_vertex_attrs(self._h2("attrs"), _p(self.pos), _p(self.tris), V, T,
                                                _p(self.extra), _p(self.adj), _p(self.vattr), self._sa("attrs")),
                       "vertex_attrs", "attrs")
            self._raster()
            self._join()
        else:
            # one hard layer: the fragment index in the rasterization's call
            fused = self.fuse_index and K == 1 and self.r == 0 and not self.band and not self._on("index")
            self._raster(attrs=True, index=fused)
            if fused:
                self._after_index()
                return
        # the backward's fragment index beside the rest of the forward
        self._fork("index")
        self._chk2(_lib.dressi_fragment_index(self._h2("index"), _p(self.tri_id), B, K, H, W, T, _p(self.frag_index),
                                              self._sa("index")), "fragment_index", "index")
        self._after_index()

    def _after_index(self):
        """The forward's per-fragment stages, after the rasterization."""
        h, s = self.ctx.handle, self._s()
        B, V, T, H, W, K = self.B, self.V, self.T, self.H, self.W, self.K
        ck = self._chk
        if self.packed:
            ck(_lib.dressi_packed_forward(h, C.byref(self._pscene), _p(self.tri_id), _p(self.bary), B, H, W,
                                          _p(self.gbuf), _p(self.uvbuf), _p(self.samp), _p(self.color),
                                          _p(self.sil), _p(self.E), _p(self.inv), s), "packed_forward")
            self._join()
            return
        ck(_lib.dressi_interpolate(h, _p(self.vattr), 1, V, self.Cv, _p(self.tris), T, _p(self.tri_id),
                                   _p(self.bary), B, K, H, W, _p(self.gbuf), s), "interpolate")
        if self.uv is not None:
            ck(_lib.dressi_interpolate(h, _p(self.uv), 1, self.uv.shape[0], 2, _p(self.uv_tris), T,
                                       _p(self.tri_id), _p(self.bary), B, K, H, W, _p(self.uvbuf), s),
               "interpolate uv")
            ck(_lib.dressi_texture(h, _p(self.tex), C.byref(self.desc), _p(self.uvbuf), _p(self.tri_id),
                                   B * K, H, W, _p(self.samp), s), "texture")
        if self.env is not None:
            ck(_lib.dressi_shade(h, self.mode, C.byref(self._fin_dir), _p(self.eye), _p(self.tri_id), B,
                                 K * H * W, None, _p(self.dir), s), "shade dir")
            ck(_lib.dressi_texture(h, _p(self.env), C.byref(self.env_desc), _p(self.dir),
                                   _p(self.tri_id), B * K, H, W, _p(self.env_s), s), "texture env")
        ck(_lib.dressi_shade(h, self.mode, C.byref(self._fin), _p(self.eye), _p(self.tri_id), B,
                             K * H * W, _p(self.layer_color), None, s), "shade")
        ck(_lib.dressi_softras(h, _p(self.layer_color), _p(self.dist), _p(self.tri_id), B, K, H, W, 3,
                               self.sigma, self.delta, self.blend, _p(self.color), _p(self.sil),
                               _p(self.E), s), "softras")
        self._join()

    def loss_and_grad(self):
        ck = self._chk
        ck(_lib.dressi_loss_l2(self.ctx.handle, _p(self.color), _p(self.sil), _p(self.target), None, self.B,
                               self.H, self.W, _p(self.loss), _p(self.g_color), _p(self.g_sil),
                               self._s()), "loss")

    def backward(self):
        with self._sparse():
            self._backward()

    def _backward(self):
        h, s = self.ctx.handle, self._s()
        B, V, T, H, W, K = self.B, self.V, self.T, self.H, self.W, self.K
        ck = self._chk
        Cv = self.Cv
        ck(_lib.dressi_softras_bwd(h, _p(self.layer_color), _p(self.dist), _p(self.tri_id), B, K, H, W, 3,
                                   self.sigma, _p(self.E), _p(self.g_color), _p(self.g_sil),
                                   _p(self.g_layer), _p(self.g_dist), s), "softras_bwd")
        Npv = K * H * W
        if self.env is not None:
            ge = Bd.FragGrad()
            ge.env, ge.env_stride = _cp(self.g_env_s, 0), 3
            ck(_lib.dressi_shade_bwd(h, self.mode, C.byref(self._fin), _p(self.eye), _p(self.tri_id), B,
                                     Npv, _p(self.g_layer), None, C.byref(ge), s), "shade_bwd env")
            self._texture_bwd(self.env, self.env_desc, self.dir, B * K, self.g_env_s, self.g_envtex, self.g_dir,
                              "texture_bwd env")
        g = Bd.FragGrad()
        g.normal, g.normal_stride = _cp(self.g_gbuf, 0), Cv
        g.pos, g.pos_stride = _cp(self.g_gbuf, 3), Cv
        if self.mode == Bd.SHADE_LAMBERT:
            g.albedo, g.albedo_stride = _cp(self.g_gbuf, 6), Cv
        else:
            g.albedo, g.albedo_stride = _cp(self.g_samp, 0), self.Ct
        if self.mode == Bd.SHADE_PHONG_ENV:
            g.tangent, g.tangent_stride = _cp(self.g_gbuf, 6), Cv
            g.nmap, g.nmap_stride = _cp(self.g_samp, 4), self.Ct
        ck(_lib.dressi_shade_bwd(h, self.mode, C.byref(self._fin), _p(self.eye), _p(self.tri_id), B, Npv,
                                 _p(self.g_layer), _p(self.g_dir), C.byref(g), s), "shade_bwd")
        gb_in = None
        if self.uv is not None:
            self._texture_bwd(self.tex, self.desc, self.uvbuf, B * K, self.g_samp, self.g_tex, self.g_uvbuf,
                              "texture_bwd")
            ck(_lib.dressi_interpolate_bwd(h, _p(self.uv), 1, self.uv.shape[0], 2, _p(self.uv_tris), T,
                                           _p(self.tri_id), _p(self.bary), B, K, H, W, _p(self.g_uvbuf),
                                           None, _p(self.frag_index), _p(self.uv_adj), None,
                                           _p(self.g_bary_uv), s), "interpolate_bwd uv")
            gb_in = self.g_bary_uv
        self._backward_geometry(gb_in)
        self._join()

    def _packed_backward(self):
        """Loss, blend, shading and texture-coordinate adjoints in one pass
        (with the inverse-UV registration), then the texture gather and the
        geometry's backward as in the separate form."""
        h, s = self.ctx.handle, self._s()
        B, H, W, K = self.B, self.H, self.W, self.K
        ck = self._chk
        # with records, the texel gather runs inside the packed backward
        # (with the loss's last sum in its launch)
        rec = self.inv_rec if self.uv is not None and self.gather_rec else None
        ck(_lib.dressi_packed_backward(h, C.byref(self._pscene), _p(self.tri_id), B, H, W, _p(self.gbuf),
                                       _p(self.uvbuf), _p(self.samp), _p(self.color), _p(self.sil),
                                       _p(self.target), None, _p(self.loss), None, None, _p(self.g_gbuf),
                                       _p(self.g_samp), _p(self.g_bary_uv), _p(self.inv), _p(rec),
                                       _p(self.g_tex if rec is not None else None), s), "packed_backward")
        gb_in = None
        if self.uv is not None:
            if rec is None:
                # the texel gather beside the geometry's backward ("texel" branch)
                self._fork("texel")
                self._gather(self._h2("texel"), self.inv, None, self._sa("texel"), "texel")
            gb_in = self.g_bary_uv
        if self.packed_geo:
            ck(_lib.dressi_geometry_bwd(h, _p(self.pos), _p(self.vattr), self.V, self.Cv, _p(self.tris), self.T,
                                        _p(self.pos_clip), _p(self.mvp), None, None, None, 0, H, W, 0,
                                        _p(self.tri_id), _p(self.bary), _p(self.g_gbuf), _p(gb_in),
                                        _p(self.frag_index), _p(self.adj), _p(self.g_vattr), _p(self.g_bary),
                                        _p(self.g_clip), _p(self.g_pos), s), "geometry_bwd")
        else:
            self._backward_geometry(gb_in)
        self._join()

    def _backward_geometry(self, gb_in):
        """Attribute interpolation, rasterization, transform and vertex
        attribute adjoints, from the G-buffer gradient (and the barycentric
        gradient gb_in of the texture coordinates)."""
        h, s = self.ctx.handle, self._s()
        B, V, T, H, W, K = self.B, self.V, self.T, self.H, self.W, self.K
        ck = self._chk
        Cv = self.Cv
        ck(_lib.dressi_interpolate_bwd(h, _p(self.vattr), 1, V, Cv, _p(self.tris), T, _p(self.tri_id),
                                       _p(self.bary), B, K, H, W, _p(self.g_gbuf), _p(gb_in),
                                       _p(self.frag_index), _p(self.adj), _p(self.g_vattr),
                                       _p(self.g_bary), s), "interpolate_bwd")
        ck(_lib.dressi_rasterize_bwd(h, _p(self.pos_clip), _p(self.tris), B, V, T, H, W, K, self.r, 0,
                                     _p(self.tri_id), _p(self.g_bary), _p(self.g_dist),
                                     _p(self.frag_index), _p(self.adj), _p(self.g_clip), s),
           "rasterize_bwd")
        ck(_lib.dressi_transform_bwd(h, _p(self.mvp), B, V, _p(self.g_clip), _p(self.g_pos_t), s),
           "transform_bwd")
        ck(_lib.dressi_vertex_attrs_bwd(h, _p(self.pos), _p(self.tris), V, T, Cv, _p(self.adj),
                                        _p(self.g_vattr), _p(self.g_pos_t), _p(self.g_pos), s),
           "vertex_attrs_bwd")

    def _whole_step(self):
        """One view, one hard layer in the packed form, every stage on the
        caller's stream: the whole step as one call (dressi_packed_step, the
        same values as the calls of forward() and the packed backward), so
        that the library can launch independent kernels of different stages
        together.  Returns False where it does not apply."""
        if not (self.whole_step and self.packed_geo and self.frame == 0 and self.fuse_index and self.r == 0
                and not self.band and self.concurrent is False and (self.uv is None or self.gather_rec)):
            return False
        if self._step_bufs is None:
            b = Bd.PackedStepBufs()
            b.pos, b.extra, b.adj, b.mvp = _p(self.pos), _p(self.extra), _p(self.adj), _p(self.mvp)
            b.H, b.W, b.target = self.H, self.W, _p(self.target)
            b.vattr, b.pos_clip, b.tri_id, b.bary = _p(self.vattr), _p(self.pos_clip), _p(self.tri_id), _p(self.bary)
            b.index, b.gbuf, b.uvbuf, b.samp = _p(self.frag_index), _p(self.gbuf), _p(self.uvbuf), _p(self.samp)
            b.color, b.sil, b.edge, b.inv, b.inv_rec = (_p(self.color), _p(self.sil), _p(self.E), _p(self.inv),
                                                        _p(self.inv_rec))
            b.loss, b.grad_gbuf, b.grad_samp = _p(self.loss), _p(self.g_gbuf), _p(self.g_samp)
            b.grad_bary_uv, b.grad_tex = _p(self.g_bary_uv), _p(self.g_tex if self.uv is not None else None)
            b.grad_vattr, b.grad_bary, b.grad_pos_clip, b.grad_pos = (_p(self.g_vattr), _p(self.g_bary),
                                                                      _p(self.g_clip), _p(self.g_pos))
            self._step_bufs = b
        self.ctx.tune(Bd.TUNE_HARD_RASTER, self.hard_raster or 0)
        self.ctx.tune(Bd.TUNE_HYBRID_WEIGHT, self.hybrid_weight)
        with self._sparse():
            self._chk(_lib.dressi_packed_step(self.ctx.handle, C.byref(self._pscene), C.byref(self._step_bufs),
                                              self._s()), "packed_step")
        return True

    def run(self):
        """One full step: forward, loss and gradient, backward.  In the packed
        form (and without inverse-UV jitter) the loss and the backward are one
        pass, which leaves g_color and g_sil unwritten."""
        packed = self.packed and self.frame == 0
        if packed and self._whole_step():
            return
        self.forward()
        if packed:
            with self._sparse():
                self._packed_backward()
            return
        self.loss_and_grad()
        self.backward()

    def check_overflow(self):
        """Raises if a rasterization since the last check (eager or a graph
        replay) overflowed the tile bins, which leaves its outputs invalid.
        The bins are calibrated on the scene at construction; a scene whose
        geometry moves (an optimisation) checks after its steps.  Host
        synchronisation; not for use while capturing."""
        need = self.ctx.check_status()
        if need > 0:
            raise Bd.DressiError(f"tile bins overflowed ({need} triangles per tile needed): "
                                 "the outputs since the last check are invalid; recalibrate")

    def rgba(self):
        """Rendered image [B,H,W,4] (colour, silhouette) as a new tensor."""
        return torch.cat([self.color, self.sil[..., None]], -1).contiguous()

    def grads(self):
        """Gradients of the loss w.r.t. the step's parameters."""
        out = {"pos": self.g_pos}
        if self.mode == Bd.SHADE_LAMBERT:
            out["color"] = self.g_vattr[:, 6:9]
        if self.g_tex is not None:
            out["tex"] = self.g_tex if self.scene.nmap is None else self.g_tex[..., :7]
        if self.g_envtex is not None:
            out["env"] = self.g_envtex
        return out


class TextureStep:
    """Texture-only optimisation of a scene whose geometry is held fixed.

    The paper's reactive cache (§3.3.3) skips graph nodes whose inputs did
    not change since they were last computed; for texture optimisation that
    removes the whole rasterization (its cross-platform table times
    texture-only and geometry iterations separately).  Here the cached nodes
    are explicit: the fragments (tri_id, barycentrics, soft distances), the
    interpolated attributes and texture coordinates, and the albedo texture's
    inverse-UV map are computed once from the wrapped Step's geometry.  A step
    then runs only what depends on the textures: sampling, shading, the blend,
    the loss, their adjoints and the texel gather from the cached map.  An
    environment map looked up along a normal-mapped reflection stays fully
    per step (its lookup direction moves with the normal map).  Images, loss
    and texture gradients are bitwise those of the full step with the same
    parameters; refresh() recomputes the cache after the geometry changed."""

    def __init__(self, step: "Step | BatchStep"):
        if step.tex is None:
            raise ValueError("a texture-only step needs a textured scene")
        self.st = step
        S = step.B * step.K
        n = int(_lib.dressi_invuv_bytes(C.byref(step.desc), S)) // 4
        self.inv = torch.empty(n, dtype=torch.int32, device=step.dev)
        self.refresh()

    def refresh(self):
        """Recomputes the cached geometry-only nodes (after the positions,
        cameras or mesh changed)."""
        st = self.st
        st.forward()
        st._chk(_lib.dressi_invuv_build(st.ctx.handle, C.byref(st.desc), _p(st.uvbuf), _p(st.tri_id), st.B * st.K,
                                        st.H, st.W, _p(self.inv), st._s()), "invuv_build")

    def forward(self):
        with self.st._sparse():
            self._forward()

    def _forward(self):
        st = self.st
        h, s, ck = st.ctx.handle, st._s(), st._chk
        B, K, H, W = st.B, st.K, st.H, st.W
        if getattr(st, "packed", False):
            # the packed pass samples, shades and blends in one kernel (it
            # recomputes the cheap interpolation beside them); the map stays
            ck(_lib.dressi_packed_forward(h, C.byref(st._pscene), _p(st.tri_id), _p(st.bary), B, H, W,
                                          _p(st.gbuf), _p(st.uvbuf), _p(st.samp), _p(st.color), _p(st.sil),
                                          _p(st.E), None, s), "packed_forward")
            return
        ck(_lib.dressi_texture(h, _p(st.tex), C.byref(st.desc), _p(st.uvbuf), _p(st.tri_id), B * K, H, W,
                               _p(st.samp), s), "texture")
        if st.env is not None:
            ck(_lib.dressi_shade(h, st.mode, C.byref(st._fin_dir), _p(st.eye), _p(st.tri_id), B, K * H * W,
                                 None, _p(st.dir), s), "shade dir")
            ck(_lib.dressi_texture(h, _p(st.env), C.byref(st.env_desc), _p(st.dir), _p(st.tri_id), B * K, H, W,
                                   _p(st.env_s), s), "texture env")
        ck(_lib.dressi_shade(h, st.mode, C.byref(st._fin), _p(st.eye), _p(st.tri_id), B, K * H * W,
                             _p(st.layer_color), None, s), "shade")
        ck(_lib.dressi_softras(h, _p(st.layer_color), _p(st.dist), _p(st.tri_id), B, K, H, W, 3, st.sigma,
                               st.delta, st.blend, _p(st.color), _p(st.sil), _p(st.E), s), "softras")

    def loss_and_grad(self):
        self.st.loss_and_grad()

    def backward(self):
        with self.st._sparse():
            self._backward()

    def _backward(self):
        st = self.st
        h, s, ck = st.ctx.handle, st._s(), st._chk
        B, K, H, W = st.B, st.K, st.H, st.W
        Npv = K * H * W
        ck(_lib.dressi_softras_bwd(h, _p(st.layer_color), _p(st.dist), _p(st.tri_id), B, K, H, W, 3, st.sigma,
                                   _p(st.E), _p(st.g_color), _p(st.g_sil), _p(st.g_layer), None, s),
           "softras_bwd")
        if st.env is not None:
            ge = Bd.FragGrad()
            ge.env, ge.env_stride = _cp(st.g_env_s, 0), 3
            ck(_lib.dressi_shade_bwd(h, st.mode, C.byref(st._fin), _p(st.eye), _p(st.tri_id), B, Npv,
                                     _p(st.g_layer), None, C.byref(ge), s), "shade_bwd env")
            st._texture_bwd(st.env, st.env_desc, st.dir, B * K, st.g_env_s, st.g_envtex, st.g_dir,
                            "texture_bwd env")
        g = Bd.FragGrad()
        g.albedo, g.albedo_stride = _cp(st.g_samp, 0), st.Ct
        if st.mode == Bd.SHADE_PHONG_ENV:
            g.nmap, g.nmap_stride = _cp(st.g_samp, 4), st.Ct
        ck(_lib.dressi_shade_bwd(h, st.mode, C.byref(st._fin), _p(st.eye), _p(st.tri_id), B, Npv, _p(st.g_layer),
                                 _p(st.g_dir), C.byref(g), s), "shade_bwd")
        ck(_lib.dressi_texture_grad_invuv(h, C.byref(st.desc), _p(st.uvbuf), _p(st.tri_id), B * K, H, W,
                                          _p(self.inv), _p(st.g_samp), _p(st.g_tex), s), "texture_grad_invuv")
        st._join()

    def run(self):
        """One texture-only step: forward, loss and gradient, backward (in the
        packed form the loss and the albedo sample's adjoint are one pass, as
        in the wrapped Step)."""
        self.forward()
        st = self.st
        if getattr(st, "packed", False):
            h, s, ck = st.ctx.handle, st._s(), st._chk
            rec = st.inv_rec if st.gather_rec else None
            with st._sparse():
                ck(_lib.dressi_packed_backward(h, C.byref(st._pscene), _p(st.tri_id), st.B, st.H, st.W,
                                               _p(st.gbuf), _p(st.uvbuf), _p(st.samp), _p(st.color), _p(st.sil),
                                               _p(st.target), _p(getattr(st, "weight", None)), _p(st.loss), None,
                                               None, None, _p(st.g_samp), None, None, _p(rec), None, s),
                   "packed_backward")
                st._gather(h, self.inv, rec, s)
            return
        self.loss_and_grad()
        self.backward()

    def grads(self):
        """Gradients of the loss w.r.t. the textures."""
        out = {"tex": self.st.grads()["tex"]}
        if self.st.g_envtex is not None:
            out["env"] = self.st.g_envtex
        return out


def make_target(scene: Scene, device="cuda", views=None) -> Step:
    """Renders the scene's target (perturbed mesh / target texture) once."""
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    params = {}
    if scene.target_pos is not None:
        params["pos"] = f32(scene.target_pos)
    if scene.target_color is not None:
        params["color"] = f32(scene.target_color)
    if scene.target_tex is not None:
        params["tex"] = f32(pack_textures(scene.target_tex, scene.nmap))
    st = Step(scene, device, views=views, params=params)
    st.forward()
    return st


# ---------------------------------------------------------------------------
# uneven batches
# ---------------------------------------------------------------------------
def pack_views(sizes, width=None):
    """Shelf packing of views (W_i, H_i) into one image: views sorted by
    height (then width, then index) fill rows left to right.  Without a
    width, every multiple of 256 from the widest view up to four times the
    side of a square of the same area is tried and the smallest image kept
    (the narrower on ties).  Returns the (x0, y0) of every view and the image
    size (Wc, Hc)."""
    n = len(sizes)
    if width is None:
        area = sum(w * h for w, h in sizes)
        w0 = max(w for w, _ in sizes)
        best = None
        for wd in range(int(math.ceil(w0 / 256.0)) * 256, max(w0, int(4 * math.sqrt(area))) + 256, 256):
            _, (wc, hc) = pack_views(sizes, wd)
            if best is None or wc * hc < best[0]:
                best = (wc * hc, wd)
        width = max(w0, best[1])
    order = sorted(range(n), key=lambda i: (-sizes[i][1], -sizes[i][0], i))
    x = y = shelf = 0
    at = [None] * n
    for i in order:
        w, h = sizes[i]
        if x + w > width:
            y += shelf
            x = shelf = 0
        at[i] = (x, y)
        x += w
        shelf = max(shelf, h)
    return at, (width, y + shelf)


class BatchStep(_TwoStreams):
    """Preallocated fwd+bwd of an uneven batch of standalone scenes (K=1,
    Phong, one 2-D texture each): the meshes are concatenated, every view is
    drawn into its own rectangle of one image and every stage is one launch
    for the whole batch.  The loss is the sum of the per-view L2 means."""

    # the whole batch is one slice of one layer, shaded with Phong and a hard
    # blend (the attributes a TextureStep reads from the step it wraps)
    B = K = 1
    mode = Bd.SHADE_PHONG
    blend = Bd.BLEND_HARD
    sigma, delta = 1.0, 0.0
    env = dist = g_dir = None

    def __init__(self, scenes_list, device="cuda", target: "BatchStep | None" = None,
                 params: list | None = None):
        dev = torch.device(device)
        self.dev = dev
        self.scenes = scenes_list
        n = self.n = len(scenes_list)
        for s in scenes_list:
            assert s.K == 1 and s.r == 0 and s.shading == "phong" and s.nmap is None, "K=1 Phong scenes only"
            assert s.tex.shape == scenes_list[0].tex.shape, "one texture size for the batch"
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
        i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(dev)
        sizes = [(s.W, s.H) for s in scenes_list]
        at, (Wc, Hc) = pack_views(sizes)
        self.at, self.W, self.H = at, Wc, Hc
        self.views_np = np.array([(at[i][0], at[i][1], sizes[i][0], sizes[i][1]) for i in range(n)], np.int32)
        V = [s.pos.shape[0] for s in scenes_list]
        T = [s.tris.shape[0] for s in scenes_list]
        Vu = [s.uv.shape[0] for s in scenes_list]
        self.vbase = np.concatenate([[0], np.cumsum(V)]).astype(np.int64)
        self.tbase = np.concatenate([[0], np.cumsum(T)]).astype(np.int64)
        ubase = np.concatenate([[0], np.cumsum(Vu)]).astype(np.int64)
        self.V, self.T = int(self.vbase[-1]), int(self.tbase[-1])
        p = params or [{} for _ in range(n)]
        pos = [p[i].get("pos", s.pos) for i, s in enumerate(scenes_list)]
        tex = [p[i].get("tex", s.tex) for i, s in enumerate(scenes_list)]
        self.pos = f32(np.concatenate(pos))
        self.tris = i32(np.concatenate([s.tris + self.vbase[i] for i, s in enumerate(scenes_list)]))
        self.uv = f32(np.concatenate([s.uv for s in scenes_list]))
        self.uv_tris = i32(np.concatenate([s.uv_tris + ubase[i] for i, s in enumerate(scenes_list)]))
        self.vert_view = i32(np.repeat(np.arange(n), V))
        self.tri_view = i32(np.repeat(np.arange(n), T))
        self.views = i32(self.views_np)
        self.mvp = f32(np.stack([s.mvp[0] for s in scenes_list]))
        self.eye = f32(np.stack([s.eyes[0] for s in scenes_list]))
        self.tex = f32(np.stack(tex))
        wu, wv = scenes_list[0].extra.get("wrap", (Bd.WRAP_REPEAT, Bd.WRAP_CLAMP))
        Ht, Wt, Ct = self.tex.shape[1:]
        self.Ct = Ct
        self.desc = Bd.TexDesc(Bd.TEX_2D_ARRAY, Ht, Wt, Ct, wu, wv, n, self.tri_view.data_ptr())
        wgt = np.zeros((Hc, Wc), np.float32)
        for i, (x0, y0, w, h) in enumerate(self.views_np):
            wgt[y0:y0 + h, x0:x0 + w] = np.float32(1.0) / np.float32(4.0 * float(w * h))
        self.weight = f32(wgt)
        e = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device=dev)
        H, W = Hc, Wc
        self.Cv = 6
        self.vattr = e(self.V, 6)
        self.pos_clip = e(self.V, 4)
        self.tri_id = e(1, 1, H, W, dt=torch.int32)
        self.bary = e(1, 1, H, W, 2)
        self.gbuf = e(1, 1, H, W, 6)
        self.uvbuf = e(1, 1, H, W, 2)
        self.samp = e(1, 1, H, W, Ct)
        self.layer_color = e(1, 1, H, W, 3)
        self.color = e(1, H, W, 3)
        self.sil = e(1, H, W)
        self.E = e(1, H, W, dt=torch.uint8)
        self.loss = e(1)
        self.target = e(1, H, W, 4) if target is None else target.rgba()
        self.g_color = e(1, H, W, 3)
        self.g_sil = e(1, H, W)
        self.g_layer = e(1, 1, H, W, 3)
        self.g_gbuf = e(1, 1, H, W, 6)
        self.g_samp = e(1, 1, H, W, Ct)
        self.g_tex = torch.empty_like(self.tex)
        self.g_uvbuf = e(1, 1, H, W, 2)
        self.g_bary_uv = e(1, 1, H, W, 2)
        self.g_bary = e(1, 1, H, W, 2)
        self.g_vattr = e(self.V, 6)
        self.g_clip = e(self.V, 4)
        self.g_pos_t = e(self.V, 3)
        self.g_pos = e(self.V, 3)
        self.ctx = Bd.context(dev.index)
        self._init_streams(dev)
        self.adj = Bd.dressi_adjacency(self.tris, self.V)
        self.uv_adj = Bd.dressi_adjacency(self.uv_tris, self.uv.shape[0])
        nbytes = int(_lib.dressi_fragment_index_bytes(1, 1, H, W, self.T))
        self.frag_index = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        fi = Bd.FragIn()
        fi.normal, fi.normal_stride = _cp(self.gbuf, 0), 6
        fi.pos, fi.pos_stride = _cp(self.gbuf, 3), 6
        fi.albedo, fi.albedo_stride, fi.albedo_channels = _cp(self.samp, 0), Ct, 4
        fi.tri_eye = C.c_void_p(self.tri_view.data_ptr())
        self._fin = fi
        # stage packing (§3.3.3) as in Step: interpolation, texture, shading
        # and blend as one forward pass, the weighted loss and their adjoints
        # as one backward pass; scenes' extra["packed"] = False keeps the
        # separate stages
        self.packed = Ct == 4 and all(bool(s.extra.get("packed", True)) for s in scenes_list)
        self.inv = None
        if self.packed:
            ps = Bd.PackedScene()
            ps.mode, ps.vattr, ps.V, ps.Cv = Bd.SHADE_PHONG, _p(self.vattr), self.V, 6
            ps.tris, ps.T, ps.eye, ps.tri_eye = _p(self.tris), self.T, _p(self.eye), _p(self.tri_view)
            ps.uv, ps.uv_tris, ps.Vuv = _p(self.uv), _p(self.uv_tris), self.uv.shape[0]
            ps.tex, ps.td = _p(self.tex), self.desc
            self._pscene = ps
            nb = int(_lib.dressi_invuv_bytes(C.byref(self.desc), 1))
            self.inv = torch.empty(nb // 4, dtype=torch.int32, device=dev)
            self.inv_rec = torch.empty((H * W, 8), dtype=torch.float32, device=dev)
        self.hard_raster = None
        self.hybrid_weight = HYBRID_WEIGHT_DEFAULT
        self._calibrate_bins()

    def _s(self):
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _chk(self, rc, what):
        if rc != 0:
            self.ctx.check(rc, what)

    def _raster(self, attrs=False):
        h, st = self.ctx.handle, self._s()
        self.ctx.tune(Bd.TUNE_HARD_RASTER, self.hard_raster or 0)
        self.ctx.tune(Bd.TUNE_HYBRID_WEIGHT, self.hybrid_weight)
        if attrs:
            self._chk(_lib.dressi_vertex_stage(h, _p(self.pos), _p(self.tris), self.V, self.T, None, _p(self.adj),
                                               _p(self.mvp), _p(self.vert_view), 1, _p(self.vattr),
                                               _p(self.pos_clip), st), "vertex_stage")
        else:
            self._chk(_lib.dressi_transform_batched(h, _p(self.pos), _p(self.vert_view), _p(self.mvp), self.V,
                                                    _p(self.pos_clip), st), "transform_batched")
        self._chk(_lib.dressi_rasterize_batched(h, _p(self.pos_clip), _p(self.tris), _p(self.tri_view),
                                                _p(self.views), self.n, self.V, self.T, self.H, self.W, 1, 0,
                                                _p(self.tri_id), _p(self.bary), st), "rasterize_batched")

    def _calibrate_bins(self):
        for _ in range(4):
            self._raster()
            need = self.ctx.check_status()
            if need <= 0:
                return
            cap = 1
            while cap < need * 5 // 4:
                cap <<= 1
            self.ctx.reserve(0, cap)
        raise RuntimeError("tile bins still overflow after growing them")

    def forward(self):
        with self._sparse():
            self._forward()

    def _forward(self):
        h, st = self.ctx.handle, self._s()
        H, W, V, T, ck = self.H, self.W, self.V, self.T, self._chk
        if self._on("attrs"):
            self._fork("attrs")
            self._chk2(_lib.dressi_vertex_attrs(self._h2("attrs"), _p(self.pos), _p(self.tris), V, T, None,
                                                _p(self.adj), _p(self.vattr), self._sa("attrs")), "vertex_attrs",
                       "attrs")
            self._raster()
            self._join()
        else:
            self._raster(attrs=True)
        self._fork("index")
        self._chk2(_lib.dressi_fragment_index(self._h2("index"), _p(self.tri_id), 1, 1, H, W, T, _p(self.frag_index),
                                              self._sa("index")), "fragment_index", "index")
        if self.packed:
            ck(_lib.dressi_packed_forward(h, C.byref(self._pscene), _p(self.tri_id), _p(self.bary), 1, H, W,
                                          _p(self.gbuf), _p(self.uvbuf), _p(self.samp), _p(self.color),
                                          _p(self.sil), _p(self.E), _p(self.inv), st), "packed_forward")
            self._join()
            return
        ck(_lib.dressi_interpolate(h, _p(self.vattr), 1, V, 6, _p(self.tris), T, _p(self.tri_id), _p(self.bary),
                                   1, 1, H, W, _p(self.gbuf), st), "interpolate")
        ck(_lib.dressi_interpolate(h, _p(self.uv), 1, self.uv.shape[0], 2, _p(self.uv_tris), T, _p(self.tri_id),
                                   _p(self.bary), 1, 1, H, W, _p(self.uvbuf), st), "interpolate uv")
        ck(_lib.dressi_texture(h, _p(self.tex), C.byref(self.desc), _p(self.uvbuf), _p(self.tri_id), 1, H, W,
                               _p(self.samp), st), "texture")
        ck(_lib.dressi_shade(h, Bd.SHADE_PHONG, C.byref(self._fin), _p(self.eye), _p(self.tri_id), 1, H * W,
                             _p(self.layer_color), None, st), "shade")
        ck(_lib.dressi_softras(h, _p(self.layer_color), None, _p(self.tri_id), 1, 1, H, W, 3, 1.0, 0.0,
                               Bd.BLEND_HARD, _p(self.color), _p(self.sil), _p(self.E), st), "softras")
        self._join()

    def loss_and_grad(self):
        self._chk(_lib.dressi_loss_l2(self.ctx.handle, _p(self.color), _p(self.sil), _p(self.target),
                                      _p(self.weight), 1, self.H, self.W, _p(self.loss), _p(self.g_color),
                                      _p(self.g_sil), self._s()), "loss")

    def backward(self):
        with self._sparse():
            self._backward()

    def _backward(self):
        h, st = self.ctx.handle, self._s()
        H, W, V, T, ck, Ct = self.H, self.W, self.V, self.T, self._chk, self.Ct
        ck(_lib.dressi_softras_bwd(h, _p(self.layer_color), None, _p(self.tri_id), 1, 1, H, W, 3, 1.0, _p(self.E),
                                   _p(self.g_color), _p(self.g_sil), _p(self.g_layer), None, st), "softras_bwd")
        g = Bd.FragGrad()
        g.normal, g.normal_stride = _cp(self.g_gbuf, 0), 6
        g.pos, g.pos_stride = _cp(self.g_gbuf, 3), 6
        g.albedo, g.albedo_stride = _cp(self.g_samp, 0), Ct
        ck(_lib.dressi_shade_bwd(h, Bd.SHADE_PHONG, C.byref(self._fin), _p(self.eye), _p(self.tri_id), 1, H * W,
                                 _p(self.g_layer), None, C.byref(g), st), "shade_bwd")
        self._texture_bwd(self.tex, self.desc, self.uvbuf, 1, self.g_samp, self.g_tex, self.g_uvbuf, "texture_bwd")
        ck(_lib.dressi_interpolate_bwd(h, _p(self.uv), 1, self.uv.shape[0], 2, _p(self.uv_tris), T,
                                       _p(self.tri_id), _p(self.bary), 1, 1, H, W, _p(self.g_uvbuf), None,
                                       _p(self.frag_index), _p(self.uv_adj), None, _p(self.g_bary_uv), st),
           "interpolate_bwd uv")
        self._backward_geometry()
        self._join()

    def _packed_backward(self):
        """Weighted loss, blend, shading and texture-coordinate adjoints in
        one pass (with the inverse-UV registration), then the texel gather
        and the geometry's backward as in the separate form."""
        h, st = self.ctx.handle, self._s()
        H, W, T = self.H, self.W, self.T
        # with records, the texel gather runs inside the packed backward
        rec = self.inv_rec if self.gather_rec else None
        self._chk(_lib.dressi_packed_backward(h, C.byref(self._pscene), _p(self.tri_id), 1, H, W, _p(self.gbuf),
                                              _p(self.uvbuf), _p(self.samp), _p(self.color), _p(self.sil),
                                              _p(self.target), _p(self.weight), _p(self.loss), None, None,
                                              _p(self.g_gbuf), _p(self.g_samp), _p(self.g_bary_uv), _p(self.inv),
                                              _p(rec), _p(self.g_tex if rec is not None else None), st),
                  "packed_backward")
        if rec is None:
            self._fork("texel")
            self._gather(self._h2("texel"), self.inv, None, self._sa("texel"), "texel")
        ck = self._chk
        V, T = self.V, self.T
        ck(_lib.dressi_geometry_bwd(h, _p(self.pos), _p(self.vattr), V, 6, _p(self.tris), T, _p(self.pos_clip),
                                    _p(self.mvp), _p(self.vert_view), _p(self.tri_view), _p(self.views), self.n, H,
                                    W, 0, _p(self.tri_id), _p(self.bary), _p(self.g_gbuf), _p(self.g_bary_uv),
                                    _p(self.frag_index), _p(self.adj), _p(self.g_vattr), _p(self.g_bary),
                                    _p(self.g_clip), _p(self.g_pos), st), "geometry_bwd")
        self._join()

    def _backward_geometry(self):
        """Attribute interpolation, rasterization, transform and vertex
        attribute adjoints from g_gbuf and the texture coordinates'
        barycentric gradient g_bary_uv."""
        h, st = self.ctx.handle, self._s()
        H, W, V, T, ck = self.H, self.W, self.V, self.T, self._chk
        ck(_lib.dressi_interpolate_bwd(h, _p(self.vattr), 1, V, 6, _p(self.tris), T, _p(self.tri_id), _p(self.bary),
                                       1, 1, H, W, _p(self.g_gbuf), _p(self.g_bary_uv), _p(self.frag_index),
                                       _p(self.adj), _p(self.g_vattr), _p(self.g_bary), st), "interpolate_bwd")
        ck(_lib.dressi_rasterize_batched_bwd(h, _p(self.pos_clip), _p(self.tris), _p(self.tri_view), _p(self.views),
                                             self.n, V, T, H, W, 1, 0, _p(self.tri_id), _p(self.g_bary),
                                             _p(self.frag_index), _p(self.adj), _p(self.g_clip), st),
           "rasterize_batched_bwd")
        ck(_lib.dressi_transform_batched_bwd(h, _p(self.mvp), _p(self.vert_view), V, _p(self.g_clip),
                                             _p(self.g_pos_t), st), "transform_batched_bwd")
        ck(_lib.dressi_vertex_attrs_bwd(h, _p(self.pos), _p(self.tris), V, T, 6, _p(self.adj), _p(self.g_vattr),
                                        _p(self.g_pos_t), _p(self.g_pos), st), "vertex_attrs_bwd")

    def run(self):
        """One step; in the packed form (without inverse-UV jitter) the loss
        and the backward are one pass, leaving g_color and g_sil unwritten."""
        packed = self.packed and self.frame == 0
        self.forward()
        if packed:
            with self._sparse():
                self._packed_backward()
            return
        self.loss_and_grad()
        self.backward()

    check_overflow = Step.check_overflow

    def rgba(self):
        return torch.cat([self.color, self.sil[..., None]], -1).contiguous()

    # per-view views of the batched buffers
    def view_rect(self, i):
        x0, y0, w, h = (int(v) for v in self.views_np[i])
        return (slice(y0, y0 + h), slice(x0, x0 + w))

    def view_tri_id(self, i):
        """tri_id of view i in its own triangle numbering (-1 = empty)."""
        t = self.tri_id[0, 0][self.view_rect(i)]
        return torch.where(t >= 0, t - int(self.tbase[i]), t)

    def grads(self):
        """Gradients of the loss w.r.t. the batch's positions and textures [n,Ht,Wt,Ct]."""
        return {"pos": self.g_pos, "tex": self.g_tex}

    def view_grads(self, i):
        return {"pos": self.g_pos[int(self.vbase[i]):int(self.vbase[i + 1])], "tex": self.g_tex[i]}


def make_batch_target(scenes_list, device="cuda") -> BatchStep:
    """Renders the targets of an uneven batch (perturbed meshes, target textures)."""
    params = [{"pos": s.target_pos, "tex": s.target_tex} for s in scenes_list]
    st = BatchStep(scenes_list, device, params=params)
    st.forward()
    return st


# ---------------------------------------------------------------------------
# autotuning
# ---------------------------------------------------------------------------
HARD_RASTER_NAMES = {None: "pixel-parallel (soft)", 0: "triangle-parallel", 1: "pixel-parallel", 2: "per-tile",
                     3: "binless (global atomics)"}
def autotune(step, reps: int = 5) -> dict:
    """Picks the hard-rasterization strategy (triangle-parallel tiles,
    pixel-parallel tiles, a choice per tile and triangle batch with one of a
    few cost weights, or, for one layer, triangle-parallel without bins) and
    the tile-bin capacity for this step's own geometry
    by timing each candidate's transform + rasterization on the device, after
    checking that it selects exactly the same layers as the first candidate
    (it must: the choice changes speed only).  The choice is stored on the
    step and applied at every later rasterization, so it is also what a
    captured graph records.  Soft rasterization (r > 0) has one strategy; only
    its bin capacity is tuned."""
    ctx = step.ctx
    if getattr(step, "r", 0.0) != 0:
        cands = [(None, HYBRID_WEIGHT_DEFAULT)]
    else:
        cands = [(0, HYBRID_WEIGHT_DEFAULT), (1, HYBRID_WEIGHT_DEFAULT)]
        if getattr(step, "K", 1) == 1:
            cands += [(2, w) for w in HYBRID_WEIGHTS] + [(3, HYBRID_WEIGHT_DEFAULT)]
    need = 0
    results = {}
    ref = None
    ref_bary = None
    for hr, w in cands:
        step.hard_raster, step.hybrid_weight = hr, w
        step._raster()
        torch.cuda.synchronize()
        need = max(need, ctx.check_status())
        tid, bary = step.tri_id.clone(), step.bary.clone()
        if ref is None:
            ref, ref_bary = tid, bary
        elif not torch.equal(ref, tid) or not torch.equal(ref_bary[ref >= 0], bary[ref >= 0]):
            raise RuntimeError(f"rasterization strategy {hr} (weight {w}) selects different layers")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step._raster()
        e1.record()
        torch.cuda.synchronize()
        results[(hr, w)] = e0.elapsed_time(e1) / reps
    best = min(results, key=results.get)
    step.hard_raster, step.hybrid_weight = best
    # bin capacity: the smallest power of two above 5/4 of the fullest tile
    cap = 0
    if need > 0:
        cap = 1
        while cap < need * 5 // 4:
            cap <<= 1
        ctx.reserve(0, cap)
    return {"hard_raster": best[0], "hybrid_weight": best[1], "ms": results, "bin_capacity": cap}


def autotune_streams(step, reps: int = 20) -> dict:
    """Chooses between issuing the whole step on the caller's stream, running
    the fragment index, the texel gather or both on a second stream, and
    running every independent branch there, by timing graph replays of the
    captured step in each mode (the results are the same)."""
    results = {}
    for mode in (False, "index", "texel", ("index", "texel"), True):
        step.concurrent = mode
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step.run()
        for _ in range(3):
            g.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        results[mode] = e0.elapsed_time(e1) / reps
        del g
    step.concurrent = min(results, key=results.get)
    return {"concurrent": step.concurrent, "ms": results}


# ---------------------------------------------------------------------------
# the optimisation loop
# ---------------------------------------------------------------------------
class Adam:
    """Adam (Kingma & Ba) on one parameter tensor: moments and the step state
    live on the device, so a captured step replays successive updates."""

    def __init__(self, param: torch.Tensor, lr: float, betas=(0.9, 0.999), eps: float = 1e-8):
        self.p = param
        self.lr, self.b1, self.b2, self.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
        self.m = torch.zeros_like(param)
        self.v = torch.zeros_like(param)
        self.state = Bd.adam_state(param.device)

    def step(self, ctx, grad: torch.Tensor, stream):
        rc = _lib.dressi_adam(ctx.handle, _p(self.p), _p(grad), _p(self.m), _p(self.v), self.p.numel(), self.lr,
                              self.b1, self.b2, self.eps, _p(self.state), stream)
        if rc != 0:
            ctx.check(rc, "adam")

    def steps_taken(self) -> int:
        return int(self.state[0].item())


class FitLoop:
    """The paper's two-stage fit (§4.1, the cross-platform application):
    first the vertex positions, from silhouettes (the image loss's colour
    gradient dropped) plus the scheduled Laplacian regulariser, then, on the
    fitted geometry, the albedo texture from the colour loss, both with Adam.
    The texture stage runs as a texture-only step (TextureStep: the
    rasterization and the inverse-UV map cached).  Every iteration allocates
    nothing and can be captured into a graph; the Adam states and the
    regulariser's schedule advance on the device."""

    def __init__(self, step: Step, lr_pos: float = 0.01, lr_tex: float = 0.01, lap0: float = 10.0,
                 lap_gamma: float = 0.99):
        self.st = step
        # the geometry moves during the fit: give every tile bin room for all
        # triangles when that is affordable, so no bin can overflow
        nt = ((step.H + 15) // 16) * ((step.W + 15) // 16)
        cap = 1 << max(0, (step.T - 1).bit_length())
        if step.B * nt * cap * 4 <= 1 << 30:
            step.ctx.reserve(0, cap)
        self.adam_pos = Adam(step.pos, lr_pos)
        self.adam_tex = Adam(step.tex, lr_tex) if step.tex is not None else None
        self.lap0, self.lap_gamma = float(lap0), float(lap_gamma)
        self.reg = torch.zeros(1, device=step.dev)
        self.ts = None

    def silhouette_iteration(self):
        st = self.st
        h, s = st.ctx.handle, st._s()
        st.forward()
        st.loss_and_grad()
        st.g_color.zero_()
        st.backward()
        st._chk(_lib.dressi_laplacian_reg(h, _p(st.pos), _p(st.tris), st.V, st.T, _p(st.adj), self.lap0,
                                          self.lap_gamma, _p(self.adam_pos.state), _p(st.g_pos), _p(st.g_pos),
                                          _p(self.reg), s), "laplacian_reg")
        self.adam_pos.step(st.ctx, st.g_pos, s)

    def start_texture_stage(self):
        """Caches the fitted geometry for the texture stage."""
        if self.ts is None:
            self.ts = TextureStep(self.st)
        else:
            self.ts.refresh()

    def texture_iteration(self):
        st = self.st
        self.ts.run()
        self.adam_tex.step(st.ctx, st.g_tex, st._s())


# ---------------------------------------------------------------------------
# image-based physically-based shading
# ---------------------------------------------------------------------------
class PbsStep:
    """Split-sum PBS lit by an environment map, on fixed geometry (the paper's
    render graph in appendix B; appendix C optimises an environment map and
    the roughness with it).  Parameters: the environment cube map, the albedo
    texture and the material (metallic, roughness; device scalars).

    Per step: the irradiance and prefiltered maps are filtered from the
    environment (dense sums, exact adjoint), the albedo is sampled, the
    lookup directions and per-level masks are formed, the maps are sampled,
    the fragments shaded and blended, and the backward runs the reverse:
    blend, shading (albedo, samples and material), the maps' texel
    gradients by the inverse UV, the filters' adjoint to the environment,
    and the albedo texture's gather from the cached inverse-UV map.  The
    geometry-only nodes (rasterization, G-buffer, UVs, the albedo inverse
    UV) are computed once by a TextureStep."""

    def __init__(self, scene: Scene, env: np.ndarray, material=(0.5, 0.5), Si: int = 16, Sp: int = 32, L: int = 5,
                 lut_n: int = 32, lut_m: int = 512, target: "PbsStep | None" = None, device="cuda",
                 params: dict | None = None):
        if scene.shading != "phong":
            raise ValueError("PBS shading runs on a textured scene without normal or environment maps")
        self.st = st = Step(scene, device, params=params)
        self.dev = st.dev
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(st.dev)
        self.env = f32(env)
        self.S = self.env.shape[1]
        self.Si, self.Sp, self.L = Si, Sp, L
        self.material = f32(np.asarray(material, np.float32))
        self.desc = Bd.IblDesc(self.S, Si, Sp, L)
        e = lambda *s, dt=torch.float32: torch.empty(s, dtype=dt, device=st.dev)
        N = st.B * st.K * st.H * st.W
        self.N = N
        self.irr, self.pref = e(6, Si, Si, 3), e(L, 6, Sp, Sp, 3)
        self.norm = e(int(_lib.dressi_ibl_norm_bytes(C.byref(self.desc))) // 8, dt=torch.float64)
        self.lut = e(lut_n, lut_n, 2)
        st._chk(_lib.dressi_brdf_lut(st.ctx.handle, lut_n, lut_m, _p(self.lut), st._s()), "brdf_lut")
        self.dir_n, self.dir_r = e(N, 3), e(N, 3)
        self.ltid = e(L, N, dt=torch.int32)
        self.irr_s, self.pref_s = e(N, 3), e(L, N, 3)
        self.g_irr_s, self.g_pref_s = e(N, 3), e(L, N, 3)
        self.g_irr, self.g_pref = e(6, Si, Si, 3), e(L, 6, Sp, Sp, 3)
        self.g_env = torch.empty_like(self.env)
        self.g_material = e(2)
        self.cube_irr = Bd.TexDesc(Bd.TEX_CUBE, Si, Si, 3, Bd.WRAP_CLAMP, Bd.WRAP_CLAMP)
        self.cube_pref = Bd.TexDesc(Bd.TEX_CUBE, Sp, Sp, 3, Bd.WRAP_CLAMP, Bd.WRAP_CLAMP)
        self.ts = TextureStep(st)
        if target is not None:
            st.target.copy_(target.rgba())
        Ct = st.Ct
        self._pin = Bd.PbsIn()
        pin = self._pin
        pin.normal, pin.normal_stride = _cp(st.gbuf, 0), st.Cv
        pin.pos, pin.pos_stride = _cp(st.gbuf, 3), st.Cv
        pin.albedo, pin.albedo_stride = _cp(st.samp, 0), Ct
        pin.irr, pin.irr_stride = _p(self.irr_s), 3
        pin.pref, pin.pref_stride, pin.pref_level_stride = _p(self.pref_s), 3, N * 3
        pin.material, pin.lut, pin.lut_n, pin.levels = _p(self.material), _p(self.lut), lut_n, L
        self._pg = Bd.PbsGrad()
        pg = self._pg
        pg.albedo, pg.albedo_stride = _cp(st.g_samp, 0), Ct
        pg.irr, pg.pref, pg.material = _p(self.g_irr_s), _p(self.g_pref_s), _p(self.g_material)

    def _pref_level(self, t, l):
        return C.c_void_p(t.data_ptr() + 4 * l * (t[0].numel()))

    def forward(self):
        st = self.st
        h, s, ck = st.ctx.handle, st._s(), st._chk
        B, K, H, W, L = st.B, st.K, st.H, st.W, self.L
        S = B * K
        ck(_lib.dressi_ibl_filter(h, _p(self.env), C.byref(self.desc), _p(self.irr), _p(self.pref), _p(self.norm),
                                  s), "ibl_filter")
        ck(_lib.dressi_texture(h, _p(st.tex), C.byref(st.desc), _p(st.uvbuf), _p(st.tri_id), S, H, W, _p(st.samp), s),
           "texture")
        ck(_lib.dressi_shade_pbs(h, C.byref(self._pin), _p(st.eye), _p(st.tri_id), B, K * H * W, None, _p(self.dir_n),
                                 _p(self.dir_r), _p(self.ltid), s), "shade_pbs dirs")
        ck(_lib.dressi_texture(h, _p(self.irr), C.byref(self.cube_irr), _p(self.dir_n), _p(st.tri_id), S, H, W,
                               _p(self.irr_s), s), "texture irradiance")
        for l in range(L):
            ck(_lib.dressi_texture(h, self._pref_level(self.pref, l), C.byref(self.cube_pref), _p(self.dir_r),
                                   self._pref_level(self.ltid, l), S, H, W, self._pref_level(self.pref_s, l), s),
               "texture prefiltered")
        ck(_lib.dressi_shade_pbs(h, C.byref(self._pin), _p(st.eye), _p(st.tri_id), B, K * H * W, _p(st.layer_color),
                                 None, None, None, s), "shade_pbs")
        ck(_lib.dressi_softras(h, _p(st.layer_color), _p(st.dist), _p(st.tri_id), B, K, H, W, 3, st.sigma, st.delta,
                               st.blend, _p(st.color), _p(st.sil), _p(st.E), s), "softras")

    def loss_and_grad(self):
        self.st.loss_and_grad()

    def backward(self):
        st = self.st
        h, s, ck = st.ctx.handle, st._s(), st._chk
        B, K, H, W, L = st.B, st.K, st.H, st.W, self.L
        S = B * K
        ck(_lib.dressi_softras_bwd(h, _p(st.layer_color), _p(st.dist), _p(st.tri_id), B, K, H, W, 3, st.sigma,
                                   _p(st.E), _p(st.g_color), _p(st.g_sil), _p(st.g_layer), None, s), "softras_bwd")
        ck(_lib.dressi_shade_pbs_bwd(h, C.byref(self._pin), _p(st.eye), _p(st.tri_id), B, K * H * W, _p(st.g_layer),
                                     None, None, C.byref(self._pg), s), "shade_pbs_bwd")
        ck(_lib.dressi_texture_bwd(h, _p(self.irr), C.byref(self.cube_irr), _p(self.dir_n), _p(st.tri_id), S, H, W,
                                   _p(self.g_irr_s), 0, _p(self.g_irr), None, s), "texture_bwd irradiance")
        for l in range(L):
            ck(_lib.dressi_texture_bwd(h, self._pref_level(self.pref, l), C.byref(self.cube_pref), _p(self.dir_r),
                                       self._pref_level(self.ltid, l), S, H, W, self._pref_level(self.g_pref_s, l),
                                       0, self._pref_level(self.g_pref, l), None, s), "texture_bwd prefiltered")
        ck(_lib.dressi_ibl_filter_bwd(h, C.byref(self.desc), _p(self.norm), _p(self.g_irr), _p(self.g_pref),
                                      _p(self.g_env), s), "ibl_filter_bwd")
        ck(_lib.dressi_texture_grad_invuv(h, C.byref(st.desc), _p(st.uvbuf), _p(st.tri_id), S, H, W, _p(self.ts.inv),
                                          _p(st.g_samp), _p(st.g_tex), s), "texture_grad_invuv")

    def run(self):
        self.forward()
        self.loss_and_grad()
        self.backward()

    def rgba(self):
        return self.st.rgba()

    def grads(self):
        return {"env": self.g_env, "material": self.g_material, "tex": self.st.g_tex}
