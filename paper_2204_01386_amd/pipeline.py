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

import ctypes as C
import math

import numpy as np
import torch

from . import binding as Bd
from .scenes import Scene

_lib = Bd._lib


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


class Step:
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
        self.blend = Bd.BLEND_HSR if self.r > 0 else Bd.BLEND_HARD
        self.sigma = self.r / 7.0 if self.r > 0 else 1.0
        self.delta = self.r
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
        # topology-only structures: built once per mesh
        self.adj = Bd.dressi_adjacency(self.tris, self.V)
        self.uv_adj = Bd.dressi_adjacency(self.uv_tris, self.uv.shape[0]) if self.uv is not None else None
        nbytes = int(_lib.dressi_fragment_index_bytes(B, K, H, W, self.T))
        self.frag_index = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._fin = self._frag_in()
        self._fin_dir = self._frag_in(with_env=False)
        self._calibrate_bins()

    def _calibrate_bins(self):
        """Rasterizes once and grows the tile-bin capacity until no tile
        overflows (dense or strongly overlapping geometry), so that later
        steps, captured or not, need no check."""
        h, st = self.ctx.handle, self._s()
        for _ in range(4):
            self._chk(_lib.dressi_transform(h, _p(self.pos), _p(self.mvp), self.B, self.V, _p(self.pos_clip), st),
                      "transform")
            self._chk(_lib.dressi_rasterize(h, _p(self.pos_clip), _p(self.tris), self.B, self.V, self.T, self.H,
                                            self.W, self.K, self.r, 0, _p(self.tri_id), _p(self.bary),
                                            _p(self.dist), st), "rasterize")
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
        h, s = self.ctx.handle, self._s()
        B, V, T, H, W, K = self.B, self.V, self.T, self.H, self.W, self.K
        ck = self._chk
        ck(_lib.dressi_vertex_attrs(h, _p(self.pos), _p(self.tris), V, T, _p(self.extra), _p(self.adj),
                                    _p(self.vattr), s), "vertex_attrs")
        ck(_lib.dressi_transform(h, _p(self.pos), _p(self.mvp), B, V, _p(self.pos_clip), s), "transform")
        ck(_lib.dressi_rasterize(h, _p(self.pos_clip), _p(self.tris), B, V, T, H, W, K, self.r, 0,
                                 _p(self.tri_id), _p(self.bary), _p(self.dist), s), "rasterize")
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

    def loss_and_grad(self):
        ck = self._chk
        ck(_lib.dressi_loss_l2(self.ctx.handle, _p(self.color), _p(self.sil), _p(self.target), self.B,
                               self.H, self.W, _p(self.loss), _p(self.g_color), _p(self.g_sil),
                               self._s()), "loss")

    def backward(self):
        h, s = self.ctx.handle, self._s()
        B, V, T, H, W, K = self.B, self.V, self.T, self.H, self.W, self.K
        ck = self._chk
        Cv = self.Cv
        ck(_lib.dressi_fragment_index(h, _p(self.tri_id), B, K, H, W, T, _p(self.frag_index), s),
           "fragment_index")
        ck(_lib.dressi_softras_bwd(h, _p(self.layer_color), _p(self.dist), _p(self.tri_id), B, K, H, W, 3,
                                   self.sigma, _p(self.E), _p(self.g_color), _p(self.g_sil),
                                   _p(self.g_layer), _p(self.g_dist), s), "softras_bwd")
        Npv = K * H * W
        if self.env is not None:
            ge = Bd.FragGrad()
            ge.env, ge.env_stride = _cp(self.g_env_s, 0), 3
            ck(_lib.dressi_shade_bwd(h, self.mode, C.byref(self._fin), _p(self.eye), _p(self.tri_id), B,
                                     Npv, _p(self.g_layer), None, C.byref(ge), s), "shade_bwd env")
            ck(_lib.dressi_texture_bwd(h, _p(self.env), C.byref(self.env_desc), _p(self.dir),
                                       _p(self.tri_id), B * K, H, W, _p(self.g_env_s), _p(self.g_envtex),
                                       _p(self.g_dir), s), "texture_bwd env")
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
            ck(_lib.dressi_texture_bwd(h, _p(self.tex), C.byref(self.desc), _p(self.uvbuf),
                                       _p(self.tri_id), B * K, H, W, _p(self.g_samp), _p(self.g_tex),
                                       _p(self.g_uvbuf), s), "texture_bwd")
            ck(_lib.dressi_interpolate_bwd(h, _p(self.uv), 1, self.uv.shape[0], 2, _p(self.uv_tris), T,
                                           _p(self.tri_id), _p(self.bary), B, K, H, W, _p(self.g_uvbuf),
                                           None, _p(self.frag_index), _p(self.uv_adj), None,
                                           _p(self.g_bary_uv), s), "interpolate_bwd uv")
            gb_in = self.g_bary_uv
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

    def run(self):
        """One full step: forward, loss and gradient, backward."""
        self.forward()
        self.loss_and_grad()
        self.backward()

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
