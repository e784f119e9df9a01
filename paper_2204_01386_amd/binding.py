"""ctypes binding of libdressi.so: argument marshalling only.

Each function has the name of the C entry point it calls, takes torch tensors
that already live on the GPU (contiguous, dtype as the C header states),
allocates the outputs with torch, and enqueues the call on torch's current
stream.  All computation happens in the HIP kernels of libdressi.so; there is
no CPU or PyTorch fallback: if the library is missing this module raises on
import.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdressi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libdressi.so not found at {LIB_PATH}; build it first "
        "(python -c 'import __graft_entry__ as g; g.build()' or python paper_2204_01386_amd/build.py)")

_lib = C.CDLL(LIB_PATH)

TEX_2D, TEX_CUBE, TEX_2D_ARRAY = 0, 1, 2
TUNE_BIN_CAPACITY, TUNE_HARD_RASTER, TUNE_HYBRID_WEIGHT, TUNE_EMPTY_SLOTS, TUNE_IV_ROWS = 1, 2, 3, 4, 5
WRAP_REPEAT, WRAP_CLAMP = 0, 1
BLEND_HSR, BLEND_AA, BLEND_SOFTRAS, BLEND_HARD = 0, 1, 2, 3

OK, EINVAL, ENOMEM, EHIP, EOVERFLOW = 0, -1, -2, -3, -4
STATUS = {OK: "ok", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", EOVERFLOW: "EOVERFLOW"}


class TexDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("Ht", C.c_int), ("Wt", C.c_int), ("Ct", C.c_int),
                ("wrap_u", C.c_int), ("wrap_v", C.c_int), ("layers", C.c_int), ("tri_layer", C.c_void_p)]


_vp, _i, _f, _i64, _sz = C.c_void_p, C.c_int, C.c_float, C.c_int64, C.c_size_t

SHADE_LAMBERT, SHADE_PHONG, SHADE_PHONG_ENV = 0, 1, 2


class FragIn(C.Structure):
    """dressi_frag_in: per-fragment shading inputs as (pointer, row stride)."""
    _fields_ = [("normal", _vp), ("normal_stride", _i), ("pos", _vp), ("pos_stride", _i),
                ("tangent", _vp), ("tangent_stride", _i), ("nmap", _vp), ("nmap_stride", _i),
                ("albedo", _vp), ("albedo_stride", _i), ("albedo_channels", _i),
                ("env", _vp), ("env_stride", _i), ("tri_eye", _vp)]


class PackedScene(C.Structure):
    """dressi_packed_scene: the inputs of the packed single-layer pass."""
    _fields_ = [("mode", _i), ("vattr", _vp), ("V", _i), ("Cv", _i), ("tris", _vp), ("T", _i),
                ("uv", _vp), ("uv_tris", _vp), ("Vuv", _i), ("tex", _vp), ("td", TexDesc), ("eye", _vp),
                ("tri_eye", _vp)]


class PackedStepBufs(C.Structure):
    """dressi_packed_step_bufs: the inputs, forward values and gradients of
    one packed step (dressi_packed_step)."""
    _fields_ = [("pos", _vp), ("extra", _vp), ("adj", _vp), ("mvp", _vp), ("H", _i), ("W", _i), ("target", _vp),
                ("vattr", _vp), ("pos_clip", _vp), ("tri_id", _vp), ("bary", _vp), ("index", _vp),
                ("gbuf", _vp), ("uvbuf", _vp), ("samp", _vp), ("color", _vp), ("sil", _vp), ("edge", _vp),
                ("inv", _vp), ("inv_rec", _vp),
                ("loss", _vp), ("grad_gbuf", _vp), ("grad_samp", _vp), ("grad_bary_uv", _vp), ("grad_tex", _vp),
                ("grad_vattr", _vp), ("grad_bary", _vp), ("grad_pos_clip", _vp), ("grad_pos", _vp)]


class FragGrad(C.Structure):
    _fields_ = [("normal", _vp), ("normal_stride", _i), ("pos", _vp), ("pos_stride", _i),
                ("tangent", _vp), ("tangent_stride", _i), ("nmap", _vp), ("nmap_stride", _i),
                ("albedo", _vp), ("albedo_stride", _i), ("env", _vp), ("env_stride", _i)]


class IblDesc(C.Structure):
    """dressi_ibl_desc: environment, irradiance and prefiltered face sizes, levels."""
    _fields_ = [("S", _i), ("Si", _i), ("Sp", _i), ("L", _i)]


class PbsIn(C.Structure):
    """dressi_pbs_in: per-fragment PBS inputs as (pointer, row stride)."""
    _fields_ = [("normal", _vp), ("normal_stride", _i), ("pos", _vp), ("pos_stride", _i),
                ("albedo", _vp), ("albedo_stride", _i), ("irr", _vp), ("irr_stride", _i),
                ("pref", _vp), ("pref_stride", _i), ("pref_level_stride", _i64),
                ("material", _vp), ("lut", _vp), ("lut_n", _i), ("levels", _i)]


class PbsGrad(C.Structure):
    _fields_ = [("normal", _vp), ("normal_stride", _i), ("pos", _vp), ("pos_stride", _i),
                ("albedo", _vp), ("albedo_stride", _i), ("irr", _vp), ("pref", _vp), ("material", _vp)]


_SIG = {
    "dressi_create": [C.POINTER(C.c_void_p), _i],
    "dressi_destroy": [_vp],
    "dressi_reserve": [_vp, _sz, _i64],
    "dressi_check_status": [_vp, C.POINTER(C.c_int64), _vp],
    "dressi_rasterize": [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _f, _i, _vp, _vp, _vp, _vp],
    "dressi_rasterize_banded": [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _f, _i, _f, _i, _vp, _vp, _vp, _vp],
    "dressi_rasterize_bwd": [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _f, _i, _vp, _vp, _vp, _vp, _vp,
                             _vp, _vp],
    "dressi_interpolate": [_vp, _vp, _i, _i, _i, _vp, _i, _vp, _vp, _i, _i, _i, _i, _vp, _vp],
    "dressi_interpolate_bwd": [_vp, _vp, _i, _i, _i, _vp, _i, _vp, _vp, _i, _i, _i, _i, _vp, _vp,
                               _vp, _vp, _vp, _vp, _vp],
    "dressi_texture": [_vp, _vp, C.POINTER(TexDesc), _vp, _vp, _i, _i, _i, _vp, _vp],
    "dressi_texture_bwd": [_vp, _vp, C.POINTER(TexDesc), _vp, _vp, _i, _i, _i, _vp, C.c_uint32, _vp, _vp, _vp],
    "dressi_ibl_filter": [_vp, _vp, C.POINTER(IblDesc), _vp, _vp, _vp, _vp],
    "dressi_ibl_filter_bwd": [_vp, C.POINTER(IblDesc), _vp, _vp, _vp, _vp, _vp],
    "dressi_brdf_lut": [_vp, _i, _i, _vp, _vp],
    "dressi_shade_pbs": [_vp, C.POINTER(PbsIn), _vp, _vp, _i, _i64, _vp, _vp, _vp, _vp, _vp],
    "dressi_shade_pbs_bwd": [_vp, C.POINTER(PbsIn), _vp, _vp, _i, _i64, _vp, _vp, _vp, C.POINTER(PbsGrad), _vp],
    "dressi_adam": [_vp, _vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, _vp, _vp],
    "dressi_laplacian_reg": [_vp, _vp, _vp, _i, _i, _vp, _f, _f, _vp, _vp, _vp, _vp, _vp],
    "dressi_invuv_build": [_vp, C.POINTER(TexDesc), _vp, _vp, _i, _i, _i, _vp, _vp],
    "dressi_texture_grad_invuv": [_vp, C.POINTER(TexDesc), _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp],
    "dressi_softras": [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _f, _f, _i, _vp, _vp, _vp, _vp],
    "dressi_softras_bwd": [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _f, _vp, _vp, _vp, _vp, _vp, _vp],
    "dressi_softras_noalloc": [_vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _f, _f, _i, _vp, _vp, _vp, _vp],
    "dressi_transform": [_vp, _vp, _vp, _i, _i, _vp, _vp],
    "dressi_transform_bwd": [_vp, _vp, _i, _i, _vp, _vp, _vp],
    "dressi_vertex_attrs": [_vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp],
    "dressi_vertex_attrs_bwd": [_vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp],
    "dressi_vertex_stage": [_vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _i, _vp, _vp, _vp],
    "dressi_adjacency": [_vp, _vp, _i, _i, _vp, _vp],
    "dressi_fragment_index": [_vp, _vp, _i, _i, _i, _i, _i, _vp, _vp],
    "dressi_rasterize_indexed": [_vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp],
    "dressi_packed_step": [_vp, _vp, _vp, _vp],
    "dressi_geometry_fwd": [_vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _i, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp],
    "dressi_shade": [_vp, _i, _vp, _vp, _vp, _i, _i64, _vp, _vp, _vp],
    "dressi_shade_bwd": [_vp, _i, _vp, _vp, _vp, _i, _i64, _vp, _vp, _vp, _vp],
    "dressi_loss_l2": [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp],
    "dressi_geometry_bwd": [_vp, _vp, _vp, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _vp, _vp,
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "dressi_packed_forward": [_vp, _vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "dressi_packed_backward": [_vp, _vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "dressi_texture_grad_invrec": [_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp],
    "dressi_transform_batched": [_vp, _vp, _vp, _vp, _i, _vp, _vp],
    "dressi_tune": [_vp, _i, _i64],
    "dressi_transform_batched_bwd": [_vp, _vp, _vp, _i, _vp, _vp, _vp],
    "dressi_rasterize_batched": [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp],
    "dressi_rasterize_batched_bwd": [_vp, _vp, _vp, _vp, _vp, _i, _i, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp,
                                     _vp, _vp],
}
for _name, _args in _SIG.items():
    fn = getattr(_lib, _name)
    fn.argtypes = _args
    fn.restype = C.c_int
_lib.dressi_last_error.argtypes = [_vp]
_lib.dressi_last_error.restype = C.c_char_p
_lib.dressi_scratch_bytes.argtypes = [_i, _i, _i, _i, _i, _i, _f, _i, _i, _i64, _i]
_lib.dressi_scratch_bytes.restype = C.c_size_t
_lib.dressi_ibl_norm_bytes.argtypes = [C.POINTER(IblDesc)]
_lib.dressi_ibl_norm_bytes.restype = C.c_size_t
_lib.dressi_invuv_bytes.argtypes = [C.POINTER(TexDesc), _i]
_lib.dressi_invuv_bytes.restype = C.c_size_t
_lib.dressi_fragment_index_bytes.argtypes = [_i, _i, _i, _i, _i]
_lib.dressi_fragment_index_bytes.restype = C.c_size_t
_lib.dressi_profile_start.argtypes = [_i]
_lib.dressi_profile_start.restype = C.c_int
_lib.dressi_profile_read.argtypes = [C.POINTER(C.c_char_p), C.POINTER(C.c_float), _i]
_lib.dressi_profile_read.restype = C.c_int

EXPORTED = sorted(list(_SIG) + ["dressi_last_error", "dressi_scratch_bytes", "dressi_fragment_index_bytes",
                                "dressi_invuv_bytes", "dressi_ibl_norm_bytes", "dressi_profile_start",
                                "dressi_profile_read"])


class Limits(C.Structure):
    """dressi_limits: the largest shapes a context will be called with."""
    _fields_ = [("B", _i), ("V", _i), ("T", _i), ("H", _i), ("W", _i), ("K", _i), ("r", _f), ("Va", _i),
                ("C", _i), ("tex_cells", _i64), ("tex_channels", _i), ("tex_slices", _i), ("jitter", _i),
                ("ibl_S", _i), ("ibl_Si", _i), ("ibl_Sp", _i), ("ibl_L", _i), ("pbs_fragments", _i64),
                ("bin_entries", _i64)]


_lib.dressi_limits_scratch_bytes.argtypes = [C.POINTER(Limits)]
_lib.dressi_limits_scratch_bytes.restype = C.c_size_t
_lib.dressi_reserve_limits.argtypes = [_vp, C.POINTER(Limits)]
_lib.dressi_reserve_limits.restype = C.c_int
EXPORTED = sorted(EXPORTED + ["dressi_limits_scratch_bytes", "dressi_reserve_limits"])


class DressiError(RuntimeError):
    pass


class Context:
    """One libdressi context (scratch arena) per device."""

    def __init__(self, device: int):
        self.device = device
        h = C.c_void_p()
        rc = _lib.dressi_create(C.byref(h), device)
        if rc != 0:
            raise DressiError(f"dressi_create failed ({STATUS.get(rc, rc)})")
        self.handle = h

    def check(self, rc, what):
        if rc != 0:
            msg = _lib.dressi_last_error(self.handle).decode()
            raise DressiError(f"{what}: {STATUS.get(rc, rc)}: {msg}")

    def reserve(self, nbytes: int = 0, bin_entries: int = 0):
        self.check(_lib.dressi_reserve(self.handle, nbytes, bin_entries), "dressi_reserve")

    def reserve_limits(self, limits: "Limits"):
        self.check(_lib.dressi_reserve_limits(self.handle, C.byref(limits)), "dressi_reserve_limits")

    def tune(self, key: int, value: int):
        self.check(_lib.dressi_tune(self.handle, key, value), "dressi_tune")

    def check_status(self, stream=None):
        needed = C.c_int64(0)
        s = _stream(stream)
        rc = _lib.dressi_check_status(self.handle, C.byref(needed), s)
        if rc == -4:
            return int(needed.value)
        self.check(rc, "dressi_check_status")
        return 0


_ctx_lock = threading.Lock()
_ctxs: dict[int, Context] = {}


def context(device=None) -> Context:
    d = torch.cuda.current_device() if device is None else int(device)
    with _ctx_lock:
        if d not in _ctxs:
            _ctxs[d] = Context(d)
        return _ctxs[d]


_aux_ctxs: dict[int, Context] = {}


def context_aux(device=None) -> Context:
    """A second context per device (its own scratch arena) for work issued on
    a second stream while the first context's calls run on the main stream."""
    d = torch.cuda.current_device() if device is None else int(device)
    with _ctx_lock:
        if d not in _aux_ctxs:
            _aux_ctxs[d] = Context(d)
        return _aux_ctxs[d]


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _need(t, dtype, name):
    if not t.is_cuda:
        raise DressiError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise DressiError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise DressiError(f"{name} must be contiguous")
    return t


def _checked_raster(ctx, call, what):
    """Runs a rasterization, then reads the device's bin-overflow status (a
    host synchronisation; skipped while the stream is being captured).  On
    overflow the bins grow to the reported need and the call runs once more;
    a second overflow raises.  Outputs are never returned from an overflowed
    call."""
    ctx.check(call(), what)
    if torch.cuda.is_current_stream_capturing():
        return
    need = ctx.check_status()
    if need > 0:
        cap = 1
        while cap < need + need // 4:
            cap <<= 1
        ctx.reserve(0, cap)
        ctx.check(call(), what)
        need = ctx.check_status()
        if need > 0:
            raise DressiError(f"{what}: tile bins still overflow ({need} triangles per tile needed)")


def scratch_bytes(B, V, T, H, W, K, r, Va=0, C_=0, tex_cells=0, tex_slices=0):
    return int(_lib.dressi_scratch_bytes(B, V, T, H, W, K, float(r), Va, C_, tex_cells, tex_slices))


# ---------------------------------------------------------------------------
def dressi_rasterize(pos_clip, tris, H, W, K=1, r=0.0, cull=0):
    _need(pos_clip, torch.float32, "pos_clip")
    _need(tris, torch.int32, "tris")
    B, V, _ = pos_clip.shape
    T = tris.shape[0]
    dev = pos_clip.device
    tri_id = torch.empty((B, K, H, W), dtype=torch.int32, device=dev)
    bary = torch.empty((B, K, H, W, 2), dtype=torch.float32, device=dev)
    dist = torch.empty((B, K, H, W), dtype=torch.float32, device=dev) if r > 0 else None
    ctx = context(dev.index)
    _checked_raster(ctx, lambda: _lib.dressi_rasterize(ctx.handle, _ptr(pos_clip), _ptr(tris), B, V, T, H, W, K,
                                                       float(r), int(cull), _ptr(tri_id), _ptr(bary),
                                                       _ptr(dist), _stream()), "dressi_rasterize")
    return tri_id, bary, dist


def dressi_rasterize_banded(pos_clip, tris, H, W, K, r, delta, mode=BLEND_HSR, cull=0):
    """Edge-band form of dressi_rasterize for a blend of the given delta and
    mode: the full layers inside the blend's edge mask, the front hard
    fragment alone outside it."""
    _need(pos_clip, torch.float32, "pos_clip")
    _need(tris, torch.int32, "tris")
    B, V, _ = pos_clip.shape
    T = tris.shape[0]
    dev = pos_clip.device
    tri_id = torch.empty((B, K, H, W), dtype=torch.int32, device=dev)
    bary = torch.empty((B, K, H, W, 2), dtype=torch.float32, device=dev)
    dist = torch.empty((B, K, H, W), dtype=torch.float32, device=dev)
    ctx = context(dev.index)
    _checked_raster(ctx, lambda: _lib.dressi_rasterize_banded(ctx.handle, _ptr(pos_clip), _ptr(tris), B, V, T, H,
                                                              W, K, float(r), int(cull), float(delta), int(mode),
                                                              _ptr(tri_id), _ptr(bary), _ptr(dist), _stream()),
                    "dressi_rasterize_banded")
    return tri_id, bary, dist


def dressi_rasterize_bwd(pos_clip, tris, tri_id, grad_bary, grad_dist=None, r=0.0, cull=0,
                         frag_index=None, adj=None):
    _need(pos_clip, torch.float32, "pos_clip")
    _need(tris, torch.int32, "tris")
    _need(tri_id, torch.int32, "tri_id")
    _need(grad_bary, torch.float32, "grad_bary")
    if grad_dist is not None:
        _need(grad_dist, torch.float32, "grad_dist")
    B, V, _ = pos_clip.shape
    _, K, H, W = tri_id.shape
    g = torch.empty_like(pos_clip)
    ctx = context(pos_clip.device.index)
    ctx.check(_lib.dressi_rasterize_bwd(ctx.handle, _ptr(pos_clip), _ptr(tris), B, V, tris.shape[0],
                                        H, W, K, float(r), int(cull), _ptr(tri_id), _ptr(grad_bary),
                                        _ptr(grad_dist), _ptr(frag_index), _ptr(adj), _ptr(g), _stream()),
              "dressi_rasterize_bwd")
    return g


def _attr3(attr):
    return attr if attr.dim() == 3 else attr.unsqueeze(0)


def dressi_interpolate(attr, attr_tris, tri_id, bary):
    a = _need(_attr3(attr), torch.float32, "attr")
    _need(attr_tris, torch.int32, "attr_tris")
    _need(tri_id, torch.int32, "tri_id")
    _need(bary, torch.float32, "bary")
    Ba, Va, Cc = a.shape
    B, K, H, W = tri_id.shape
    out = torch.empty((B, K, H, W, Cc), dtype=torch.float32, device=a.device)
    ctx = context(a.device.index)
    ctx.check(_lib.dressi_interpolate(ctx.handle, _ptr(a), Ba, Va, Cc, _ptr(attr_tris),
                                      attr_tris.shape[0], _ptr(tri_id), _ptr(bary), B, K, H, W,
                                      _ptr(out), _stream()), "dressi_interpolate")
    return out


def dressi_interpolate_bwd(attr, attr_tris, tri_id, bary, grad_out, need_attr=True, need_bary=True,
                           grad_bary_in=None, frag_index=None, adj=None):
    a = _need(_attr3(attr), torch.float32, "attr")
    _need(grad_out, torch.float32, "grad_out")
    Ba, Va, Cc = a.shape
    B, K, H, W = tri_id.shape
    ga = torch.empty_like(a) if need_attr else None
    gb = torch.empty_like(bary) if need_bary else None
    ctx = context(a.device.index)
    ctx.check(_lib.dressi_interpolate_bwd(ctx.handle, _ptr(a), Ba, Va, Cc, _ptr(attr_tris),
                                          attr_tris.shape[0], _ptr(tri_id), _ptr(bary), B, K, H, W,
                                          _ptr(grad_out), _ptr(grad_bary_in), _ptr(frag_index), _ptr(adj),
                                          _ptr(ga), _ptr(gb), _stream()), "dressi_interpolate_bwd")
    if ga is not None and attr.dim() == 2:
        ga = ga[0]
    return ga, gb


def _desc(tex, kind, wrap_u, wrap_v, tri_layer=None):
    if kind == TEX_2D_ARRAY:
        L, Ht, Wt, Ct = tex.shape
        _need(tri_layer, torch.int32, "tri_layer")
        return TexDesc(kind, Ht, Wt, Ct, wrap_u, wrap_v, L, tri_layer.data_ptr())
    if kind == TEX_CUBE:
        _, Ht, Wt, Ct = tex.shape
    else:
        Ht, Wt, Ct = tex.shape
    return TexDesc(kind, Ht, Wt, Ct, wrap_u, wrap_v)


def dressi_texture(tex, coord, tri_id, kind=TEX_2D, wrap_u=WRAP_REPEAT, wrap_v=WRAP_CLAMP, tri_layer=None):
    """coord [S,H,W,2|3], tri_id [S,H,W] (or [B,K,H,W] flattened to S=B*K)."""
    _need(tex, torch.float32, "tex")
    _need(coord, torch.float32, "coord")
    d = _desc(tex, kind, wrap_u, wrap_v, tri_layer)
    lead = coord.shape[:-1]
    H, W = lead[-2], lead[-1]
    S = coord.numel() // (coord.shape[-1] * H * W)
    out = torch.empty(lead + (d.Ct,), dtype=torch.float32, device=coord.device)
    ctx = context(coord.device.index)
    ctx.check(_lib.dressi_texture(ctx.handle, _ptr(tex), C.byref(d), _ptr(coord),
                                  _ptr(tri_id) if tri_id is not None else None, S, H, W, _ptr(out),
                                  _stream()), "dressi_texture")
    return out


def dressi_texture_bwd(tex, coord, tri_id, grad_out, kind=TEX_2D, wrap_u=WRAP_REPEAT,
                       wrap_v=WRAP_CLAMP, need_tex=True, need_coord=True, tri_layer=None, frame=0):
    _need(grad_out, torch.float32, "grad_out")
    d = _desc(tex, kind, wrap_u, wrap_v, tri_layer)
    lead = coord.shape[:-1]
    H, W = lead[-2], lead[-1]
    S = coord.numel() // (coord.shape[-1] * H * W)
    gt = torch.empty_like(tex) if need_tex else None
    gc = torch.empty_like(coord) if need_coord else None
    ctx = context(coord.device.index)
    ctx.check(_lib.dressi_texture_bwd(ctx.handle, _ptr(tex), C.byref(d), _ptr(coord), _ptr(tri_id),
                                      S, H, W, _ptr(grad_out), int(frame), _ptr(gt), _ptr(gc), _stream()),
              "dressi_texture_bwd")
    return gt, gc


def dressi_invuv_build(tex, coord, tri_id, kind=TEX_2D, wrap_u=WRAP_REPEAT, wrap_v=WRAP_CLAMP, tri_layer=None):
    """The inverse-UV map [S,F,Ht,Wt] int32 of coord/tri_id for a texture shaped like `tex`."""
    _need(coord, torch.float32, "coord")
    if tri_id is not None:
        _need(tri_id, torch.int32, "tri_id")
    d = _desc(tex, kind, wrap_u, wrap_v, tri_layer)
    lead = coord.shape[:-1]
    H, W = lead[-2], lead[-1]
    S = coord.numel() // (coord.shape[-1] * H * W)
    n = int(_lib.dressi_invuv_bytes(C.byref(d), S)) // 4
    inv = torch.empty(n, dtype=torch.int32, device=coord.device)
    ctx = context(coord.device.index)
    ctx.check(_lib.dressi_invuv_build(ctx.handle, C.byref(d), _ptr(coord), _ptr(tri_id), S, H, W, _ptr(inv),
                                      _stream()), "dressi_invuv_build")
    return inv


def dressi_texture_grad_invuv(tex, coord, tri_id, inv, grad_out, kind=TEX_2D, wrap_u=WRAP_REPEAT,
                              wrap_v=WRAP_CLAMP, tri_layer=None):
    """Texture gradient gathered through a map from dressi_invuv_build."""
    _need(grad_out, torch.float32, "grad_out")
    _need(inv, torch.int32, "inv")
    d = _desc(tex, kind, wrap_u, wrap_v, tri_layer)
    lead = coord.shape[:-1]
    H, W = lead[-2], lead[-1]
    S = coord.numel() // (coord.shape[-1] * H * W)
    if inv.numel() * 4 != int(_lib.dressi_invuv_bytes(C.byref(d), S)):
        raise ValueError("inverse-UV map of the wrong size for this texture and coordinate set")
    gt = torch.empty_like(tex)
    ctx = context(coord.device.index)
    ctx.check(_lib.dressi_texture_grad_invuv(ctx.handle, C.byref(d), _ptr(coord), _ptr(tri_id), S, H, W,
                                             _ptr(inv), _ptr(grad_out), _ptr(gt), _stream()),
              "dressi_texture_grad_invuv")
    return gt


def dressi_ibl_filter(env, Si, Sp, L):
    """env [6,S,S,3] -> (irr [6,Si,Si,3], pref [L,6,Sp,Sp,3], norm float64)."""
    _need(env, torch.float32, "env")
    S = env.shape[1]
    d = IblDesc(S, Si, Sp, L)
    dev = env.device
    irr = torch.empty((6, Si, Si, 3), dtype=torch.float32, device=dev)
    pref = torch.empty((L, 6, Sp, Sp, 3), dtype=torch.float32, device=dev)
    norm = torch.empty(int(_lib.dressi_ibl_norm_bytes(C.byref(d))) // 8, dtype=torch.float64, device=dev)
    ctx = context(dev.index)
    ctx.check(_lib.dressi_ibl_filter(ctx.handle, _ptr(env), C.byref(d), _ptr(irr), _ptr(pref), _ptr(norm),
                                     _stream()), "dressi_ibl_filter")
    return irr, pref, norm


def dressi_ibl_filter_bwd(S, norm, grad_irr, grad_pref):
    Si, L, Sp = grad_irr.shape[1], grad_pref.shape[0], grad_pref.shape[2]
    d = IblDesc(S, Si, Sp, L)
    g = torch.empty((6, S, S, 3), dtype=torch.float32, device=grad_irr.device)
    ctx = context(grad_irr.device.index)
    ctx.check(_lib.dressi_ibl_filter_bwd(ctx.handle, C.byref(d), _ptr(norm), _ptr(grad_irr), _ptr(grad_pref),
                                         _ptr(g), _stream()), "dressi_ibl_filter_bwd")
    return g


def dressi_brdf_lut(N, M, device=None):
    lut = torch.empty((N, N, 2), dtype=torch.float32, device=device or "cuda")
    ctx = context(lut.device.index)
    ctx.check(_lib.dressi_brdf_lut(ctx.handle, N, M, _ptr(lut), _stream()), "dressi_brdf_lut")
    return lut


def pbs_in(normal, pos, material, lut, albedo=None, irr=None, pref=None, levels=None):
    """A dressi_pbs_in over [N,3] rows (pref [L,N,3]); keeps no references."""
    pin = PbsIn()
    pin.normal, pin.normal_stride = _ptr(normal), normal.shape[-1]
    pin.pos, pin.pos_stride = _ptr(pos), pos.shape[-1]
    if albedo is not None:
        pin.albedo, pin.albedo_stride = _ptr(albedo), albedo.shape[-1]
    if irr is not None:
        pin.irr, pin.irr_stride = _ptr(irr), 3
    if pref is not None:
        pin.pref, pin.pref_stride = _ptr(pref), 3
        pin.pref_level_stride = pref[0].numel()
    pin.material = _ptr(material)
    pin.lut, pin.lut_n = _ptr(lut), lut.shape[0]
    pin.levels = levels if levels is not None else (pref.shape[0] if pref is not None else 2)
    return pin


ADAM_STATE_BYTES = 16


def adam_state(device=None):
    """A zeroed Adam step state (DRESSI_ADAM_STATE_BYTES on the device)."""
    return torch.zeros(ADAM_STATE_BYTES // 4, dtype=torch.int32, device=device or "cuda")


def dressi_adam(param, grad, m, v, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One in-place Adam step on param, m, v (all float32, same size)."""
    for t, nm in ((param, "param"), (grad, "grad"), (m, "m"), (v, "v")):
        _need(t, torch.float32, nm)
    _need(state, torch.int32, "state")
    n = param.numel()
    if grad.numel() != n or m.numel() != n or v.numel() != n or state.numel() * 4 != ADAM_STATE_BYTES:
        raise DressiError("dressi_adam: size mismatch")
    ctx = context(param.device.index)
    ctx.check(_lib.dressi_adam(ctx.handle, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), n, lr, beta1, beta2, eps,
                               _ptr(state), _stream()), "dressi_adam")


def dressi_laplacian_reg(pos, tris, lam0, gamma=1.0, state=None, grad_in=None, adj=None, need_grad=True):
    """(grad_out [V,3] or None, value [1]) of the Laplacian regulariser."""
    _need(pos, torch.float32, "pos")
    _need(tris, torch.int32, "tris")
    V, T = pos.shape[0], tris.shape[0]
    g = torch.empty_like(pos) if need_grad else None
    val = torch.empty(1, dtype=torch.float32, device=pos.device)
    ctx = context(pos.device.index)
    ctx.check(_lib.dressi_laplacian_reg(ctx.handle, _ptr(pos), _ptr(tris), V, T, _ptr(adj), lam0, gamma,
                                        _ptr(state), _ptr(grad_in), _ptr(g), _ptr(val), _stream()),
              "dressi_laplacian_reg")
    return g, val


def dressi_softras(color, dist, tri_id, sigma, delta, mode=BLEND_HSR):
    _need(color, torch.float32, "color")
    _need(tri_id, torch.int32, "tri_id")
    if dist is not None:
        _need(dist, torch.float32, "dist")
    B, K, H, W = tri_id.shape
    Cc = color.shape[-1]
    dev = color.device
    oc = torch.empty((B, H, W, Cc), dtype=torch.float32, device=dev)
    os_ = torch.empty((B, H, W), dtype=torch.float32, device=dev)
    E = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
    ctx = context(dev.index)
    ctx.check(_lib.dressi_softras(ctx.handle, _ptr(color), _ptr(dist), _ptr(tri_id), B, K, H, W, Cc,
                                  float(sigma), float(delta), int(mode), _ptr(oc), _ptr(os_), _ptr(E),
                                  _stream()), "dressi_softras")
    return oc, os_, E


SOFTRAS_NOALLOC_MAX_PIXELS = 16 * 1024 * 1024


def dressi_softras_noalloc(color, dist, tri_id, sigma, delta, mode=BLEND_HSR, out=None):
    """dressi_softras through its allocation-free entry point.  `out` =
    (out_color [B,H,W,Cc], out_sil [B,H,W], edge_mask [B,H,W] uint8) given by
    the caller, or None to allocate them here (the library call allocates
    nothing either way)."""
    _need(color, torch.float32, "color")
    _need(tri_id, torch.int32, "tri_id")
    if dist is not None:
        _need(dist, torch.float32, "dist")
    B, K, H, W = tri_id.shape
    Cc = color.shape[-1]
    dev = color.device
    if out is None:
        out = (torch.empty((B, H, W, Cc), dtype=torch.float32, device=dev),
               torch.empty((B, H, W), dtype=torch.float32, device=dev),
               torch.empty((B, H, W), dtype=torch.uint8, device=dev))
    oc, os_, E = out
    _need(oc, torch.float32, "out_color")
    _need(os_, torch.float32, "out_sil")
    _need(E, torch.uint8, "edge_mask")
    ctx = context(dev.index)
    ctx.check(_lib.dressi_softras_noalloc(ctx.handle, _ptr(color), _ptr(dist), _ptr(tri_id), B, K, H, W, Cc,
                                          float(sigma), float(delta), int(mode), _ptr(oc), _ptr(os_),
                                          _ptr(E), _stream()), "dressi_softras_noalloc")
    return oc, os_, E


def dressi_softras_bwd(color, dist, tri_id, sigma, edge_mask, grad_color, grad_sil, need_dist=True):
    _need(grad_color, torch.float32, "grad_color")
    if grad_sil is not None:
        _need(grad_sil, torch.float32, "grad_sil")
    B, K, H, W = tri_id.shape
    Cc = color.shape[-1]
    gl = torch.empty_like(color)
    gd = torch.empty_like(dist) if (dist is not None and need_dist) else None
    ctx = context(color.device.index)
    ctx.check(_lib.dressi_softras_bwd(ctx.handle, _ptr(color), _ptr(dist), _ptr(tri_id), B, K, H, W,
                                      Cc, float(sigma), _ptr(edge_mask), _ptr(grad_color),
                                      _ptr(grad_sil), _ptr(gl), _ptr(gd), _stream()),
              "dressi_softras_bwd")
    return gl, gd


def dressi_transform(pos, mvp):
    _need(pos, torch.float32, "pos")
    _need(mvp, torch.float32, "mvp")
    B, V = mvp.shape[0], pos.shape[0]
    out = torch.empty((B, V, 4), dtype=torch.float32, device=pos.device)
    ctx = context(pos.device.index)
    ctx.check(_lib.dressi_transform(ctx.handle, _ptr(pos), _ptr(mvp), B, V, _ptr(out), _stream()),
              "dressi_transform")
    return out


def dressi_transform_batched(pos, vert_view, mvp):
    """pos [V,3], vert_view [V] int32, mvp [n,4,4] -> pos_clip [V,4]."""
    _need(pos, torch.float32, "pos")
    _need(vert_view, torch.int32, "vert_view")
    V = pos.shape[0]
    out = torch.empty((V, 4), dtype=torch.float32, device=pos.device)
    ctx = context(pos.device.index)
    ctx.check(_lib.dressi_transform_batched(ctx.handle, _ptr(pos), _ptr(vert_view), _ptr(mvp), V, _ptr(out),
                                            _stream()), "dressi_transform_batched")
    return out


def dressi_transform_batched_bwd(mvp, vert_view, grad_clip):
    V = grad_clip.shape[0]
    out = torch.empty((V, 3), dtype=torch.float32, device=grad_clip.device)
    ctx = context(grad_clip.device.index)
    ctx.check(_lib.dressi_transform_batched_bwd(ctx.handle, _ptr(mvp), _ptr(vert_view), V, _ptr(grad_clip),
                                                _ptr(out), _stream()), "dressi_transform_batched_bwd")
    return out


def dressi_rasterize_batched(pos_clip, tris, tri_view, views, H, W, K=1, cull=0):
    """pos_clip [V,4], tris [T,3], tri_view [T] int32, views [n,4] int32 (x0, y0, W, H)
    -> tri_id [1,K,H,W], bary [1,K,H,W,2]."""
    _need(pos_clip, torch.float32, "pos_clip")
    _need(views, torch.int32, "views")
    V, T, n = pos_clip.shape[0], tris.shape[0], views.shape[0]
    dev = pos_clip.device
    tid = torch.empty((1, K, H, W), dtype=torch.int32, device=dev)
    bary = torch.empty((1, K, H, W, 2), dtype=torch.float32, device=dev)
    ctx = context(dev.index)
    _checked_raster(ctx, lambda: _lib.dressi_rasterize_batched(ctx.handle, _ptr(pos_clip), _ptr(tris),
                                                               _ptr(tri_view), _ptr(views), n, V, T, H, W, K,
                                                               cull, _ptr(tid), _ptr(bary), _stream()),
                    "dressi_rasterize_batched")
    return tid, bary


def dressi_rasterize_batched_bwd(pos_clip, tris, tri_view, views, tri_id, grad_bary, cull=0, frag_index=None,
                                 adj=None):
    V, T, n = pos_clip.shape[0], tris.shape[0], views.shape[0]
    _, K, H, W = tri_id.shape
    out = torch.empty((V, 4), dtype=torch.float32, device=pos_clip.device)
    ctx = context(pos_clip.device.index)
    ctx.check(_lib.dressi_rasterize_batched_bwd(ctx.handle, _ptr(pos_clip), _ptr(tris), _ptr(tri_view),
                                                _ptr(views), n, V, T, H, W, K, cull, _ptr(tri_id), _ptr(grad_bary),
                                                _ptr(frag_index), _ptr(adj), _ptr(out), _stream()),
              "dressi_rasterize_batched_bwd")
    return out


def dressi_transform_bwd(mvp, grad_clip):
    _need(grad_clip, torch.float32, "grad_clip")
    B, V, _ = grad_clip.shape
    out = torch.empty((V, 3), dtype=torch.float32, device=grad_clip.device)
    ctx = context(grad_clip.device.index)
    ctx.check(_lib.dressi_transform_bwd(ctx.handle, _ptr(mvp), B, V, _ptr(grad_clip), _ptr(out),
                                        _stream()), "dressi_transform_bwd")
    return out


def dressi_vertex_attrs(pos, tris, extra=None, adj=None):
    _need(pos, torch.float32, "pos")
    _need(tris, torch.int32, "tris")
    V, T = pos.shape[0], tris.shape[0]
    C_ = 9 if extra is not None else 6
    out = torch.empty((V, C_), dtype=torch.float32, device=pos.device)
    ctx = context(pos.device.index)
    ctx.check(_lib.dressi_vertex_attrs(ctx.handle, _ptr(pos), _ptr(tris), V, T, _ptr(extra), _ptr(adj),
                                       _ptr(out), _stream()), "dressi_vertex_attrs")
    return out


def dressi_vertex_attrs_bwd(pos, tris, grad_out, grad_pos_in=None, adj=None):
    _need(grad_out, torch.float32, "grad_out")
    V, T = pos.shape[0], tris.shape[0]
    out = torch.empty((V, 3), dtype=torch.float32, device=pos.device)
    ctx = context(pos.device.index)
    ctx.check(_lib.dressi_vertex_attrs_bwd(ctx.handle, _ptr(pos), _ptr(tris), V, T, grad_out.shape[1],
                                           _ptr(adj), _ptr(grad_out), _ptr(grad_pos_in), _ptr(out),
                                           _stream()),
              "dressi_vertex_attrs_bwd")
    return out


def _col(t, off=0):
    """(pointer to column `off` of a row-major tensor, row stride in floats)."""
    if t is None:
        return None, 0
    return C.c_void_p(t.data_ptr() + 4 * off), int(t.shape[-1])


def frag_in(normal, pos=None, tangent=None, nmap=None, albedo=None, env=None):
    """Each argument is (tensor, column offset) or None."""
    f = FragIn()
    for name, v in (("normal", normal), ("pos", pos), ("tangent", tangent), ("nmap", nmap),
                    ("albedo", albedo), ("env", env)):
        if v is None:
            continue
        t, off = v
        p, st = _col(t, off)
        setattr(f, name, p)
        setattr(f, name + "_stride", st)
    if albedo is not None:
        t, off = albedo
        f.albedo_channels = min(4, t.shape[-1] - off)
    return f


def frag_grad(**kw):
    g = FragGrad()
    for name, v in kw.items():
        if v is None:
            continue
        t, off = v
        p, st = _col(t, off)
        setattr(g, name, p)
        setattr(g, name + "_stride", st)
    return g


def dressi_shade(mode, fin, eye, tri_id, color=None, dir=None):
    B = tri_id.shape[0]
    Npv = tri_id.numel() // B
    ctx = context(tri_id.device.index)
    ctx.check(_lib.dressi_shade(ctx.handle, mode, C.byref(fin), _ptr(eye), _ptr(tri_id), B, Npv,
                                _ptr(color), _ptr(dir), _stream()), "dressi_shade")


def dressi_shade_bwd(mode, fin, eye, tri_id, grad_color, grad_dir, fgrad):
    B = tri_id.shape[0]
    Npv = tri_id.numel() // B
    ctx = context(tri_id.device.index)
    ctx.check(_lib.dressi_shade_bwd(ctx.handle, mode, C.byref(fin), _ptr(eye), _ptr(tri_id), B, Npv,
                                    _ptr(grad_color), _ptr(grad_dir), C.byref(fgrad), _stream()),
              "dressi_shade_bwd")


def dressi_loss_l2(color, sil, target, loss=None, grad_color=None, grad_sil=None, weight=None):
    B, H, W = sil.shape
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=sil.device)
    ctx = context(sil.device.index)
    ctx.check(_lib.dressi_loss_l2(ctx.handle, _ptr(color), _ptr(sil), _ptr(target), _ptr(weight), B, H, W,
                                  _ptr(loss), _ptr(grad_color), _ptr(grad_sil), _stream()),
              "dressi_loss_l2")
    return loss


def dressi_adjacency(tris, V):
    """Vertex -> corner adjacency of a mesh (int32 [V + 1 + 3T]); build once per mesh."""
    _need(tris, torch.int32, "tris")
    T = tris.shape[0]
    adj = torch.empty(V + 1 + 3 * T, dtype=torch.int32, device=tris.device)
    ctx = context(tris.device.index)
    ctx.check(_lib.dressi_adjacency(ctx.handle, _ptr(tris), T, V, _ptr(adj), _stream()), "dressi_adjacency")
    return adj


def dressi_fragment_index(tri_id, T, out=None):
    """Per-tile triangle-sorted fragment index of tri_id (opaque uint8 buffer)."""
    _need(tri_id, torch.int32, "tri_id")
    B, K, H, W = tri_id.shape
    nbytes = int(_lib.dressi_fragment_index_bytes(B, K, H, W, T))
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device=tri_id.device)
    ctx = context(tri_id.device.index)
    ctx.check(_lib.dressi_fragment_index(ctx.handle, _ptr(tri_id), B, K, H, W, T, _ptr(out), _stream()),
              "dressi_fragment_index")
    return out
