"""torch.autograd.Functions over the libdressi entry points.

Each stage's backward is the hand-written adjoint kernel of the library; the
Functions only save what the backward needs (inputs, tri_id and the edge
mask — never per-pixel fragment lists) and route gradients.
"""
from __future__ import annotations

import torch

from . import binding as B


class Rasterize(torch.autograd.Function):
    """(pos_clip [B,V,4], tris [T,3]) -> tri_id [B,K,H,W], bary [B,K,H,W,2](, dist [B,K,H,W])."""

    @staticmethod
    def forward(ctx, pos_clip, tris, H, W, K, r, cull):
        tri_id, bary, dist = B.dressi_rasterize(pos_clip, tris, H, W, K, r, cull)
        ctx.save_for_backward(pos_clip, tris, tri_id)
        ctx.params = (float(r), int(cull))
        ctx.mark_non_differentiable(tri_id)
        if dist is None:
            return tri_id, bary
        return tri_id, bary, dist

    @staticmethod
    def backward(ctx, *grads):
        pos_clip, tris, tri_id = ctx.saved_tensors
        r, cull = ctx.params
        g_bary = grads[1]
        g_dist = grads[2] if len(grads) > 2 else None
        if g_bary is None:
            g_bary = torch.zeros(tri_id.shape + (2,), dtype=torch.float32, device=tri_id.device)
        gp = B.dressi_rasterize_bwd(pos_clip, tris, tri_id, g_bary.contiguous(),
                                    g_dist.contiguous() if g_dist is not None else None, r, cull)
        return gp, None, None, None, None, None, None


class Interpolate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, attr, attr_tris, tri_id, bary):
        out = B.dressi_interpolate(attr, attr_tris, tri_id, bary)
        ctx.save_for_backward(attr, attr_tris, tri_id, bary)
        return out

    @staticmethod
    def backward(ctx, g):
        attr, attr_tris, tri_id, bary = ctx.saved_tensors
        ga, gb = B.dressi_interpolate_bwd(attr, attr_tris, tri_id, bary, g.contiguous(),
                                          need_attr=ctx.needs_input_grad[0],
                                          need_bary=ctx.needs_input_grad[3])
        return ga, None, None, gb


class Texture(torch.autograd.Function):
    @staticmethod
    def forward(ctx, tex, coord, tri_id, kind, wrap_u, wrap_v):
        out = B.dressi_texture(tex, coord, tri_id, kind, wrap_u, wrap_v)
        ctx.save_for_backward(tex, coord, tri_id)
        ctx.params = (kind, wrap_u, wrap_v)
        return out

    @staticmethod
    def backward(ctx, g):
        tex, coord, tri_id = ctx.saved_tensors
        kind, wu, wv = ctx.params
        gt, gc = B.dressi_texture_bwd(tex, coord, tri_id, g.contiguous(), kind, wu, wv,
                                      need_tex=ctx.needs_input_grad[0],
                                      need_coord=ctx.needs_input_grad[1])
        return gt, gc, None, None, None, None


class SoftRas(torch.autograd.Function):
    @staticmethod
    def forward(ctx, color, dist, tri_id, sigma, delta, mode):
        oc, os_, E = B.dressi_softras(color, dist, tri_id, sigma, delta, mode)
        ctx.save_for_backward(color, dist, tri_id, E)
        ctx.params = (float(sigma),)
        return oc, os_

    @staticmethod
    def backward(ctx, g_color, g_sil):
        color, dist, tri_id, E = ctx.saved_tensors
        (sigma,) = ctx.params
        if g_color is None:
            g_color = torch.zeros(E.shape + (color.shape[-1],), dtype=torch.float32, device=E.device)
        gl, gd = B.dressi_softras_bwd(color, dist, tri_id, sigma, E, g_color.contiguous(),
                                      g_sil.contiguous() if g_sil is not None else None,
                                      need_dist=dist is not None and ctx.needs_input_grad[1])
        return gl, gd, None, None, None, None


def rasterize(pos_clip, tris, H, W, K=1, r=0.0, cull=0):
    out = Rasterize.apply(pos_clip, tris, H, W, K, r, cull)
    if len(out) == 2:
        return out[0], out[1], None
    return out


def interpolate(attr, attr_tris, tri_id, bary):
    return Interpolate.apply(attr, attr_tris, tri_id, bary)


def texture(tex, coord, tri_id, kind=B.TEX_2D, wrap_u=B.WRAP_REPEAT, wrap_v=B.WRAP_CLAMP):
    return Texture.apply(tex, coord, tri_id, kind, wrap_u, wrap_v)


def softras(color, dist, tri_id, sigma, delta, mode=B.BLEND_HSR):
    return SoftRas.apply(color, dist, tri_id, sigma, delta, mode)


# ---------------------------------------------------------------------------
# image-based PBS and the Laplacian regulariser
# ---------------------------------------------------------------------------
class IblFilter(torch.autograd.Function):
    """env [6,S,S,3] -> (irradiance [6,Si,Si,3], prefiltered [L,6,Sp,Sp,3]);
    the backward is the filters' exact adjoint (saved: the denominators)."""

    @staticmethod
    def forward(ctx, env, Si, Sp, L):
        irr, pref, norm = B.dressi_ibl_filter(env.contiguous(), Si, Sp, L)
        ctx.save_for_backward(norm)
        ctx.shape = (env.shape[1], Si, Sp, L)
        return irr, pref

    @staticmethod
    def backward(ctx, g_irr, g_pref):
        (norm,) = ctx.saved_tensors
        S, Si, Sp, L = ctx.shape
        dev = norm.device
        gi = g_irr.contiguous() if g_irr is not None else torch.zeros((6, Si, Si, 3), device=dev)
        gp = g_pref.contiguous() if g_pref is not None else torch.zeros((L, 6, Sp, Sp, 3), device=dev)
        return B.dressi_ibl_filter_bwd(S, norm, gi, gp), None, None, None


class PbsDirs(torch.autograd.Function):
    """(normal [N,3], pos [N,3]) of fragments -> the lookup directions
    dir_n, dir_r [N,3] (differentiable) and the per-level masks level_tri_id
    [L,N] (not), for the material's roughness."""

    @staticmethod
    def forward(ctx, normal, pos, eye, tri_id, material, lut, L, Npv):
        N = normal.shape[0]
        dev = normal.device
        dn = torch.empty((N, 3), device=dev)
        dr = torch.empty((N, 3), device=dev)
        ltid = torch.empty((L, N), dtype=torch.int32, device=dev)
        pin = B.pbs_in(normal, pos, material, lut, levels=L)
        c = B.context(dev.index)
        c.check(B._lib.dressi_shade_pbs(c.handle, B.C.byref(pin), B._ptr(eye), B._ptr(tri_id), N // Npv, Npv, None,
                                        B._ptr(dn), B._ptr(dr), B._ptr(ltid), B._stream()), "shade_pbs dirs")
        ctx.save_for_backward(normal, pos, eye, tri_id, material, lut)
        ctx.L, ctx.Npv = L, Npv
        ctx.mark_non_differentiable(ltid)
        return dn, dr, ltid

    @staticmethod
    def backward(ctx, g_dn, g_dr, _):
        normal, pos, eye, tri_id, material, lut = ctx.saved_tensors
        L, Npv = ctx.L, ctx.Npv
        N = normal.shape[0]
        dev = normal.device
        z3 = torch.zeros((N, 3), device=dev)
        zl = torch.zeros((L, N, 3), device=dev)
        pin = B.pbs_in(normal, pos, material, lut, albedo=z3, irr=z3, pref=zl, levels=L)
        gn, gp = torch.empty((N, 3), device=dev), torch.empty((N, 3), device=dev)
        pg = B.PbsGrad()
        pg.normal, pg.normal_stride, pg.pos, pg.pos_stride = B._ptr(gn), 3, B._ptr(gp), 3
        gdn = (g_dn if g_dn is not None else z3).contiguous()
        gdr = (g_dr if g_dr is not None else z3).contiguous()
        gdr_l = torch.zeros((L, N, 3), device=dev)
        gdr_l[0] = gdr
        c = B.context(dev.index)
        c.check(B._lib.dressi_shade_pbs_bwd(c.handle, B.C.byref(pin), B._ptr(eye), B._ptr(tri_id), N // Npv, Npv,
                                            B._ptr(z3), B._ptr(gdn), B._ptr(gdr_l), B.C.byref(pg), B._stream()),
                "shade_pbs_bwd dirs")
        return gn, gp, None, None, None, None, None, None


class PbsShade(torch.autograd.Function):
    """Split-sum shading of fragments from their samples: (normal, pos,
    albedo [N,3], irr_s [N,3], pref_s [L,N,3], material [2]) -> colour [N,3]."""

    @staticmethod
    def forward(ctx, normal, pos, albedo, irr_s, pref_s, material, eye, tri_id, lut, Npv):
        N = normal.shape[0]
        L = pref_s.shape[0]
        dev = normal.device
        col = torch.empty((N, 3), device=dev)
        ins = [t.contiguous() for t in (normal, pos, albedo, irr_s, pref_s)]
        pin = B.pbs_in(ins[0], ins[1], material, lut, albedo=ins[2], irr=ins[3], pref=ins[4])
        c = B.context(dev.index)
        c.check(B._lib.dressi_shade_pbs(c.handle, B.C.byref(pin), B._ptr(eye), B._ptr(tri_id), N // Npv, Npv,
                                        B._ptr(col), None, None, None, B._stream()), "shade_pbs")
        ctx.save_for_backward(*ins, material, eye, tri_id, lut)
        ctx.Npv = Npv
        return col

    @staticmethod
    def backward(ctx, g):
        normal, pos, albedo, irr_s, pref_s, material, eye, tri_id, lut = ctx.saved_tensors
        N, L, Npv = normal.shape[0], pref_s.shape[0], ctx.Npv
        dev = normal.device
        pin = B.pbs_in(normal, pos, material, lut, albedo=albedo, irr=irr_s, pref=pref_s)
        e3 = lambda: torch.empty((N, 3), device=dev)
        gn, gp, ga, gi = e3(), e3(), e3(), e3()
        gpr = torch.empty((L, N, 3), device=dev)
        gm = torch.empty(2, device=dev)
        pg = B.PbsGrad()
        pg.normal, pg.normal_stride, pg.pos, pg.pos_stride = B._ptr(gn), 3, B._ptr(gp), 3
        pg.albedo, pg.albedo_stride = B._ptr(ga), 3
        pg.irr, pg.pref, pg.material = B._ptr(gi), B._ptr(gpr), B._ptr(gm)
        gc = g.contiguous()
        c = B.context(dev.index)
        c.check(B._lib.dressi_shade_pbs_bwd(c.handle, B.C.byref(pin), B._ptr(eye), B._ptr(tri_id), N // Npv, Npv,
                                            B._ptr(gc), None, None, B.C.byref(pg), B._stream()), "shade_pbs_bwd")
        return gn, gp, ga, gi, gpr, gm, None, None, None, None


class LaplacianReg(torch.autograd.Function):
    """pos [V,3] -> R (a [1] tensor), the Laplacian regulariser with weight lam."""

    @staticmethod
    def forward(ctx, pos, tris, lam):
        g, val = B.dressi_laplacian_reg(pos.contiguous(), tris, float(lam), 1.0)
        ctx.save_for_backward(g)
        return val

    @staticmethod
    def backward(ctx, gR):
        (g,) = ctx.saved_tensors
        return g * gR, None, None


def ibl_filter(env, Si, Sp, L):
    return IblFilter.apply(env, Si, Sp, L)


def pbs_dirs(normal, pos, eye, tri_id, material, lut, L, Npv):
    return PbsDirs.apply(normal, pos, eye, tri_id, material, lut, L, Npv)


def pbs_shade(normal, pos, albedo, irr_s, pref_s, material, eye, tri_id, lut, Npv):
    return PbsShade.apply(normal, pos, albedo, irr_s, pref_s, material, eye, tri_id, lut, Npv)


def laplacian_reg(pos, tris, lam):
    return LaplacianReg.apply(pos, tris, lam)
