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
