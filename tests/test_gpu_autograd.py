"""The core torch.autograd.Functions (ops.rasterize, interpolate, texture,
softras) chained as a renderer chains them, against the oracle's
composition of the same stages in double precision; and central finite
differences of the HIP adjoints through autograd: attributes and
barycentrics of the interpolation, texels and coordinates of the sampler,
layer colours and signed distances of the blend (§3.4.3: every stage has a
hand-written adjoint; the rasterizer's selection has none)."""
import numpy as np
import pytest
import torch

import oracle
from helpers import to_clip
from test_gpu_parity import assert_grad_close, dev, host
from paper_2204_01386_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_01386_amd import ops as O
    return O


def _scene(seed=0, views=2):
    p, tris = scenes.noisy_sphere(3, seed)
    uv, uv_tris = scenes.spherical_uv(p, tris)
    pc = to_clip(p, scenes.view_proj(scenes.camera_ring(views, seed)))
    return pc, tris, uv.astype(np.float32), uv_tris


@pytest.mark.parametrize("K,r", [(1, 0.0), (2, 0.04), (3, 0.06)])
def test_autograd_chain_matches_the_oracle(ops, K, r):
    """pos_clip -> Rasterize -> (Interpolate colour, Interpolate UV ->
    Texture) -> per-layer product -> SoftRas -> weighted sum: every leaf
    gradient (clip positions, vertex colours, per-corner UVs, texels) against
    the oracle's stages composed with the same chain rule."""
    from paper_2204_01386_amd import binding as Bd
    H, W = 72, 80
    pc, tris, uv, uv_tris = _scene(seed=K)
    rng = np.random.default_rng(K)
    V = pc.shape[1]
    col = rng.random((V, 3)).astype(np.float32)
    tex = rng.random((48, 64, 3)).astype(np.float32)
    sigma, delta = (r / 7, r) if r > 0 else (1.0, 0.0)
    mode = Bd.BLEND_HSR if r > 0 else Bd.BLEND_HARD
    w_c = rng.standard_normal((pc.shape[0], H, W, 3))
    w_s = rng.standard_normal((pc.shape[0], H, W))
    # ---- GPU: autograd through the Functions
    P = dev(pc).requires_grad_(True)
    Cv = dev(col).requires_grad_(True)
    U = dev(uv).requires_grad_(True)
    X = dev(tex).requires_grad_(True)
    tid, bary, dist = ops.rasterize(P, dev(tris), H, W, K, r)
    c = ops.interpolate(Cv, dev(tris), tid, bary)
    uvf = ops.interpolate(U, dev(uv_tris), tid, bary)
    smp = ops.texture(X, uvf, tid)
    layer = (c * smp).contiguous()
    oc, osil = ops.softras(layer, dist, tid, sigma, delta, mode)
    loss = (oc * dev(w_c.astype(np.float32))).sum() + (osil * dev(w_s.astype(np.float32))).sum()
    loss.backward()
    # ---- oracle: the same chain in double
    tid_o, hard_o, bary_o, dist_o = oracle.rasterize(pc, tris, H, W, K=K, r=r)
    assert np.array_equal(host(tid), tid_o)
    c_o = oracle.interpolate(col.astype(np.float64), tris, tid_o, bary_o)
    uv_o = oracle.interpolate_f32(uv, uv_tris, tid_o, bary_o.astype(np.float32))   # selects texels
    s_o = oracle.texture(tex, uv_o, tid_o)
    lay_o = c_o * s_o
    d_o = dist_o if r > 0 else None
    oc_o, os_o, E_o = oracle.softras(lay_o, d_o, tid_o, sigma, delta, mode)
    g_lay, g_dist = oracle.softras_bwd(lay_o, d_o, tid_o, sigma, E_o, w_c, w_s)
    g_c, g_s = g_lay * s_o, g_lay * c_o
    g_col, g_b1 = oracle.interpolate_bwd(col.astype(np.float64), tris, tid_o, bary_o, g_c)
    S = pc.shape[0] * K
    rs = lambda a: a.reshape((S,) + a.shape[2:])
    g_uvf = oracle.texture_bwd_coord(tex, uv_o, g_s, tid_o)
    g_tex = oracle.texture_bwd_tex(tex.shape, rs(uv_o), rs(tid_o), rs(g_s))
    g_uv, g_b2 = oracle.interpolate_bwd(uv.astype(np.float64), uv_tris, tid_o, bary_o, g_uvf)
    g_pc = oracle.rasterize_bwd(pc, tris, tid_o, hard_o, g_b1 + g_b2, g_dist if r > 0 else None)
    assert_grad_close(host(Cv.grad), g_col, what="vertex colours")
    assert_grad_close(host(U.grad), g_uv, what="per-corner UVs")
    assert_grad_close(host(X.grad), g_tex, what="texels")
    assert_grad_close(host(P.grad), g_pc, what="clip positions")
    assert np.all(host(P.grad)[..., 2] == 0)


def _fd_check(f, x, eps, tol=1e-3, what="", shape=None):
    """Central difference of the scalar f between x - eps v and x + eps v
    (rounded to float, as the GPU sees them) against the autograd gradient
    times their exact difference, along the gradient's own direction
    v = g / max|g| (optionally reshaped by `shape`, which keeps |v| <= 1):
    every term of the directional derivative is then non-negative, so float
    rounding of the outputs is not magnified by cancellation.  f sums the
    GPU's float outputs in double on the host."""
    x = x.detach().clone().requires_grad_(True)
    y = f(x)
    y.backward()
    g = x.grad.detach()
    v = g / g.abs().max()
    if shape is not None:
        v = shape(v)
    with torch.no_grad():
        xp, xm = x + eps * v, x - eps * v
        step = xp.double() - xm.double()
        ana = float((g.double() * step).sum())
        fd = float(f(xp)) - float(f(xm))
    assert ana > 0, f"{what}: the step should follow the gradient"
    assert abs(fd - ana) <= tol * abs(ana), f"{what}: difference {fd:.9g} vs adjoint {ana:.9g}"


def _weighted(out, w):
    return (out.double() * w).sum()


def test_fd_interpolate_attributes_and_barycentrics(ops):
    pc, tris, uv, uv_tris = _scene(seed=4, views=1)
    from paper_2204_01386_amd import binding as Bd
    tid, bary, _ = Bd.dressi_rasterize(dev(pc), dev(tris), 40, 40, 2, 0.05, 0)
    rng = np.random.default_rng(4)
    attr = dev(rng.standard_normal((pc.shape[1], 5)).astype(np.float32))
    w = torch.from_numpy(rng.standard_normal(tuple(tid.shape) + (5,))).cuda()
    T = dev(tris)
    _fd_check(lambda a: _weighted(ops.interpolate(a, T, tid, bary), w), attr, 0.5,
              what="interpolate / attributes")
    _fd_check(lambda b: _weighted(ops.interpolate(attr, T, tid, b), w), bary, 1e-2,
              what="interpolate / barycentrics")


def test_fd_texture_texels_and_coordinates(ops):
    """Texels: one pixel per texture cell (the image is coarser than the
    texture), so the inverse-UV gradient is the exact adjoint and the
    difference quotient of this linear map is exact.  Coordinates: samples
    kept away from texel centres, where the bilinear weights are smooth."""
    rng = np.random.default_rng(5)
    Ht, Wt = 40, 48
    tex = dev(rng.random((Ht, Wt, 4)).astype(np.float32))
    S, H, W = 2, 12, 15
    cx = rng.permutation(Wt)[:W]
    cy = rng.permutation(Ht)[:H]
    fr = rng.uniform(0.1, 0.4, (S, H, W, 2)) + rng.integers(0, 2, (S, H, W, 2)) * 0.5
    u = (cx[None, None, :] + fr[..., 0]) / Wt
    v = (cy[None, :, None] + fr[..., 1]) / Ht
    uv = dev(np.stack([u, v], -1).astype(np.float32))
    tid = dev(np.zeros((S, H, W), np.int32))
    w = torch.from_numpy(rng.standard_normal((S, H, W, 4))).cuda()
    _fd_check(lambda t: _weighted(ops.texture(t, uv, tid), w), tex, 0.5, what="texture / texels")
    # steps of at most 2e-3 texel: no sample crosses a texel centre
    _fd_check(lambda q: _weighted(ops.texture(tex, q, tid), w), uv, 2e-3 / Wt, what="texture / coordinates")


@pytest.mark.parametrize("mode", [0, 2])
def test_fd_softras_colours_and_distances(ops, mode):
    pc, tris, _, _ = _scene(seed=6, views=2)
    from paper_2204_01386_amd import binding as Bd
    r = 0.06
    sigma = r / 7
    tid, _, dist = Bd.dressi_rasterize(dev(pc), dev(tris), 48, 48, 3, r, 0)
    rng = np.random.default_rng(6)
    col = dev(rng.random(tuple(tid.shape) + (3,)).astype(np.float32))
    wc = torch.from_numpy(rng.standard_normal((2, 48, 48, 3))).cuda()
    ws = torch.from_numpy(rng.standard_normal((2, 48, 48))).cuda()

    def f_col(c):
        oc, os_ = ops.softras(c, dist, tid, sigma, r, mode)
        return _weighted(oc, wc) + _weighted(os_, ws)

    def f_dist(d):
        oc, os_ = ops.softras(col, d, tid, sigma, r, mode)
        return _weighted(oc, wc) + _weighted(os_, ws)

    _fd_check(f_col, col, 1e-2, what="softras / colours")
    # distances: steps of at most 0.01 sigma, only where the sign (the hard
    # flag, which selects the edge mask) cannot flip
    keep = dist.abs() > 0.05 * sigma
    _fd_check(f_dist, dist, 1e-2 * sigma, what="softras / distances", shape=lambda v: v * keep)
