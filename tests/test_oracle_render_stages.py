"""Pins for the oracle's vertex transform, vertex normals, normal mapping,
reflection, shading and loss: closed forms and central finite differences."""
import numpy as np
import pytest

import oracle
from helpers import rel_err, to_clip
from paper_2204_01386_amd import scenes


def fd_check(fwd, x, g, h=1e-6, tol=1e-6, mask=None):
    """Directional central difference of <fwd(x), g> along random directions."""
    rng = np.random.default_rng(0)
    out = []
    for _ in range(3):
        d = rng.standard_normal(x.shape)
        if mask is not None:
            d = d * mask
        fp = (fwd(x + h * d) * g).sum()
        fm = (fwd(x - h * d) * g).sum()
        out.append(((fp - fm) / (2 * h), d))
    return out


# ---------------------------------------------------------------------------
def test_transform_closed_forms():
    p = np.random.default_rng(1).standard_normal((10, 3))
    out = oracle.transform(p, np.eye(4))
    assert np.array_equal(out[0, :, :3], p) and (out[0, :, 3] == 1).all()
    # origin seen from (0,0,3): centre of the image, w = 3, z/w inside (0,1)
    mvp = scenes.view_proj(np.array([[0.0, 0.0, 3.0]]))
    c = oracle.transform(np.zeros((1, 3)), mvp)[0, 0]
    assert abs(c[0]) < 1e-6 and abs(c[1]) < 1e-6 and abs(c[3] - 3.0) < 1e-6
    zn = c[2] / c[3]
    assert abs(zn - 10.0 * (3.0 - 0.1) / (3.0 * (10.0 - 0.1))) < 1e-6
    # a unit sphere at distance 3 (fov 60) covers a disc of NDC radius tan(asin(1/3))/tan(30deg)
    pos, tris = scenes.icosphere(5)
    H = W = 256
    tid, _, _, _ = oracle.rasterize(oracle.transform(pos, mvp).astype(np.float32), tris, H, W)
    R = np.tan(np.arcsin(1 / 3)) / np.tan(np.radians(30)) * W / 2
    area = (tid[0, 0] >= 0).sum()
    assert abs(R - 156.8 * 256 / 512) < 0.1
    assert abs(area - np.pi * R * R) / (np.pi * R * R) < 0.01


def test_transform_adjoint():
    rng = np.random.default_rng(2)
    p = rng.standard_normal((7, 3))
    m = rng.standard_normal((3, 4, 4))
    g = rng.standard_normal((3, 7, 4))
    y = oracle.transform(p, m)
    gp = oracle.transform_bwd(m, g)
    d = rng.standard_normal(p.shape)
    assert abs(((oracle.transform(p + d, m) - y) * g).sum() - (gp * d).sum()) < 1e-10


def test_vertex_normals_closed_forms():
    pos, tris = scenes.icosphere(2)
    n = oracle.vertex_normals(pos, tris)
    # the 12 base vertices are symmetric: the area-weighted normal is radial
    assert np.abs(n[:12] - pos[:12]).max() < 1e-12
    # every normal of a sphere mesh is close to radial
    assert np.abs(n - pos).max() < 0.03
    # a planar fan has the plane normal everywhere
    fan = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [-1, 0.5, 0]], np.float64)
    ft = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 4]], np.int32)
    assert np.allclose(oracle.vertex_normals(fan, ft), [0, 0, 1], atol=1e-15)


def test_vertex_normals_bwd_fd():
    pos, tris = scenes.noisy_sphere(1, 3)
    pos = pos.astype(np.float64)
    g = np.random.default_rng(3).standard_normal(pos.shape)
    ana = oracle.vertex_normals_bwd(pos, tris, g)
    for fd, d in fd_check(lambda x: oracle.vertex_normals(x, tris), pos, g):
        assert abs(fd - (ana * d).sum()) < 1e-6 * max(1, abs(fd))


def _frag_vectors(rng, N, unit=False):
    v = rng.standard_normal((N, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True) if unit else v


def test_normal_map_closed_forms_and_fd():
    rng = np.random.default_rng(4)
    N = 50
    n = _frag_vectors(rng, N)
    t = _frag_vectors(rng, N)
    tid = np.zeros(N, np.int32)
    nh = n / np.linalg.norm(n, axis=1, keepdims=True)
    up = np.tile([0.0, 0.0, 1.0], (N, 1))
    assert np.abs(oracle.normal_map(n, t, up, tid) - nh).max() < 1e-14
    tt = t - (t * nh).sum(1, keepdims=True) * nh
    tt /= np.linalg.norm(tt, axis=1, keepdims=True)
    ex = np.tile([1.0, 0.0, 0.0], (N, 1))
    assert np.abs(oracle.normal_map(n, t, ex, tid) - tt).max() < 1e-14
    ey = np.tile([0.0, 1.0, 0.0], (N, 1))
    assert np.abs(oracle.normal_map(n, t, ey, tid) - np.cross(nh, tt)).max() < 1e-14
    m = _frag_vectors(rng, N) * 0.3 + up
    g = rng.standard_normal((N, 3))
    gn, gt, gm = oracle.normal_map_bwd(n, t, m, tid, g)
    for fd, d in fd_check(lambda x: oracle.normal_map(x, t, m, tid), n, g):
        assert abs(fd - (gn * d).sum()) < 1e-6 * max(1, abs(fd))
    for fd, d in fd_check(lambda x: oracle.normal_map(n, x, m, tid), t, g):
        assert abs(fd - (gt * d).sum()) < 1e-6 * max(1, abs(fd))
    for fd, d in fd_check(lambda x: oracle.normal_map(n, t, x, tid), m, g):
        assert abs(fd - (gm * d).sum()) < 1e-6 * max(1, abs(fd))


def test_reflect_closed_form_and_fd():
    tid = np.zeros((1, 1), np.int32)
    n = np.array([[[0.0, 0.0, 2.0]]])
    pos = np.zeros((1, 1, 3))
    eye = np.array([[1.0, 0.0, 1.0]])
    d = oracle.reflect(n, pos, eye, tid)
    assert np.allclose(d[0, 0], np.array([-1.0, 0.0, 1.0]) / np.sqrt(2), atol=1e-15)
    rng = np.random.default_rng(5)
    B, N = 2, 30
    n = rng.standard_normal((B, N, 3))
    pos = rng.standard_normal((B, N, 3))
    eye = rng.standard_normal((B, 3)) * 4
    tid = np.zeros((B, N), np.int32)
    g = rng.standard_normal((B, N, 3))
    gn, gp = oracle.reflect_bwd(n, pos, eye, tid, g)
    for fd, dd in fd_check(lambda x: oracle.reflect(x, pos, eye, tid), n, g):
        assert abs(fd - (gn * dd).sum()) < 1e-6 * max(1, abs(fd))
    for fd, dd in fd_check(lambda x: oracle.reflect(n, x, eye, tid), pos, g):
        assert abs(fd - (gp * dd).sum()) < 1e-6 * max(1, abs(fd))


L = np.array([1.0, 1.0, 2.0]) / np.sqrt(6.0)


def test_shade_closed_forms():
    tid = np.zeros((1, 3), np.int32)
    a = np.array([[[0.2, 0.4, 0.6], [0.2, 0.4, 0.6], [0.2, 0.4, 0.6]]])
    perp = np.cross(L, [1.0, 0, 0])
    n = np.stack([L * 3.0, perp, -L])[None]
    c = oracle.shade(oracle.SHADE_LAMBERT, n, None, a, None, np.zeros((1, 3)), tid)
    assert np.allclose(c[0, 0], a[0, 0], atol=1e-15)          # n = l: full light
    assert np.allclose(c[0, 1], 0.1 * a[0, 1], atol=1e-15)    # grazing
    assert np.allclose(c[0, 2], 0.1 * a[0, 2], atol=1e-15)    # facing away
    # Phong: the mirror direction of l about n^ seen along it gives the full highlight
    nrm = np.array([0.0, 0.0, 1.0])
    r = 2 * np.dot(nrm, L) * nrm - L
    pos = np.zeros((1, 1, 3))
    eye = (r * 5.0)[None]
    a4 = np.array([[[0.5, 0.25, 0.125, 0.8]]])
    c = oracle.shade(oracle.SHADE_PHONG, nrm[None, None], pos, a4, None, eye, np.zeros((1, 1), np.int32))
    expect = a4[0, 0, :3] * (0.1 + 0.8 * np.dot(nrm, L)) + 0.2 * 0.8
    assert np.allclose(c[0, 0], expect, atol=1e-14)
    env = np.array([[[0.3, 0.6, 0.9]]])
    c2 = oracle.shade(oracle.SHADE_PHONG_ENV, nrm[None, None], pos, a4, env, eye, np.zeros((1, 1), np.int32))
    assert np.allclose(c2[0, 0], expect + 0.5 * 0.8 * env[0, 0], atol=1e-14)
    # empty fragments are black
    c = oracle.shade(oracle.SHADE_LAMBERT, n, None, a, None, np.zeros((1, 3)), -np.ones((1, 3), np.int32))
    assert (c == 0).all()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_shade_bwd_fd(mode):
    rng = np.random.default_rng(6 + mode)
    B, N = 2, 40
    n = rng.standard_normal((B, N, 3))
    pos = rng.standard_normal((B, N, 3)) * 0.5
    Ca = 3 if mode == 0 else 4
    a = rng.random((B, N, Ca))
    env = rng.random((B, N, 3)) if mode == 2 else None
    eye = rng.standard_normal((B, 3)) * 3
    tid = rng.integers(-1, 3, (B, N)).astype(np.int32)
    g = rng.standard_normal((B, N, 3))
    gn, gp, ga, ge = oracle.shade_bwd(mode, n, pos if mode else None, a, env, eye, tid, g)
    f = lambda **kw: oracle.shade(mode, kw.get("n", n), kw.get("p", pos) if mode else None,
                                  kw.get("a", a), kw.get("e", env), eye, tid)
    for fd, d in fd_check(lambda x: f(n=x), n, g, h=1e-7):
        assert abs(fd - (gn * d).sum()) < 1e-5 * max(1, abs(fd))
    for fd, d in fd_check(lambda x: f(a=x), a, g):
        assert abs(fd - (ga * d).sum()) < 1e-6 * max(1, abs(fd))
    if mode:
        for fd, d in fd_check(lambda x: f(p=x), pos, g, h=1e-7):
            assert abs(fd - (gp * d).sum()) < 1e-5 * max(1, abs(fd))
    if mode == 2:
        for fd, d in fd_check(lambda x: f(e=x), env, g):
            assert abs(fd - (ge * d).sum()) < 1e-6 * max(1, abs(fd))


def test_loss_l2():
    rng = np.random.default_rng(7)
    c = rng.random((2, 5, 6, 3))
    s = rng.random((2, 5, 6))
    t = rng.random((2, 5, 6, 4))
    Lv, gc, gs = oracle.loss_l2(c, s, t)
    rgba = np.concatenate([c, s[..., None]], -1)
    assert abs(Lv - ((rgba - t) ** 2).mean()) < 1e-15
    d = rng.standard_normal(c.shape)
    h = 1e-6
    fd = (oracle.loss_l2(c + h * d, s, t)[0] - oracle.loss_l2(c - h * d, s, t)[0]) / (2 * h)
    assert abs(fd - (gc * d).sum()) < 1e-8
