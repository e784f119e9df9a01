"""Pins for the oracle's interpolation, texture sampling, inverse-UV gradient
and HardSoftRas blend against closed forms, adjoint identities, library
routines (scipy morphology) and brute force."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from helpers import rel_err, screen_to_clip, to_clip
from paper_2204_01386_amd import scenes


# ---------------------------------------------------------------------------
# interpolation
# ---------------------------------------------------------------------------
def test_interpolated_position_is_ray_plane_hit():
    """Interpolating view-space positions with perspective-correct barycentrics
    gives the point where the pixel ray meets the quad's plane."""
    H = W = 32
    P = scenes.perspective()
    Vq = np.array([[-1.0, -0.8, -2.5], [1.2, -0.7, -4.0], [1.1, 0.9, -4.2], [-0.9, 1.0, -2.6]])
    # make it planar: project the 4th corner onto the plane of the first three
    n = np.cross(Vq[1] - Vq[0], Vq[2] - Vq[0])
    n /= np.linalg.norm(n)
    Vq[3] -= np.dot(Vq[3] - Vq[0], n) * n
    pc = to_clip(Vq, P[None])
    c = pc[0].astype(np.float64)
    Pv = np.stack([c[:, 0] / P[0, 0], c[:, 1] / P[1, 1], -c[:, 3]], 1)
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    tid, hard, _, _ = oracle.rasterize(pc, tris, H, W)
    bu, _ = oracle.resolve(pc, tris, tid, hard, snap=False)
    out = oracle.interpolate(Pv, tris, tid, bu)
    ys, xs = np.nonzero(tid[0, 0] >= 0)
    assert len(xs) > 100
    for x, y in zip(xs, ys):
        t = tid[0, 0, y, x]
        q = Pv[tris[t]]
        nn = np.cross(q[1] - q[0], q[2] - q[0])
        d = np.array([((x + 0.5) / (W / 2) - 1) / P[0, 0], (1 - (y + 0.5) / (H / 2)) / P[1, 1], -1.0])
        X = d * np.dot(q[0], nn) / np.dot(d, nn)
        assert np.abs(out[0, 0, y, x] - X).max() < 1e-9


def test_flat_fullscreen_quad_reproduces_colour():
    H = W = 24
    xy = np.array([[-0.5, -0.5], [W + 0.5, -0.5], [W + 0.5, H + 0.5], [-0.5, H + 0.5]])
    pc = screen_to_clip(xy, H, W, z=0.5, w=np.array([1.0, 2.0, 1.5, 0.8]))
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    col = np.tile(np.array([[0.2, 0.5, 0.9]]), (4, 1))
    tid, hard, bary, _ = oracle.rasterize(pc, tris, H, W, K=2)
    assert (tid[0, 0] >= 0).all() and (tid[0, 1] < 0).all()
    out = oracle.interpolate(col, tris, tid, bary)
    assert np.abs(out[0, 0] - col[0]).max() < 1e-12


@pytest.mark.parametrize("Ba", [1, 2])
def test_interpolate_adjoint_identity_and_bary_grad(Ba):
    rng = np.random.default_rng(2)
    B, K, H, W, T, Va, Cc = 2, 2, 8, 9, 5, 7, 3
    tid = rng.integers(-1, T, (B, K, H, W)).astype(np.int32)
    bary = rng.uniform(-0.2, 1.0, (B, K, H, W, 2))
    at = rng.integers(0, Va, (T, 3)).astype(np.int32)
    a = rng.standard_normal((Ba, Va, Cc))
    g = rng.standard_normal((B, K, H, W, Cc))
    y = oracle.interpolate(a, at, tid, bary)
    ga, gb = oracle.interpolate_bwd(a, at, tid, bary, g)
    # <interp(a), g> = <a, interp^T(g)>  (linear in a)
    assert abs((y * g).sum() - (a * ga).sum()) < 1e-10
    # linear in bary too: exact directional derivative
    d = rng.standard_normal(bary.shape)
    y2 = oracle.interpolate(a, at, tid, bary + d)
    assert abs(((y2 - y) * g).sum() - (gb * d).sum()) < 1e-10
    assert (y[tid < 0] == 0).all()


# ---------------------------------------------------------------------------
# texture sampling
# ---------------------------------------------------------------------------
def test_texel_centres_constant_and_ramp():
    rng = np.random.default_rng(4)
    Ht, Wt = 8, 16
    tex = rng.random((Ht, Wt, 3))
    ys, xs = np.meshgrid(np.arange(Ht), np.arange(Wt), indexing="ij")
    uv = np.stack([(xs + 0.5) / Wt, (ys + 0.5) / Ht], -1).astype(np.float32)
    out = oracle.texture(tex, uv)
    assert np.abs(out - tex).max() < 1e-15
    const = np.full((Ht, Wt, 2), 0.7)
    q = rng.uniform(-1.5, 2.5, (500, 2)).astype(np.float32)
    assert np.abs(oracle.texture(const, q) - 0.7).max() < 1e-15
    ramp = (0.3 * xs + 1.7 * ys + 0.25)[..., None].astype(np.float64)
    q = np.stack([rng.uniform(1.0 / Wt, 1 - 1.0 / Wt, 300), rng.uniform(0.5 / Ht, 1 - 0.5 / Ht, 300)],
                 -1).astype(np.float32)
    s = q[:, 0].astype(np.float64) * Wt - 0.5
    t = q[:, 1].astype(np.float64) * Ht - 0.5
    expect = 0.3 * s + 1.7 * t + 0.25
    got = oracle.texture(ramp, q, wrap_u=oracle.WRAP_CLAMP, wrap_v=oracle.WRAP_CLAMP)[:, 0]
    assert np.abs(got - expect).max() < 1e-12


def test_repeat_wrap_is_periodic_and_clamp_saturates():
    rng = np.random.default_rng(6)
    tex = rng.random((6, 10, 2))
    q = rng.uniform(0, 1, (200, 2)).astype(np.float32)
    q2 = q.copy()
    q2[:, 0] += 1.0
    a = oracle.texture(tex, q)
    b = oracle.texture(tex, q2.astype(np.float32))
    assert np.abs(a - b).max() < 1e-5      # u + 1 rounds in float32
    lo = np.array([[0.3, -0.7]], np.float32)
    assert np.allclose(oracle.texture(tex, lo), oracle.texture(tex, np.array([[0.3, 0.0]], np.float32)))


def test_texture_coord_grad_finite_differences():
    rng = np.random.default_rng(8)
    tex = rng.random((12, 12, 3))
    uv = rng.uniform(0.05, 0.95, (60, 2)).astype(np.float32)
    g = rng.standard_normal((60, 3))
    ana = oracle.texture_bwd_coord(tex, uv, g)
    fd = np.zeros_like(ana)
    h = 1e-3   # the forward's frac is single precision: keep the step well above its ulp
    for j in range(2):
        up, um = uv.copy(), uv.copy()
        up[:, j] += h
        um[:, j] -= h
        step = up[:, j].astype(np.float64) - um[:, j].astype(np.float64)
        fd[:, j] = ((oracle.texture(tex, up) - oracle.texture(tex, um)) * g).sum(-1) / step
    # drop samples whose stencil crosses a texel centre (kink of the bilinear)
    s = uv.astype(np.float64) * 12 - 0.5
    ok = (np.abs(s - np.round(s)) > 0.05).all(-1)
    assert ok.sum() > 40
    assert rel_err(ana[ok], fd[ok]) < 1e-4


def test_cube_faces():
    S = 4
    rng = np.random.default_rng(9)
    cube = rng.random((6, S, S, 1))
    axes = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    d = np.array(axes, np.float32)
    out = oracle.texture(cube, d, kind=oracle.TEX_CUBE)[:, 0]
    centre = cube[:, S // 2 - 1:S // 2 + 1, S // 2 - 1:S // 2 + 1, 0].mean((1, 2))
    assert np.abs(out - centre).max() < 1e-15
    # +X face: u grows with -z, v grows with -y; texel (row 0, col 3) centre
    u, v = (3 + 0.5) / S, (0 + 0.5) / S
    dx = np.array([[1.0, -(2 * v - 1), -(2 * u - 1)]], np.float32)
    assert abs(oracle.texture(cube, dx, kind=oracle.TEX_CUBE)[0, 0] - cube[0, 0, 3, 0]) < 1e-6
    # -Z face: u grows with -x, v with -y; texel (row 2, col 1)
    u, v = (1 + 0.5) / S, (2 + 0.5) / S
    dz = np.array([[-(2 * u - 1), -(2 * v - 1), -1.0]], np.float32)
    assert abs(oracle.texture(cube, dz, kind=oracle.TEX_CUBE)[0, 0] - cube[5, 2, 1, 0]) < 1e-6
    # scale invariance of the direction
    q = rng.standard_normal((50, 3)).astype(np.float32)
    a = oracle.texture(cube, q, kind=oracle.TEX_CUBE)
    b = oracle.texture(cube, (q * 4.0).astype(np.float32), kind=oracle.TEX_CUBE)
    assert np.abs(a - b).max() < 1e-6


def test_cube_direction_grad_finite_differences():
    rng = np.random.default_rng(10)
    cube = rng.random((6, 8, 8, 2))
    q = rng.standard_normal((80, 3)).astype(np.float32)
    g = rng.standard_normal((80, 2))
    ana = oracle.texture_bwd_coord(cube, q, g, kind=oracle.TEX_CUBE)
    fd = np.zeros_like(ana)
    h = 1e-4
    for j in range(3):
        qp, qm = q.copy(), q.copy()
        qp[:, j] += h
        qm[:, j] -= h
        step = qp[:, j].astype(np.float64) - qm[:, j].astype(np.float64)
        fp = oracle.texture(cube, qp, kind=oracle.TEX_CUBE)
        fm = oracle.texture(cube, qm, kind=oracle.TEX_CUBE)
        fd[:, j] = ((fp - fm) * g).sum(-1) / step
    ok = np.abs(ana - fd).max(-1) < 10  # drop samples crossing a face edge or texel centre
    a = np.abs(q)
    srt = np.sort(a, -1)
    ok &= (srt[:, 2] - srt[:, 1]) > 1e-2
    assert ok.sum() > 60
    assert rel_err(ana[ok], fd[ok]) < 1e-3


def test_texture_exact_adjoint_identity():
    rng = np.random.default_rng(12)
    tex = rng.random((7, 9, 2))
    uv = rng.uniform(-0.3, 1.3, (4, 5, 5, 2)).astype(np.float32)
    tid = rng.integers(-1, 3, (4, 5, 5)).astype(np.int32)
    g = rng.standard_normal((4, 5, 5, 2))
    y = oracle.texture(tex, uv, tid)
    gt = oracle.texture_adjoint(tex.shape, uv, tid, g)
    assert abs((y * g).sum() - (tex * gt).sum()) < 1e-10


# ---------------------------------------------------------------------------
# inverse UV
# ---------------------------------------------------------------------------
def _bf_inverse_uv_grad(tex_shape, uv, tid, g, wrap_u, wrap_v):
    """Brute force: per slice and cell the largest covered pixel index wins;
    the winner's gradient goes to all four of its bilinear taps."""
    Ht, Wt, Ct = tex_shape
    out = np.zeros(tex_shape)
    S = tid.shape[0]
    for s in range(S):
        win = {}
        flat_uv = uv[s].reshape(-1, 2)
        flat_t = tid[s].ravel()
        for i in range(flat_t.size):
            if flat_t[i] < 0:
                continue
            u, v = flat_uv[i]
            cx = int(np.floor(np.float32(u) * np.float32(Wt)))
            cy = int(np.floor(np.float32(v) * np.float32(Ht)))
            cx = cx % Wt if wrap_u == oracle.WRAP_REPEAT else min(max(cx, 0), Wt - 1)
            cy = cy % Ht if wrap_v == oracle.WRAP_REPEAT else min(max(cy, 0), Ht - 1)
            win[(cy, cx)] = max(win.get((cy, cx), -1), i)
        gs = g[s].reshape(-1, Ct)
        for (cy, cx), i in win.items():
            one = np.zeros((1, 2), np.float32)
            one[0] = flat_uv[i]
            out += oracle.texture_adjoint(tex_shape, one, None, gs[i:i + 1], wrap_u=wrap_u, wrap_v=wrap_v)
    return out


@pytest.mark.parametrize("wrap", [(oracle.WRAP_REPEAT, oracle.WRAP_CLAMP),
                                  (oracle.WRAP_CLAMP, oracle.WRAP_CLAMP),
                                  (oracle.WRAP_REPEAT, oracle.WRAP_REPEAT)])
def test_inverse_uv_matches_winner_only_bruteforce(wrap):
    rng = np.random.default_rng(13)
    tex_shape = (6, 7, 2)
    S, H, W = 3, 6, 6
    uv = rng.uniform(-0.2, 1.2, (S, H, W, 2)).astype(np.float32)
    tid = rng.integers(-1, 4, (S, H, W)).astype(np.int32)
    g = rng.standard_normal((S, H, W, 2))
    got = oracle.texture_bwd_tex(tex_shape, uv, tid, g, wrap_u=wrap[0], wrap_v=wrap[1])
    bf = _bf_inverse_uv_grad(tex_shape, uv, tid, g, *wrap)
    assert np.abs(got - bf).max() < 1e-12
    inv = oracle.invuv_build(tex_shape, uv, tid, wrap_u=wrap[0], wrap_v=wrap[1])
    assert inv.max() < H * W and (inv >= -1).all()


def test_inverse_uv_equals_exact_adjoint_without_collisions():
    """Minification with one pixel per cell: the inverse-UV gradient is the
    exact bilinear adjoint."""
    rng = np.random.default_rng(14)
    Ht = Wt = 32
    tex_shape = (Ht, Wt, 3)
    H = W = 8
    cells = rng.permutation(Ht * Wt)[:H * W]
    cy, cx = cells // Wt, cells % Wt
    uv = np.stack([(cx + rng.uniform(0.05, 0.95, H * W)) / Wt,
                   (cy + rng.uniform(0.05, 0.95, H * W)) / Ht], -1).reshape(1, H, W, 2).astype(np.float32)
    tid = np.zeros((1, H, W), np.int32)
    g = rng.standard_normal((1, H, W, 3))
    got = oracle.texture_bwd_tex(tex_shape, uv, tid, g)
    exact = oracle.texture_adjoint(tex_shape, uv, tid, g)
    assert np.abs(got - exact).max() < 1e-12


def test_inverse_uv_cube():
    rng = np.random.default_rng(15)
    S = 4
    tex_shape = (6, S, S, 2)
    q = rng.standard_normal((2, 5, 5, 3)).astype(np.float32)
    tid = rng.integers(-1, 2, (2, 5, 5)).astype(np.int32)
    g = rng.standard_normal((2, 5, 5, 2))
    got = oracle.texture_bwd_tex(tex_shape, q, tid, g, kind=oracle.TEX_CUBE)
    # brute force per slice: winner per (face, cell), adjoint of the winner only
    bf = np.zeros(tex_shape)
    for s in range(2):
        win = {}
        for i in range(25):
            if tid[s].ravel()[i] < 0:
                continue
            d = q[s].reshape(-1, 3)[i]
            a = np.abs(d)
            f = 0 if (a[0] >= a[1] and a[0] >= a[2]) else (1 if a[1] >= a[2] else 2)
            f = 2 * f + (0 if d[f] >= 0 else 1)
            key = (f,) + tuple(_cube_cell(d, f, S))
            win[key] = max(win.get(key, -1), i)
        for key, i in win.items():
            bf += oracle.texture_adjoint(tex_shape, q[s].reshape(-1, 3)[i:i + 1], None,
                                         g[s].reshape(-1, 2)[i:i + 1], kind=oracle.TEX_CUBE)
    assert np.abs(got - bf).max() < 1e-12


def _cube_cell(d, f, S):
    x, y, z = [np.float32(c) for c in d]
    sc, tc, ma = {0: (-z, -y, x), 1: (z, -y, -x), 2: (x, z, y), 3: (x, -z, -y),
                  4: (x, -y, z), 5: (-x, -y, -z)}[f]
    u = (sc / ma + np.float32(1)) * np.float32(0.5)
    v = (tc / ma + np.float32(1)) * np.float32(0.5)
    cx = min(max(int(np.floor(u * np.float32(S))), 0), S - 1)
    cy = min(max(int(np.floor(v * np.float32(S))), 0), S - 1)
    return cy, cx


# ---------------------------------------------------------------------------
# HardSoftRas blend
# ---------------------------------------------------------------------------
def _layers(rng, B, K, H, W, p_empty=0.3):
    tid = rng.integers(0, 50, (B, K, H, W)).astype(np.int32)
    n = rng.integers(0, K + 1, (B, H, W))           # layers fill front to back
    for k in range(K):
        tid[:, k][k >= n] = -1
    dist = rng.uniform(-0.05, 0.05, (B, K, H, W))
    dist[tid < 0] = 0.0
    # hard layers first: sign of dist non-increasing over k
    for k in range(1, K):
        m = dist[:, k - 1] < 0
        dist[:, k][m] = -np.abs(dist[:, k][m])
    return tid, dist


def test_edge_mask_matches_scipy_morphology():
    rng = np.random.default_rng(16)
    B, K, H, W = 2, 2, 40, 40
    tid = np.full((B, K, H, W), -1, np.int32)
    dist = np.zeros((B, K, H, W))
    yy, xx = np.mgrid[:H, :W]
    tid[0, 0][(xx - 20) ** 2 + (yy - 18) ** 2 < 120] = 1
    tid[1, 0][(xx > 5) & (xx < 30) & (yy > 2)] = 2
    dist[:, 0] = 0.01
    dist[0, 0][(xx < 18)] = -0.0       # soft fragments do not count as S^H
    for delta in [0.02, 0.1, 0.0251]:
        E = oracle.edge_mask(tid, dist, delta)
        rho = int(np.ceil(np.float32(delta) * np.float32(W))) - 1
        for b in range(B):
            S = (tid[b, 0] >= 0) & ~np.signbit(dist[b, 0])
            cross = ndimage.generate_binary_structure(2, 1)
            inner = S & ~ndimage.binary_erosion(S, cross, border_value=1)
            outer = ~S & ndimage.binary_dilation(S, cross, border_value=0)
            bnd = inner | outer
            ref = ndimage.binary_dilation(bnd, np.ones((2 * rho + 1,) * 2, bool)) if rho >= 0 else bnd * 0
            np.testing.assert_array_equal(E[b].astype(bool), ref)
    assert (oracle.edge_mask(tid, dist, 0.1, oracle.BLEND_SOFTRAS) == 1).all()
    E_aa = oracle.edge_mask(tid, dist, 0.1, oracle.BLEND_AA)
    np.testing.assert_array_equal(E_aa, oracle.edge_mask(tid, dist, 1.0 / W))


def test_blend_special_cases():
    rng = np.random.default_rng(17)
    B, K, H, W, Cc = 1, 3, 10, 10, 3
    tid, dist = _layers(rng, B, K, H, W)
    col = rng.random((B, K, H, W, Cc))
    sigma = 0.01 / 7
    # E == 0: exactly S^H C_1 and S^H
    oc, os_, E = oracle.softras(col, dist, tid, sigma, 0.1, oracle.BLEND_HARD)
    SH = (tid[:, 0] >= 0) & ~np.signbit(dist[:, 0])
    assert (E == 0).all()
    assert np.array_equal(oc, col[:, 0] * SH[..., None])
    assert np.array_equal(os_, SH.astype(np.float64))
    # K = 1, E == 1, present pixel: I_c = C_1, I_s = D_1
    oc, os_, _ = oracle.softras(col[:, :1], dist[:, :1], tid[:, :1], sigma, 0.1, oracle.BLEND_SOFTRAS)
    m = tid[:, 0] >= 0
    assert np.abs(oc[m] - col[:, 0][m]).max() < 1e-15
    D1 = 1 / (1 + np.exp(-dist[:, 0] / sigma))
    assert np.abs(os_[m] - D1[m]).max() < 1e-15
    # all D ~ 1: silhouette 1 and plain mean of the present layers
    big = np.where(tid >= 0, 1.0, 0.0)
    oc, os_, _ = oracle.softras(col, big, tid, 1e-3, 0.1, oracle.BLEND_SOFTRAS)
    n = (tid >= 0).sum(1)
    m = n > 0
    mean = (col * (tid >= 0)[..., None]).sum(1) / np.maximum(n, 1)[..., None]
    assert np.abs(oc[m] - mean[m]).max() < 1e-12 and np.abs(os_[m] - 1).max() < 1e-12
    assert (oc[~m] == 0).all() and (os_[~m] == 0).all()
    # D at +-r with sigma = r / 7
    r = 0.01
    d = np.array([r, -r]).reshape(1, 2, 1, 1)
    t2 = np.zeros((1, 2, 1, 1), np.int32)
    _, s1, _ = oracle.softras(np.ones((1, 1, 1, 1, 1)), d[:, :1], t2[:, :1], r / 7, 0.1, oracle.BLEND_SOFTRAS)
    _, s2, _ = oracle.softras(np.ones((1, 1, 1, 1, 1)), d[:, 1:], t2[:, 1:], r / 7, 0.1, oracle.BLEND_SOFTRAS)
    assert abs(s1[0, 0, 0] - 0.9990889488055994) < 1e-12
    assert abs(s2[0, 0, 0] - 9.110511944006454e-4) < 1e-12


@pytest.mark.parametrize("mode", [oracle.BLEND_HSR, oracle.BLEND_SOFTRAS])
def test_blend_bwd_finite_differences(mode):
    rng = np.random.default_rng(18)
    B, K, H, W, Cc = 1, 3, 12, 12, 3
    tid, dist = _layers(rng, B, K, H, W)
    col = rng.random((B, K, H, W, Cc))
    sigma, delta = 0.01, 0.15
    oc, os_, E = oracle.softras(col, dist, tid, sigma, delta, mode)
    gc = rng.standard_normal(oc.shape)
    gs = rng.standard_normal(os_.shape)
    glc, gld = oracle.softras_bwd(col, dist, tid, sigma, E, gc, gs)

    def L(c, d):
        a, b, _ = oracle.softras(c, d, tid, sigma, delta, mode)
        return (a * gc).sum() + (b * gs).sum()

    h = 1e-6
    dc = rng.standard_normal(col.shape)
    fd_c = (L(col + h * dc, dist) - L(col - h * dc, dist)) / (2 * h)
    assert abs(fd_c - (glc * dc).sum()) < 1e-6 * max(1, abs(fd_c))
    dd = rng.standard_normal(dist.shape) * (tid >= 0)
    # keep signs (hardness) fixed
    sgn = np.where(np.signbit(dist), -1.0, 1.0)
    dp = sgn * np.abs(dist + h * dd * sgn)
    dm = sgn * np.abs(dist - h * dd * sgn)
    keep = (np.abs(dist) > 2 * h)
    dd = dd * keep
    dp = np.where(keep, dist + h * dd, dist)
    dm = np.where(keep, dist - h * dd, dist)
    fd_d = (L(col, dp) - L(col, dm)) / (2 * h)
    assert abs(fd_d - (gld * dd).sum()) < 1e-5 * max(1, abs(fd_d))
