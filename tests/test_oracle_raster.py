"""Pins for the oracle's rasterization (coverage, depth key, K layers, soft
distance, barycentrics) against what the method and geometry fix independently
of the oracle: a tiling covers every pixel exactly once, a brute-force
set-based rendering of tiny scenes, ray/plane intersections, closed-form
distances, the Shift ordering invariant and finite differences."""
import numpy as np
import pytest

import oracle
from helpers import rel_err, screen_to_clip, to_clip
from paper_2204_01386_amd import scenes


# ---------------------------------------------------------------------------
# tiling: every pixel covered exactly once
# ---------------------------------------------------------------------------
def _separate(tris_xy, H, W, depths=None):
    """Unshared vertices per triangle, each triangle at its own constant depth."""
    T = len(tris_xy)
    xy = np.asarray(tris_xy, np.float64).reshape(-1, 2)
    if depths is None:
        depths = 0.1 + 0.8 * (np.arange(T) + 0.5) / T
    z = np.repeat(depths, 3)
    pc = screen_to_clip(xy, H, W, z=z)
    tris = np.arange(3 * T, dtype=np.int32).reshape(T, 3)
    return pc, tris


def _grid_triangulation(H, W, step, jitter, rng, fan=False):
    xs = np.arange(-step + 0.5, W + step, step)
    ys = np.arange(-step + 0.5, H + step, step)
    P = np.stack(np.meshgrid(xs, ys, indexing="xy"), -1).astype(np.float64)
    if jitter:
        J = rng.uniform(-jitter, jitter, P.shape)
        J = np.round(J * 256) / 256                   # keep positions dyadic
        J[rng.random(P.shape[:2]) < 0.3] = 0.0        # some vertices exactly on pixel centres
        P = P + J
    tri = []
    for i in range(P.shape[0] - 1):
        for j in range(P.shape[1] - 1):
            a, b, c, d = P[i, j], P[i, j + 1], P[i + 1, j + 1], P[i + 1, j]
            if fan:
                m = (a + c) / 2
                tri += [(a, b, m), (b, c, m), (c, d, m), (d, a, m)]
            elif (i + j) % 2:
                tri += [(a, b, c), (a, c, d)]
            else:
                tri += [(a, b, d), (b, c, d)]
    return tri


@pytest.mark.parametrize("case", ["jitter", "pixel_centres", "fans", "reversed"])
def test_tiling_covers_every_pixel_once(case):
    H = W = 32
    rng = np.random.default_rng(3)
    if case == "jitter":
        tri = _grid_triangulation(H, W, 5, 2.0, rng)
    elif case == "pixel_centres":
        tri = _grid_triangulation(H, W, 4, 0.0, rng)      # axis-aligned edges through centres
    elif case == "fans":
        tri = _grid_triangulation(H, W, 4, 0.0, rng, fan=True)
    else:
        tri = [t[::-1] for t in _grid_triangulation(H, W, 6, 1.5, rng)]  # other winding
    pc, tris = _separate(tri, H, W)
    tid, hard, _, _ = oracle.rasterize(pc, tris, H, W, K=2)
    assert (tid[0, 0] >= 0).all(), "a pixel is not covered"
    assert (tid[0, 1] == -1).all(), "a pixel is covered twice"
    assert hard[0, 0].all()


def test_shared_edge_goes_to_one_side_only():
    """Two triangles sharing a diagonal through pixel centres: union covers the
    square exactly once, and each pixel on the diagonal goes to exactly one."""
    H = W = 16
    a, b, c, d = (0.5, 0.5), (12.5, 0.5), (12.5, 12.5), (0.5, 12.5)
    pc, tris = _separate([(a, b, c), (a, c, d)], H, W)
    tid, _, _, _ = oracle.rasterize(pc, tris, H, W, K=2)
    inside = np.zeros((H, W), bool)
    inside[1:13, 1:13] = True   # centres strictly inside the square
    # centres on the square's border: the top-left rule takes top and left edges
    inside[0:13, 0] = False
    cov = tid[0, 0] >= 0
    assert (tid[0, 1] == -1).all()
    diag = [(i, i) for i in range(1, 12)]
    assert all(cov[y, x] for y, x in diag)


# ---------------------------------------------------------------------------
# brute force on tiny scenes (set definition of the K layers)
# ---------------------------------------------------------------------------
def _bf_snap(c, w, half, is_y):
    n = np.float32(c) / np.float32(w)
    p = (np.float32(1) - n) * np.float32(half) if is_y else (n + np.float32(1)) * np.float32(half)
    return int(np.rint(p * np.float32(256)))


def _bf_render(pc, tris, H, W, K, r):
    """Brute force: collect every fragment of every pixel, sort by (key, id),
    keep the first id of each distinct key, take K.  Coverage by the symbolic
    perturbation P + (eps, eps^2) without reordering the vertices."""
    frags = [[[] for _ in range(W)] for _ in range(H)]
    for t, tv in enumerate(tris):
        v = pc[tv]
        if (v[:, 3] <= 0).any():
            continue
        X = [_bf_snap(v[i, 0], v[i, 3], W * 0.5, False) for i in range(3)]
        Y = [_bf_snap(v[i, 1], v[i, 3], H * 0.5, True) for i in range(3)]
        A = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0])
        if A == 0:
            continue
        sgn = 1 if A > 0 else -1
        order = [0, 1, 2] if A > 0 else [0, 2, 1]
        zn = [np.float32(v[i, 2]) / np.float32(v[i, 3]) for i in range(3)]
        Xo, Yo, zo = [X[i] for i in order], [Y[i] for i in order], [zn[i] for i in order]
        for y in range(H):
            for x in range(W):
                px, py = 256 * x + 128, 256 * y + 128
                inside = True
                for i in range(3):
                    a, b = (i + 1) % 3, (i + 2) % 3
                    dx, dy = X[b] - X[a], Y[b] - Y[a]
                    E = dx * (py - Y[a]) - dy * (px - X[a])
                    lex = (E, -dy, dx)
                    pos = next((s for s in lex if s != 0), 0) * sgn
                    inside &= pos > 0
                if inside:
                    E1 = (Xo[0] - Xo[2]) * (py - Yo[2]) - (Yo[0] - Yo[2]) * (px - Xo[2])
                    E2 = (Xo[1] - Xo[0]) * (py - Yo[0]) - (Yo[1] - Yo[0]) * (px - Xo[0])
                    Af = np.float32(abs(A))
                    l1, l2 = np.float32(E1) / Af, np.float32(E2) / Af
                    z = (zo[0] + l1 * (zo[1] - zo[0])) + l2 * (zo[2] - zo[0])
                    if not (np.float32(0) < z < np.float32(1)):
                        continue
                    frags[y][x].append((np.float32(0.5) * z, t))
                elif r > 0:
                    # distance to the triangle: the nearest of the three segments
                    P = np.array([x + 0.5, y + 0.5])
                    best = np.inf
                    for i in range(3):
                        A_ = np.array([X[i], Y[i]]) / 256.0
                        B_ = np.array([X[(i + 1) % 3], Y[(i + 1) % 3]]) / 256.0
                        e = B_ - A_
                        tt = np.clip(np.dot(P - A_, e) / np.dot(e, e), 0, 1)
                        best = min(best, np.linalg.norm(P - (A_ + tt * e)))
                    dn = np.float32(best / W)
                    if dn <= np.float32(r):
                        frags[y][x].append((np.float32(0.5) * dn + np.float32(0.5), t))
    tid = -np.ones((K, H, W), np.int32)
    hard = np.zeros((K, H, W), np.uint8)
    for y in range(H):
        for x in range(W):
            fl = sorted(frags[y][x], key=lambda f: (f[0], f[1]))
            keep, last = [], None
            for key, t in fl:
                if key != last:
                    keep.append((key, t))
                    last = key
            for k, (key, t) in enumerate(keep[:K]):
                tid[k, y, x] = t
                hard[k, y, x] = key < 0.5
    return tid, hard


@pytest.mark.parametrize("seed,K,r", [(0, 1, 0.0), (1, 2, 0.0), (2, 3, 0.12), (3, 2, 0.2), (4, 5, 0.1)])
def test_bruteforce_tiny_scenes(seed, K, r):
    rng = np.random.default_rng(seed)
    H = W = 16
    T = 7
    xy = rng.uniform(-2, 18, (T * 3, 2))
    z = rng.uniform(0.05, 0.95, T * 3)
    w = rng.uniform(0.5, 2.0, T * 3)
    pc = screen_to_clip(xy, H, W, z=z, w=w)
    tris = rng.permutation(T * 3).reshape(T, 3).astype(np.int32)
    # a duplicate of triangle 0 (equal keys everywhere) and a shared-vertex neighbour
    tris = np.concatenate([tris, tris[:1], tris[1:2, [1, 0, 2]]]).astype(np.int32)
    tid, hard, _, _ = oracle.rasterize(pc, tris, H, W, K=K, r=r)
    btid, bhard = _bf_render(pc, tris, H, W, K, r)
    np.testing.assert_array_equal(tid[0], btid)
    np.testing.assert_array_equal(hard[0], bhard)
    # the duplicate never shows up: equal keys keep the smaller id
    assert not (tid == T).any()


def test_shift_puts_hard_before_soft_and_no_pseudo_occlusion():
    """Two adjacent triangles (Fig. 4): blue in front of red, K=2.  Every pixel
    hard-covered by either triangle has a hard front layer, hard layers precede
    soft ones, and soft keys grow with distance."""
    H = W = 48
    xy = np.array([[6, 6], [40, 8], [20, 40], [40, 8], [44, 44], [20, 40]], np.float64)
    z = np.array([0.3, 0.3, 0.3, 0.6, 0.6, 0.6])
    pc = screen_to_clip(xy, H, W, z=z)
    tris = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    tid, hard, _, dist = oracle.rasterize(pc, tris, H, W, K=2, r=0.1)
    tid_h, _, _, _ = oracle.rasterize(pc, tris, H, W, K=1, r=0.0)
    covered = tid_h[0, 0] >= 0
    assert hard[0, 0][covered].all()
    np.testing.assert_array_equal(tid[0, 0][covered], tid_h[0, 0][covered])
    # hard flags are non-increasing over layers
    assert (hard[0, 1] <= hard[0, 0]).all()
    # soft layers are ordered by |dist|
    both_soft = (tid[0, 0] >= 0) & (tid[0, 1] >= 0) & (hard[0, 0] == 0)
    assert (np.abs(dist[0, 0][both_soft]) <= np.abs(dist[0, 1][both_soft])).all()
    # signs carry hardness
    assert (np.signbit(dist[0][tid[0] >= 0]) == (hard[0][tid[0] >= 0] == 0)).all()
    # soft reach: |dist| <= r for soft fragments
    soft = (tid[0] >= 0) & (hard[0] == 0)
    assert soft.any()
    assert (np.abs(dist[0][soft]) <= 0.1 + 1e-7).all()


def test_soft_distance_closed_form():
    """Right triangle (8,8),(24,8),(8,24) px: outside distances are to the legs,
    the hypotenuse or the corners; inside ones to the nearest side."""
    H = W = 40
    xy = np.array([[8, 8], [24, 8], [8, 24]], np.float64)
    pc = screen_to_clip(xy, H, W, z=0.5)
    tris = np.array([[0, 1, 2]], np.int32)
    tid, hard, _, dist = oracle.rasterize(pc, tris, H, W, K=1, r=0.5)
    A, B_, C_ = xy
    for y in range(H):
        for x in range(W):
            P = np.array([x + 0.5, y + 0.5])
            d = min(_segdist(P, A, B_), _segdist(P, B_, C_), _segdist(P, C_, A))
            assert (tid[0, 0, y, x] >= 0) == (d / W <= 0.5)
            if tid[0, 0, y, x] < 0:
                continue
            assert abs(abs(dist[0, 0, y, x]) - d / W) < 1e-12
            inside = x + 0.5 > 8 and y + 0.5 > 8 and (x + 0.5 - 8) + (y + 0.5 - 8) < 16
            assert bool(hard[0, 0, y, x]) == inside
    # sampled boundary check (independent of the segment formula)
    t = np.linspace(0, 1, 20001)[:, None]
    bnd = np.concatenate([A + t * (B_ - A), B_ + t * (C_ - B_), C_ + t * (A - C_)])
    for (x, y) in [(2, 30), (24, 24), (16, 3), (12, 12), (26, 5)]:
        P = np.array([x + 0.5, y + 0.5])
        d = np.min(np.linalg.norm(bnd - P, axis=1))
        assert abs(abs(dist[0, 0, y, x]) * W - d) < 1e-3


def _segdist(P, A, B):
    e = B - A
    t = np.clip(np.dot(P - A, e) / np.dot(e, e), 0, 1)
    return np.linalg.norm(P - (A + t * e))


def test_soft_probability_range():
    """D = sigmoid(dist / sigma) with sigma = r/7 spans sigmoid(-7)..1 over soft
    pixels: every soft fragment has |dist| <= r."""
    H = W = 64
    s = scenes.config1()
    pc = to_clip(s.pos, s.mvp)
    pc = np.ascontiguousarray(pc)
    # 64x64 render of the icosphere with r = 0.05
    tid, hard, _, dist = oracle.rasterize(pc, s.tris, H, W, K=3, r=0.05)
    soft = (tid >= 0) & (hard == 0)
    assert soft.any()
    assert (np.abs(dist[soft]) <= 0.05 + 1e-7).all()


# ---------------------------------------------------------------------------
# barycentrics: ray / plane intersection
# ---------------------------------------------------------------------------
def test_perspective_bary_equals_ray_plane_hit():
    """In view space (eye at the origin looking down -z, w = -z_view) the
    perspective-correct barycentrics of a pixel are the barycentrics of the
    point where the ray through the pixel centre meets the triangle's plane.
    The view-space vertices are rebuilt from the float32 clip x, y, w that the
    rasterizer consumes, so both sides see the same triangle."""
    rng = np.random.default_rng(5)
    H = W = 40
    P = scenes.perspective()
    f = P[1, 1]
    for trial in range(4):
        V = rng.uniform(-0.9, 0.9, (3, 3))
        V[:, 2] = rng.uniform(-4.0, -2.0, 3)            # strong depth variation
        pc = to_clip(V, P[None])
        tris = np.array([[0, 1, 2]], np.int32)
        tid, hard, bary, _ = oracle.rasterize(pc, tris, H, W)
        bu, _ = oracle.resolve(pc, tris, tid, hard, snap=False)
        ys, xs = np.nonzero(tid[0, 0] >= 0)
        assert len(xs) > 10
        c = pc[0].astype(np.float64)
        Pv = np.stack([c[:, 0] / P[0, 0], c[:, 1] / f, -c[:, 3]], 1)
        n = np.cross(Pv[1] - Pv[0], Pv[2] - Pv[0])
        for x, y in zip(xs, ys):
            xn = (x + 0.5) / (W / 2) - 1
            yn = 1 - (y + 0.5) / (H / 2)
            d = np.array([xn / P[0, 0], yn / f, -1.0])
            X = d * np.dot(Pv[0], n) / np.dot(d, n)
            M = np.stack([Pv[0] - Pv[2], Pv[1] - Pv[2]], 1)
            w01, *_ = np.linalg.lstsq(M, X - Pv[2], rcond=None)
            assert abs(bu[0, 0, y, x, 0] - w01[0]) < 1e-9
            assert abs(bu[0, 0, y, x, 1] - w01[1]) < 1e-9
        # snapped values stay within the 1/256-pixel snap of the exact ones
        cov = tid[0, 0] >= 0
        assert np.abs(bary[0, 0][cov] - bu[0, 0][cov]).max() < 0.05


def test_bary_is_lambda_when_w_equal():
    H = W = 32
    xy = np.array([[2.25, 3.5], [30.0, 5.75], [10.5, 29.0]])
    pc = screen_to_clip(xy, H, W, z=0.5, w=1.7)
    tris = np.array([[0, 1, 2]], np.int32)
    tid, hard, bary, _ = oracle.rasterize(pc, tris, H, W)
    for y, x in zip(*np.nonzero(tid[0, 0] >= 0)):
        P = np.array([x + 0.5, y + 0.5])
        M = np.stack([xy[0] - xy[2], xy[1] - xy[2]], 1)
        l = np.linalg.solve(M, P - xy[2])
        assert np.allclose(bary[0, 0, y, x], l, atol=1e-9)


# ---------------------------------------------------------------------------
# backward: frozen-visibility central finite differences
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("K,r", [(1, 0.0), (2, 0.15)])
def test_rasterize_bwd_finite_differences(K, r):
    rng = np.random.default_rng(11)
    H = W = 20
    T = 4
    xy = rng.uniform(0, 20, (T * 3, 2))
    z = rng.uniform(0.2, 0.8, T * 3)
    w = rng.uniform(0.7, 1.6, T * 3)
    pc = screen_to_clip(xy, H, W, z=z, w=w)
    tris = np.arange(T * 3, dtype=np.int32).reshape(T, 3)
    tid, hard, _, _ = oracle.rasterize(pc, tris, H, W, K=K, r=r)
    gb = rng.standard_normal(tid.shape + (2,))
    gd = rng.standard_normal(tid.shape) if r > 0 else None
    ana = oracle.rasterize_bwd(pc, tris, tid, hard, gb, gd, snap=False)

    def loss(p):
        b, d = oracle.resolve(p, tris, tid, hard, snap=False)
        L = (b * gb).sum()
        if gd is not None:
            L += (d * gd).sum()
        return L

    fd = np.zeros_like(ana)
    for v in range(pc.shape[0]):
        for c in range(4):
            pp, pm = pc.copy(), pc.copy()
            h = 1e-5 * max(1.0, abs(float(pc[v, c])))
            pp[v, c] = np.float32(pc[v, c] + h)
            pm[v, c] = np.float32(pc[v, c] - h)
            step = float(pp[v, c]) - float(pm[v, c])
            fd[0, v, c] = (loss(pp) - loss(pm)) / step
    assert np.all(ana[0, :, 2] == 0.0)
    assert rel_err(ana, fd) < 1e-3


def test_window_equals_crop_of_full_image():
    """The windowed rasterizer (used for sampled checks of large images) visits
    only the window's pixels but considers every triangle: its layers are the
    crop of the full image's."""
    from paper_2204_01386_amd import scenes
    s = scenes.config1()
    pc = oracle.transform_f32(s.pos, s.mvp)
    full = oracle.rasterize(pc, s.tris, 128, 128, K=3, r=0.05)
    for win in [(0, 0, 128, 128), (20, 30, 50, 40), (127, 0, 1, 128), (60, 60, 7, 3)]:
        x0, y0, w, h = win
        part = oracle.rasterize_window(pc, s.tris, 128, 128, win, K=3, r=0.05)
        for a, b in zip(full, part):
            assert np.array_equal(a[:, :, y0:y0 + h, x0:x0 + w], b)


def test_window_adjoint_equals_full_adjoint_with_gradient_only_there():
    """The window form of the rasterization adjoint (used for sampled checks
    of large images) equals the full-image adjoint whose incoming gradients
    are zero outside the window."""
    s = scenes.config1()
    pc = oracle.transform_f32(s.pos, s.mvp)
    H = W = 96
    tid, hard, _, _ = oracle.rasterize(pc, s.tris, H, W, K=3, r=0.05)
    rng = np.random.default_rng(5)
    gb = rng.standard_normal(tid.shape + (2,))
    gd = rng.standard_normal(tid.shape)
    for win in [(0, 0, W, H), (10, 40, 60, 56), (0, 70, W, 26), (47, 3, 1, 50)]:
        x0, y0, w, h = win
        mask = np.zeros(tid.shape, bool)
        mask[:, :, y0:y0 + h, x0:x0 + w] = True
        full = oracle.rasterize_bwd(pc, s.tris, tid, hard, gb * mask[..., None], gd * mask)
        cut = lambda a: np.ascontiguousarray(a[:, :, y0:y0 + h, x0:x0 + w])
        part = oracle.rasterize_bwd(pc, s.tris, cut(tid), cut(hard), cut(gb), cut(gd),
                                    image=(H, W), window=win)
        assert np.abs(full).max() > 0
        assert np.allclose(part, full, rtol=1e-12, atol=1e-12 * np.abs(full).max())
