"""Pins of the oracle's inverse-UV jitter (§3.3.2: the sampling positions move
by quasi-random Sobol offsets per frame): the Sobol points against the net
property that defines the sequence, and the moved samples against a plane
(bilinear sampling reproduces it at the moved point) and the zero offset."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("k", range(1, 11))
def test_sobol_points_form_a_base2_net(k):
    """The first 2^k points of the 2-D Sobol sequence are a (0, k, 2)-net in
    base 2: every box [i / 2^a, (i+1) / 2^a) x [j / 2^b, (j+1) / 2^b) with
    a + b = k holds exactly one of them.  A wrong direction number breaks it."""
    pts = np.array([oracle.sobol2(f) for f in range(2 ** k)])
    for a in range(k + 1):
        b = k - a
        cells = (np.floor(pts[:, 0] * 2 ** a).astype(int) * 2 ** b + np.floor(pts[:, 1] * 2 ** b).astype(int))
        assert np.array_equal(np.sort(cells), np.arange(2 ** k)), (k, a)


def test_sobol_first_points_and_range():
    assert oracle.sobol2(0) == (0.0, 0.0)
    assert oracle.sobol2(1) == (0.5, 0.5)
    pts = np.array([oracle.sobol2(f) for f in range(1, 5000)])
    assert (pts >= 0).all() and (pts < 1).all()
    assert len({tuple(p) for p in pts}) == len(pts)


def _scene(seed=0, S=2, H=13, W=17, cd=2, Ct=3):
    rng = np.random.default_rng(seed)
    tid = rng.integers(-1, 5, (S, H, W)).astype(np.int32)
    tid[:, 3:9, 4:12] = 2                      # a covered block
    coord = rng.random((S, H, W, cd)).astype(np.float32)
    grad = rng.standard_normal((S, H, W, Ct))
    return coord, tid, grad


def test_frame_one_is_the_unmoved_sample():
    """Sobol point 1 is (1/2, 1/2): no offset.  A pixel registers its own
    coordinate and gradient, when it and its right, lower and lower-right
    neighbours are covered."""
    coord, tid, grad = _scene()
    jc, jt, jg = oracle.jitter_samples(coord, tid, grad, 1)
    cov = tid >= 0
    ok = np.zeros_like(cov)
    ok[:, :-1, :-1] = cov[:, :-1, :-1] & cov[:, :-1, 1:] & cov[:, 1:, :-1] & cov[:, 1:, 1:]
    assert np.array_equal(jt >= 0, ok)
    assert np.array_equal(jc[ok], coord[ok]) and np.array_equal(jg[ok], grad[ok])


@pytest.mark.parametrize("frame", [2, 3, 5, 12, 1000, 77777])
def test_moved_sample_of_a_plane(frame):
    """A coordinate plane c(x, y) = c0 + a x + b y sampled bilinearly at the
    moved centre is the plane there, (x + 1/2 + o_x, y + 1/2 + o_y) with
    o = Sobol(frame) - 1/2, up to float rounding; a constant gradient stays."""
    S, H, W = 1, 11, 15
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    plane = lambda X, Y: np.stack([0.1 + 0.03 * X - 0.01 * Y, 0.7 - 0.02 * X + 0.04 * Y], -1)
    coord = plane(xs, ys)[None].astype(np.float32)
    tid = np.zeros((S, H, W), np.int32)
    grad = np.full((S, H, W, 2), 1.25)
    jc, jt, jg = oracle.jitter_samples(coord, tid, grad, frame)
    u, v = oracle.sobol2(frame)
    want = plane(xs + (u - 0.5), ys + (v - 0.5))[None]
    ok = jt >= 0
    assert ok.sum() >= (H - 1) * (W - 1)
    assert np.abs(jc[ok] - want[ok]).max() < 4e-7
    assert np.allclose(jg[ok], 1.25, rtol=0, atol=1e-15)
    # the pixels on the border the offset leaves without taps do not register
    dx, dy = int(np.floor(u - 0.5)), int(np.floor(v - 0.5))
    xs_i, ys_i = np.meshgrid(np.arange(W), np.arange(H))
    inside = (xs_i + dx >= 0) & (ys_i + dy >= 0) & (xs_i + dx + 1 < W) & (ys_i + dy + 1 < H)
    assert np.array_equal(ok[0], inside)
