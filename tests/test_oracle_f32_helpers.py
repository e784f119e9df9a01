"""Pins of the oracle's single-precision helpers: the values that feed
discrete decisions (clip coordinates are snapped, texture coordinates select
texels and inverse-UV cells, a normal-map sample steers the cube lookup and
the shading kinks) are computed in float32 with a fixed operation order on
both sides.  Each helper is held here to its double-precision counterpart
within the textbook rounding-error bound of its float operations (unit
roundoff u = 2^-24, gamma_n = n u / (1 - n u)), so a wrong index, operand or
sign in it fails although the GPU is compared against it bit for bit."""
import numpy as np

import oracle
from paper_2204_01386_amd import scenes

U = 2.0 ** -24


def gamma(n):
    return n * U / (1 - n * U)


def test_transform_f32_within_dot_product_bound():
    """o_r = sum_j M_rj p_j (p_3 = 1): four products and three sums, so
    |fl(o_r) - o_r| <= gamma_4 sum_j |M_rj p_j| (every input is a float)."""
    rng = np.random.default_rng(0)
    s = scenes.config3(n_views=4, subdiv=2)
    pos = np.concatenate([s.pos, rng.uniform(-3, 3, (200, 3))]).astype(np.float32)
    mvp = np.concatenate([s.mvp, rng.standard_normal((3, 4, 4))]).astype(np.float32)
    out = oracle.transform_f32(pos, mvp).astype(np.float64)
    ref = oracle.transform(pos.astype(np.float64), mvp.astype(np.float64))
    ph = np.concatenate([pos, np.ones((len(pos), 1), np.float32)], 1).astype(np.float64)
    mag = np.einsum("bij,vj->bvi", np.abs(mvp.astype(np.float64)), np.abs(ph))
    err = np.abs(out - ref)
    assert (err <= gamma(4) * mag).all(), (err / np.maximum(mag, 1e-300)).max()
    # the bound is tight enough to notice a transposed matrix or a dropped term
    bad = oracle.transform_f32(pos, np.ascontiguousarray(np.swapaxes(mvp, 1, 2))).astype(np.float64)
    assert not (np.abs(bad - ref) <= gamma(4) * mag).all()


def test_interpolate_f32_within_rounding_bound():
    """out = (b0 a0 + b1 a1) + b2' a2 with b2' = fl(fl(1 - b0) - b1): the
    third weight carries |b2' - b2| <= 2u (|1 - b0| + |b1|) (1 + u), and the
    three products and two sums add gamma_3 of the sum of magnitudes.  Soft
    fragments extrapolate, so barycentrics run outside [0, 1] as well."""
    rng = np.random.default_rng(1)
    V, C, T = 50, 5, 40
    attr = rng.standard_normal((V, C)).astype(np.float32) * rng.uniform(0.1, 30, (V, 1)).astype(np.float32)
    tris = rng.integers(0, V, (T, 3)).astype(np.int32)
    tid = rng.integers(-1, T, (2, 3, 9, 11)).astype(np.int32)
    bary = rng.uniform(-1.5, 2.5, tid.shape + (2,)).astype(np.float32)
    bary[0, 0] = rng.uniform(0, 0.5, bary[0, 0].shape)   # ordinary interior fragments too
    out = oracle.interpolate_f32(attr, tris, tid, bary).astype(np.float64)
    ref = oracle.interpolate(attr.astype(np.float64), tris, tid, bary.astype(np.float64))
    b = bary.astype(np.float64)
    b0, b1 = b[..., 0], b[..., 1]
    b2 = 1.0 - b0 - b1
    a = np.abs(attr.astype(np.float64))[tris[np.maximum(tid, 0)]]     # [...,3,C]
    mag = (np.abs(b0)[..., None] * a[..., 0, :] + np.abs(b1)[..., None] * a[..., 1, :]
           + (np.abs(b2)[..., None] + 4 * U) * a[..., 2, :])
    w2err = 2 * U * (1 + U) * (np.abs(1 - b0) + np.abs(b1))
    bound = gamma(3) * mag + (1 + gamma(3)) * w2err[..., None] * a[..., 2, :]
    bound[tid < 0] = 0.0
    err = np.abs(out - ref)
    assert (err <= bound).all(), (err - bound).max()
    assert (out[tid < 0] == 0).all()
    # a swapped corner is far outside the bound
    bad = oracle.interpolate_f32(attr, tris[:, [1, 0, 2]], tid, bary).astype(np.float64)
    assert not (np.abs(bad - ref) <= bound).all()


def test_texture_f32_within_rounding_bound():
    """Bilinear sample in float: each weight is a product of two rounded
    complements (gamma_3 relative), each term one more product, three sums:
    |fl(out) - out| <= gamma_7 sum |w_i t_i|, with the same taps as the
    double sampler; 2-D (repeat, clamp) and cube maps."""
    rng = np.random.default_rng(2)
    tex = rng.uniform(-2, 3, (7, 9, 5)).astype(np.float32)
    uv = rng.uniform(-0.7, 1.7, (3, 41, 2)).astype(np.float32)
    cx = np.array([[0, 0], [2, 1], [4, 2], [6, 3], [8, 4], [1, 6]])       # (column, row) of texels
    uv[0, :6] = ((cx + 0.5) / np.array([9, 7])).astype(np.float32)        # their centres
    tid = rng.integers(-1, 4, (3, 41)).astype(np.int32)
    for wu, wv in [(oracle.WRAP_REPEAT, oracle.WRAP_CLAMP), (oracle.WRAP_CLAMP, oracle.WRAP_REPEAT)]:
        out = oracle.texture_f32(tex, uv, tid, wrap_u=wu, wrap_v=wv).astype(np.float64)
        ref = oracle.texture(tex.astype(np.float64), uv, tid, wrap_u=wu, wrap_v=wv)
        mag = oracle.texture(np.abs(tex.astype(np.float64)), uv, tid, wrap_u=wu, wrap_v=wv)
        assert (np.abs(out - ref) <= gamma(7) * mag).all()
        assert (out[tid < 0] == 0).all()
        # the texel centres return their texel exactly
        for j in range(6):
            if tid[0, j] >= 0:
                assert np.array_equal(out[0, j], tex[cx[j, 1], cx[j, 0]].astype(np.float64))
    # swapped coordinates (u taken along rows) are caught
    bad = oracle.texture_f32(tex, np.ascontiguousarray(uv[..., ::-1]), tid).astype(np.float64)
    ref = oracle.texture(tex.astype(np.float64), uv, tid)
    mag = oracle.texture(np.abs(tex.astype(np.float64)), uv, tid)
    assert not (np.abs(bad - ref) <= gamma(7) * mag).all()
    cube = rng.uniform(0, 1, (6, 8, 8, 3)).astype(np.float32)
    d = rng.standard_normal((200, 3)).astype(np.float32)
    out = oracle.texture_f32(cube, d, kind=oracle.TEX_CUBE).astype(np.float64)
    ref = oracle.texture(cube.astype(np.float64), d, kind=oracle.TEX_CUBE)
    assert (np.abs(out - ref) <= gamma(7) * ref).all()   # non-negative texels: |t| = t
