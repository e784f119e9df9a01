"""Pins for the oracle of image-based PBS: the cube texel geometry against the
sampler and the sphere's solid angle; the irradiance filter against the
closed form of a linear environment; the prefilter against the irradiance
filter (alpha = 1 makes D constant) and against the environment itself (a
lobe narrower than a texel); the BRDF table against an independent
quadrature and its smooth-surface limit; the shading's autograd against
finite differences; the filters' adjoint identity."""
import math

import numpy as np
import torch

import oracle as O
from oracle import pbs as P


def test_cube_texels_geometry():
    S = 8
    d, om = P.cube_texels(S)
    assert d.shape == (6 * S * S, 3)
    assert abs(om.sum() - 4 * math.pi) < 1e-12
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    # the sampler maps each texel's direction back to that texel (weights at the centre)
    tex = np.arange(6 * S * S, dtype=np.float32).reshape(6, S, S, 1)
    got = O.texture(tex, d.astype(np.float32).reshape(1, 1, -1, 3), None, kind=O.TEX_CUBE)
    assert np.allclose(got.reshape(-1), np.arange(6 * S * S), atol=1e-3)


def test_irradiance_of_linear_environment():
    """env(w) = w_z: the normalised cosine convolution gives (2/3) n_z (the
    hemisphere's first moment over its cosine integral)."""
    S, Si = 48, 8
    w, _ = P.cube_texels(S)
    env = w[:, 2].reshape(6, S, S, 1)
    irr, _ = P.ibl_filter(env, Si, 4, 2)
    n, _ = P.cube_texels(Si)
    assert np.abs(irr.reshape(-1) - 2.0 / 3.0 * n[:, 2]).max() < 3e-3


def test_prefilter_limits():
    S = 16
    # alpha = 1: D = 1/pi everywhere, the prefilter is the cosine convolution
    assert np.abs(P.prefilter_matrix(S, 8, 1.0) - P.irradiance_matrix(S, 8)).max() < 1e-12
    # a lobe much narrower than a texel keeps the texel itself (Sp = S)
    M = P.prefilter_matrix(S, S, 1e-3)
    assert np.diag(M).min() > 0.99


def test_brdf_lut_against_quadrature():
    N, M = 8, 1024
    lut = P.brdf_lut(N, M)
    assert (lut >= 0).all() and (lut.sum(-1) <= 1.0 + 1e-9).all()
    # smooth limit (alpha -> 0): h -> n and l -> the mirror of v, so
    # A -> (1 - (1 - c)^5) G1(c)^2 and B -> (1 - c)^5 G1(c)^2
    N0 = 32
    lut0 = P.brdf_lut(N0, M)[0]
    r0 = 0.5 / N0
    k0 = r0 ** 4 / 2.0
    c = (np.arange(N0) + 0.5) / N0
    G2 = (c / (c * (1 - k0) + k0)) ** 2
    fc = (1 - c) ** 5
    # (away from grazing views, where part of even a narrow lobe dips below the horizon)
    ok = c >= 0.1
    assert np.abs(lut0[ok, 0] - ((1 - fc) * G2)[ok]).max() < 3e-3
    assert np.abs(lut0[ok, 1] - (fc * G2)[ok]).max() < 3e-3
    # independent quadrature over light directions (midpoint rule in theta, phi)
    def ref(c, r):
        a = r * r
        k = a / 2.0
        nt, nph = 800, 400
        th = (np.arange(nt) + 0.5) / nt * (math.pi / 2)
        ph = (np.arange(nph) + 0.5) / nph * 2 * math.pi
        T, Ph = np.meshgrid(th, ph, indexing="ij")
        l = np.stack([np.sin(T) * np.cos(Ph), np.sin(T) * np.sin(Ph), np.cos(T)], -1)
        v = np.array([math.sqrt(1 - c * c), 0.0, c])
        h = l + v
        h /= np.linalg.norm(h, axis=-1, keepdims=True)
        ndl, ndh, vdh = l[..., 2], h[..., 2], h @ v
        D = P.ggx_d(ndh, a)
        g1 = lambda q: q / (q * (1 - k) + k)
        f = D * g1(c) * g1(ndl) / (4 * ndl * c)        # specular BRDF without Fresnel
        dw = np.sin(T) * (math.pi / 2 / nt) * (2 * math.pi / nph)
        fc = (1 - vdh) ** 5
        return ((1 - fc) * f * ndl * dw).sum(), (fc * f * ndl * dw).sum()
    for j, i in ((3, 2), (5, 6), (7, 1)):
        A, B = ref((i + 0.5) / N, (j + 0.5) / N)
        assert abs(lut[j, i, 0] - A) < 2e-2 * max(A, 0.05) and abs(lut[j, i, 1] - B) < 2e-2 * max(B, 0.05), \
            (j, i, lut[j, i], A, B)


def test_shading_autograd_matches_finite_differences():
    rng = np.random.default_rng(0)
    n = rng.standard_normal((5, 3))
    p = 0.3 * rng.standard_normal((5, 3))
    eye = np.array([0.2, 0.4, 3.0])
    n[:, 2] = np.abs(n[:, 2]) + 1.0          # facing the eye
    alb = rng.uniform(0.1, 0.9, (5, 3))
    irr = rng.uniform(0.1, 1.0, (5, 3))
    L = 5
    pref = rng.uniform(0.1, 1.0, (L, 5, 3))
    lut = P.brdf_lut(8, 256)
    m, r = 0.3, 0.37
    g = rng.standard_normal((5, 3))
    tid = np.zeros(5, np.int32)
    _, gr = P.shade_and_grads(n, p, eye, alb, m, r, irr, pref, lut, L, tid, g)

    def f(**kw):
        a = dict(n=n, p=p, albedo=alb, metallic=m, roughness=r, irr_s=irr, pref_s=pref)
        a.update(kw)
        t = lambda x: torch.tensor(np.asarray(x, np.float64))
        out = P.pbs_shade(t(a["n"]), t(a["p"]), t(eye), t(a["albedo"]), t(a["metallic"]), t(a["roughness"]),
                          t(a["irr_s"]), t(a["pref_s"]), t(lut), L)
        return float((out.numpy() * g).sum())
    h = 1e-6
    for name, val in (("metallic", m), ("roughness", r)):
        fd = (f(**{name: val + h}) - f(**{name: val - h})) / (2 * h)
        assert abs(fd - gr[name]) < 1e-6 * max(1.0, abs(fd)), (name, fd, gr[name])
    for name, arr in (("n", n), ("p", p), ("albedo", alb), ("irr_s", irr)):
        key = {"n": "normal", "p": "pos"}.get(name, name)
        for idx in ((0, 0), (3, 2)):
            q = arr.copy()
            q[idx] += h
            fp = f(**{name: q})
            q[idx] -= 2 * h
            fm = f(**{name: q})
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gr[key][idx]) < 1e-6 * max(1.0, abs(fd)), (name, idx, fd, gr[key][idx])


def test_filter_adjoint_identity():
    rng = np.random.default_rng(1)
    S, Si, Sp, L = 8, 4, 4, 3
    x = rng.standard_normal((6, S, S, 3))
    gi = rng.standard_normal((6, Si, Si, 3))
    gp = rng.standard_normal((L, 6, Sp, Sp, 3))
    irr, pref = P.ibl_filter(x, Si, Sp, L)
    gx = P.ibl_filter_bwd(S, Si, Sp, L, gi, gp)
    lhs = (irr * gi).sum() + (pref * gp).sum()
    assert abs(lhs - (x * gx).sum()) < 1e-10 * abs(lhs)
