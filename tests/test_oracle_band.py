"""Pins of the oracle's edge-band form of the layers (band_layers): the reading
that, outside the blend's edge mask E, only the front hard fragment reaches
the image (§3.4.3: there I = S^H C_1 and the silhouette is S^H).  Checked
against the blend itself: the banded layers give the same image, silhouette
and edge mask as the full layers, and the blend's adjoint is the same on
every kept entry and zero on every emptied one."""
import numpy as np
import pytest

import oracle
from helpers import to_clip
from paper_2204_01386_amd import scenes


def _layers(K, r, H=72, W=88, views=2, seed=3):
    p, tris = scenes.noisy_sphere(3, seed)
    pc = to_clip(p, scenes.view_proj(scenes.camera_ring(views, seed)))
    return oracle.rasterize(pc, tris, H, W, K=K, r=r)


@pytest.mark.parametrize("mode,K,r,delta", [(oracle.BLEND_HSR, 3, 0.05, 0.05), (oracle.BLEND_HSR, 2, 0.06, 0.02),
                                            (oracle.BLEND_AA, 3, 0.05, 0.0), (oracle.BLEND_HARD, 2, 0.05, 0.0)])
def test_band_keeps_the_blend(mode, K, r, delta):
    full = _layers(K, r)
    band = oracle.band_layers(*full, delta, mode)
    rng = np.random.default_rng(K)
    col = rng.random(full[0].shape + (3,))
    sigma = r / 7
    oc_f, os_f, E_f = oracle.softras(col, full[3], full[0], sigma, delta, mode)
    oc_b, os_b, E_b = oracle.softras(col, band[3], band[0], sigma, delta, mode)
    assert np.array_equal(E_f, E_b)
    assert np.array_equal(oc_f, oc_b) and np.array_equal(os_f, os_b)
    gc = rng.standard_normal(oc_f.shape)
    gs = rng.standard_normal(os_f.shape)
    gl_f, gd_f = oracle.softras_bwd(col, full[3], full[0], sigma, E_f, gc, gs)
    gl_b, gd_b = oracle.softras_bwd(col, band[3], band[0], sigma, E_b, gc, gs)
    kept = band[0] >= 0
    assert np.array_equal(gl_b[kept], gl_f[kept]) and np.array_equal(gd_b[kept], gd_f[kept])
    dropped = (full[0] >= 0) & ~kept
    assert dropped.any(), "the band should empty some entries"
    assert not gl_f[dropped].any() and not gd_f[dropped].any(), "an emptied entry had a gradient"
    # inside E nothing changes; outside E only front hard fragments remain
    inE = np.broadcast_to(E_f.astype(bool)[:, None], full[0].shape)
    assert np.array_equal(band[0][inE], full[0][inE])
    out = ~inE
    assert (band[0][:, 1:][out[:, 1:]] == -1).all()
    assert (band[1][:, 0][out[:, 0] & (band[0][:, 0] >= 0)] == 1).all()


def test_band_in_softras_mode_is_the_full_form():
    full = _layers(3, 0.05)
    band = oracle.band_layers(*full, 0.0, oracle.BLEND_SOFTRAS)
    for a, b in zip(full, band):
        assert np.array_equal(a, b)
