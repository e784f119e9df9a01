"""Pins of the oracle's HardSoftRas blend against the constants the paper fixes
(tests/golden/hardsoftras_constants.json, each with its citation)."""
import json
import math
import os

import numpy as np

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hardsoftras_constants.json")))


def test_golden_sigmoid_values_are_the_closed_form():
    b = GOLD["blend"]
    assert abs(b["D_at_plus_r"] - 1 / (1 + math.exp(-7))) < 1e-15
    assert abs(b["D_at_minus_r"] - 1 / (1 + math.exp(7))) < 1e-15
    assert abs(b["sigma_over_r"] - 1 / 7) < 1e-15


def test_blend_probability_at_the_soft_reach():
    """One soft layer at distance r from its face (SoftRas mode: every pixel
    an edge pixel, K=1): the silhouette is D = sigmoid(dist / sigma) with
    sigma = r/7, i.e. sigmoid(+-7) at dist = +-r."""
    b = GOLD["blend"]
    r = b["r"]
    sigma = r * b["sigma_over_r"]
    tid = np.zeros((1, 1, 1, 2), np.int32)
    dist = np.array([[[[r, -r]]]], np.float64)
    col = np.full((1, 1, 1, 2, 3), 0.5)
    _, sil, E = oracle.softras(col, dist, tid, sigma, r, oracle.BLEND_SOFTRAS)
    assert (E == 1).all()
    assert abs(sil[0, 0, 0] - b["D_at_plus_r"]) < 1e-12
    assert abs(sil[0, 0, 1] - b["D_at_minus_r"]) < 1e-12


def test_shift_keys_order_the_oracle_layers():
    """The four Shift-equation entries of the golden file (§3.4.2), built as
    four triangles over one pixel p of a 250 x 250 image (one screen unit =
    250 pixels): two faces covering p at depths 0.3 (50 px inside) and 0.9
    (p exactly on its left edge, which the fill rule owns), and two faces
    missing p by 1 px (|dist| = 0.004) and by 250 px (|dist| = 1, reach r = 1).
    The oracle's K = 4 layers at p must come in the order of the golden keys,
    with the golden signed distances (+ hard, - soft, +0 on the edge)."""
    from helpers import screen_to_clip
    sh = GOLD["shift"]
    for e in sh:   # the file's keys are the Shift equation of its own entries
        key = 0.5 * e["depth"] if e["dist"] >= 0 else 0.5 * abs(e["dist"]) + 0.5
        assert abs(key - e["key"]) < 1e-12
    H = W = 250
    px, py = 125, 125
    faces = {   # golden entry -> (pixel-space corners, depth)
        0: ([(75.5, 75.5), (475.5, 75.5), (75.5, 475.5)], sh[0]["depth"]),
        1: ([(125.5, -100.0), (125.5, 350.0), (400.0, 125.5)], sh[1]["depth"]),
        2: ([(126.5, 100.5), (126.5, 150.5), (200.5, 125.5)], sh[2]["depth"]),
        3: ([(375.5, -200.0), (375.5, 450.0), (700.0, 125.5)], sh[3]["depth"]),
    }
    order = [3, 1, 2, 0]          # triangle t draws golden entry order[t]
    xy = np.concatenate([np.array(faces[e][0]) for e in order])
    z = np.repeat([faces[e][1] for e in order], 3)
    pc = screen_to_clip(xy, H, W, z=z, w=1.0)
    tris = np.arange(12, dtype=np.int32).reshape(4, 3)
    tid, hard, _, dist = oracle.rasterize(pc, tris, H, W, K=4, r=1.0)
    want = np.argsort([e["key"] for e in sh])            # entries by key
    got = [order[t] for t in tid[0, :, py, px]]
    assert got == list(want), got
    for k, e in enumerate(np.array(sh)[want]):
        d = dist[0, k, py, px]
        assert abs(d - e["dist"]) <= 1e-6, (k, d, e)
        assert bool(hard[0, k, py, px]) == (e["dist"] >= 0)
        assert np.signbit(d) == (e["dist"] < 0)          # +0 on the owned edge
