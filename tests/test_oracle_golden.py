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
