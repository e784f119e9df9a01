"""Oracle of the optimisation loop around the render step (test
infrastructure: only the tests, smoke() and the benchmark's CPU baseline use
anything under oracle/).  Plain NumPy/SciPy in float64, written from the
definitions below; it shares nothing with the GPU library.

The paper optimises vertex positions with Adam under a scheduled Laplacian
regulariser, then the albedo texture with Adam (§4.1, the cross-platform
application; §4.2 and §4.3 use the same regulariser), but gives neither the
Laplacian's weights nor the schedule.  The readings taken here:

* Laplacian.  For vertex v with triangle fan F(v),
      delta_v = p_v - 1 / (2 |F(v)|) * sum over t in F(v) of the two other
                corners of t,
  i.e. every fan triangle weighs the same.  On a closed manifold mesh every
  1-ring neighbour lies in exactly two fan triangles, so delta_v is p_v minus
  the mean of its 1-ring (the uniform "umbrella" Laplacian).  A vertex in no
  triangle has delta_v = 0.
  Regulariser R = lam / V * sum_v |delta_v|^2, with lam = lam0 * gamma^i at
  iteration i (i = steps already taken by the positions' optimiser).
* Adam: Kingma & Ba (2015), Algorithm 1, with t the 1-based step number:
      m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
      m^ = m / (1 - b1^t),  v^ = v / (1 - b2^t),  p <- p - lr m^ / (sqrt(v^) + eps).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def laplacian_matrix(tris: np.ndarray, V: int) -> sp.csr_matrix:
    """L = I - A as a sparse float64 matrix, delta = L @ pos (fan-averaged
    umbrella operator as defined above)."""
    tris = np.asarray(tris, np.int64)
    rows, cols, vals = [], [], []
    fan = np.bincount(tris.ravel(), minlength=V).astype(np.float64)
    for i in range(3):
        v = tris[:, i]
        for j in (1, 2):
            u = tris[:, (i + j) % 3]
            rows.append(v)
            cols.append(u)
            vals.append(-0.5 / fan[v])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(V, V))
    diag = (fan > 0).astype(np.float64)
    return (sp.diags(diag) + A).tocsr()


def laplacian_reg(pos: np.ndarray, tris: np.ndarray, lam: float):
    """(R, dR/dpos) of R = lam / V * sum_v |delta_v|^2."""
    V = pos.shape[0]
    L = laplacian_matrix(tris, V)
    p = np.asarray(pos, np.float64)
    d = L @ p
    R = lam / V * float((d * d).sum())
    g = 2.0 * lam / V * (L.T @ d)
    return R, g


def lap_weight(lam0: float, gamma: float, i: int) -> float:
    """The scheduled regulariser weight at iteration i."""
    return lam0 * gamma ** i


def adam(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t = 1-based step number); returns new (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
