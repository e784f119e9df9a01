"""Pins for the oracle of the optimisation loop: the fan-averaged Laplacian
against an independent 1-ring construction, invariants and brute-force
finite differences; Adam against its closed-form first step and against
torch.optim.Adam (a library routine) over many steps."""
import numpy as np
import torch

from oracle import optim as oo
from paper_2204_01386_amd import scenes


def test_laplacian_is_umbrella_on_closed_mesh():
    """On a closed manifold mesh delta_v = p_v - mean of the 1-ring, with the
    1-ring taken from the mesh's unique edges."""
    p, tris = scenes.noisy_sphere(2, 3)
    p = p.astype(np.float64)
    V = p.shape[0]
    ring = [set() for _ in range(V)]
    for a, b, c in tris:
        for x, y in ((a, b), (b, c), (c, a)):
            ring[x].add(y)
            ring[y].add(x)
    ref = np.stack([p[v] - p[sorted(ring[v])].mean(0) for v in range(V)])
    d = oo.laplacian_matrix(tris, V) @ p.astype(np.float64)
    assert np.abs(d - ref).max() < 1e-12


def test_laplacian_invariants():
    """Rows sum to zero (translations are free); the interior of a flat,
    affinely mapped regular grid has delta = 0; an isolated vertex has 0."""
    p, tris = scenes.noisy_sphere(2, 4)
    V = p.shape[0]
    L = oo.laplacian_matrix(tris, V)
    assert np.abs(L @ np.ones(V)).max() < 1e-12
    R0, g0 = oo.laplacian_reg(p, tris, 0.7)
    R1, g1 = oo.laplacian_reg(p + np.array([0.3, -2.0, 5.0]), tris, 0.7)
    assert abs(R0 - R1) < 1e-12 * R0 and np.abs(g0 - g1).max() < 1e-12
    nu, nv = 12, 9
    A = np.array([[1.0, 0.3, 0.2], [-0.4, 2.0, 0.5]])

    def plane(U, Vv):
        return np.stack([U, Vv], -1) @ A + np.array([0.1, 0.2, 0.3])
    pos, gt, U, Vv = scenes.grid_surface(nu, nv, plane, wrap_v=False)
    d = oo.laplacian_matrix(gt, pos.shape[0]) @ pos
    rows = nv + 1
    i, j = np.arange(pos.shape[0]) // rows, np.arange(pos.shape[0]) % rows
    interior = (i >= 2) & (i <= nu - 3) & (j >= 1) & (j <= nv - 1)
    assert interior.sum() > 40 and np.abs(d[interior]).max() < 1e-12
    assert np.abs(d[~interior]).max() > 1e-3   # the seam and rim are not flat neighbourhoods
    # an extra vertex in no triangle
    Lx = oo.laplacian_matrix(tris, V + 1)
    assert Lx[V].nnz == 0 or np.abs(Lx[V].toarray()).max() == 0


def test_laplacian_gradient_finite_differences():
    p, tris = scenes.noisy_sphere(1, 5)
    lam = 1.3
    _, g = oo.laplacian_reg(p, tris, lam)
    rng = np.random.default_rng(0)
    h = 1e-6
    for v, c in zip(rng.integers(0, p.shape[0], 12), rng.integers(0, 3, 12)):
        q = p.astype(np.float64).copy()
        q[v, c] += h
        Rp, _ = oo.laplacian_reg(q, tris, lam)
        q[v, c] -= 2 * h
        Rm, _ = oo.laplacian_reg(q, tris, lam)
        fd = (Rp - Rm) / (2 * h)
        assert abs(fd - g[v, c]) <= 1e-6 * max(1.0, abs(g[v, c])), (v, c, fd, g[v, c])


def test_adam_first_step_closed_form():
    """At t = 1 the bias corrections give m^ = g, v^ = g^2: the step is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p, g = rng.standard_normal(50), rng.standard_normal(50)
    z = np.zeros(50)
    p1, m1, v1 = oo.adam(p, g, z, z, 1, 0.01, 0.9, 0.999, 1e-8)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(200)
    grads = rng.standard_normal((25, 200))
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=0.02, betas=(0.8, 0.99), eps=1e-6)
    p, m, v = p0.copy(), np.zeros(200), np.zeros(200)
    for t in range(1, 26):
        opt.zero_grad()
        tp.grad = torch.tensor(grads[t - 1])
        opt.step()
        p, m, v = oo.adam(p, grads[t - 1], m, v, t, 0.02, 0.8, 0.99, 1e-6)
    assert np.abs(p - tp.detach().numpy()).max() < 1e-12


def test_lap_weight_schedule():
    assert oo.lap_weight(2.0, 0.5, 0) == 2.0 and oo.lap_weight(2.0, 0.5, 3) == 0.25
