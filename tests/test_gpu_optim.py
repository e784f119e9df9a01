"""The optimisation loop on the GPU: Adam and the Laplacian regulariser
against the oracle, the first silhouette iteration's position gradient
against the oracle, and the two-stage fit (positions from silhouettes, then
the albedo texture on the cached geometry): it reduces both losses, and
graph replays of its iterations reproduce the eager loop bit for bit."""
import numpy as np
import pytest
import torch

from oracle import optim as oo
from oracle import step as ostep
from paper_2204_01386_amd import scenes
from test_gpu_parity import assert_grad_close, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_01386_amd import binding
    return binding


U32 = 2.0 ** -24   # unit roundoff of float32


def _within(a, ref, tol, what):
    err = np.abs(a.astype(np.float64) - ref)
    assert (err <= tol).all(), f"{what}: max excess {(err - tol).max():.3e}"


@pytest.mark.parametrize("n", [4096, 1001, 0])
def test_adam_matches_oracle(B, n):
    rng = np.random.default_rng(n)
    p0 = rng.standard_normal(n).astype(np.float32)
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    p, m, v = dev(p0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    state = B.adam_state()
    po, mo, vo = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 8):
        g = (rng.standard_normal(n) * (0.1 if t % 2 else 3.0)).astype(np.float32)
        if n:
            g[: n // 10] = 0.0          # parameters without gradient
        B.dressi_adam(p, dev(g), m, v, state, lr, b1, b2, eps)
        # the oracle continues from the GPU's float32 parameters and moments
        # (each step's rounding is checked, not a drift over steps)
        pp, mp, vp = host(p).astype(np.float64), host(m).astype(np.float64), host(v).astype(np.float64)
        # the hyperparameters cross the ABI as float32: the oracle takes those values
        f = lambda x: float(np.float32(x))
        fl, f1, f2, fe = f(lr), f(b1), f(b2), f(eps)
        po_n, mo_n, vo_n = oo.adam(po, g, mo, vo, t, fl, f1, f2, fe)
        # float32 error bounds of each update (two products and a sum, which
        # can cancel for m), and of the parameter step through m's error
        tol_m = 3 * U32 * (np.abs(f1 * mo) + np.abs((1 - f1) * g))
        tol_v = 3 * U32 * (f2 * vo + (1 - f2) * g.astype(np.float64) ** 2)
        c1, c2 = 1 - f1 ** t, 1 - f2 ** t
        den = np.sqrt(vo_n / c2) + fe
        step = fl * np.abs(mo_n) / c1 / den
        tol_p = 2 * U32 * np.abs(po_n) + 10 * U32 * step + fl * tol_m / c1 / den
        _within(pp, po_n, tol_p, f"param, step {t}")
        _within(mp, mo_n, tol_m, f"m, step {t}")
        _within(vp, vo_n, tol_v, f"v, step {t}")
        po, mo, vo = pp, mp, vp
    assert int(host(state)[0]) == 7


def test_adam_rejects_bad_arguments(B):
    p = torch.zeros(8, device="cuda")
    with pytest.raises(B.DressiError):
        B.dressi_adam(p, p, p.clone(), p.clone(), B.adam_state(), 0.01, beta1=1.0)
    with pytest.raises(B.DressiError):
        B.dressi_adam(p, p, p.clone(), p.clone(), B.adam_state(), 0.01, eps=0.0)


@pytest.mark.parametrize("mesh", ["noisy_sphere", "fit_target", "torus_open"])
def test_laplacian_matches_oracle(B, mesh):
    if mesh == "noisy_sphere":
        p, tris = scenes.noisy_sphere(3, 2)
    elif mesh == "fit_target":
        s = scenes.fit_scene()
        p, tris = s.target_pos, s.tris
    else:
        # an open grid (a torus cut open along v) with an unused extra vertex
        p, tris, _, _ = scenes.grid_surface(24, 9, lambda U, V: np.stack(
            [np.cos(6.28 * U) * (1 + 0.3 * V), 0.5 * V, np.sin(6.28 * U) * (1 + 0.3 * V)], -1), wrap_v=False)
        p = np.concatenate([p, [[5.0, 5.0, 5.0]]]).astype(np.float32)
    p = p.astype(np.float32)
    V = p.shape[0]
    rng = np.random.default_rng(V)
    gin = rng.standard_normal((V, 3)).astype(np.float32)
    lam0, gamma, t = 2.5, 0.9, 3
    state = B.adam_state()
    state[0] = t
    g, val = B.dressi_laplacian_reg(dev(p), dev(tris), lam0, gamma, state, grad_in=dev(gin))
    R, gr = oo.laplacian_reg(p, tris, oo.lap_weight(lam0, gamma, t))
    assert abs(float(host(val)[0]) - R) <= 1e-6 * R, (float(host(val)[0]), R)
    assert_grad_close(host(g), gr + gin, what="laplacian grad + grad_in")
    g0, _ = B.dressi_laplacian_reg(dev(p), dev(tris), lam0, gamma, state)
    assert_grad_close(host(g0), gr, what="laplacian grad")
    # in place, with the adjacency given: bitwise the same
    adj = B.dressi_adjacency(dev(tris), V)
    gi = dev(gin)
    B.dressi_laplacian_reg(dev(p), dev(tris), lam0, gamma, state, grad_in=gi, adj=adj)
    ctx = B.context()
    from paper_2204_01386_amd.pipeline import _p
    pd, td, vbuf = dev(p), dev(tris), torch.empty(1, device="cuda")
    ctx.check(B._lib.dressi_laplacian_reg(ctx.handle, _p(pd), _p(td), V, tris.shape[0], _p(adj), lam0, gamma,
                                          _p(state), _p(gi), _p(gi), _p(vbuf), B._stream()), "in place")
    assert np.array_equal(host(gi), host(g))
    # no schedule state: lam = lam0
    _, v0 = B.dressi_laplacian_reg(dev(p), dev(tris), lam0, gamma, None, need_grad=False)
    R0, _ = oo.laplacian_reg(p, tris, lam0)
    assert abs(float(host(v0)[0]) - R0) <= 1e-6 * R0


def _fit_loop(scene):
    from paper_2204_01386_amd.pipeline import FitLoop, Step, make_target
    st = Step(scene, target=make_target(scene))
    return FitLoop(st)


def _sil_l2(st):
    return float(((st.sil - st.target[..., 3]) ** 2).mean().item())


def _col_l2(st):
    m = st.target[..., 3:4] > 0
    return float((((st.color - st.target[..., :3]) ** 2) * m).sum().item() / max(1, int(m.sum().item())))


def test_first_silhouette_iteration_gradient_matches_oracle(B):
    """Silhouette-only image gradient (the oracle's loss against a target
    whose colour equals its own render, so only the silhouette residual
    remains) plus the regulariser's gradient, before the Adam update."""
    from paper_2204_01386_amd.pipeline import _p
    s = scenes.fit_scene(subdiv=3, H=128)
    fl = _fit_loop(s)
    st = fl.st
    st.forward()
    st.loss_and_grad()
    st.g_color.zero_()
    st.backward()
    ctx = st.ctx
    ctx.check(B._lib.dressi_laplacian_reg(ctx.handle, _p(st.pos), _p(st.tris), st.V, st.T, _p(st.adj), fl.lap0,
                                          fl.lap_gamma, _p(fl.adam_pos.state), _p(st.g_pos), _p(st.g_pos),
                                          _p(fl.reg), B._stream()), "laplacian")
    torch.cuda.synchronize()
    tgt = ostep.forward(s, target=True)["rgba"]
    o = ostep.forward(s)
    tgt = tgt.copy()
    tgt[..., :3] = o["color"]
    og = ostep.backward(s, o, tgt)
    _, lg = oo.laplacian_reg(s.pos, s.tris, fl.lap0)
    assert np.array_equal(host(st.tri_id), o["tid"]), "tri_id differs"
    assert np.abs(og["pos"]).max() > 0
    assert_grad_close(host(st.g_pos), og["pos"] + lg, what="silhouette-stage position gradient")


def test_fit_loop_converges_and_replays(B):
    s = scenes.fit_scene()
    n_sil, n_tex = 150, 60
    # eager
    fl = _fit_loop(s)
    st = fl.st
    st.forward()
    sil0 = _sil_l2(st)
    for _ in range(n_sil):
        fl.silhouette_iteration()
    st.forward()
    torch.cuda.synchronize()
    sil1 = _sil_l2(st)
    fl.start_texture_stage()
    fl.ts.forward()
    col0 = _col_l2(st)
    for _ in range(n_tex):
        fl.texture_iteration()
    fl.ts.forward()
    torch.cuda.synchronize()
    col1 = _col_l2(st)
    assert fl.adam_pos.steps_taken() == n_sil and fl.adam_tex.steps_taken() == n_tex
    assert sil1 < 0.25 * sil0, (sil0, sil1)
    assert col1 < 0.5 * col0, (col0, col1)
    eager_pos, eager_tex = host(st.pos).copy(), host(st.tex).copy()
    # the same loop as graph replays, from the same start
    fl2 = _fit_loop(s)
    st2 = fl2.st
    fl2.silhouette_iteration()     # eager warm-up: sizes the scratch
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fl2.silhouette_iteration()
    for _ in range(n_sil - 1):     # the capture itself runs nothing
        g.replay()
    torch.cuda.synchronize()
    assert fl2.adam_pos.steps_taken() == n_sil
    assert np.array_equal(host(st2.pos), eager_pos), "silhouette stage: graph replays differ from eager"
    fl2.start_texture_stage()
    fl2.texture_iteration()
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        fl2.texture_iteration()
    for _ in range(n_tex - 1):
        g2.replay()
    torch.cuda.synchronize()
    assert np.array_equal(host(st2.tex), eager_tex), "texture stage: graph replays differ from eager"
    assert B.context().check_status() == 0
