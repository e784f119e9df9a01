"""Texture-only steps on fixed geometry (the rasterization, interpolated
attributes and the albedo texture's inverse-UV map computed once and reused):
the split inverse-UV entry points give bitwise what the one-call texture
backward gives, and a texture-only step gives bitwise the full step's image,
loss and texture gradients, also after the textures changed, eager and
replayed as a graph; its texture gradient matches the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from oracle import step as ostep
from paper_2204_01386_amd import scenes
from test_gpu_parity import assert_grad_close, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_01386_amd import binding
    return binding


CASES = ["2d_repeat_clamp", "2d_clamp", "2d_repeat", "cube", "empty_slice"]


@pytest.mark.parametrize("case", CASES)
def test_invuv_split_matches_texture_bwd(B, case):
    rng = np.random.default_rng(CASES.index(case))
    S, H, W = 3, 37, 29
    tid = rng.integers(-1, 5, (S, H, W)).astype(np.int32)
    if case == "cube":
        tex = rng.random((6, 16, 16, 3)).astype(np.float32)
        coord = rng.standard_normal((S, H, W, 3)).astype(np.float32)
        kw = dict(kind=B.TEX_CUBE)
    else:
        wrap = {"2d_repeat_clamp": (0, 1), "2d_clamp": (1, 1), "2d_repeat": (0, 0), "empty_slice": (0, 1)}[case]
        tex = rng.random((33, 40, 4)).astype(np.float32)
        coord = rng.uniform(-0.3, 1.3, (S, H, W, 2)).astype(np.float32)
        kw = dict(kind=B.TEX_2D, wrap_u=wrap[0], wrap_v=wrap[1])
        if case == "empty_slice":
            tid[1] = -1
    g = rng.standard_normal(coord.shape[:-1] + (tex.shape[-1],)).astype(np.float32)
    ref, _ = B.dressi_texture_bwd(dev(tex), dev(coord), dev(tid), dev(g), need_coord=False, **kw)
    inv = B.dressi_invuv_build(dev(tex), dev(coord), dev(tid), **kw)
    gt = B.dressi_texture_grad_invuv(dev(tex), dev(coord), dev(tid), inv, dev(g), **kw)
    assert np.array_equal(host(gt), host(ref))
    # the map is only read: a second gather with other gradients is exact too
    g2 = rng.standard_normal(g.shape).astype(np.float32)
    ref2, _ = B.dressi_texture_bwd(dev(tex), dev(coord), dev(tid), dev(g2), need_coord=False, **kw)
    assert np.array_equal(host(B.dressi_texture_grad_invuv(dev(tex), dev(coord), dev(tid), inv, dev(g2), **kw)),
                          host(ref2))
    # the map is the oracle's, bit-exact
    F, Ht, Wt = (6, tex.shape[1], tex.shape[2]) if case == "cube" else (1, tex.shape[0], tex.shape[1])
    cells = host(inv).reshape(S, F, Ht, Wt)
    want = oracle.invuv_build(tex.shape, coord, tid, **kw)
    assert np.array_equal(cells, want.reshape(S, F, Ht, Wt)), "inverse-UV cells differ from the oracle's"
    if case == "empty_slice":
        assert (cells[1] == -1).all()


def test_invuv_errors(B):
    tex = torch.zeros((8, 8, 4), device="cuda")
    coord = torch.zeros((1, 4, 4, 2), device="cuda")
    tid = torch.zeros((1, 4, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(B.DressiError):
        B.dressi_invuv_build(tex, coord, None)
    inv = B.dressi_invuv_build(tex, coord, tid)
    with pytest.raises(ValueError):
        B.dressi_texture_grad_invuv(tex, coord, tid, inv[:-1], torch.zeros((1, 4, 4, 4), device="cuda"))
    with pytest.raises(B.DressiError):   # repeat wrap needs 3 texels
        B.dressi_invuv_build(torch.zeros((2, 2, 4), device="cuda"), coord, tid)


def _texture_state(st):
    g = st.grads()
    out = {"rgba": host(st.rgba()).copy(), "loss": host(st.loss).copy(), "tex": host(g["tex"]).copy()}
    if "env" in g:
        out["env"] = host(g["env"]).copy()
    return out


def _assert_same(a, b, what):
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"


def _scene(name):
    if name == "config2_small":
        return scenes.config2(H=128, subdiv=4, tex_size=256)
    return scenes.config3(n_views=3, subdiv=4, H=128, tex_size=256, env_size=16)


@pytest.mark.parametrize("name", ["config2_small", "config3_small"])
def test_texture_step_matches_full_step(B, name):
    from paper_2204_01386_amd.pipeline import Step, TextureStep, make_target
    s = _scene(name)
    st = Step(s, target=make_target(s))
    st.run()
    torch.cuda.synchronize()
    full = _texture_state(st)
    ts = TextureStep(st)
    ts.run()
    torch.cuda.synchronize()
    _assert_same(full, _texture_state(ts.st), "texture-only step")
    # a gradient step on the textures: the cache stays valid
    with torch.no_grad():
        st.tex.sub_(0.5 * st.g_tex)
        if st.env is not None:
            st.env.sub_(0.5 * st.g_envtex)
    st.run()
    torch.cuda.synchronize()
    full2 = _texture_state(st)
    assert not np.array_equal(full2["rgba"], full["rgba"])
    ts.run()
    torch.cuda.synchronize()
    _assert_same(full2, _texture_state(ts.st), "texture-only step after an update")


def test_texture_step_config2_oracle(B):
    """The texture-only gradient of the config-2 step (512^2, 81,920
    triangles, 1024^2 texture) against the oracle's."""
    from paper_2204_01386_amd.pipeline import Step, TextureStep, make_target
    s = scenes.config2()
    st = Step(s, target=make_target(s))
    ts = TextureStep(st)
    ts.run()
    torch.cuda.synchronize()
    _, _, o_g = ostep.step(s)
    assert_grad_close(host(ts.grads()["tex"]), o_g["tex"], what="grad texture (texture-only step)")
    L = float(host(st.loss)[0])
    assert abs(L - o_g["loss"]) <= 1e-5 * o_g["loss"], (L, o_g["loss"])


@pytest.mark.parametrize("concurrent", [False, "index", True])
def test_texture_step_graph_replay(B, concurrent):
    from paper_2204_01386_amd.pipeline import Step, TextureStep, make_target
    s = _scene("config3_small")
    st = Step(s, target=make_target(s))
    st.concurrent = concurrent
    ts = TextureStep(st)
    ts.run()
    torch.cuda.synchronize()
    ref = _texture_state(st)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ts.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        ts.run()
    for rep in range(3):
        for v in ts.grads().values():
            v.fill_(123.0)
        st.color.fill_(5.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _assert_same(ref, _texture_state(st), f"replay {rep}")


def test_texture_step_uneven_batch(B):
    """Texture-only steps of an uneven batch (texture array, one layer per
    instance): bitwise the full batched step's image, loss and texture
    gradients, before and after a texture update."""
    from paper_2204_01386_amd.pipeline import BatchStep, TextureStep, make_batch_target
    sl = scenes.config4(seed=3, n=5, t_min=200, t_max=2e4, sizes=(128, 256), tex_size=64)
    bs = BatchStep(sl, target=make_batch_target(sl))
    bs.run()
    torch.cuda.synchronize()
    full = _texture_state(bs)
    ts = TextureStep(bs)
    ts.run()
    torch.cuda.synchronize()
    _assert_same(full, _texture_state(bs), "uneven texture-only step")
    with torch.no_grad():
        bs.tex.sub_(0.5 * bs.g_tex)
    bs.run()
    torch.cuda.synchronize()
    full2 = _texture_state(bs)
    ts.run()
    torch.cuda.synchronize()
    _assert_same(full2, _texture_state(bs), "uneven texture-only step after an update")
