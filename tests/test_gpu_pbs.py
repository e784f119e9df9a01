"""Image-based PBS on the GPU against the oracle: the irradiance and GGX
prefilter convolutions and their exact adjoint, the BRDF integration table,
and split-sum shading forward and backward (lookup directions, per-level
masks, every gradient including the material's scalars)."""
import numpy as np
import pytest
import torch

from oracle import pbs as OP
from test_gpu_parity import assert_grad_close, assert_vals_close, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2204_01386_amd import binding
    return binding


@pytest.mark.parametrize("S,Si,Sp,L", [(16, 4, 8, 4), (12, 5, 3, 2)])
def test_ibl_filter_and_adjoint(B, S, Si, Sp, L):
    rng = np.random.default_rng(S + L)
    env = rng.random((6, S, S, 3)).astype(np.float32)
    irr, pref, norm = B.dressi_ibl_filter(dev(env), Si, Sp, L)
    irr_o, pref_o = OP.ibl_filter(env, Si, Sp, L)
    assert_vals_close(host(irr), irr_o, what="irradiance")
    assert_vals_close(host(pref), pref_o, what="prefiltered")
    gi = rng.standard_normal(irr_o.shape).astype(np.float32)
    gp = rng.standard_normal(pref_o.shape).astype(np.float32)
    ge = B.dressi_ibl_filter_bwd(S, norm, dev(gi), dev(gp))
    assert_grad_close(host(ge), OP.ibl_filter_bwd(S, Si, Sp, L, gi, gp), what="environment gradient")


def test_brdf_lut(B):
    lut = B.dressi_brdf_lut(16, 128)
    ref = OP.brdf_lut(16, 128)
    assert np.abs(host(lut) - ref).max() < 1e-6


def _frags(rng, Bv, Npv, L):
    n = rng.standard_normal((Bv, Npv, 3))
    n[..., 2] = np.abs(n[..., 2]) + 0.2
    p = 0.4 * rng.standard_normal((Bv, Npv, 3))
    eye = np.stack([[0.3, 0.5, 3.0], [-0.4, 0.2, 2.7]])[:Bv]
    alb = rng.uniform(0.05, 0.95, (Bv, Npv, 3))
    irr = rng.uniform(0.05, 1.0, (Bv, Npv, 3))
    pref = rng.uniform(0.05, 1.0, (L, Bv, Npv, 3))
    tid = rng.integers(-1, 40, (Bv, Npv)).astype(np.int32)
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return f32(n), f32(p), f32(eye), f32(alb), f32(irr), f32(pref), tid


@pytest.mark.parametrize("m,r", [(0.3, 0.37), (0.8, 0.9), (0.0, 1.0), (0.5, 0.0), (0.4, -0.2), (0.4, 1.3)])
def test_shade_pbs_forward_and_backward(B, m, r):
    rng = np.random.default_rng(int(100 * (m + r)))
    Bv, Npv, L = 2, 700, 5
    n, p, eye, alb, irr, pref, tid = _frags(rng, Bv, Npv, L)
    lut = OP.brdf_lut(8, 256).astype(np.float32)
    mat = np.array([m, r], np.float32)
    N = Bv * Npv
    t = {k: dev(v) for k, v in dict(n=n.reshape(N, 3), p=p.reshape(N, 3), a=alb.reshape(N, 3),
                                     i=irr.reshape(N, 3), pr=pref.reshape(L, N, 3), m=mat, lut=lut,
                                     eye=eye, tid=tid.reshape(N)).items()}
    pin = B.pbs_in(t["n"], t["p"], t["m"], t["lut"], albedo=t["a"], irr=t["i"], pref=t["pr"])
    ctx = B.context()
    dir_n = torch.empty((N, 3), device="cuda")
    dir_r = torch.empty((N, 3), device="cuda")
    ltid = torch.empty((L, N), dtype=torch.int32, device="cuda")
    col = torch.empty((N, 3), device="cuda")
    P = lambda x: B._ptr(x)
    ctx.check(B._lib.dressi_shade_pbs(ctx.handle, B.C.byref(pin), P(t["eye"]), P(t["tid"]), Bv, Npv, P(col),
                                      P(dir_n), P(dir_r), P(ltid), B._stream()), "shade_pbs")
    # oracle, one eye per fragment
    eye_f = np.repeat(eye[:, None, :], Npv, 1)
    g = rng.standard_normal((Bv, Npv, 3))
    out_o, gr = OP.shade_and_grads(n, p, eye_f, alb, m, r, irr, pref, lut.astype(np.float64), L, tid, g)
    cov = tid >= 0
    assert_vals_close(host(col).reshape(Bv, Npv, 3), out_o, what="pbs colour")
    assert np.abs(host(dir_n).reshape(Bv, Npv, 3)[cov] - gr["dir_n"][cov]).max() < 1e-6
    assert np.abs(host(dir_r).reshape(Bv, Npv, 3)[cov] - gr["dir_r"][cov]).max() < 1e-6
    l0 = min(int(np.floor(min(max(r, 0.0), 1.0) * (L - 1))), L - 2)
    want = np.where(cov[None], tid[None], -1).repeat(L, 0)
    for l in range(L):
        if l not in (l0, l0 + 1):
            want[l] = -1
    assert np.array_equal(host(ltid).reshape(L, Bv, Npv), want)
    # backward, with direction gradients from the lookups
    gdn = rng.standard_normal((N, 3)).astype(np.float32)
    gdr = rng.standard_normal((L, N, 3)).astype(np.float32)
    outs = {k: torch.empty((N, 3), device="cuda") for k in ("normal", "pos", "albedo", "irr")}
    gpref = torch.empty((L, N, 3), device="cuda")
    gmat = torch.empty(2, device="cuda")
    pg = B.PbsGrad()
    pg.normal, pg.normal_stride = P(outs["normal"]), 3
    pg.pos, pg.pos_stride = P(outs["pos"]), 3
    pg.albedo, pg.albedo_stride = P(outs["albedo"]), 3
    pg.irr, pg.pref, pg.material = P(outs["irr"]), P(gpref), P(gmat)
    # (device copies kept alive: a pointer of a temporary tensor could be
    # handed to the next allocation before the kernel runs)
    gd = dev(g.reshape(N, 3).astype(np.float32))
    tgdn, tgdr = dev(gdn), dev(gdr)
    ctx.check(B._lib.dressi_shade_pbs_bwd(ctx.handle, B.C.byref(pin), P(t["eye"]), P(t["tid"]), Bv, Npv, P(gd),
                                          P(tgdn), P(tgdr), B.C.byref(pg), B._stream()), "shade_pbs_bwd")
    # the oracle with the same float32 output gradient
    _, gr = OP.shade_and_grads(n, p, eye_f, alb, m, r, irr, pref, lut.astype(np.float64), L, tid,
                               g.astype(np.float32))
    vn, vp = OP.dirs_vjp(n, p, eye_f, gdn.reshape(Bv, Npv, 3).astype(np.float64),
                         gdr.sum(0).reshape(Bv, Npv, 3).astype(np.float64))
    c3 = cov[..., None]
    sh = lambda x: host(x).reshape(Bv, Npv, 3)
    assert_grad_close(sh(outs["albedo"]), gr["albedo"], what="albedo")
    assert_grad_close(sh(outs["irr"]), gr["irr_s"], what="irradiance sample")
    assert_grad_close(host(gpref).reshape(L, Bv, Npv, 3), gr["pref_s"], what="prefiltered samples")
    assert_grad_close(sh(outs["normal"]), gr["normal"] + np.where(c3, vn, 0.0), what="normal")
    assert_grad_close(sh(outs["pos"]), gr["pos"] + np.where(c3, vp, 0.0), what="position")
    gm = host(gmat).astype(np.float64)
    for k, name in enumerate(("metallic", "roughness")):
        ref = gr[name]
        assert abs(gm[k] - ref) <= 1e-5 * max(abs(ref), 1e-3), (name, gm[k], ref)


def test_pbs_step_matches_oracle(B):
    """The whole PBS step on fixed geometry (2 views 64^2, HardSoftRas K = 2):
    image, loss and the gradients of the environment map, the material and
    the albedo texture against the oracle's step."""
    from paper_2204_01386_amd import scenes
    from paper_2204_01386_amd.pipeline import PbsStep
    s = scenes.fit_scene(subdiv=3, H=64, n_views=2, tex_size=64)
    env_t = scenes.cube_env_map(8, 5)
    env0 = np.full_like(env_t, 0.5)
    Si, Sp, L, N, M = 4, 8, 4, 16, 128
    mat_t, mat0 = np.array([0.7, 0.3], np.float32), np.array([0.4, 0.6], np.float32)
    tgt = PbsStep(s, env_t, mat_t, Si, Sp, L, N, M, params={"tex": torch.from_numpy(s.target_tex).cuda()})
    tgt.forward()
    ps = PbsStep(s, env0, mat0, Si, Sp, L, N, M, target=tgt)
    ps.run()
    torch.cuda.synchronize()
    lut = OP.brdf_lut(N, M)
    t_o = OP.pbs_forward(s, env_t, mat_t, s.target_tex, Si, Sp, L, lut)
    f, g = OP.pbs_step(s, env0, mat0, s.tex, t_o["rgba"], Si, Sp, L, lut)
    assert np.array_equal(host(ps.st.tri_id), f["tid"])
    assert_vals_close(host(tgt.rgba()), t_o["rgba"], what="target image")
    assert_vals_close(host(ps.rgba()), f["rgba"], what="image")
    Lg = float(host(ps.st.loss)[0])
    assert abs(Lg - g["loss"]) <= 1e-5 * g["loss"], (Lg, g["loss"])
    assert_grad_close(host(ps.g_env), g["env"], what="environment gradient")
    assert_grad_close(host(ps.st.g_tex), g["tex"], what="albedo texture gradient")
    gm = host(ps.g_material).astype(np.float64)
    assert np.abs(gm - g["material"]).max() <= 1e-4 * np.abs(g["material"]).max(), (gm, g["material"])


def test_new_entry_points_empty_and_rejected(B):
    """Empty inputs do nothing (or write the empty sum); bad arguments are
    rejected before any launch."""
    ctx = B.context()
    P, S = B._ptr, B._stream()
    # the Laplacian of an empty mesh: value 0
    val = torch.full((1,), 7.0, device="cuda")
    ctx.check(B._lib.dressi_laplacian_reg(ctx.handle, None, None, 0, 0, None, 1.0, 1.0, None, None, None, P(val),
                                          S), "empty laplacian")
    torch.cuda.synchronize()
    assert float(val.item()) == 0.0
    # shading of no fragment: nothing written, the material gradient is 0
    pin = B.PbsIn()
    pin.levels = 2
    pg = B.PbsGrad()
    gm = torch.full((2,), 3.0, device="cuda")
    pg.material = P(gm)
    assert B._lib.dressi_shade_pbs(ctx.handle, B.C.byref(pin), None, None, 0, 0, None, None, None, None, S) == 0
    assert B._lib.dressi_shade_pbs_bwd(ctx.handle, B.C.byref(pin), None, None, 0, 0, None, None, None,
                                       B.C.byref(pg), S) == 0
    torch.cuda.synchronize()
    assert (gm == 0).all()
    # an inverse-UV map of zero slices
    tex = torch.zeros((8, 8, 4), device="cuda")
    inv = B.dressi_invuv_build(tex, torch.zeros((0, 4, 4, 2), device="cuda"),
                               torch.zeros((1, 4, 4), dtype=torch.int32, device="cuda"))
    assert inv.numel() == 0
    # rejected descriptors and sizes
    bad = B.IblDesc(8, 4, 4, 1)   # L < 2
    e = torch.zeros((6, 8, 8, 3), device="cuda")
    assert B._lib.dressi_ibl_filter(ctx.handle, P(e), B.C.byref(bad), P(e), P(e), P(e), S) == B.EINVAL
    assert B._lib.dressi_brdf_lut(ctx.handle, 0, 16, P(e), S) == B.EINVAL
    pin.levels = 1
    pin.normal, pin.normal_stride, pin.pos, pin.pos_stride, pin.material = P(e), 3, P(e), 3, P(e)
    assert B._lib.dressi_shade_pbs(ctx.handle, B.C.byref(pin), P(e), P(e), 1, 4, None, P(e), None, None,
                                   S) == B.EINVAL
    mis = torch.zeros(4, dtype=torch.int32, device="cuda")[1:]   # a state not 16-byte aligned
    p = torch.zeros(4, device="cuda")
    assert B._lib.dressi_adam(ctx.handle, P(p), P(p), P(p), P(p), 4, 0.01, 0.9, 0.999, 1e-8, P(mis), S) == B.EINVAL


def test_pbs_autograd_chain_matches_oracle(B):
    """The autograd Functions chained as a renderer would: environment ->
    filters -> lookup directions -> cube lookups (inverse-UV texel gradients
    and coordinate gradients) -> shading; every leaf's gradient against the
    oracle's composition of the same steps."""
    import oracle as O
    from paper_2204_01386_amd import ops
    rng = np.random.default_rng(21)
    Bv, H, W, L, S, Si, Sp = 2, 16, 20, 4, 8, 4, 6
    Npv = H * W
    N = Bv * Npv
    n, p, eye, alb, _, _, tid = _frags(rng, Bv, Npv, L)
    env = rng.uniform(0.05, 1.0, (6, S, S, 3)).astype(np.float32)
    lut = OP.brdf_lut(8, 128).astype(np.float32)
    m, r = 0.6, 0.45
    G = rng.standard_normal((N, 3)).astype(np.float32)
    # GPU, through autograd
    env_t = dev(env).requires_grad_()
    n_t = dev(n.reshape(N, 3)).requires_grad_()
    p_t = dev(p.reshape(N, 3)).requires_grad_()
    a_t = dev(alb.reshape(N, 3)).requires_grad_()
    mat = dev(np.array([m, r], np.float32)).requires_grad_()
    eye_t, tid_t, lut_t = dev(eye), dev(tid.reshape(N)), dev(lut)
    irr, pref = ops.ibl_filter(env_t, Si, Sp, L)
    dn, dr, ltid = ops.pbs_dirs(n_t, p_t, eye_t, tid_t, mat, lut_t, L, Npv)
    cube = lambda tex, d, t: ops.texture(tex, d.view(Bv, H, W, 3), t.view(Bv, H, W), kind=B.TEX_CUBE).view(N, 3)
    irr_s = cube(irr, dn, tid_t)
    pref_s = torch.stack([cube(pref[l], dr, ltid[l]) for l in range(L)])
    col = ops.pbs_shade(n_t, p_t, a_t, irr_s, pref_s, mat, eye_t, tid_t, lut_t, Npv)
    (col * dev(G)).sum().backward()
    # the oracle
    eye_f = np.repeat(eye[:, None, :], Npv, 1)
    cov = tid >= 0
    irr_o, pref_o = OP.ibl_filter(env, Si, Sp, L)
    with torch.no_grad():
        nn_, R_ = OP.pbs_dirs(torch.tensor(n.astype(np.float64)), torch.tensor(p.astype(np.float64)),
                              torch.tensor(eye_f))
    dn32 = np.where(cov[..., None], nn_.numpy(), 0.0).astype(np.float32).reshape(Bv, H, W, 3)
    dr32 = np.where(cov[..., None], R_.numpy(), 0.0).astype(np.float32).reshape(Bv, H, W, 3)
    t3 = tid.reshape(Bv, H, W)
    l0 = min(int(np.floor(float(np.float32(r)) * (L - 1))), L - 2)
    tid_l = [np.where(t3 >= 0, t3, -1) if l in (l0, l0 + 1) else np.full_like(t3, -1) for l in range(L)]
    irr_s_o = OP.cube_sample(irr_o, dn32, t3)
    pref_s_o = np.stack([OP.cube_sample(pref_o[l], dr32, tid_l[l]) for l in range(L)])
    sh = lambda a: a.reshape(Bv, Npv, 3)
    out_o, gr = OP.shade_and_grads(n, p, eye_f, alb, float(np.float32(m)), float(np.float32(r)), sh(irr_s_o),
                                   pref_s_o.reshape(L, Bv, Npv, 3), lut.astype(np.float64), L, tid, sh(G))
    assert_vals_close(host(col.detach()).reshape(Bv, Npv, 3), out_o, what="colour")
    gi = gr["irr_s"].reshape(Bv, H, W, 3)
    gpf = gr["pref_s"].reshape(L, Bv, H, W, 3)
    g_dn = O.texture_bwd_coord(irr_o, dn32, gi, t3, kind=O.TEX_CUBE)
    g_dr = sum(O.texture_bwd_coord(pref_o[l], dr32, gpf[l], tid_l[l], kind=O.TEX_CUBE) for l in range(L))
    vn, vp = OP.dirs_vjp(n, p, eye_f, g_dn.reshape(Bv, Npv, 3), g_dr.reshape(Bv, Npv, 3))
    g_irr = O.texture_bwd_tex(irr_o.shape, dn32, t3, gi, kind=O.TEX_CUBE)
    g_pref = np.stack([O.texture_bwd_tex(pref_o[l].shape, dr32, tid_l[l], gpf[l], kind=O.TEX_CUBE)
                       for l in range(L)])
    g_env = OP.ibl_filter_bwd(S, Si, Sp, L, g_irr, g_pref)
    c3 = cov[..., None]
    assert_grad_close(host(env_t.grad), g_env, what="environment")
    assert_grad_close(host(a_t.grad).reshape(Bv, Npv, 3), gr["albedo"], what="albedo")
    assert_grad_close(host(n_t.grad).reshape(Bv, Npv, 3), gr["normal"] + np.where(c3, vn, 0.0), what="normal")
    assert_grad_close(host(p_t.grad).reshape(Bv, Npv, 3), gr["pos"] + np.where(c3, vp, 0.0), what="position")
    gm = host(mat.grad).astype(np.float64)
    ref = np.array([gr["metallic"], gr["roughness"]])
    assert np.abs(gm - ref).max() <= 1e-4 * np.abs(ref).max(), (gm, ref)


def test_laplacian_autograd(B):
    from oracle import optim as oo
    from paper_2204_01386_amd import ops, scenes
    p, tris = scenes.noisy_sphere(3, 7)
    pos = dev(p).requires_grad_()
    R = ops.laplacian_reg(pos, dev(tris), 3.0)
    (2.5 * R).sum().backward()
    Ro, go = oo.laplacian_reg(p, tris, 3.0)
    assert abs(float(R.item()) - Ro) <= 1e-6 * Ro
    assert_grad_close(host(pos.grad), 2.5 * go, what="laplacian autograd")
