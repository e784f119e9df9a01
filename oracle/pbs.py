"""Oracle of physically-based shading with image-based lighting (test
infrastructure: only the tests, smoke() and the benchmark's CPU baseline use
anything under oracle/).  float64 NumPy and PyTorch-CPU (autograd as the
differentiation primitive), written from the definitions below; it shares
nothing with the GPU library.

The paper's render graph (appendix B) shades with PBS from three maps built
from the environment image: an irradiance map, a prefiltered environment map
for glossy reflection and a BRDF integration map (the split-sum image-based
lighting of the cited course notes); appendix C optimises an environment
map jointly with the PBS roughness.  It gives none of the filters'
definitions.  The readings taken here:

* Cube texels.  Face f, column i, row j of an S x S face has centre
  (a, b) = (2 (i + 1/2) / S - 1, 2 (j + 1/2) / S - 1) and direction
  +X: (1, -b, -a), -X: (-1, -b, a), +Y: (a, 1, b), -Y: (a, -1, -b),
  +Z: (a, -b, 1), -Z: (-a, -b, -1) (the sampler's major-axis convention),
  and exact solid angle F(a1,b1) - F(a0,b1) - F(a1,b0) + F(a0,b0),
  F(a, b) = atan2(a b, sqrt(a^2 + b^2 + 1)), over the texel's square.
* Irradiance, the cosine convolution as a normalised discrete sum over all
  environment texels j (direction w_j, solid angle O_j):
      irr(n) = sum_j env_j max(0, n.w_j) O_j / sum_j max(0, n.w_j) O_j.
* Prefiltered level l of L (roughness r_l = l / (L - 1), GGX alpha
  a_l = max(r_l^2, 1e-3)), with n = v = R (the split sum's assumption):
      pref_l(R) = sum_j env_j W_j / sum_j W_j,
      W_j = max(0, R.w_j) D(h_j) O_j,  h_j = normalize(R + w_j),
      D(h) = a^2 / (pi ((R.h)^2 (a^2 - 1) + 1)^2).
* BRDF integration table, N x N, n.v = (i + 1/2) / N along columns,
  roughness (j + 1/2) / N along rows, alpha = roughness^2: the mean over the
  M-point Hammersley set (x_k = (k + 1/2) / M, y_k = radical inverse base 2 of
  k) of GGX-sampled half vectors h (cos theta = sqrt((1 - y) / (1 + (a^2 - 1) y)),
  phi = 2 pi x), l = reflect(-v, h), kept when n.l > 0:
      A += (1 - Fc) Gv,  B += Fc Gv,  Fc = (1 - v.h)^5,
      Gv = G (v.h) / ((n.h)(n.v)),  G = G1(n.v) G1(n.l),  G1(c) = c / (c (1 - k) + k),  k = alpha / 2.
* Shading of a fragment with shading normal n' = normalize(n), position p,
  albedo a (rgb), metallic m and roughness r (scalars of the material):
      v = normalize(eye - p),  c = max(n'.v, 1e-4),  R = 2 (n'.v) n' - v,
      F0 = 0.04 (1 - m) + a m,  F = F0 + (max(1 - r, F0) - F0)(1 - c)^5,
      x = clamp(r, 0, 1) (L - 1), l0 = min(floor(x), L - 2), f = x - l0,
      P = (1 - f) pref_l0(R) + f pref_l0+1(R)   (bilinear cube lookups),
      (A, B) = the table sampled bilinearly (clamped) at (c, r),
      C = (1 - F)(1 - m) a irr(n') + P (F0 A + B),   out = C / (1 + C).
  Lookups of irr and pref use the sampler's bilinear cube filtering.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle as O


# ---------------------------------------------------------------------------
# cube geometry
# ---------------------------------------------------------------------------
def _face_dir(f, a, b):
    one = np.ones_like(a)
    return {0: (one, -b, -a), 1: (-one, -b, a), 2: (a, one, b), 3: (a, -one, -b),
            4: (a, -b, one), 5: (-a, -b, -one)}[f]


def cube_texels(S: int):
    """(directions [6*S*S, 3] unit, solid angles [6*S*S]) in face, row, column order."""
    c = (np.arange(S) + 0.5) / S * 2.0 - 1.0
    e = np.arange(S + 1) / S * 2.0 - 1.0
    B, A = np.meshgrid(c, c, indexing="ij")              # row j -> b, column i -> a
    F = lambda a, b: np.arctan2(a * b, np.sqrt(a * a + b * b + 1.0))
    jb, ia = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
    ax0, ax1 = e[ia], e[ia + 1]
    by0, by1 = e[jb], e[jb + 1]
    om = F(ax1, by1) - F(ax0, by1) - F(ax1, by0) + F(ax0, by0)
    dirs, oms = [], []
    for f in range(6):
        d = np.stack(_face_dir(f, A, B), -1)
        dirs.append((d / np.linalg.norm(d, axis=-1, keepdims=True)).reshape(-1, 3))
        oms.append(om.reshape(-1))
    return np.concatenate(dirs), np.concatenate(oms)


# ---------------------------------------------------------------------------
# the filters as explicit matrices: out = M @ env (rows normalised)
# ---------------------------------------------------------------------------
def irradiance_matrix(S: int, Si: int) -> np.ndarray:
    w, om = cube_texels(S)
    n, _ = cube_texels(Si)
    K = np.maximum(0.0, n @ w.T) * om[None, :]
    return K / K.sum(1, keepdims=True)


def ggx_d(ndh, alpha):
    a2 = alpha * alpha
    t = ndh * ndh * (a2 - 1.0) + 1.0
    return a2 / (math.pi * t * t)


def level_alpha(l: int, L: int) -> float:
    r = l / (L - 1)
    return max(r * r, 1e-3)


def prefilter_matrix(S: int, Sp: int, alpha: float) -> np.ndarray:
    w, om = cube_texels(S)
    R, _ = cube_texels(Sp)
    ndl = R @ w.T
    h = R[:, None, :] + w[None, :, :]
    hn = np.linalg.norm(h, axis=-1)
    ndh = np.where(hn > 0, (R[:, None, :] * h).sum(-1) / np.where(hn > 0, hn, 1.0), 0.0)
    K = np.maximum(0.0, ndl) * ggx_d(ndh, alpha) * om[None, :]
    return K / K.sum(1, keepdims=True)


def ibl_filter(env: np.ndarray, Si: int, Sp: int, L: int):
    """env [6,S,S,C] -> (irr [6,Si,Si,C], pref [L,6,Sp,Sp,C])."""
    S, C = env.shape[1], env.shape[-1]
    e = env.reshape(-1, C).astype(np.float64)
    irr = (irradiance_matrix(S, Si) @ e).reshape(6, Si, Si, C)
    pref = np.stack([(prefilter_matrix(S, Sp, level_alpha(l, L)) @ e).reshape(6, Sp, Sp, C) for l in range(L)])
    return irr, pref


def ibl_filter_bwd(S: int, Si: int, Sp: int, L: int, g_irr: np.ndarray, g_pref: np.ndarray) -> np.ndarray:
    """The adjoint: g_env = M_irr^T g_irr + sum_l M_l^T g_pref_l."""
    C = g_irr.shape[-1]
    g = irradiance_matrix(S, Si).T @ g_irr.reshape(-1, C).astype(np.float64)
    for l in range(L):
        g += prefilter_matrix(S, Sp, level_alpha(l, L)).T @ g_pref[l].reshape(-1, C).astype(np.float64)
    return g.reshape(6, S, S, C)


# ---------------------------------------------------------------------------
# BRDF integration table
# ---------------------------------------------------------------------------
def radical_inverse2(k: np.ndarray) -> np.ndarray:
    k = k.astype(np.uint64)
    out = np.zeros(k.shape, np.float64)
    f = 0.5
    kk = k.copy()
    while kk.any():
        out += f * (kk & np.uint64(1)).astype(np.float64)
        kk >>= np.uint64(1)
        f *= 0.5
    return out


def brdf_lut(N: int, M: int) -> np.ndarray:
    """[N, N, 2] (rows: roughness, columns: n.v) of (A, B)."""
    k = np.arange(M)
    x = (k + 0.5) / M
    y = radical_inverse2(k)
    out = np.zeros((N, N, 2))
    for j in range(N):
        r = (j + 0.5) / N
        a = r * r
        kk = a / 2.0
        ct = np.sqrt((1.0 - y) / (1.0 + (a * a - 1.0) * y))
        st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
        ph = 2.0 * math.pi * x
        h = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1)   # n = +z
        for i in range(N):
            c = (i + 0.5) / N
            v = np.array([math.sqrt(1.0 - c * c), 0.0, c])
            vdh = h @ v
            l = 2.0 * vdh[:, None] * h - v
            ndl = l[:, 2]
            ok = ndl > 0
            g1 = lambda q: q / (q * (1.0 - kk) + kk)
            G = g1(c) * g1(np.maximum(ndl, 1e-30))
            gv = G * vdh / (h[:, 2] * c)
            fc = (1.0 - vdh) ** 5
            out[j, i, 0] = np.where(ok, (1.0 - fc) * gv, 0.0).sum() / M
            out[j, i, 1] = np.where(ok, fc * gv, 0.0).sum() / M
    return out


# ---------------------------------------------------------------------------
# shading (torch float64: the backward is its autograd)
# ---------------------------------------------------------------------------
def _bilinear_clamped(table: torch.Tensor, u: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """table [N,N,C] sampled at (u along columns, v along rows), texel centres
    at (i + 1/2)/N, clamped at the borders (piecewise linear in u and v)."""
    N = table.shape[0]
    s = u * N - 0.5
    t = v * N - 0.5
    x0 = torch.floor(s)
    y0 = torch.floor(t)
    fx, fy = s - x0, t - y0
    cl = lambda q: q.clamp(0, N - 1).long()
    X0, X1, Y0, Y1 = cl(x0), cl(x0 + 1), cl(y0), cl(y0 + 1)
    w00 = ((1 - fx) * (1 - fy))[..., None]
    w01 = (fx * (1 - fy))[..., None]
    w10 = ((1 - fx) * fy)[..., None]
    w11 = (fx * fy)[..., None]
    return w00 * table[Y0, X0] + w01 * table[Y0, X1] + w10 * table[Y1, X0] + w11 * table[Y1, X1]


def pbs_dirs(n, p, eye):
    """(n' = normalize(n), R = 2 (n'.v) n' - v) as torch tensors."""
    nn = n / torch.linalg.norm(n, dim=-1, keepdim=True)
    v = eye - p
    v = v / torch.linalg.norm(v, dim=-1, keepdim=True)
    R = 2.0 * (nn * v).sum(-1, keepdim=True) * nn - v
    return nn, R


def pbs_shade(n, p, eye, albedo, metallic, roughness, irr_s, pref_s, lut, L):
    """Torch float64 shading.  pref_s [L, ..., 3]: every level sampled at R
    (only the two around the roughness are used)."""
    nn, R = pbs_dirs(n, p, eye)
    v = eye - p
    v = v / torch.linalg.norm(v, dim=-1, keepdim=True)
    c = torch.clamp((nn * v).sum(-1), min=1e-4)
    F0 = 0.04 * (1.0 - metallic) + albedo * metallic
    w5 = ((1.0 - c) ** 5)[..., None]
    F = F0 + (torch.maximum(1.0 - roughness, F0) - F0) * w5
    x = torch.clamp(roughness, 0.0, 1.0) * (L - 1)
    l0 = int(min(math.floor(float(x.detach())), L - 2))
    f = x - l0
    P = (1.0 - f) * pref_s[l0] + f * pref_s[l0 + 1]
    AB = _bilinear_clamped(lut, c, roughness.expand_as(c))
    spec = P * (F0 * AB[..., 0:1] + AB[..., 1:2])
    C = (1.0 - F) * (1.0 - metallic) * albedo * irr_s + spec
    return C / (1.0 + C)


def shade_and_grads(n, p, eye, albedo, metallic, roughness, irr_s, pref_s, lut, L, tri_id, grad_out):
    """Forward and every gradient of the shading of covered fragments
    (tri_id >= 0; others give 0): returns (out, grads dict) as float64
    arrays; 'dir_n' and 'dir_r' are the lookup directions."""
    T = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    tn, tp, ta, tirr, tpref = T(n), T(p), T(albedo), T(irr_s), T(pref_s)
    tm, tr = T(metallic), T(roughness)
    te = torch.tensor(np.asarray(eye, np.float64))
    lut_t = torch.tensor(np.asarray(lut, np.float64))
    out = pbs_shade(tn, tp, te, ta, tm, tr, tirr, tpref, lut_t, L)
    mask = torch.tensor(np.asarray(tri_id) >= 0)[..., None]
    out = torch.where(mask, out, torch.zeros_like(out))
    out.backward(torch.tensor(np.asarray(grad_out, np.float64)))
    with torch.no_grad():
        nn, R = pbs_dirs(tn, tp, te)
    g = lambda t: t.grad.numpy()
    return out.detach().numpy(), {"normal": g(tn), "pos": g(tp), "albedo": g(ta), "irr_s": g(tirr),
                                  "pref_s": g(tpref), "metallic": float(tm.grad), "roughness": float(tr.grad),
                                  "dir_n": nn.numpy(), "dir_r": R.numpy()}


def dirs_vjp(n, p, eye, g_dir_n, g_dir_r):
    """Gradients to n and p of the lookup directions' gradients."""
    tn = torch.tensor(np.asarray(n, np.float64), requires_grad=True)
    tp = torch.tensor(np.asarray(p, np.float64), requires_grad=True)
    te = torch.tensor(np.asarray(eye, np.float64))
    nn, R = pbs_dirs(tn, tp, te)
    (nn * torch.tensor(g_dir_n) + R * torch.tensor(g_dir_r)).sum().backward()
    return tn.grad.numpy(), tp.grad.numpy()


def cube_sample(tex, d, tri_id):
    """The oracle's bilinear cube lookup (float32 directions, as the kernels get them)."""
    return O.texture(tex, np.asarray(d, np.float32), tri_id, kind=O.TEX_CUBE)


# ---------------------------------------------------------------------------
# the whole PBS step on fixed geometry
# ---------------------------------------------------------------------------
def pbs_forward(scene, env, material, tex, Si, Sp, L, lut):
    """Geometry from the oracle's step (rasterization, G-buffer, UVs), then
    the filters, lookups, shading and blend.  Returns the state dict."""
    from oracle import step as ostep
    g = ostep.forward(scene)
    tid = g["tid"]
    Bv, K, H, W = tid.shape
    gb = g["gbuf"]
    n, p = gb[..., 0:3], gb[..., 3:6]
    wu, wv = scene.extra.get("wrap", (O.WRAP_REPEAT, O.WRAP_CLAMP))
    albedo = O.texture(tex, g["uv"], tid, wrap_u=wu, wrap_v=wv)[..., 0:3]
    irr, pref = ibl_filter(env, Si, Sp, L)
    eye = np.broadcast_to(np.asarray(scene.eyes, np.float64)[:, None, None, None, :], n.shape)
    cov = tid >= 0
    # lookup directions in double, handed to the sampler in float32
    nsafe = np.where(cov[..., None], n, 1.0)
    with torch.no_grad():
        nn, R = pbs_dirs(torch.tensor(nsafe), torch.tensor(p), torch.tensor(np.ascontiguousarray(eye)))
    dn = np.where(cov[..., None], nn.numpy(), 0.0).astype(np.float32)
    dr = np.where(cov[..., None], R.numpy(), 0.0).astype(np.float32)
    m, r = float(material[0]), float(material[1])
    l0 = min(int(math.floor(min(max(r, 0.0), 1.0) * (L - 1))), L - 2)
    tid_l = [np.where(cov, tid, -1) if l in (l0, l0 + 1) else np.full_like(tid, -1) for l in range(L)]
    irr_s = cube_sample(irr, dn, tid)
    pref_s = np.stack([cube_sample(pref[l], dr, tid_l[l]) for l in range(L)])
    out, _ = shade_and_grads(nsafe, p, eye, albedo, m, r, irr_s, pref_s, lut, L, tid, np.zeros(n.shape))
    blend = {"hsr": O.BLEND_HSR, "aa": O.BLEND_AA, "softras": O.BLEND_SOFTRAS,
             "hard": O.BLEND_HARD}[scene.extra.get("blend", "hsr" if scene.r > 0 else "hard")]
    oc, os_, E = O.softras(out, g["dist"], tid, g["sigma"], float(scene.r), blend)
    return {"geo": g, "tid": tid, "tid_l": tid_l, "n": nsafe, "p": p, "eye": eye, "albedo": albedo, "irr": irr,
            "pref": pref, "dn": dn, "dr": dr, "irr_s": irr_s, "pref_s": pref_s, "layer": out, "color": oc,
            "sil": os_, "E": E, "rgba": np.concatenate([oc, os_[..., None]], -1), "m": m, "r": r}


def pbs_step(scene, env, material, tex, target_rgba, Si, Sp, L, lut):
    """Forward, L2 loss against target_rgba, and the gradients of the
    environment map, the material and the albedo texture."""
    f = pbs_forward(scene, env, material, tex, Si, Sp, L, lut)
    tid = f["tid"]
    loss, g_c, g_s = O.loss_l2(f["color"], f["sil"], target_rgba)
    gl, _ = O.softras_bwd(f["layer"], f["geo"]["dist"], tid, f["geo"]["sigma"], f["E"], g_c, g_s)
    _, gr = shade_and_grads(f["n"], f["p"], f["eye"], f["albedo"], f["m"], f["r"], f["irr_s"], f["pref_s"], lut, L,
                            tid, gl)
    S = tid.shape[0] * tid.shape[1]
    rs = lambda a: a.reshape((S,) + a.shape[2:])
    g_irr = O.texture_bwd_tex(f["irr"].shape, rs(f["dn"]), rs(tid), rs(gr["irr_s"]), kind=O.TEX_CUBE)
    g_pref = np.stack([O.texture_bwd_tex(f["pref"][l].shape, rs(f["dr"]), rs(f["tid_l"][l]), rs(gr["pref_s"][l]),
                                         kind=O.TEX_CUBE) for l in range(L)])
    g_env = ibl_filter_bwd(env.shape[1], Si, Sp, L, g_irr, g_pref)
    wu, wv = scene.extra.get("wrap", (O.WRAP_REPEAT, O.WRAP_CLAMP))
    g_samp = np.concatenate([gr["albedo"], np.zeros(gr["albedo"].shape[:-1] + (1,))], -1)
    g_tex = O.texture_bwd_tex(tex.shape, rs(f["geo"]["uv"]), rs(tid), rs(g_samp), wrap_u=wu, wrap_v=wv)
    return f, {"loss": loss, "env": g_env, "material": np.array([gr["metallic"], gr["roughness"]]), "tex": g_tex}
