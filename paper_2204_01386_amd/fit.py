"""The two-stage fit of the paper's cross-platform application (§4.1) run to
convergence on the GPU: vertex positions from silhouettes under the
scheduled Laplacian regulariser, then the albedo texture on the fitted
geometry.  Both stages run as captured graphs replayed once per iteration.
Reports the convergence curve (silhouette and colour L2, and the mean
distance of the fitted vertices to the target surface) and the time of one
iteration of each stage."""
from __future__ import annotations

import numpy as np
import torch
from scipy.spatial import cKDTree

from .pipeline import FitLoop, Step, make_target
from .scenes import Scene


def surface_samples(pos: np.ndarray, tris: np.ndarray, n: int = 6) -> np.ndarray:
    """Points on every triangle at the barycentric grid of step 1/n (interior
    and edges)."""
    ij = [(i, j) for i in range(n + 1) for j in range(n + 1 - i)]
    w = np.array([(i / n, j / n, 1.0 - (i + j) / n) for i, j in ij])
    p = pos[tris].astype(np.float64)                       # [T,3,3]
    return np.einsum("kc,tcd->tkd", w, p).reshape(-1, 3)


def mean_surface_distance(pos: np.ndarray, tree: cKDTree) -> float:
    d, _ = tree.query(pos.astype(np.float64))
    return float(d.mean())


def _sil_l2(st) -> float:
    return float(((st.sil - st.target[..., 3]) ** 2).mean().item())


def _col_l2(st) -> float:
    m = st.target[..., 3:4] > 0
    return float((((st.color - st.target[..., :3]) ** 2) * m).sum().item() / max(1, int(m.sum().item())))


def _capture(fn):
    fn()                      # eager: sizes the scratch, takes the first iteration
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def _time(g, n: int) -> float:
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(n):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def run_fit(scene: Scene, n_sil: int = 300, n_tex: int = 200, every: int = 25, lr_pos: float = 0.01,
            lr_tex: float = 0.01, lap0: float = 10.0, lap_gamma: float = 0.99, time_reps: int = 50) -> dict:
    """Runs the fit and returns its curve and timings.  The timing replays
    run after the curve on copies of the final state, so they do not change
    the reported fit."""
    st = Step(scene, target=make_target(scene))
    fl = FitLoop(st, lr_pos=lr_pos, lr_tex=lr_tex, lap0=lap0, lap_gamma=lap_gamma)
    tree = cKDTree(surface_samples(scene.target_pos, scene.tris))
    curve = []

    def record(stage, it):
        torch.cuda.synchronize()
        curve.append({"stage": stage, "iteration": it, "sil_l2": round(_sil_l2(st), 6),
                      "color_l2": round(_col_l2(st), 6),
                      "surface_distance": round(mean_surface_distance(st.pos.cpu().numpy(), tree), 5),
                      "laplacian": round(float(fl.reg.item()), 6)})

    st.forward()
    record("silhouette", 0)
    g_sil = _capture(fl.silhouette_iteration)
    done = 1
    while done < n_sil:
        k = min(every - done % every, n_sil - done)
        for _ in range(k):
            g_sil.replay()
        done += k
        if done % every == 0 or done == n_sil:
            st.forward()
            record("silhouette", done)
    fl.start_texture_stage()
    fl.ts.forward()
    record("texture", 0)
    g_tex = _capture(fl.texture_iteration)
    done = 1
    while done < n_tex:
        k = min(every - done % every, n_tex - done)
        for _ in range(k):
            g_tex.replay()
        done += k
        if done % every == 0 or done == n_tex:
            fl.ts.forward()
            record("texture", done)
    status = st.ctx.check_status()
    # timing: replays on the fitted state (positions and texture saved and restored)
    saved = (st.pos.clone(), st.tex.clone(), fl.adam_pos.m.clone(), fl.adam_pos.v.clone(),
             fl.adam_pos.state.clone(), fl.adam_tex.m.clone(), fl.adam_tex.v.clone(), fl.adam_tex.state.clone())
    ms_sil = _time(g_sil, time_reps)
    ms_tex = _time(g_tex, time_reps)
    for dst, src in zip((st.pos, st.tex, fl.adam_pos.m, fl.adam_pos.v, fl.adam_pos.state, fl.adam_tex.m,
                         fl.adam_tex.v, fl.adam_tex.state), saved):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"workload": scene.name, "views": int(st.B), "H": st.H, "W": st.W, "triangles": int(st.T),
            "K": st.K, "r": st.r, "lr_pos": lr_pos, "lr_tex": lr_tex, "lap0": lap0, "lap_gamma": lap_gamma,
            "iterations": {"silhouette": n_sil, "texture": n_tex}, "bin_overflow": status != 0,
            "ms_per_iteration": {"silhouette": round(ms_sil, 4), "texture": round(ms_tex, 4)},
            "curve": curve}


def kr_sweep(Ks=(1, 2, 3, 4, 5), r_px=(1, 2, 3, 5, 7), checkpoints=(500, 2500), seed: int = 0,
             blend: str = "hsr", lap_gamma: float = 0.999) -> dict:
    """The paper's validation of HardSoftRas settings (§4.3: a heatmap over K
    and r of the fitted geometry's distance to the target, early and late in
    the optimisation) on the sphere-to-pear silhouette fit: for every (K, r)
    the target is rendered with the same setting, and the mean distance of
    the fitted vertices to the target surface is recorded at each checkpoint
    (iterations of the silhouette stage).  The regulariser decays by
    lap_gamma per iteration (0.999: to a tenth over the 2,500 iterations;
    a schedule that reaches zero lets the silhouette-only fit drift)."""
    out = {"checkpoints": list(checkpoints), "K": list(Ks), "r_px": list(r_px), "blend": blend, "lap_gamma": lap_gamma,
           "surface_distance": {}, "ms_per_iteration": {}}
    base = None
    for K in Ks:
        for rp in r_px:
            from .scenes import fit_scene
            scene = fit_scene(seed, K=K, r=rp / 256.0, blend=blend)
            if base is None:
                base = cKDTree(surface_samples(scene.target_pos, scene.tris))
            st = Step(scene, target=make_target(scene))
            fl = FitLoop(st, lap_gamma=lap_gamma)
            g = _capture(fl.silhouette_iteration)
            done, dists = 1, []
            for cp in checkpoints:
                for _ in range(cp - done):
                    g.replay()
                done = cp
                torch.cuda.synchronize()
                dists.append(round(mean_surface_distance(st.pos.cpu().numpy(), base), 5))
            key = f"K={K},r={rp}px"
            out["surface_distance"][key] = dists
            out["ms_per_iteration"][key] = round(_time(g, 20), 4)
            if st.ctx.check_status() != 0:
                out.setdefault("bin_overflow", []).append(key)
            del g, fl, st
            torch.cuda.empty_cache()
    return out


def run_env_fit(n_iter: int = 300, every: int = 50, S: int = 32, Si: int = 8, Sp: int = 16, L: int = 5,
                n_views: int = 20, H: int = 256, material_t=(0.9, 0.25), rough0: float = 0.6, lr_env: float = 0.02,
                lr_rough: float = 0.01, seed: int = 0, time_reps: int = 30) -> dict:
    """The environment-map fit of the paper's appendix C on synthetic data:
    a metallic pear (fixed geometry, 20 fixed views) rendered with split-sum
    PBS under a ground-truth environment map and roughness; the environment
    map starts uniform grey and the roughness elsewhere, and both are fitted
    with Adam to the ground-truth images (metallic and albedo held).  Every
    iteration is one captured graph.  Reports the image loss, the
    environment map's relative error and the roughness at checkpoints, and
    the time of one iteration."""
    from .pipeline import Adam, PbsStep
    from .scenes import cube_env_map, fit_scene
    s = fit_scene(seed, n_views=n_views, H=H)
    s.pos = s.target_pos                              # the pear itself
    s.tex = s.target_tex
    env_t = cube_env_map(S, seed + 11)
    tgt = PbsStep(s, env_t, np.asarray(material_t, np.float32), Si, Sp, L)
    tgt.forward()
    ps = PbsStep(s, np.full_like(env_t, 0.5), np.asarray([material_t[0], rough0], np.float32), Si, Sp, L,
                 target=tgt)
    env_t_d = torch.from_numpy(env_t).to(ps.dev)
    adam_env = Adam(ps.env, lr_env)
    rough = ps.material[1:2]
    adam_r = Adam(rough, lr_rough)
    g_rough = ps.g_material[1:2]
    st = ps.st

    def iteration():
        ps.run()
        adam_env.step(st.ctx, ps.g_env, st._s())
        adam_r.step(st.ctx, g_rough, st._s())

    curve = []

    def record(it):
        ps.forward()
        ps.loss_and_grad()
        torch.cuda.synchronize()
        curve.append({"iteration": it, "loss": float(f"{float(st.loss.item()):.4e}"),
                      "env_rel_error": round(float(((ps.env - env_t_d).norm() / env_t_d.norm()).item()), 5),
                      "roughness": round(float(rough.item()), 5)})

    record(0)
    g = _capture(iteration)
    done = 1
    while done < n_iter:
        k = min(every - done % every, n_iter - done)
        for _ in range(k):
            g.replay()
        done += k
        if done % every == 0 or done == n_iter:
            record(done)
    saved = [t.clone() for t in (ps.env, ps.material, adam_env.m, adam_env.v, adam_env.state, adam_r.m, adam_r.v,
                                 adam_r.state)]
    ms = _time(g, time_reps)
    kernels = _profile(iteration)
    for dst, src in zip((ps.env, ps.material, adam_env.m, adam_env.v, adam_env.state, adam_r.m, adam_r.v,
                         adam_r.state), saved):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"workload": f"metallic pear ({st.T} triangles), {n_views} views {H}x{H}, HardSoftRas K={st.K}, "
                        f"env 6x{S}^2, irradiance 6x{Si}^2, prefiltered {L}x6x{Sp}^2",
            "material_target": list(material_t), "roughness_start": rough0, "iterations": n_iter,
            "ms_per_iteration": round(ms, 4), "kernels": kernels, "curve": curve}


def _profile(fn, cap: int = 4096) -> list:
    """Per-kernel time of one eager call of fn (the library's event profiler:
    each launch timed from its own dispatch), largest first."""
    import ctypes as C

    from . import binding as Bd
    torch.cuda.synchronize()
    Bd._lib.dressi_profile_start(cap)
    fn()
    torch.cuda.synchronize()
    names = (C.c_char_p * cap)()
    ms = (C.c_float * cap)()
    n = Bd._lib.dressi_profile_read(names, ms, cap)
    Bd._lib.dressi_profile_start(0)
    tot = {}
    for i in range(max(n, 0)):
        k = names[i].decode()
        tot[k] = tot.get(k, 0.0) + ms[i]
    return [[k, round(v, 4)] for k, v in sorted(tot.items(), key=lambda kv: -kv[1])]
