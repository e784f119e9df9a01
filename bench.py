#!/usr/bin/env python
"""Forward+backward throughput of the Dressi rasterization hot path on one
MI355X (gfx950).

Workload (the configuration the headline metric is quoted on): a noisy
icosphere of 40,962 vertices / 81,920 triangles seen by one 512x512 camera,
spherical UVs on a 1024x1024 RGBA fp32 value-noise texture, hard
rasterization (K=1), Phong shading, L2 loss against a render of a perturbed
mesh and texture, backward to vertex positions and texels (texels through the
inverse-UV gather).  All inputs are seeded and synthetic.

One step = vertex normals + transform, rasterize, interpolate, texture,
shade, blend, loss, and every adjoint.  "batched" replays the whole step as
one captured hipGraph; "plain" issues the same calls eagerly (for multi-view
configurations: one view per call).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The paper's own fwd+bwd timings nearest to the measured workloads (§5.1,
# the non-textured and textured timing tables; one NVIDIA GeForce RTX 2080,
# Vulkan, the average over six views of 1,000 frames).  Context only: the
# meshes, shaders and soft-rasterization settings differ from these configs.
PAPER_CONTEXT = [
    {"workload": "512x512 window, 51,414 triangles, white vertex colour (silhouette)",
     "hardware": "NVIDIA GeForce RTX 2080", "ms_per_view": 0.502, "Mpix_s": round(512 * 512 / 0.502e-3 / 1e6, 1)},
    {"workload": "2048x2048 window, 55,704 triangles, 1024^2 albedo texture",
     "hardware": "NVIDIA GeForce RTX 2080", "ms_per_view": 2.929, "Mpix_s": round(2048 * 2048 / 2.929e-3 / 1e6, 1)},
    {"workload": "one optimisation iteration of the cross-platform application (a sphere fitted to images of "
                 "a pear): vertex positions vs albedo texture only, scene size not given",
     "hardware": "NVIDIA GeForce RTX 2080", "ms_geometry_iteration": 3.0, "ms_texture_iteration": 2.0},
]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 5])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=8.0)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--hard-raster", type=int, default=None, choices=[0, 1, 2, 3],
                    help="fix the headline's hard rasterization strategy after autotuning (profiling runs)")
    ap.add_argument("--only-graph", action="store_true",
                    help="only the captured-step replays (for external profilers)")
    ap.add_argument("--no-multiview", dest="multiview", action="store_false",
                    help="skip the 16-view batched-vs-plain measurement")
    ap.add_argument("--multiview-steps", type=int, default=30)
    ap.add_argument("--no-large", dest="large", action="store_false",
                    help="skip the large configuration (8 views 2048^2, 1 M triangles)")
    ap.add_argument("--no-uneven", dest="uneven", action="store_false",
                    help="skip the 64-instance uneven batch measurement")
    ap.add_argument("--uneven-steps", type=int, default=20)
    ap.add_argument("--fits-only", action="store_true",
                    help="only the two-stage fit and the environment-map fit (one JSON line)")
    ap.add_argument("--kr-sweep", action="store_true",
                    help="only the K x r sweep of the sphere-to-pear silhouette fit (one JSON line)")
    ap.add_argument("--no-fit", dest="fit", action="store_false",
                    help="skip the two-stage fit (sphere to pear, positions then texture)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (reference for HBM counters)")
    ap.add_argument("--paper-table", action="store_true",
                    help="instead: fwd+bwd time per view on workloads shaped like the paper's non-textured "
                         "timing table (windows 256^2-2048^2, three mesh sizes, six views, white Lambert)")
    return ap.parse_args()


# The paper's non-textured fwd+bwd time per view (ms) on one RTX 2080 (§5.1
# table), by window and by mesh (682, 14,208 and 51,414 triangles).
PAPER_TABLE_MS = {256: (0.304, 0.308, 0.364), 512: (0.442, 0.480, 0.502), 1024: (1.034, 1.106, 1.104),
                  2048: (3.301, 3.545, 3.469)}
PAPER_TABLE_TRIS = (682, 14208, 51414)


def paper_table(steps, warmup):
    """Each cell: six views of one mesh rendered and differentiated as one
    graph-captured step; time per view = step time / 6."""
    from paper_2204_01386_amd import scenes
    rows = []
    for H, paper_ms in PAPER_TABLE_MS.items():
        for T, pm in zip(PAPER_TABLE_TRIS, paper_ms):
            sc = scenes.paper_table_scene(T, H)
            m = measure(sc, steps, warmup, -1)
            per_view = m["ms_per_step"] / sc.mvp.shape[0]
            rows.append({"window": H, "triangles": int(sc.tris.shape[0]), "paper_triangles": T,
                         "views": int(sc.mvp.shape[0]), "ms_per_view": round(per_view, 4),
                         "Mpix_s": round(H * H / (per_view * 1e-3) / 1e6, 1),
                         "paper_ms_per_view": pm, "paper_hardware": "NVIDIA GeForce RTX 2080"})
            del m
    return rows


def scene_for(cfg):
    from paper_2204_01386_amd import scenes
    if cfg == 1:
        return scenes.config1(), "icosphere s3 (642 v, 1,280 t), 1 view 128x128, per-vertex RGB, K=1, Lambert"
    if cfg == 2:
        return scenes.config2(), ("noisy icosphere s6 (40,962 v, 81,920 t), 1 view 512x512, "
                                  "1024x1024 RGBA fp32 texture, K=1, Phong")
    if cfg == 3:
        return scenes.config3(), ("noisy icosphere s6 (81,920 t), 16 views 512x512, 1024^2 RGBA texture + "
                                  "1024^2 normal map, 6x128^2 env map, HardSoftRas K=3 r=0.01, Phong+env")
    return scenes.config5(), ("torus-knot tube (524,288 v, 1,048,576 t), 8 views 2048x2048, 4096^2 RGBA "
                              "texture, HardSoftRas K=3 r=0.01, Phong")


# ---------------------------------------------------------------------------
# Algorithmic bytes.  A tensor that crosses the library boundary (a stage's
# input or output) is read once and written once at its dtype, where the
# method needs it: every per-fragment stage reads tri_id at each of the
# N = B*K*H*W fragment slots (it decides which slots are empty) and reads and
# writes the other per-fragment planes only at the covered fragments; the
# rasterizer writes every slot.  A texture read counts only the texels that
# can be touched, min(Ht*Wt, 4 * covered fragments); each inverse-UV slice is
# cleared and read once in full and written once per covered fragment.
# Internal scratch (setup records, bins, fragment index, per-tile partial
# sums) is not counted, so implementation overhead shows up as a lower
# fraction of the roofline.
# ---------------------------------------------------------------------------
# HBM traffic per launch from two rocprofv3 counter runs of this script on the
# headline workload (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).  Each
# counter is scaled by its reading for a plain 256 MiB device copy
# (torch copy_, same runs): FETCH_SIZE read 131,083.5 KiB for 262,144 KiB moved
# (x2.0), WRITE_SIZE 262,144 KiB (x1.0).  "sha" fingerprints the kernel's
# source file when the counters were taken; the figure is reported as null
# once that file has changed.
FETCH_SCALE, WRITE_SCALE = 262144.0 / 131083.5, 1.0
TRAFFIC = {
    "k_invuv_gather": {"src": "paper_2204_01386_amd/csrc/texture.hip",
                       "sha": "c152c7215b4175a8581336317d50255a6df16017110a081b438998f3ec178ce4",
                       "fetch_kib": 10434.1875, "write_kib": 16384.03125},
    "k_packed_bwd": {"src": "paper_2204_01386_amd/csrc/shade.hip",
                     "sha": "d294fd08a604b8564d2e85916e3fd85935d080b02776a2876d1a9dbe346b2797",
                     "fetch_kib": 10422.375, "write_kib": 7253.0},
}


def traffic_bytes(kernel):
    t = TRAFFIC.get(kernel)
    if t is None:
        return None
    import hashlib
    with open(os.path.join(ROOT, t["src"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha"]:
            return None
    return int(round((t["fetch_kib"] * FETCH_SCALE + t["write_kib"] * WRITE_SCALE) * 1024))


class Shapes:
    def __init__(self, st, cov):
        self.B, self.K, self.H, self.W = st.B, st.K, st.H, st.W
        self.N = st.B * st.K * st.H * st.W          # fragment slots
        self.P = st.B * st.H * st.W                 # pixels
        self.cov = cov                              # covered fragments
        self.V, self.T, self.Cv = st.V, st.T, st.Cv
        self.soft = st.r > 0
        self.mode = st.mode
        self.ex = st.extra is not None
        self.Vuv = 0 if st.uv is None else st.uv.shape[0]
        # channels the method samples (a packed texture's zero padding channel is overhead)
        self.Ct = st.Ct - (1 if st.Ct and st.scene.nmap is not None else 0)
        self.cells = 0 if st.tex is None else st.tex.shape[0] * st.tex.shape[1]
        self.env = st.env is not None
        self.ecells = 0 if st.env is None else st.env.shape[0] * st.env.shape[1] * st.env.shape[2]
        self.S = st.B * st.K
        self.adj = (st.V + 1 + 3 * st.T) * 4
        self.uvadj = (self.Vuv + 1 + 3 * st.T) * 4
        # the packed single-layer pass replaces the per-fragment stages
        self.packed = bool(getattr(st, "packed", False))
        # its texel gather reads one 32-byte record per kept pixel
        self.rec = self.packed and bool(getattr(st, "gather_rec", False)) and getattr(st, "inv_rec", None) is not None

    def touched(self, cells, C):
        return min(cells, 4 * self.cov) * C * 4


def _shade_in(z: Shapes):
    """Per-fragment shading inputs (bytes per covered fragment): normal,
    position (Phong), albedo (sampled) or colour (Lambert), tangent and
    normal-map sample and environment sample (with the environment map)."""
    b = 12 + (0 if z.mode == 0 else 12) + (z.Ct * 4 if z.Ct else 12)
    return b + (12 + 12 if z.env else 0)


def _win_bytes(z: Shapes):
    """Bytes the texel gather reads per kept pixel: its record, or its
    coordinate and sample gradient."""
    return 32 if z.rec else 8 + z.Ct * 4


def call_bytes(z: Shapes):
    """Algorithmic bytes of every library call of one step, by call."""
    N, P, V, T, Cv, B, c = z.N, z.P, z.V, z.T, z.Cv, z.B, z.cov
    d = 4 if z.soft else 0
    sh_in = N * 4 + c * _shade_in(z) + B * 12
    g_geo = 12 + (0 if z.mode == 0 else 12) + (12 if z.env else 0)      # normal, pos, tangent gradients
    out = {
        "vertex_attrs": V * 12 + T * 12 + z.adj + (V * 12 if z.ex else 0) + V * Cv * 4,
        "transform": V * 12 + B * 64 + B * V * 16,
        "rasterize": B * V * 16 + T * 12 + N * (4 + 8 + d),
        "interpolate": V * Cv * 4 + T * 12 + N * 4 + c * 8 + c * Cv * 4,
        "softras": N * 4 + c * (12 + d) + P * (12 + 4 + 1),
        "loss_l2": P * (12 + 4 + 16) + P * 16,
        "softras_bwd": N * 4 + c * (12 + d) + P * (1 + 12 + 4) + c * (12 + d),
        "shade": sh_in + c * 12,
        "shade_bwd": sh_in + c * 12 + c * (g_geo + (z.Ct * 4 if z.Ct else 12)),
        "interpolate_bwd": N * 4 + c * (8 + Cv * 4) + V * Cv * 4 + T * 12 + z.adj + (c * 8 if z.Ct else 0)
                           + V * Cv * 4 + c * 8,
        "rasterize_bwd": B * V * 16 + T * 12 + z.adj + N * 4 + c * (8 + d) + B * V * 16,
        "transform_bwd": B * V * 16 + B * 64 + V * 12,
        "vertex_attrs_bwd": V * 12 + T * 12 + z.adj + V * Cv * 4 + V * 12 + V * 12,
    }
    if z.Ct:
        win = min(c, z.S * z.cells)
        out["interpolate uv"] = z.Vuv * 8 + T * 12 + N * 4 + c * 8 + c * 8
        out["texture"] = N * 4 + c * 8 + z.touched(z.cells, z.Ct) + c * z.Ct * 4
        out["interpolate_bwd uv"] = z.Vuv * 8 + T * 12 + N * 4 + c * (8 + 8) + c * 8
        out["texture_bwd"] = (N * 4 + c * (8 + z.Ct * 4) + z.touched(z.cells, z.Ct) + c * 8
                              + z.S * z.cells * 4 * 2 + c * 4 + win * (8 + z.Ct * 4) + z.cells * z.Ct * 4)
    if z.packed:
        # interpolation, texture, shading, blend, loss and their adjoints as
        # one forward and one backward pass: only what leaves the pass moves
        for k in ("interpolate", "interpolate uv", "texture", "shade", "softras", "loss_l2", "softras_bwd",
                  "shade_bwd", "texture_bwd", "interpolate_bwd uv"):
            out.pop(k, None)
        tex_in = (z.Vuv * 8 + T * 12 + z.touched(z.cells, z.Ct)) if z.Ct else 0
        g_gbuf = Cv * 4 if z.mode == 0 else 24          # normal, position (, colour) gradients
        out["packed_forward"] = (N * 4 + c * 8 + V * Cv * 4 + T * 12 + tex_in + B * 12
                                 + c * Cv * 4 + (c * (8 + z.Ct * 4) + z.S * z.cells * 4 if z.Ct else 0)
                                 + P * (12 + 4 + 1))
        out["packed_backward"] = (N * 4 + c * Cv * 4 + (c * (8 + z.Ct * 4) + tex_in if z.Ct else 0)
                                  + P * (12 + 4 + 16) + B * 12
                                  + c * g_gbuf + (c * (z.Ct * 4 + 8 + 4) if z.Ct else 0)
                                  + (c * 32 if z.rec else 0))
        if z.Ct:
            win = min(c, z.S * z.cells)
            out["texture_grad_invuv"] = z.S * z.cells * 4 + win * _win_bytes(z) + z.cells * z.Ct * 4
    if z.env:
        ewin = min(c, z.S * z.ecells)
        out["shade dir"] = N * 4 + c * (12 + 12 + 12 + 12) + B * 12 + c * 12
        out["texture env"] = N * 4 + c * 12 + z.touched(z.ecells, 3) + c * 12
        out["shade_bwd env"] = sh_in + c * 12 + c * 12
        out["texture_bwd env"] = (N * 4 + c * (12 + 12) + z.touched(z.ecells, 3) + c * 12
                                  + z.S * z.ecells * 4 * 2 + c * 4 + ewin * (12 + 12) + z.ecells * 12)
    return out


def kernel_bytes(name, z: Shapes):
    """Algorithmic bytes per launch of a kernel (same accounting as above),
    or None for kernels that only move internal scratch."""
    N, P, V, T, Cv, B, c = z.N, z.P, z.V, z.T, z.Cv, z.B, z.cov
    d = 4 if z.soft else 0
    cb = call_bytes(z)
    if z.packed and name in ("k_interp", "k_tex_fwd", "k_shade", "k_shade_bwd", "k_blend", "k_blend_bwd",
                             "k_loss_l2", "k_tex_bwd_pixel"):
        return None
    if name in ("k_raster", "k_raster_list"):
        return cb["rasterize"] - B * V * 16 - T * 12
    if name == "k_setup_bin":
        return B * V * 16 + T * 12
    if name == "k_interp":        # per-vertex attributes and (textured) UVs: mean per launch
        return cb["interpolate"] if not z.Ct else (cb["interpolate"] + cb["interpolate uv"]) // 2
    if name == "k_tex_fwd":       # albedo (and environment) lookups: mean per launch
        return cb["texture"] if not z.env else (cb["texture"] + cb["texture env"]) // 2
    if name == "k_invuv_gather" and not z.env:
        return z.S * z.cells * 4 + min(c, z.S * z.cells) * _win_bytes(z) + z.cells * z.Ct * 4
    if name == "k_tex_bwd_pixel" and not z.env:
        return N * 4 + c * (8 + z.Ct * 4) + z.touched(z.cells, z.Ct) + c * 8 + c * 4
    if name == "k_packed_fwd":
        return cb.get("packed_forward")
    if name == "k_packed_bwd":
        return cb.get("packed_backward")
    if name == "k_blend":
        return cb.get("softras")
    if name == "k_blend_bwd":
        return cb.get("softras_bwd")
    if name == "k_loss_l2":
        return cb.get("loss_l2")
    if name == "k_interp_bwd_tile":
        return N * 4 + c * (8 + Cv * 4) + V * Cv * 4 + T * 12 + (c * 8 if z.Ct else 0) + c * 8
    if name == "k_interp_bwd_bary":
        return z.Vuv * 8 + T * 12 + N * 4 + c * (8 + 8) + c * 8
    if name == "k_interp_bwd_vertex":
        return z.adj + V * Cv * 4
    if name == "k_rast_bwd_tile":
        return B * V * 16 + T * 12 + N * 4 + c * (8 + d)
    if name == "k_geo_tile":          # both per-tile adjoints: one read of the fragments
        return (N * 4 + c * (8 + Cv * 4) + V * Cv * 4 + T * 12 + (c * 8 if z.Ct else 0) + c * 8
                + B * V * 16)
    if name == "k_geo_vertex":        # both vertex sums, the transform and normal-sum adjoints
        return z.adj + V * 12 + T * 12 + B * V * 16 + B * 64 + V * Cv * 4 + B * V * 16
    if name == "k_vertex_attrs_bwd2":
        return z.adj + V * 12 + T * 12 + V * 12 + V * 12 + V * 12
    if name == "k_rast_bwd_vertex":
        return z.adj + B * V * 16 + B * V * 16
    if name == "k_fragsort":
        return N * 4
    if name == "k_transform":
        return cb["transform"]
    if name == "k_transform_bwd":
        return cb["transform_bwd"]
    if name == "k_vertex_attrs":
        return cb["vertex_attrs"]
    if name == "k_shade_bwd" and not z.env:
        return cb["shade_bwd"]
    if name == "k_shade" and not z.env:
        return cb["shade"]
    return None


def measure(scene, steps, warmup, prof_steps, plain_steps_min=10, hard_raster=None):
    """Times one scene: captured-graph replays ("batched"), eager per-view
    calls ("plain"), and a per-kernel breakdown (one event pair per launch,
    stamped from the kernel's own dispatch)."""
    import ctypes as C

    import torch

    from paper_2204_01386_amd import binding as Bd
    from paper_2204_01386_amd.pipeline import Step, autotune, autotune_streams, make_target

    B = scene.mvp.shape[0]
    tgt = make_target(scene)
    st = Step(scene, target=tgt)
    ctx = Bd.context()

    # ---- warm-up (grows the scratch arena), then capture the step --------
    for _ in range(3):
        st.run()
    torch.cuda.synchronize()
    if ctx.check_status() != 0:
        raise SystemExit("tile-bin capacity overflow during warm-up")
    tuned = autotune(st)
    if hard_raster is not None:
        # a fixed strategy (profiling runs: the profiler's own cost can change
        # the autotuner's choice)
        st.hard_raster = hard_raster
        tuned["hard_raster_fixed"] = hard_raster
    tuned["streams"] = autotune_streams(st)
    st.run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        st.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        st.run()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()

    # ---- batched: K replays of the captured step ---------------------------
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_batched = e0.elapsed_time(e1) / steps
    if ctx.check_status() != 0:
        raise SystemExit("tile-bin capacity overflow in the timed region")
    res = {"ms_per_step": ms_batched, "wall_s_timed": t_wall, "graph": graph, "step": st, "tuned": tuned}
    if prof_steps < 0:
        return res
    if st.tex is not None:
        res["texture_only_ms_per_step"] = texture_only_ms(st, steps, warmup)

    # ---- plain: eager calls on one stream, one view per call ---------------
    conc, st.concurrent = st.concurrent, False
    if B == 1:
        plain_steps = [st]
    else:
        plain_steps = [Step(scene, views=slice(v, v + 1), target=None) for v in range(B)]
        for v, ps in enumerate(plain_steps):
            ps.target.copy_(tgt.rgba()[v:v + 1])
            ps.hard_raster, ps.hybrid_weight = st.hard_raster, st.hybrid_weight
    for _ in range(3):
        for ps in plain_steps:
            ps.run()
    torch.cuda.synchronize()
    n_plain = max(plain_steps_min, steps // 4)
    e0.record()
    for _ in range(n_plain):
        for ps in plain_steps:
            ps.run()
    e1.record()
    torch.cuda.synchronize()
    res["plain_ms_per_step"] = e0.elapsed_time(e1) / n_plain
    del plain_steps

    # ---- per-kernel timing (one stream: every kernel timed alone) ---------
    cap = 400 * max(prof_steps, 1)
    Bd._lib.dressi_profile_start(cap)
    for _ in range(prof_steps):
        st.run()
    torch.cuda.synchronize()
    st.concurrent = conc
    names = (C.c_char_p * cap)()
    ms = (C.c_float * cap)()
    n = Bd._lib.dressi_profile_read(names, ms, cap)
    Bd._lib.dressi_profile_start(0)
    if n < 0:
        raise SystemExit(f"kernel profiler failed ({n})")
    per = {}
    per_launch = {}   # (name, occurrence within the step) -> total ms
    for i in range(n):
        k = names[i].decode()
        tot, cnt = per.get(k, (0.0, 0))
        per[k] = (tot + ms[i], cnt + 1)
    launches = n // prof_steps if prof_steps else 0
    for i in range(n):
        k = names[i].decode()
        j = i % launches if launches else i
        per_launch.setdefault((j, k), 0.0)
        per_launch[(j, k)] += ms[i]
    res["table"] = sorted(((k, tot / prof_steps, tot / cnt, cnt // prof_steps)
                           for k, (tot, cnt) in per.items()), key=lambda x: -x[1])
    res["launches"] = sorted(((f"{k}@{j}", tot / prof_steps) for (j, k), tot in per_launch.items()),
                             key=lambda x: -x[1])
    res["cov"] = int((st.tri_id >= 0).sum().item())
    return res


def texture_only_ms(st, steps, warmup):
    """A texture-only step on the same scene (geometry held fixed: the
    rasterization and the albedo texture's inverse-UV map cached), captured
    and replayed like the full step."""
    import torch

    from paper_2204_01386_amd.pipeline import TextureStep

    ts = TextureStep(st)
    ts.run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        ts.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        ts.run()
    for _ in range(warmup):
        graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    del graph, ts
    return e0.elapsed_time(e1) / steps


def measure_batch(scene_list, steps, warmup, prof_steps):
    """The uneven batch: one captured step of the whole batch (every stage one
    launch) against a loop of standalone per-view steps issued eagerly."""
    import ctypes as C

    import torch

    from paper_2204_01386_amd import binding as Bd
    from paper_2204_01386_amd.pipeline import (BatchStep, Step, autotune, autotune_streams, make_batch_target,
                                               make_target)

    bs = BatchStep(scene_list, target=make_batch_target(scene_list))
    tuned = autotune(bs)
    tuned["streams"] = autotune_streams(bs, reps=5)
    ctx = Bd.context()
    for _ in range(3):
        bs.run()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        bs.run()
    for _ in range(warmup):
        graph.replay()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / steps
    if ctx.check_status() != 0:
        raise SystemExit("tile-bin capacity overflow in the timed region")
    del graph
    ms_tex = texture_only_ms(bs, steps, warmup)
    # plain: one standalone step per view, eager
    plain = [Step(sc, target=make_target(sc)) for sc in scene_list]
    for ps in plain:
        autotune(ps, reps=2)
        ps.run()
    torch.cuda.synchronize()
    n_plain = max(3, steps // 4)
    e0.record()
    for _ in range(n_plain):
        for ps in plain:
            ps.run()
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1) / n_plain
    step_bytes = 0
    for ps in plain:
        step_bytes += sum(call_bytes(Shapes(ps, int((ps.tri_id >= 0).sum().item()))).values())
    del plain
    # per-kernel times of the batched step (one stream: every kernel timed alone)
    bs.concurrent = False
    cap = 400 * max(prof_steps, 1)
    Bd._lib.dressi_profile_start(cap)
    for _ in range(prof_steps):
        bs.run()
    torch.cuda.synchronize()
    names = (C.c_char_p * cap)()
    ms = (C.c_float * cap)()
    n = Bd._lib.dressi_profile_read(names, ms, cap)
    Bd._lib.dressi_profile_start(0)
    per = {}
    for i in range(n):
        k = names[i].decode()
        per[k] = per.get(k, 0.0) + ms[i]
    table = sorted(((k, v / max(prof_steps, 1)) for k, v in per.items()), key=lambda x: -x[1])
    return {"ms_per_step": ms_batched, "plain_ms_per_step": ms_plain, "step_alg_bytes": step_bytes,
            "texture_only_ms_per_step": ms_tex,
            "table": table, "T": bs.T, "pixels": int(sum(s.H * s.W for s in scene_list)),
            "canvas": (bs.W, bs.H), "tuned": tuned}


def uneven_line(steps, prof_steps):
    from paper_2204_01386_amd import scenes
    sl = scenes.config4()
    m = measure_batch(sl, steps, 3, prof_steps)
    return {"workload": "64 uneven instances: UV spheres and tori of 1k-200k triangles (log-uniform, "
                        f"{m['T']:,} in all), {{256,512,768,1024}}^2 views ({m['pixels'] / 1e6:.1f} Mpix, "
                        f"packed into a {m['canvas'][0]}x{m['canvas'][1]} image), 512^2 RGBA texture each, "
                        "K=1, Phong, per-view L2",
            "ms_per_step": round(m["ms_per_step"], 4),
            "value": round(m["pixels"] / (m["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpix/s",
            "tris_per_s": round(m["T"] / (m["ms_per_step"] * 1e-3), 1),
            "plain_ms_per_step": round(m["plain_ms_per_step"], 4),
            "batched_vs_plain_speedup": round(m["plain_ms_per_step"] / m["ms_per_step"], 3),
            "texture_only_ms_per_step": round(m["texture_only_ms_per_step"], 4),
            "step_alg_bytes": m["step_alg_bytes"],
            "step_hbm_frac": round(m["step_alg_bytes"] / (m["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "autotune": _tuned_json(m["tuned"]),
            "kernels": [{"kernel": k, "ms_per_step": round(v, 5)} for k, v in m["table"][:12]]}


def _strategy_name(hr, w):
    from paper_2204_01386_amd.pipeline import HARD_RASTER_NAMES
    return HARD_RASTER_NAMES[hr] + (f" (weight {w}/16)" if hr == 2 else "")


def _tuned_json(t):
    name = {False: "one stream", "index": "fragment index on a second stream",
            "texel": "texel gather on a second stream",
            ("index", "texel"): "fragment index and texel gather on a second stream", True: "two streams"}
    return {"hard_raster": _strategy_name(t["hard_raster"], t["hybrid_weight"]),
            "raster_ms": {_strategy_name(*k): round(v, 4) for k, v in t["ms"].items()},
            "schedule": name[t["streams"]["concurrent"]],
            "step_ms": {name[k]: round(v, 4) for k, v in t["streams"]["ms"].items()}}


def _host_cpu() -> str:
    """The host CPU's model name and the number of logical CPUs this process may use."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return f"{model} ({n} logical CPUs available)"


def copy_bandwidth(mib: int = 1024, reps: int = 20) -> dict:
    """Achieved HBM bandwidth of a plain device-to-device copy of `mib` MiB
    (read once, written once), the practical ceiling the step's algorithmic
    bytes are also compared with."""
    import torch
    src = torch.ones(mib * (1 << 18), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"gbs": round(2 * mib * (1 << 20) / (ms * 1e-3) / 1e9, 1), "bytes_per_copy": 2 * mib * (1 << 20),
            "ms_per_copy": round(ms, 4), "kind": "torch copy_ (device to device), read + write"}


def _log(msg):
    """One progress line per finished phase, on stderr (stdout carries the
    single JSON result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def oracle_rate(scene, seconds, threads, views=None, view_threads=1, max_steps=200):
    """Times the C oracle's whole fwd+bwd step (forward of the current scene,
    loss against the target, backward) on the host: `threads` OpenMP threads
    and row bands inside each step, or `view_threads` Python threads taking a
    view each (the oracle's C calls release the interpreter lock).  Returns
    (ms per step, steps run, pixels per step)."""
    import oracle
    from oracle import step as ostep
    from concurrent.futures import ThreadPoolExecutor
    n = scene.mvp.shape[0]
    sel = list(range(n)) if views is None else list(views)
    oracle.set_threads(threads)
    try:
        if view_threads > 1:
            with ThreadPoolExecutor(view_threads) as ex:
                tg = dict(zip(sel, ex.map(lambda v: ostep.forward(scene, slice(v, v + 1), target=True)["rgba"],
                                          sel)))
        else:
            tg = {None: ostep.forward(scene, None if views is None else slice(sel[0], sel[-1] + 1),
                                      target=True, threads=threads)["rgba"]}

        def one(v):
            sl = slice(v, v + 1) if v is not None else (None if views is None else slice(sel[0], sel[-1] + 1))
            o = ostep.forward(scene, sl, threads=threads)
            ostep.backward(scene, o, tg[v])

        t0 = time.perf_counter()
        nrun = 0
        while True:
            if view_threads > 1:
                with ThreadPoolExecutor(view_threads) as ex:
                    list(ex.map(one, sel))
            else:
                one(None)
            nrun += 1
            if time.perf_counter() - t0 > seconds or nrun >= max_steps:
                break
        tc = (time.perf_counter() - t0) / nrun
    finally:
        oracle.set_threads(1)
    return tc * 1e3, nrun, len(sel) * scene.H * scene.W


def _ncpu():
    try:
        return max(1, min(len(os.sched_getaffinity(0)), 16))
    except AttributeError:
        return max(1, min(os.cpu_count() or 1, 16))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (one MI355X per box); --gpus {args.gpus} is not "
              f"supported. The path shards by views/instances; see the design notes.", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.paper_table:
        print(json.dumps({"paper_table": paper_table(min(args.steps, 50), min(args.warmup, 5)),
                          "note": "white Lambert spheres here, silhouette shading in the paper; context only"}))
        return
    if args.fits_only:
        from paper_2204_01386_amd import scenes as _sc
        from paper_2204_01386_amd.fit import run_env_fit, run_fit
        fr = run_fit(_sc.fit_scene())
        er = run_env_fit()
        print(json.dumps({"fit": {k: fr[k] for k in ("workload", "ms_per_iteration", "iterations")},
                          "pbs_env_fit": {k: er[k] for k in ("workload", "ms_per_iteration", "iterations",
                                                             "kernels")}}))
        return
    if args.kr_sweep:
        from paper_2204_01386_amd.fit import kr_sweep
        print(json.dumps({"kr_sweep": kr_sweep()}))
        return
    if args.copy_ref:
        src = torch.ones(args.copy_ref * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    scene, desc = scene_for(args.config)
    B = scene.mvp.shape[0]
    m = measure(scene, args.steps, args.warmup, -1 if args.only_graph else args.profile_steps,
                hard_raster=args.hard_raster)
    ms_batched = m["ms_per_step"]
    _log(f"config {args.config}: {ms_batched:.4f} ms/step")
    if args.only_graph:
        print(json.dumps({"ms_per_step": ms_batched}))
        return
    st, table, cov = m["step"], m["table"], m["cov"]
    z = Shapes(st, cov)
    step_bytes = sum(call_bytes(z).values())
    # the HBM roofline's kernel: the one whose launches move the most
    # algorithmic bytes per step; the longest byte-modelled kernel is
    # reported beside it (at this size it can be a latency-bound one)
    modelled = [row for row in table if kernel_bytes(row[0], z) is not None]
    dom = max(modelled, key=lambda row: kernel_bytes(row[0], z) * row[3]) if modelled else table[0]
    dom_bytes = kernel_bytes(dom[0], z)
    achieved = dom_bytes / (dom[2] * 1e-3) / 1e9 if dom_bytes else None
    longest = modelled[0] if modelled else None
    longest_json = None if longest is None else {
        "kernel": longest[0], "ms_per_launch": round(longest[2], 5),
        "alg_bytes_per_launch": kernel_bytes(longest[0], z),
        "hbm_frac": round(kernel_bytes(longest[0], z) / (longest[2] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    kernel_rows = [{"kernel": k, "ms_per_step": round(a, 5), "ms_per_launch": round(b, 5),
                    "launches_per_step": c, "alg_bytes": kernel_bytes(k, z)} for k, a, b, c in table]
    ms_plain = m["plain_ms_per_step"]
    ms_tex = m.get("texture_only_ms_per_step")
    launch_rows = [{"launch": k, "ms": round(a, 5)} for k, a in m["launches"][:16]]
    tuned = _tuned_json(m["tuned"])
    del m

    # ---- the 16-view batched configuration beside its per-view form -------
    multi = None
    if args.multiview and args.config == 2:
        s3, d3 = scene_for(3)
        m3 = measure(s3, args.multiview_steps, 5, args.profile_steps // 4, plain_steps_min=3)
        z3 = Shapes(m3["step"], m3["cov"])
        b3 = sum(call_bytes(z3).values())
        pix3 = s3.mvp.shape[0] * s3.H * s3.W
        # the same 16 views with the full form of the layers (graph replays only)
        s3f, _ = scene_for(3)
        s3f.extra["band"] = False
        ms_full = measure(s3f, args.multiview_steps, 5, -1)["ms_per_step"]
        multi = {"workload": d3, "views": int(s3.mvp.shape[0]),
                 "layers": "edge-band form (full layers where the blend's edge mask reaches)",
                 "full_form_ms_per_step": round(ms_full, 4),
                 "ms_per_step": round(m3["ms_per_step"], 4),
                 "value": round(pix3 / (m3["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpix/s",
                 "tris_per_s": round(s3.mvp.shape[0] * s3.tris.shape[0] / (m3["ms_per_step"] * 1e-3), 1),
                 "plain_ms_per_step": round(m3["plain_ms_per_step"], 4),
                 "batched_vs_plain_speedup": round(m3["plain_ms_per_step"] / m3["ms_per_step"], 3),
                 "texture_only_ms_per_step": round(m3["texture_only_ms_per_step"], 4),
                 "step_alg_bytes": b3,
                 "step_hbm_frac": round(b3 / (m3["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "kernels": [{"kernel": k, "ms_per_step": round(a, 5), "launches_per_step": c}
                             for k, a, b, c in m3["table"][:12]],
                 "launches": [{"launch": k, "ms": round(a, 5)} for k, a in m3["launches"][:16]]}
        del m3
        _log(f"16 views: {multi['ms_per_step']} ms/step (full form {multi['full_form_ms_per_step']})")

    # ---- the large configuration: 8 views at 2048^2, 1 M triangles ---------
    large = None
    if args.large and args.config == 2:
        s5, d5 = scene_for(5)
        m5 = measure(s5, 10, 2, 2, plain_steps_min=2)
        z5 = Shapes(m5["step"], m5["cov"])
        b5 = sum(call_bytes(z5).values())
        pix5 = s5.mvp.shape[0] * s5.H * s5.W
        large = {"workload": d5, "views": int(s5.mvp.shape[0]), "layers": "full form",
                 "ms_per_step": round(m5["ms_per_step"], 3),
                 "value": round(pix5 / (m5["ms_per_step"] * 1e-3) / 1e6, 2), "unit": "Mpix/s",
                 "tris_per_s": round(s5.mvp.shape[0] * s5.tris.shape[0] / (m5["ms_per_step"] * 1e-3), 1),
                 "plain_ms_per_step": round(m5["plain_ms_per_step"], 3),
                 "batched_vs_plain_speedup": round(m5["plain_ms_per_step"] / m5["ms_per_step"], 3),
                 "step_alg_bytes": b5,
                 "step_hbm_frac": round(b5 / (m5["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "kernels": [{"kernel": k, "ms_per_step": round(a, 4), "launches_per_step": c}
                             for k, a, b, c in m5["table"][:12]]}
        del m5
        _log(f"large: {large['ms_per_step']} ms/step")

    # ---- the uneven 64-instance batch beside its per-instance form ---------
    uneven = uneven_line(args.uneven_steps, max(1, args.profile_steps // 4)) if args.uneven and args.config == 2 else None
    if uneven:
        _log(f"uneven: {uneven['ms_per_step']} ms/step")

    # ---- the two-stage fit of the cross-platform application ---------------
    fit = None
    if args.fit and args.config == 2:
        from paper_2204_01386_amd import scenes as _sc
        from paper_2204_01386_amd.fit import run_fit
        fr = run_fit(_sc.fit_scene())
        _log(f"fit: {fr['ms_per_iteration']} ms/iteration")
        c = fr["curve"]
        first = next(x for x in c if x["stage"] == "silhouette")
        last_sil = [x for x in c if x["stage"] == "silhouette"][-1]
        t0 = next(x for x in c if x["stage"] == "texture")
        last = c[-1]
        fit = {"workload": fr["workload"], "views": fr["views"], "H": fr["H"], "triangles": fr["triangles"],
               "iterations": fr["iterations"], "ms_per_iteration": fr["ms_per_iteration"],
               "silhouette_l2": [first["sil_l2"], last_sil["sil_l2"]],
               "surface_distance": [first["surface_distance"], last_sil["surface_distance"]],
               "color_l2": [t0["color_l2"], last["color_l2"]], "bin_overflow": fr["bin_overflow"]}

    # ---- image-based PBS: the environment-map fit -------------------------
    pbs = None
    if args.fit and args.config == 2:
        from paper_2204_01386_amd.fit import run_env_fit
        er = run_env_fit()
        _log(f"environment-map fit: {er['ms_per_iteration']} ms/iteration")
        c0, c1 = er["curve"][0], er["curve"][-1]
        pbs = {"workload": er["workload"], "iterations": er["iterations"], "ms_per_iteration": er["ms_per_iteration"],
               "loss": [c0["loss"], c1["loss"]], "env_rel_error": [c0["env_rel_error"], c1["env_rel_error"]],
               "roughness": [c0["roughness"], c1["roughness"]], "roughness_target": er["material_target"][1],
               "kernels_ms": er["kernels"][:10]}

    # ---- CPU baseline: the oracle's step on the same workload --------------
    cpu = None
    if not args.no_cpu:
        nc = _ncpu()
        ms1, n1, px = oracle_rate(scene, args.cpu_seconds, 1)
        _log(f"oracle, one core: {ms1:.1f} ms/step")
        msa, na, _ = oracle_rate(scene, args.cpu_seconds, nc)
        _log(f"oracle, {nc} threads: {msa:.1f} ms/step")
        cpu = {"value": round(px / (msa * 1e-3) / 1e6, 4), "unit": "Mpix/s", "cores": nc, "kind": "oracle",
               "sample": f"{na} full fwd+bwd steps of the same workload (C oracle, fp64), {msa:.1f} ms/step "
                         f"with {nc} threads (OpenMP per-pixel and per-texel loops, rasterization in row bands), "
                         f"on {_host_cpu()}",
               "single_core": {"value": round(px / (ms1 * 1e-3) / 1e6, 4), "unit": "Mpix/s", "cores": 1,
                               "sample": f"{n1} steps, {ms1:.1f} ms/step, one thread"}}
        if multi:
            s3, _ = scene_for(3)
            ms1, n1, px1 = oracle_rate(s3, 1.0, 1, views=range(2))
            _log(f"oracle, 16 views sample, one core: {ms1:.0f} ms/step")
            msa, na, pxa = oracle_rate(s3, 1.0, 1, view_threads=nc)
            _log(f"oracle, 16 views, {nc} threads: {msa:.0f} ms/step")
            multi["cpu_baseline"] = {
                "value": round(pxa / (msa * 1e-3) / 1e6, 4), "unit": "Mpix/s", "cores": nc, "kind": "oracle",
                "sample": f"{na} steps of all 16 views, one view per thread, {msa:.0f} ms/step",
                "single_core": {"value": round(px1 / (ms1 * 1e-3) / 1e6, 4), "unit": "Mpix/s", "cores": 1,
                                "sample": f"{n1} steps of views 1-2, one thread, {ms1:.0f} ms/step"}}
        if uneven:
            from paper_2204_01386_amd import scenes as _sc
            sub = _sc.config4()[:8]
            tms1 = tmsa = px1 = pxa = 0.0
            for sc in sub[:2]:
                m_, _, p_ = oracle_rate(sc, 0.0, 1)
                tms1, px1 = tms1 + m_, px1 + p_
            from concurrent.futures import ThreadPoolExecutor
            t0 = time.perf_counter()
            with ThreadPoolExecutor(nc) as ex:
                pxa = sum(p_ for _, _, p_ in ex.map(lambda sc: oracle_rate(sc, 0.0, 1), sub))
            tmsa = (time.perf_counter() - t0) * 1e3
            uneven["cpu_baseline"] = {
                "value": round(pxa / (tmsa * 1e-3) / 1e6, 4), "unit": "Mpix/s", "cores": nc, "kind": "oracle",
                "sample": f"one step of instances 1-8 ({pxa / 1e6:.2f} Mpix), one instance per thread, "
                          f"{tmsa:.0f} ms",
                "single_core": {"value": round(px1 / (tms1 * 1e-3) / 1e6, 4), "unit": "Mpix/s", "cores": 1,
                                "sample": f"one step of instances 1-2 ({px1 / 1e6:.2f} Mpix), one thread, "
                                          f"{tms1:.0f} ms"}}

    pix = B * scene.H * scene.W
    cbw = copy_bandwidth()

    def copy_frac(nbytes, ms):
        return round(nbytes / (ms * 1e-3) / 1e9 / cbw["gbs"], 4)

    if multi:
        multi["step_copy_frac"] = copy_frac(multi["step_alg_bytes"], multi["ms_per_step"])
    if uneven and uneven.get("step_alg_bytes"):
        uneven["step_copy_frac"] = copy_frac(uneven["step_alg_bytes"], uneven["ms_per_step"])
    if large:
        large["step_copy_frac"] = copy_frac(large["step_alg_bytes"], large["ms_per_step"])
    res = {
        "metric": "fwd+bwd Mpix/s & tris/s at 512^2 80k tris; batched vs plain speedup, %HBM roofline",
        "value": round(pix / (ms_batched * 1e-3) / 1e6, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_batched, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded meshes, value-noise textures)",
        "config": {"workload": desc, "views": B, "H": scene.H, "W": scene.W,
                   "triangles": int(scene.tris.shape[0]), "vertices": int(scene.pos.shape[0]),
                   "K": scene.K, "r": scene.r},
        "tris_per_s": round(B * scene.tris.shape[0] / (ms_batched * 1e-3), 1),
        "plain": {"ms_per_step": round(ms_plain, 5),
                  "value": round(pix / (ms_plain * 1e-3) / 1e6, 3), "unit": "Mpix/s"},
        "batched_vs_plain_speedup": round(ms_plain / ms_batched, 3),
        "autotune": tuned,
        "texture_only": None if ms_tex is None else {
            "ms_per_step": round(ms_tex, 5), "full_over_texture_only": round(ms_batched / ms_tex, 3),
            "note": "textures optimised on fixed geometry: rasterization and inverse-UV map cached"},
        "step_alg_bytes": step_bytes,
        "step_hbm_frac": round(step_bytes / (ms_batched * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "step_copy_frac": copy_frac(step_bytes, ms_batched),
        "hbm_copy": cbw,
        "roofline": {"bound": "hbm", "kernel": dom[0],
                     "achieved": round(achieved, 2) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": traffic_bytes(dom[0]),
                     "alg_bytes_per_launch": dom_bytes,
                     "ms_per_launch": round(dom[2], 5),
                     "selection": "most algorithmic bytes per step"},
        "longest_kernel": longest_json,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "fit": fit,
        "pbs_env_fit": pbs,
        "multiview": multi,
        "uneven": uneven,
        "large": large,
        "kernels": kernel_rows,
        "launches": launch_rows,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
