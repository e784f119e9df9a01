"""Seeded synthetic workloads shaped like the paper's experiments (§5.1, §4.3, appendix).

This module only *generates inputs*: meshes, per-corner UVs, value-noise textures,
normal maps, cube environment maps and camera matrices.  It holds none of the
renderer's arithmetic (no projection of vertices, no rasterization, no shading),
so both the HIP path and the CPU oracle can consume its arrays without sharing
any computation.

Every generator takes an explicit ``seed`` and draws from
``numpy.random.default_rng(seed)``.  Arrays are returned as float32 / int32
numpy arrays in the layouts the C-ABI expects:

* positions ``[V,3]``, triangles ``[T,3]`` (counter-clockwise seen from outside),
* per-corner attribute tables ``[Va,C]`` indexed by ``attr_tris [T,3]``,
* textures ``[Ht,Wt,Ct]`` (row 0 = v in [0, 1/Ht)), cube maps ``[6,S,S,C]``
  in the face order +X, -X, +Y, -Y, +Z, -Z,
* view-projection matrices ``[B,4,4]`` mapping ``[x,y,z,1]`` (column vector)
  to clip space with ``w = -z_view`` and ``z/w`` in [0,1] between the near and
  far planes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NEAR = 0.1
FAR = 10.0
FOV_Y_DEG = 60.0


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def icosphere(subdiv: int):
    """Unit icosphere: 10*4^s+2 vertices, 20*4^s triangles."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = f
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts, dtype=np.float64), np.array(faces, dtype=np.int32)


def vertex_neighbours(tris: np.ndarray, V: int):
    nb = [set() for _ in range(V)]
    for a, b, c in tris:
        nb[a].update((b, c))
        nb[b].update((a, c))
        nb[c].update((a, b))
    return [np.fromiter(s, dtype=np.int64) for s in nb]


def smooth_noise(rng, tris, V, iters=5):
    """N(0,1) per vertex smoothed by `iters` Jacobi neighbour-averaging passes."""
    n = rng.standard_normal(V)
    nb = vertex_neighbours(tris, V)
    lens = np.array([len(x) for x in nb], dtype=np.float64)
    flat = np.concatenate(nb)
    seg = np.repeat(np.arange(V), [len(x) for x in nb])
    for _ in range(iters):
        s = np.zeros(V)
        np.add.at(s, seg, n[flat])
        n = s / np.maximum(lens, 1)
    return n


def noisy_sphere(subdiv: int, seed: int, amp: float = 0.05):
    """Icosphere whose radius is scaled per vertex by 1 + amp * smoothed N(0,1)."""
    rng = np.random.default_rng(seed)
    p, tris = icosphere(subdiv)
    n = smooth_noise(rng, tris, len(p))
    p = p * (1.0 + amp * n)[:, None]
    return p.astype(np.float32), tris


def spherical_uv(pos: np.ndarray, tris: np.ndarray):
    """Per-corner spherical UVs u = 1/2 + atan2(z,x)/2pi, v = acos(y)/pi.

    Triangles crossing the u seam get +1 on their small-u corners, so u stays
    continuous inside every triangle (sampled with repeat in u).  Corners are
    de-duplicated into a UV vertex table indexed by ``uv_tris``.
    """
    d = pos / np.linalg.norm(pos, axis=1, keepdims=True)
    u = 0.5 + np.arctan2(d[:, 2], d[:, 0]) / (2 * math.pi)
    v = np.arccos(np.clip(d[:, 1], -1, 1)) / math.pi
    cu = u[tris]                      # [T,3]
    cv = v[tris]
    span = cu.max(1) - cu.min(1)
    seam = span > 0.5
    shift = seam[:, None] & (cu < 0.5)
    cu = cu + shift
    key = tris.astype(np.int64) * 2 + shift.astype(np.int64)
    uniq, inv = np.unique(key.ravel(), return_inverse=True)
    uv = np.zeros((len(uniq), 2), dtype=np.float64)
    uv[inv, 0] = cu.ravel()
    uv[inv, 1] = cv.ravel()
    return uv.astype(np.float32), inv.reshape(-1, 3).astype(np.int32)


def grid_surface(nu: int, nv: int, fn, wrap_v: bool):
    """Parametric quad grid (u wraps, v wraps if `wrap_v`), two triangles per quad."""
    us = np.arange(nu) / nu
    rows = nv if wrap_v else nv + 1
    vs = np.arange(rows) / (nv if wrap_v else nv)
    U, Vv = np.meshgrid(us, vs, indexing="ij")        # [nu, rows]
    P = fn(U, Vv)                                      # [nu, rows, 3]
    pos = P.reshape(-1, 3)
    idx = lambda i, j: (i % nu) * rows + (j % rows)
    tris = []
    for i in range(nu):
        for j in range(nv):
            a, b = idx(i, j), idx(i + 1, j)
            c, d = idx(i + 1, j + 1), idx(i, j + 1)
            tris.append((a, b, c))
            tris.append((a, c, d))
    return pos, np.array(tris, dtype=np.int32), U.ravel(), Vv.ravel()


def torus(nu: int, nv: int, R=0.7, r=0.3):
    """Torus (major radius R, tube radius r) as an nu x nv quad grid, outward CCW."""
    def fn(U, V):
        a, b = 2 * math.pi * U, 2 * math.pi * V
        return np.stack([(R + r * np.cos(b)) * np.cos(a), r * np.sin(b),
                         (R + r * np.cos(b)) * np.sin(a)], -1)
    pos, tris, _, _ = grid_surface(nu, nv, fn, wrap_v=True)
    # outward = away from the core circle of radius R in the xz plane
    c = pos[tris].mean(1)
    n = np.cross(pos[tris[:, 1]] - pos[tris[:, 0]], pos[tris[:, 2]] - pos[tris[:, 0]])
    ring = c[:, [0, 2]] / np.linalg.norm(c[:, [0, 2]], axis=1, keepdims=True) * R
    out = c - np.stack([ring[:, 0], np.zeros(len(c)), ring[:, 1]], -1)
    if (n * out).sum(1).mean() < 0:
        tris = tris[:, [0, 2, 1]].copy()
    return pos, tris


def grid_tris(nu: int, nv: int):
    """Triangles of an nu x nv quad grid wrapping in both directions (vertex
    (i, j) has index i * nv + j), two per quad, vectorised."""
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = i * nv + j
    b = ((i + 1) % nu) * nv + j
    c = ((i + 1) % nu) * nv + (j + 1) % nv
    d = i * nv + (j + 1) % nv
    t = np.stack([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], 2)
    return t.reshape(-1, 3).astype(np.int32)


def smooth_noise_edges(rng, tris, V, iters=5):
    """N(0,1) per vertex smoothed by `iters` Jacobi neighbour-averaging passes
    (neighbours from the unique edges; vectorised for large meshes)."""
    n = rng.standard_normal(V)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.concatenate([e, e[:, ::-1]]).astype(np.int64)
    e = np.unique(e[:, 0] * V + e[:, 1])
    src, dst = e // V, e % V
    deg = np.bincount(src, minlength=V).astype(np.float64)
    for _ in range(iters):
        n = np.bincount(src, weights=n[dst], minlength=V) / np.maximum(deg, 1)
    return n


def torus_knot(nu: int = 2048, nv: int = 256, p: int = 2, q: int = 3, radius: float = 0.15,
               seed: int = 0, amp: float = 0.05):
    """(p,q) torus-knot tube: core curve ((2 + cos qt) cos pt, (2 + cos qt) sin pt,
    sin qt), Frenet frame, tube radius radius * (1 + amp * smoothed N(0,1)) per
    vertex, scaled to fit the unit sphere.  nu x nv grid wrapping both ways:
    V = nu nv, T = 2 nu nv, outward counter-clockwise.  Per-corner UVs
    (8 i / nu, j / nv) on an (nu+1) x (nv+1) UV grid (seams split), repeat."""
    t = 2 * math.pi * np.arange(nu) / nu
    r = 2.0 + np.cos(q * t)
    c = np.stack([r * np.cos(p * t), r * np.sin(p * t), np.sin(q * t)], -1)
    dr = -q * np.sin(q * t)
    d1 = np.stack([dr * np.cos(p * t) - p * r * np.sin(p * t),
                   dr * np.sin(p * t) + p * r * np.cos(p * t), q * np.cos(q * t)], -1)
    ddr = -q * q * np.cos(q * t)
    d2 = np.stack([ddr * np.cos(p * t) - 2 * p * dr * np.sin(p * t) - p * p * r * np.cos(p * t),
                   ddr * np.sin(p * t) + 2 * p * dr * np.cos(p * t) - p * p * r * np.sin(p * t),
                   -q * q * np.sin(q * t)], -1)
    T_ = d1 / np.linalg.norm(d1, axis=1, keepdims=True)
    N_ = d2 - (d2 * T_).sum(1, keepdims=True) * T_
    N_ /= np.linalg.norm(N_, axis=1, keepdims=True)
    B_ = np.cross(T_, N_)
    tris = grid_tris(nu, nv)
    V = nu * nv
    rng = np.random.default_rng(seed)
    rad = radius * (1.0 + amp * smooth_noise_edges(rng, tris, V)).reshape(nu, nv)
    phi = 2 * math.pi * np.arange(nv) / nv
    ring = np.cos(phi)[None, :, None] * N_[:, None, :] + np.sin(phi)[None, :, None] * B_[:, None, :]
    pos = (c[:, None, :] + rad[:, :, None] * ring).reshape(-1, 3)
    pos = pos / np.linalg.norm(pos, axis=1).max()
    # outward: away from the (equally scaled) core curve
    ctr = np.repeat(c / np.linalg.norm(c[:, None, :] + rad[:, :, None] * ring, axis=2).max(), nv, 0)
    fn = np.cross(pos[tris[:, 1]] - pos[tris[:, 0]], pos[tris[:, 2]] - pos[tris[:, 0]])
    out = pos[tris].mean(1) - ctr[tris[:, 0]]
    if (fn * out).sum(1).mean() < 0:
        tris = tris[:, [0, 2, 1]].copy()
    # UVs: corner (i, j) -> (8 i / nu, j / nv) with i, j unwrapped at the seams
    iu = np.arange(nu + 1)
    jv = np.arange(nv + 1)
    U, Vv = np.meshgrid(8.0 * iu / nu, jv / nv, indexing="ij")
    uv = np.stack([U, Vv], -1).reshape(-1, 2)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = i * (nv + 1) + j
    b = (i + 1) * (nv + 1) + j
    cc = (i + 1) * (nv + 1) + j + 1
    d = i * (nv + 1) + j + 1
    uv_tris = np.stack([np.stack([a, b, cc], -1), np.stack([a, cc, d], -1)], 2).reshape(-1, 3)
    if not np.array_equal(tris, grid_tris(nu, nv)):
        uv_tris = uv_tris[:, [0, 2, 1]]
    return pos.astype(np.float32), tris, uv.astype(np.float32), uv_tris.astype(np.int32)


def uv_sphere(nu: int, nv: int, seed: int, amp: float = 0.05):
    """Latitude-longitude sphere: nu columns (wrapping) x (nv + 1) rows from
    pole to pole (the pole rows are coincident vertices), 2 nu nv triangles,
    radius scaled per vertex by 1 + amp * smoothed N(0,1).  Per-corner UVs
    (i / nu, j / nv) on an (nu+1) x (nv+1) grid (seam split)."""
    i, j = np.meshgrid(np.arange(nu), np.arange(nv + 1), indexing="ij")
    th, ph = 2 * math.pi * i / nu, math.pi * j / nv
    pos = np.stack([np.sin(ph) * np.cos(th), np.cos(ph), np.sin(ph) * np.sin(th)], -1).reshape(-1, 3)
    R = nv + 1
    ii, jj = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = ii * R + jj
    b = ((ii + 1) % nu) * R + jj
    c = ((ii + 1) % nu) * R + jj + 1
    d = ii * R + jj + 1
    tris = np.stack([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], 2).reshape(-1, 3).astype(np.int32)
    rng = np.random.default_rng(seed)
    pos = pos * (1.0 + amp * smooth_noise_edges(rng, tris, len(pos)))[:, None]
    U, Vv = np.meshgrid(np.arange(nu + 1) / nu, np.arange(nv + 1) / nv, indexing="ij")
    uv = np.stack([U, Vv], -1).reshape(-1, 2)
    ua = ii * (nv + 1) + jj
    ub = (ii + 1) * (nv + 1) + jj
    uc = (ii + 1) * (nv + 1) + jj + 1
    ud = ii * (nv + 1) + jj + 1
    uv_tris = np.stack([np.stack([ua, ub, uc], -1), np.stack([ua, uc, ud], -1)], 2).reshape(-1, 3)
    return pos.astype(np.float32), tris, uv.astype(np.float32), uv_tris.astype(np.int32)


def noisy_torus(nu: int, nv: int, seed: int, R: float = 0.7, r: float = 0.3, amp: float = 0.05):
    """Torus as an nu x nv grid wrapping both ways (2 nu nv triangles, outward
    counter-clockwise), tube radius r * (1 + amp * smoothed N(0,1)) per vertex.
    Per-corner UVs (i / nu, j / nv) on an (nu+1) x (nv+1) grid (seams split)."""
    tris = grid_tris(nu, nv)
    rng = np.random.default_rng(seed)
    rad = r * (1.0 + amp * smooth_noise_edges(rng, tris, nu * nv)).reshape(nu, nv)
    a = 2 * math.pi * np.arange(nu)[:, None] / nu
    b = 2 * math.pi * np.arange(nv)[None, :] / nv
    pos = np.stack([(R + rad * np.cos(b)) * np.cos(a), rad * np.sin(b), (R + rad * np.cos(b)) * np.sin(a)],
                   -1).reshape(-1, 3)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    ua = i * (nv + 1) + j
    ub = (i + 1) * (nv + 1) + j
    uc = (i + 1) * (nv + 1) + j + 1
    ud = i * (nv + 1) + j + 1
    uv_tris = np.stack([np.stack([ua, ub, uc], -1), np.stack([ua, uc, ud], -1)], 2).reshape(-1, 3)
    # outward orientation: away from the core circle of radius R in the xz plane
    c = pos[tris].mean(1)
    n = np.cross(pos[tris[:, 1]] - pos[tris[:, 0]], pos[tris[:, 2]] - pos[tris[:, 0]])
    ring = c[:, [0, 2]] / np.linalg.norm(c[:, [0, 2]], axis=1, keepdims=True) * R
    out = c - np.stack([ring[:, 0], np.zeros(len(c)), ring[:, 1]], -1)
    if (n * out).sum(1).mean() < 0:
        tris = tris[:, [0, 2, 1]].copy()
        uv_tris = uv_tris[:, [0, 2, 1]]
    U, Vv = np.meshgrid(np.arange(nu + 1) / nu, np.arange(nv + 1) / nv, indexing="ij")
    uv = np.stack([U, Vv], -1).reshape(-1, 2)
    return pos.astype(np.float32), tris, uv.astype(np.float32), uv_tris.astype(np.int32)


# --------------------------------------------------------------------------
# textures
# --------------------------------------------------------------------------
def value_noise(H: int, W: int, C: int, seed: int, octaves: int = 4, base: int = 8):
    """Tileable value noise in [0,1]: `octaves` octaves, lattice `base` cells
    doubling per octave, smoothstep interpolation, amplitude 1/2^o, each channel
    independent, normalized to [0,1] per channel."""
    rng = np.random.default_rng(seed)
    out = np.zeros((H, W, C), dtype=np.float64)
    ys = (np.arange(H) + 0.5) / H
    xs = (np.arange(W) + 0.5) / W
    for o in range(octaves):
        n = base * (2 ** o)
        lat = rng.random((n, n, C))
        fy, fx = ys * n, xs * n
        y0, x0 = np.floor(fy).astype(int), np.floor(fx).astype(int)
        ty, tx = fy - y0, fx - x0
        sy, sx = ty * ty * (3 - 2 * ty), tx * tx * (3 - 2 * tx)
        y1, x1 = (y0 + 1) % n, (x0 + 1) % n
        y0, x0 = y0 % n, x0 % n
        # interpolate every lattice row along x once, then between rows along y
        a = lat[:, x0]
        lx = a + (lat[:, x1] - a) * sx[None, :, None]          # [n, W, C]
        for r0 in range(0, H, 256):                            # row bands bound the temporaries
            r1 = min(H, r0 + 256)
            top = lx[y0[r0:r1]]
            bot = lx[y1[r0:r1]]
            out[r0:r1] += (top + (bot - top) * sy[r0:r1, None, None]) * (0.5 ** o)
    lo = out.min(axis=(0, 1), keepdims=True)
    hi = out.max(axis=(0, 1), keepdims=True)
    return ((out - lo) / np.maximum(hi - lo, 1e-12)).astype(np.float32)


def normal_map(H: int, W: int, seed: int, strength: float = 0.3):
    """Tangent-space normal map: normalize((0,0,1) + s*(2n1-1, 2n2-1, 0))."""
    n = value_noise(H, W, 2, seed).astype(np.float64)
    m = np.zeros((H, W, 3))
    m[..., 0] = strength * (2 * n[..., 0] - 1)
    m[..., 1] = strength * (2 * n[..., 1] - 1)
    m[..., 2] = 1.0
    m /= np.linalg.norm(m, axis=-1, keepdims=True)
    return m.astype(np.float32)


def cube_env_map(S: int, seed: int, C: int = 3):
    """6xSxSxC sky-gradient cube map (+0.2 value noise), faces +X,-X,+Y,-Y,+Z,-Z."""
    noise = value_noise(S, S * 6, C, seed).reshape(S, 6, S, C).transpose(1, 0, 2, 3)
    out = np.zeros((6, S, S, C), dtype=np.float64)
    t = (np.arange(S) + 0.5) / S
    sky = np.array([0.35, 0.55, 0.9])[:C]
    ground = np.array([0.3, 0.25, 0.2])[:C]
    for f in range(6):
        if f == 2:
            g = np.ones((S, S))
        elif f == 3:
            g = np.zeros((S, S))
        else:
            g = np.repeat((1.0 - t)[:, None], S, 1)   # row 0 = up on side faces
        out[f] = ground + (sky - ground) * g[..., None]
    out += 0.2 * noise
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(np.dot(f, up)) > 0.999:
        up = np.array([0.0, 0.0, 1.0])
    s = np.cross(f, up)
    s /= np.linalg.norm(s)
    u = np.cross(s, f)
    M = np.eye(4)
    M[0, :3], M[1, :3], M[2, :3] = s, u, -f
    M[:3, 3] = -M[:3, :3] @ eye
    return M


def perspective(fov_y_deg=FOV_Y_DEG, aspect=1.0, near=NEAR, far=FAR):
    """Clip w = -z_view = d, z_clip/w = far (d - near) / (d (far - near)) in [0,1]."""
    f = 1.0 / math.tan(math.radians(fov_y_deg) / 2)
    P = np.zeros((4, 4))
    P[0, 0] = f / aspect
    P[1, 1] = f
    P[2, 2] = -far / (far - near)
    P[2, 3] = -far * near / (far - near)
    P[3, 2] = -1.0
    return P


def camera_ring(n: int, seed: int, radius=3.0, elev_deg=60.0):
    """n cameras at `radius`, azimuth ~U(0,2pi), elevation ~U(-elev, elev)."""
    rng = np.random.default_rng(seed)
    az = rng.uniform(0, 2 * math.pi, n)
    el = np.radians(rng.uniform(-elev_deg, elev_deg, n))
    eyes = np.stack([radius * np.cos(el) * np.sin(az), radius * np.sin(el),
                     radius * np.cos(el) * np.cos(az)], -1)
    return eyes


def view_proj(eyes):
    P = perspective()
    return np.stack([P @ look_at(e) for e in np.atleast_2d(eyes)]).astype(np.float32)


# --------------------------------------------------------------------------
# the five benchmark scenes
# --------------------------------------------------------------------------
@dataclass
class Scene:
    name: str
    pos: np.ndarray                 # [V,3] f32
    tris: np.ndarray                # [T,3] i32
    mvp: np.ndarray                 # [B,4,4] f32
    eyes: np.ndarray                # [B,3] f32 camera positions (world)
    H: int
    W: int
    K: int = 1
    r: float = 0.0
    shading: str = "lambert"
    color: np.ndarray | None = None         # [V,3] per-vertex colour (lambert)
    uv: np.ndarray | None = None            # [Vuv,2]
    uv_tris: np.ndarray | None = None       # [T,3]
    tex: np.ndarray | None = None           # [Ht,Wt,4]
    nmap: np.ndarray | None = None          # [Hn,Wn,3]
    env: np.ndarray | None = None           # [6,S,S,3]
    target_pos: np.ndarray | None = None
    target_color: np.ndarray | None = None
    target_tex: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def config1(seed: int = 0) -> Scene:
    """Icosphere s3 (642 v, 1280 t), radius 1, per-vertex RGB ~U(0,1), camera at
    (0,0,3), 128x128, K=1, r=0, Lambert; target = positions + N(0,0.02)."""
    rng = np.random.default_rng(seed)
    p, tris = icosphere(3)
    color = rng.random((len(p), 3)).astype(np.float32)
    trng = np.random.default_rng([seed, 1])
    tpos = p + trng.normal(0.0, 0.02, p.shape)
    eyes = np.array([[0.0, 0.0, 3.0]])
    return Scene("icosphere3-128", p.astype(np.float32), tris, view_proj(eyes),
                 eyes.astype(np.float32), 128, 128, 1, 0.0, "lambert",
                 color=color, target_pos=tpos.astype(np.float32), target_color=color)


def config2(seed: int = 0, H: int = 512, subdiv: int = 6, tex_size: int = 1024) -> Scene:
    """Noisy icosphere s6 (40962 v, 81920 t), spherical UVs, 1024^2 RGBA value
    noise, one view at 512^2, K=1, Phong.  Target: perturbed mesh, texture seed+1."""
    p, tris = noisy_sphere(subdiv, seed)
    uv, uv_tris = spherical_uv(p, tris)
    tex = value_noise(tex_size, tex_size, 4, seed)
    tp, _ = noisy_sphere(subdiv, seed + 1)
    eyes = np.array([[0.0, 0.0, 3.0]])
    return Scene(f"noisy-icosphere{subdiv}-{H}", p, tris, view_proj(eyes),
                 eyes.astype(np.float32), H, H, 1, 0.0, "phong",
                 uv=uv, uv_tris=uv_tris, tex=tex, target_pos=tp,
                 target_tex=value_noise(tex_size, tex_size, 4, seed + 1))


def config3(seed: int = 0, n_views: int = 16, H: int = 512, subdiv: int = 6,
            tex_size: int = 1024, env_size: int = 128) -> Scene:
    """Config-2 mesh/texture seen by 16 random cameras (radius 3, elevation in
    +-60 deg), 1024^2 tangent-space normal map, 6x128^2 cube env map,
    HardSoftRas K=3, r=0.01, Phong + env reflection."""
    s = config2(seed, H, subdiv, tex_size)
    eyes = camera_ring(n_views, seed)
    s.name = f"noisy-icosphere{subdiv}-{n_views}x{H}-hsr"
    s.mvp = view_proj(eyes)
    s.eyes = eyes.astype(np.float32)
    s.K, s.r = 3, 0.01
    s.shading = "phong_env"
    s.nmap = normal_map(tex_size, tex_size, seed + 7)
    s.env = cube_env_map(env_size, seed + 11)
    s.extra["tangent"] = sphere_tangents(s.pos)
    return s


def config4(seed: int = 0, n: int = 64, t_min: float = 1e3, t_max: float = 2e5,
            sizes=(256, 512, 768, 1024), tex_size: int = 512) -> list:
    """Uneven batch: n instances, T_i = round(exp(U(ln t_min, ln t_max)))
    triangles, each a latitude-longitude sphere (nu = 2 nv) or a torus
    (nu = 3 nv) with 2 nu nv close to T_i and radial noise as in config 2,
    seen by its own camera (radius 3, random direction) at a resolution drawn
    from `sizes`, with its own tex_size^2 RGBA value-noise texture; K=1,
    Phong, repeat wrap.  Target: noise seed+1, texture seed+1.  Returns one
    standalone Scene per instance."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        T = int(round(math.exp(rng.uniform(math.log(t_min), math.log(t_max)))))
        torus_kind = bool(rng.integers(2))
        res = int(sizes[rng.integers(len(sizes))])
        s_i = 1000 * (seed + 1) + i
        if torus_kind:
            nv = max(3, int(round(math.sqrt(T / 6.0))))
            nu = max(3, int(round(T / (2.0 * nv))))
            p, tris, uv, uv_tris = noisy_torus(nu, nv, s_i)
            tp, _, _, _ = noisy_torus(nu, nv, s_i + 1)
        else:
            nv = max(3, int(round(math.sqrt(T / 4.0))))
            nu = max(3, int(round(T / (2.0 * nv))))
            p, tris, uv, uv_tris = uv_sphere(nu, nv, s_i)
            tp, _, _, _ = uv_sphere(nu, nv, s_i + 1)
        eyes = camera_ring(1, s_i)
        sc = Scene(f"inst{i}-{'torus' if torus_kind else 'sphere'}{nu}x{nv}-{res}", p, tris, view_proj(eyes),
                   eyes.astype(np.float32), res, res, 1, 0.0, "phong", uv=uv, uv_tris=uv_tris,
                   tex=value_noise(tex_size, tex_size, 4, s_i), target_pos=tp,
                   target_tex=value_noise(tex_size, tex_size, 4, s_i + 1))
        sc.extra["wrap"] = (0, 0)   # repeat in u and v
        out.append(sc)
    return out


def config5(seed: int = 0, n_views: int = 8, H: int = 2048, nu: int = 2048, nv: int = 256,
            tex_size: int = 4096) -> Scene:
    """(2,3) torus-knot tube, 2048 x 256 grid (1,048,576 triangles, 524,288
    vertices), per-corner UVs (8 i/2048, j/256) on a 4096^2 RGBA fp32 value-noise
    texture (repeat), 8 cameras as in config 3 at 2048^2, HardSoftRas K=3,
    r=0.01, Phong.  Target: tube noise seed+1, texture seed+1."""
    p, tris, uv, uv_tris = torus_knot(nu, nv, seed=seed)
    tp, _, _, _ = torus_knot(nu, nv, seed=seed + 1)
    eyes = camera_ring(n_views, seed)
    s = Scene(f"torus-knot-{nu}x{nv}-{n_views}x{H}-hsr", p, tris, view_proj(eyes), eyes.astype(np.float32),
              H, H, 3, 0.01, "phong", uv=uv, uv_tris=uv_tris,
              tex=value_noise(tex_size, tex_size, 4, seed), target_pos=tp,
              target_tex=value_noise(tex_size, tex_size, 4, seed + 1))
    s.extra["wrap"] = (0, 0)   # repeat in u and v
    # the full form of the layers: at this reach (20 px) the blend's edge band
    # covers nearly the whole tube, so the edge-band form saves no soft work
    s.extra["band"] = False
    return s


def paper_table_scene(triangles: int, H: int, n_views: int = 6, seed: int = 0) -> Scene:
    """A workload shaped like the paper's non-textured timing table (§5.1):
    a noisy latitude-longitude sphere with about `triangles` triangles
    (2 nu nv with nu = 2 nv), white vertex colour, Lambert, K = 1, seen by
    `n_views` cameras on the ring of config 3 at H x H; target: positions +
    N(0, 0.02)."""
    nv = max(3, int(round(math.sqrt(triangles / 4.0))))
    p, tris, _, _ = uv_sphere(2 * nv, nv, seed)
    white = np.ones((len(p), 3), np.float32)
    trng = np.random.default_rng([seed, 1])
    tpos = (p + trng.normal(0.0, 0.02, p.shape)).astype(np.float32)
    eyes = camera_ring(n_views, seed)
    return Scene(f"paper-table-{len(tris)}-{H}", p, tris, view_proj(eyes), eyes.astype(np.float32), H, H, 1, 0.0,
                 "lambert", color=white, target_pos=tpos, target_color=white)


def sphere_tangents(pos: np.ndarray):
    """Raw per-vertex tangent (-sin phi, 0, cos phi), phi = atan2(z, x): the
    direction of growing u of the spherical UVs (orthogonalised per pixel)."""
    phi = np.arctan2(pos[:, 2].astype(np.float64), pos[:, 0].astype(np.float64))
    return np.stack([-np.sin(phi), np.zeros_like(phi), np.cos(phi)], -1).astype(np.float32)


def pear_surface(d: np.ndarray) -> np.ndarray:
    """A smooth pear-like closed surface over unit directions d [N,3]: a
    radius that narrows towards +y, a wider bulb towards -y, stretched along y."""
    y = d[:, 1]
    rad = 0.62 - 0.16 * y + 0.10 * np.cos(2.4 * (y + 0.35)) + 0.04 * d[:, 0] * d[:, 2]
    p = d * rad[:, None]
    p[:, 1] = 1.3 * p[:, 1] + 0.27    # centred on the origin
    return p


def fit_scene(seed: int = 0, subdiv: int = 4, H: int = 256, tex_size: int = 256, n_views: int = 6,
              K: int = 2, r: float = 0.01, blend: str = "hsr") -> Scene:
    """The optimisation workload of the paper's cross-platform application
    (§4.1): a white sphere with a white albedo texture fitted to images of a
    pear, in 6 views of 256^2 with a 256^2 albedo texture.  The pear here is
    synthetic: the same icosphere topology mapped onto `pear_surface`, with a
    value-noise albedo.  HardSoftRas K = 2, r = 0.01, sigma = r/7, delta = r
    (the listing's parameters); Phong; cameras on the ring of config 3.
    `blend` picks another setting of the blend ("aa", "softras")."""
    p, tris = icosphere(subdiv)
    uv, uv_tris = spherical_uv(p.astype(np.float32), tris)
    start = (0.7 * p).astype(np.float32)
    target = pear_surface(p).astype(np.float32)
    white = np.ones((tex_size, tex_size, 4), np.float32)
    eyes = camera_ring(n_views, seed)
    return Scene(f"fit-sphere{subdiv}-to-pear-{n_views}x{H}", start, tris, view_proj(eyes), eyes.astype(np.float32),
                 H, H, K, r, "phong", uv=uv, uv_tris=uv_tris, tex=white, target_pos=target,
                 target_tex=value_noise(tex_size, tex_size, 4, seed + 3), extra={"blend": blend})
