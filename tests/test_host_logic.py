"""Host-side logic that runs without a GPU: workload generators and the
packing of uneven batches."""
import numpy as np
import pytest

from paper_2204_01386_amd import scenes


def _pack():
    # pipeline imports torch and the binding only lazily through Step
    from paper_2204_01386_amd.pipeline import pack_views
    return pack_views


def test_pack_views_disjoint_tile_aligned_rectangles():
    pack_views = _pack()
    rng = np.random.default_rng(0)
    sizes = [(int(s), int(s)) for s in rng.choice([256, 512, 768, 1024], 64)]
    at, (Wc, Hc) = pack_views(sizes)
    occ = np.zeros((Hc // 16, Wc // 16), np.int32)
    for (x0, y0), (w, h) in zip(at, sizes):
        assert x0 % 16 == 0 and y0 % 16 == 0 and x0 + w <= Wc and y0 + h <= Hc
        occ[y0 // 16:(y0 + h) // 16, x0 // 16:(x0 + w) // 16] += 1
    assert occ.max() == 1, "views overlap"
    assert occ.sum() * 256 == sum(w * h for w, h in sizes)
    assert Wc * Hc < 1.6 * sum(w * h for w, h in sizes), "packing wastes too much"


def test_torus_knot_sizes_and_orientation():
    p, tris, uv, uv_tris = scenes.torus_knot(256, 32)
    assert p.shape == (256 * 32, 3) and tris.shape == (2 * 256 * 32, 3)
    assert abs(np.linalg.norm(p, axis=1).max() - 1.0) < 1e-6
    assert uv.shape == (257 * 33, 2) and uv_tris.shape == tris.shape
    # corner (i, j) of a triangle maps to UV grid corner (i, j) with the seams split
    nv = 32
    vi, vj = tris // nv, tris % nv
    ui, uj = uv_tris // (nv + 1), uv_tris % (nv + 1)
    assert np.array_equal(vi, ui % 256) and np.array_equal(vj, uj % nv)
    assert np.allclose(uv[uv_tris][..., 0], 8.0 * ui / 256) and np.allclose(uv[uv_tris][..., 1], uj / nv)


def test_config5_shape():
    p, tris, uv, uv_tris = scenes.torus_knot()
    assert tris.shape[0] == 1048576 and p.shape[0] == 524288


def test_config4_instances():
    sl = scenes.config4(n=64, tex_size=16)
    T = np.array([s.tris.shape[0] for s in sl])
    assert len(sl) == 64 and T.min() >= 700 and T.max() <= 2.1e5
    # log-uniform sizes: about half the instances below the geometric mean
    assert 20 <= (T < np.sqrt(1e3 * 2e5)).sum() <= 44
    assert {s.H for s in sl} <= {256, 512, 768, 1024} and all(s.H == s.W for s in sl)
    kinds = ["torus" in s.name for s in sl]
    assert 16 <= sum(kinds) <= 48
    for s in sl[:8]:
        # outward-facing: the (area-weighted) face normals point away from the centre on average
        fn = np.cross(s.pos[s.tris[:, 1]] - s.pos[s.tris[:, 0]], s.pos[s.tris[:, 2]] - s.pos[s.tris[:, 0]])
        c = s.pos[s.tris].mean(1)
        assert (fn * c).sum() > 0


@pytest.mark.parametrize("H,W,C", [(64, 48, 4), (33, 17, 3)])
def test_value_noise_range_and_tiling(H, W, C):
    t = scenes.value_noise(H, W, C, 3)
    assert t.shape == (H, W, C) and t.dtype == np.float32
    assert t.min() >= 0.0 and t.max() <= 1.0
    assert np.allclose(t.min(axis=(0, 1)), 0.0) and np.allclose(t.max(axis=(0, 1)), 1.0)


def test_paper_table_scene_shapes():
    """Sphere sizes near the paper's table meshes, six views, white Lambert."""
    for T in (682, 14208, 51414):
        sc = scenes.paper_table_scene(T, 256)
        assert abs(sc.tris.shape[0] - T) / T < 0.02
        assert sc.mvp.shape == (6, 4, 4) and sc.shading == "lambert" and sc.K == 1
        assert np.all(sc.color == 1.0) and sc.tris.max() < sc.pos.shape[0]


def test_fit_scene_and_surface_distance():
    """The fit scene: a sphere and a pear of one topology, both closed and
    outward-facing; the surface-distance metric is 0 on the surface itself,
    equals an offset of a sphere, and the start lies off the target."""
    from paper_2204_01386_amd.fit import mean_surface_distance, surface_samples
    from scipy.spatial import cKDTree
    s = scenes.fit_scene(subdiv=3)
    assert s.pos.shape == s.target_pos.shape and s.tris.max() < s.pos.shape[0]
    assert s.K == 2 and abs(s.r - 0.01) < 1e-12 and s.extra["blend"] == "hsr" and s.mvp.shape[0] == 6
    # every edge shared by exactly two triangles (closed), outward normals
    e = np.sort(np.concatenate([s.tris[:, [0, 1]], s.tris[:, [1, 2]], s.tris[:, [2, 0]]]), 1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    assert (cnt == 2).all()
    for p in (s.pos, s.target_pos):
        fn = np.cross(p[s.tris[:, 1]] - p[s.tris[:, 0]], p[s.tris[:, 2]] - p[s.tris[:, 0]])
        assert (fn * p[s.tris].mean(1)).sum() > 0
    tree = cKDTree(surface_samples(s.target_pos, s.tris))
    assert mean_surface_distance(s.target_pos, tree) == 0.0
    assert mean_surface_distance(s.pos, tree) > 0.02
    # a unit sphere's samples against points at radius 1.5: distance 0.5 (up to the sampling)
    p, tris = scenes.icosphere(3)
    tree = cKDTree(surface_samples(p, tris, n=8))
    d = mean_surface_distance(1.5 * p, tree)
    assert abs(d - 0.5) < 2e-3
