"""Pins for the oracle's rasteriser (Eq. 14), CPU only:
  * coverage and the chosen face against FP64 ray casting (Moller-Trumbore)
    through each pixel centre, away from edges and depth ties;
  * perspective-correct interpolation: radiance linear in world position is
    reproduced exactly at the ray's hit point on a tilted plane;
  * constant radiance gives a constant image (the weights sum to 1);
  * ties in depth go to the lower face index;
  * gradients against central finite differences."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import raster

W, H = 48, 40


def camera(f=40.0, cx=24.0, cy=20.0, R=None, t=(0.0, 0.0, 4.0)):
    R = np.eye(3) if R is None else R
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1.0]])
    return (K @ np.concatenate([R, np.asarray(t)[:, None]], 1)).astype(np.float32)


def icosphere_mesh(level=2, radius=1.0):
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    v = [np.array(p, float) / np.linalg.norm(p) for p in v]
    for _ in range(level):
        cache, nf = {}, []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return (np.array(v) * radius).astype(np.float32), np.array(f, np.int32)


def ray_cast(vertices, faces, P, i, j):
    """Nearest hit (face, distance) of the ray through pixel centre (i, j), FP64."""
    P = P.astype(np.float64)
    M, p4 = P[:, :3], P[:, 3]
    origin = -np.linalg.solve(M, p4)
    d = np.linalg.solve(M, np.array([i + 0.5, j + 0.5, 1.0]))
    best = (np.inf, -1)
    for fi, (a, b, c) in enumerate(faces):
        v0, v1, v2 = (vertices[k].astype(np.float64) for k in (a, b, c))
        e1, e2 = v1 - v0, v2 - v0
        pv = np.cross(d, e2)
        det = e1 @ pv
        if abs(det) < 1e-14:
            continue
        tv = origin - v0
        u = (tv @ pv) / det
        qv = np.cross(tv, e1)
        vv = (d @ qv) / det
        tt = (e2 @ qv) / det
        if u >= 0 and vv >= 0 and u + vv <= 1 and tt > 0 and tt < best[0]:
            best = (tt, fi)
    return best


def test_faces_match_ray_casting_away_from_edges():
    verts, faces = icosphere_mesh(2)
    P = camera()
    fid = raster.rasterize_ids(verts, faces, P, W, H)
    sx, sy, w = raster.project_f32(verts, P)
    checked = 0
    for j in range(0, H, 2):
        for i in range(0, W, 2):
            tt, f = ray_cast(verts, faces, P, i, j)
            if f < 0:
                continue
            a, b, c = faces[f]
            X, Y = [sx[a], sx[b], sx[c]], [sy[a], sy[b], sy[c]]
            area = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0])
            px, py = i + 0.5, j + 0.5
            lam = [((X[1] - px) * (Y[2] - py) - (X[2] - px) * (Y[1] - py)) / area,
                   ((X[2] - px) * (Y[0] - py) - (X[0] - px) * (Y[2] - py)) / area,
                   ((X[0] - px) * (Y[1] - py) - (X[1] - px) * (Y[0] - py)) / area]
            if min(lam) < 1e-3:
                continue                      # near an edge: either neighbour is valid
            assert fid[j, i] == f
            checked += 1
    assert checked > 50
    # pixels far outside the sphere's silhouette are background
    assert fid[0, 0] == -1 and fid[H - 1, W - 1] == -1


def test_perspective_correct_interpolation_of_a_linear_function():
    """A tilted square (two triangles) with B = a . x + c at its corners: the
    interpolated value at each covered pixel equals a . X + c at the ray's
    hit point X on the plane."""
    verts = np.array([[-1.0, -1.0, 0.6], [1.2, -1.0, -0.5], [1.2, 1.1, -0.5], [-1.0, 1.1, 0.6]], np.float32)
    faces = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    a, c0 = np.array([0.3, -0.7, 1.1]), 0.4
    B = (verts.astype(np.float64) @ a + c0).astype(np.float32)
    P = camera()
    fid, img = raster.render(verts, faces, B, P, W, H)
    Pd = P.astype(np.float64)
    M, p4 = Pd[:, :3], Pd[:, 3]
    origin = -np.linalg.solve(M, p4)
    v = verts.astype(np.float64)
    n = np.cross(v[1] - v[0], v[2] - v[0])
    covered = np.argwhere(fid >= 0)
    assert len(covered) > 200
    for j, i in covered:
        d = np.linalg.solve(M, np.array([i + 0.5, j + 0.5, 1.0]))
        t = ((v[0] - origin) @ n) / (d @ n)
        X = origin + t * d
        assert abs(float(img[j, i]) - (X @ a + c0)) < 2e-5


def test_constant_radiance_gives_a_constant_image():
    verts, faces = icosphere_mesh(1)
    B = np.full(len(verts), 0.75, np.float32)
    fid, img = raster.render(verts, faces, B, camera(), W, H)
    on = fid >= 0
    assert on.sum() > 300
    assert torch.allclose(img[torch.as_tensor(on)], torch.full((int(on.sum()),), 0.75, dtype=torch.float64),
                          rtol=0, atol=1e-12)
    assert not img[torch.as_tensor(~on)].any()


def test_depth_ties_go_to_the_lower_face_index_and_nearer_wins():
    tri = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float32)
    verts = np.concatenate([tri, tri, tri + np.array([0, 0, -0.5], np.float32)])
    faces = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)
    fid = raster.rasterize_ids(verts, faces, camera(), W, H)
    vals = set(np.unique(fid)) - {-1}
    assert vals == {2}                      # the nearer copy (z = -0.5 is nearer to a camera at z = -4)
    fid2 = raster.rasterize_ids(verts[:6], faces[:2], camera(), W, H)
    assert set(np.unique(fid2)) - {-1} == {0}


def test_gradients_against_central_differences():
    verts, faces = icosphere_mesh(1)
    rng = np.random.default_rng(0)
    B = rng.uniform(0.2, 1.0, len(verts)).astype(np.float32)
    P = camera()
    fid, img = raster.render(verts, faces, B, P, W, H)
    gI = rng.standard_normal((H, W)).astype(np.float32)
    gB, gv = raster.render_backward(verts, faces, B, P, fid, gI)
    v64 = torch.as_tensor(verts).double()
    B64 = torch.as_tensor(B).double()
    P64 = torch.as_tensor(P).double()
    gI64 = torch.as_tensor(gI).double()

    def loss(v, b):
        return float((raster.shade_pixels(v, faces, b, P64, fid) * gI64).sum())
    h = 1e-6
    for k in rng.choice(len(verts), 6, replace=False):
        e = torch.zeros_like(B64)
        e[k] = h
        fd = (loss(v64, B64 + e) - loss(v64, B64 - e)) / (2 * h)
        assert abs(fd - float(gB[k])) < 1e-7 * max(1.0, abs(fd))
        for d in range(3):
            e = torch.zeros_like(v64)
            e[k, d] = h
            fd = (loss(v64 + e, B64) - loss(v64 - e, B64)) / (2 * h)
            assert abs(fd - float(gv[k, d])) < 1e-5 * max(1.0, abs(fd))


def test_stress_scene_loads_the_binning_as_intended():
    """The rasteriser's stress scene (its GPU parity test relies on this):
    faces spanning more than 16 tiles, a tile list of several 64-entry chunks,
    and pixels whose nearest face has an exact twin later in the list; the
    twins never win (ties go to the lower index)."""
    sc = scenegen.scene_raster_stress()
    v, f, P, W, H = sc["points"], sc["faces"], sc["camera"], sc["width"], sc["height"]
    sx, sy, w = raster.project_f32(v, P)
    assert (w > 1.0).all()
    tiles = np.zeros(((H + 7) // 8, (W + 7) // 8), int)
    spanning = 0
    for a, b, c in f:
        xs, ys = sx[[a, b, c]], sy[[a, b, c]]
        i0, i1 = max(int(np.floor(xs.min() - 0.5)), 0), min(int(np.ceil(xs.max() - 0.5)), W - 1)
        j0, j1 = max(int(np.floor(ys.min() - 0.5)), 0), min(int(np.ceil(ys.max() - 0.5)), H - 1)
        if i0 > i1 or j0 > j1:
            continue
        if (i1 // 8 - i0 // 8 + 1) * (j1 // 8 - j0 // 8 + 1) > 16:
            spanning += 1
        else:
            tiles[j0 // 8:j1 // 8 + 1, i0 // 8:i1 // 8 + 1] += 1
    assert spanning > 64 and tiles.max() > 8 * 64
    fid = raster.rasterize_ids(v, f, P, W, H)
    n_dup = sc["n_dup"]
    assert (fid >= 0).mean() > 0.9
    assert np.isin(fid, np.arange(n_dup)).sum() > 1000
    assert not (fid >= len(f) - n_dup).any()
