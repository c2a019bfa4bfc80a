"""Pins for the FP64 oracle of the scene parameterisation (embedded deformation
driven by the spheres plus a global rigid pose), against library routines
(SciPy's rotation-vector conversion and k-d tree), closed forms and finite
differences.  CPU only."""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import scenegen
from oracle import deform

DT = torch.float64


def small_scene(P=300, S=12, seed=3):
    sc = scenegen.scene_random_shell(seed, P, S, 4)
    return sc


@pytest.mark.parametrize("scale", [0.0, 1e-7, 1e-4, 1e-2, 0.7, 3.0])
def test_rodrigues_matches_scipy_rotation_vectors(scale):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((20, 3)) * scale
    R = deform.rodrigues(torch.tensor(a)).numpy()
    ref = Rotation.from_rotvec(a).as_matrix()
    assert np.abs(R - ref).max() < 1e-14
    assert np.abs(R @ R.transpose(0, 2, 1) - np.eye(3)).max() < 1e-14


def test_skew_is_the_cross_product():
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal((5, 3)), rng.standard_normal((5, 3))
    out = (deform.skew(torch.tensor(a)) @ torch.tensor(b)[..., None])[..., 0].numpy()
    assert np.allclose(out, np.cross(a, b), rtol=0, atol=1e-15)


def test_attachment_is_the_k_nearest_vertices():
    sc = small_scene()
    K = 40
    idx, u = deform.attach(sc["points"], sc["spheres"][:, :3], K)
    tree = cKDTree(np.asarray(sc["points"], np.float64))
    d, ref = tree.query(np.asarray(sc["spheres"][:, :3], np.float64), k=K + 1)
    for k in range(idx.shape[0]):
        assert list(idx[k]) == list(ref[k, :K])            # distinct distances: same order
        dk = np.linalg.norm(sc["points"][idx[k]].astype(np.float64) - sc["spheres"][k, :3], axis=1)
        assert np.allclose(u[k], (1.0 - dk / d[k, K]) ** 2, rtol=1e-12, atol=0)


def test_attachment_ties_go_to_the_lower_index():
    v = np.array([[1.0, 0, 0], [0, 1.0, 0], [-1.0, 0, 0], [0, 0, 2.0]], np.float32)
    idx, u = deform.attach(v, np.zeros((1, 3), np.float32), 2)
    assert list(idx[0]) == [0, 1]
    assert np.all(u == 0.0)       # the third vertex is as near as the attached ones


def _graph(sc, K):
    idx, u = deform.attach(sc["points"], sc["spheres"][:, :3], K)
    w = deform.normalised_weights(idx, u, sc["points"].shape[0])
    return torch.tensor(idx), torch.tensor(w)


def _tensors(sc):
    return (torch.tensor(sc["points"], dtype=DT), torch.tensor(sc["normals"], dtype=DT),
            torch.tensor(sc["spheres"], dtype=DT))


def test_weights_of_an_attached_vertex_sum_to_one():
    sc = small_scene()
    idx, w = _graph(sc, 40)
    tot = torch.zeros(sc["points"].shape[0], dtype=DT).index_add(0, idx.reshape(-1), w.reshape(-1))
    att = tot > 0
    assert att.sum() > 0.5 * len(tot)
    assert torch.allclose(tot[att], torch.ones_like(tot[att]), rtol=0, atol=1e-14)


def test_zero_parameters_leave_the_template():
    sc = small_scene()
    idx, w = _graph(sc, 40)
    v, m, s = _tensors(sc)
    x, n, c = deform.deform(torch.zeros(s.shape[0] + 1, 6, dtype=DT), v, m, s, idx, w)
    assert torch.allclose(x, v, rtol=0, atol=1e-15)
    assert torch.allclose(n, m, rtol=0, atol=1e-15)
    assert torch.equal(c, s)


def test_common_translation_moves_attached_vertices_rigidly():
    sc = small_scene()
    idx, w = _graph(sc, 40)
    v, m, s = _tensors(sc)
    prm = torch.zeros(s.shape[0] + 1, 6, dtype=DT)
    t = torch.tensor([0.1, -0.2, 0.05], dtype=DT)
    prm[:-1, 3:] = t
    x, n, c = deform.deform(prm, v, m, s, idx, w)
    tot = torch.zeros(v.shape[0], dtype=DT).index_add(0, idx.reshape(-1), w.reshape(-1))
    att = tot > 0
    assert torch.allclose(x[att], v[att] + t, rtol=0, atol=1e-14)
    assert torch.equal(x[~att], v[~att])
    assert torch.allclose(n, m, rtol=0, atol=1e-15)
    assert torch.allclose(c[:, :3], s[:, :3] + t, rtol=0, atol=1e-15)


def test_global_pose_is_a_rigid_motion():
    sc = small_scene()
    idx, w = _graph(sc, 40)
    v, m, s = _tensors(sc)
    prm = torch.zeros(s.shape[0] + 1, 6, dtype=DT)
    a0 = np.array([0.3, -0.5, 0.2])
    t0 = np.array([1.0, 2.0, -0.5])
    prm[-1, :3] = torch.tensor(a0)
    prm[-1, 3:] = torch.tensor(t0)
    x, n, c = deform.deform(prm, v, m, s, idx, w)
    R0 = Rotation.from_rotvec(a0).as_matrix()
    assert np.allclose(x.numpy(), v.numpy() @ R0.T + t0, rtol=0, atol=1e-13)
    assert np.allclose(n.numpy(), m.numpy() @ R0.T, rtol=0, atol=1e-13)
    assert np.allclose(c[:, :3].numpy(), s[:, :3].numpy() @ R0.T + t0, rtol=0, atol=1e-13)
    assert torch.equal(c[:, 3], s[:, 3])


def test_single_attachment_closed_form():
    """One sphere, one vertex, K = 1 of 2 vertices: the vertex follows that
    sphere with weight 1: y = R (v - g) + g + t."""
    v = torch.tensor([[0.3, 0.1, 0.0], [3.0, 0.0, 0.0]], dtype=DT)
    m = torch.tensor([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]], dtype=DT)
    s = torch.tensor([[0.0, 0.0, 0.0, 0.2]], dtype=DT)
    idx, u = deform.attach(v.numpy(), s[:, :3].numpy(), 1)
    w = torch.tensor(deform.normalised_weights(idx, u, 2))
    assert list(idx[0]) == [0] and float(w[0, 0]) == 1.0
    a = np.array([0.0, 0.0, np.pi / 2])
    t = np.array([0.0, 0.0, 1.0])
    prm = torch.zeros(2, 6, dtype=DT)
    prm[0, :3], prm[0, 3:] = torch.tensor(a), torch.tensor(t)
    x, n, c = deform.deform(prm, v, m, s, torch.tensor(idx), w)
    assert np.allclose(x[0].numpy(), [-0.1, 0.3, 1.0], atol=1e-15)   # (0.3, 0.1) turned by 90 degrees, lifted
    assert np.allclose(x[1].numpy(), [3.0, 0.0, 0.0], atol=0)        # unattached vertex
    assert np.allclose(n[0].numpy(), [0.0, 0.0, 1.0], atol=1e-15)    # axis-aligned normal unchanged
    assert np.allclose(c[0, :3].numpy(), [0.0, 0.0, 1.0], atol=0)


def test_gradients_match_central_differences():
    sc = small_scene(P=120, S=6, seed=5)
    idx, w = _graph(sc, 30)
    v, m, s = _tensors(sc)
    rng = np.random.default_rng(4)
    prm0 = torch.tensor(rng.standard_normal((7, 6)) * 0.3)
    gx, gn, gc = (torch.tensor(rng.standard_normal(x.shape)) for x in (v, m, s))

    def f(p):
        x, n, c = deform.deform(p, v, m, s, idx, w)
        return (x * gx).sum() + (n * gn).sum() + (c * gc).sum()

    p = prm0.clone().requires_grad_(True)
    g = torch.autograd.grad(f(p), p)[0]
    h = 1e-5
    fd = torch.zeros_like(prm0)
    for i in range(prm0.shape[0]):
        for j in range(6):
            e = torch.zeros_like(prm0)
            e[i, j] = h
            fd[i, j] = (f(prm0 + e) - f(prm0 - e)) / (2 * h)
    assert torch.allclose(g, fd, rtol=1e-7, atol=1e-7)


def test_render_loss_gradient_matches_central_differences():
    """The inverse problem's gradient through deformation and shading."""
    sc = small_scene(P=40, S=5, seed=8)
    idx, w = _graph(sc, 12)
    rng = np.random.default_rng(9)
    target = rng.uniform(0.5, 2.0, 40)
    prm0 = rng.standard_normal((6, 6)) * 0.05
    loss, g = deform.render_loss(prm0, sc, idx, w, target, 4)
    h = 1e-6
    for (i, j) in [(0, 0), (1, 4), (3, 2), (5, 0), (5, 5), (2, 3)]:
        e = np.zeros_like(prm0)
        e[i, j] = h
        lp, _ = deform.render_loss(prm0 + e, sc, idx, w, target, 4)
        lm, _ = deform.render_loss(prm0 - e, sc, idx, w, target, 4)
        fd = float(lp - lm) / (2 * h)
        assert abs(float(g[i, j]) - fd) <= 1e-6 * max(1.0, abs(fd)), (i, j, float(g[i, j]), fd)


def test_image_loss_gradient_matches_central_differences():
    """The image-space loss of Eqs. 14-16 through deformation, visibility,
    shading and the rasteriser's perspective-correct weights: with the face
    map held fixed (the loss is then smooth in the parameters) its autograd
    gradient equals FP64 central differences, on every parameter kind
    (per-sphere rotation and translation, global pose)."""
    sc = scenegen.scene_mesh_body(n_bands=4, width=40, height=40, spacing=0.06)
    P, S = sc["points"].shape[0], sc["spheres"].shape[0]
    idx, u = deform.attach(sc["points"], sc["spheres"][:, :3], 8)
    w = deform.normalised_weights(idx, u, P)
    rng = np.random.default_rng(11)
    target = rng.uniform(0.0, 1.0, (40, 40))
    prm0 = np.zeros((S + 1, 6))
    prm0[:, :3] = rng.standard_normal((S + 1, 3)) * 0.02
    prm0[:, 3:] = rng.standard_normal((S + 1, 3)) * 0.005
    loss, g, fid = deform.image_loss(prm0, sc, idx, w, target, 4)
    assert (fid >= 0).sum() > 100
    # the parameters of the spheres that reach the most covered pixels, and the global pose
    hits = np.bincount(idx.reshape(-1), minlength=P)
    k_busy = [int(k) for k in np.argsort([-(hits[idx[k]]).sum() for k in range(S)])[:2]]
    h = 1e-6
    checked = 0
    for i, j in [(k_busy[0], 0), (k_busy[0], 4), (k_busy[1], 2), (k_busy[1], 3), (S, 1), (S, 5)]:
        e = np.zeros_like(prm0)
        e[i, j] = h
        lp, _, _ = deform.image_loss(prm0 + e, sc, idx, w, target, 4, face_id=fid)
        lm, _, _ = deform.image_loss(prm0 - e, sc, idx, w, target, 4, face_id=fid)
        fd = float(lp - lm) / (2 * h)
        assert abs(float(g[i, j]) - fd) <= 1e-6 * max(abs(fd), 1e-3 * float(g.abs().max())), (i, j, float(g[i, j]), fd)
        checked += abs(fd) > 0
    assert checked >= 4
