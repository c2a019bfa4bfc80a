"""Edge cases, error paths and determinism of the HIP library (GPU)."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import lib, rel_l2, rel_max, run_hip, run_oracle, run_render, to_dev

pytestmark = pytest.mark.gpu


def test_no_spheres_is_unoccluded():
    sc = scenegen.scene_random_shell(3, 300, 0, 8)
    sc["spheres"] = np.zeros((0, 4), np.float32)
    w = sc["grad_radiance"]
    h = run_hip(sc, w)
    o = run_oracle(sc, w)
    e0 = np.zeros(64)
    e0[0] = np.sqrt(4 * np.pi)
    assert np.abs(h["V"] - e0).max() < 1e-5
    assert rel_max(h["B"], o["B"]) < 1e-5
    assert h["grad_spheres"].shape == (0, 4)
    assert np.all(h["grad_points"] == 0)
    assert rel_l2(h["grad_light"], o["grad_light"]) < 1e-4


def test_single_receiver_and_single_sphere():
    sc = scenegen.scene_random_shell(4, 1, 1, 5)
    w = sc["grad_radiance"]
    h = run_hip(sc, w)
    o = run_oracle(sc, w)
    assert rel_max(h["B"], o["B"]) < 1e-5
    for key in ("grad_points", "grad_spheres", "grad_light", "grad_normals", "grad_albedo"):
        assert rel_l2(h[key], o[key]) < 1e-4, key


def test_receiver_inside_sphere_and_centred_sphere():
    """r >= d gives a hemisphere cap (t = 0, no gradient through t); a sphere
    centred exactly on the receiver contributes nothing."""
    sc = scenegen.scene_random_shell(6, 64, 6, 6)
    sph = sc["spheres"].copy()
    p0 = sc["points"][0]
    sph[0, :3] = p0 + np.float32(0.05) * sc["normals"][0]
    sph[0, 3] = 0.2                           # receiver 0 inside sphere 0
    sph[1, :3] = sc["points"][1]              # sphere 1 centred on receiver 1
    sph[1, 3] = 0.1
    sc["spheres"] = sph
    w = sc["grad_radiance"]
    h = run_hip(sc, w)
    o = run_oracle(sc, w)
    assert rel_l2(h["V"], o["V"]) < 1e-5
    assert rel_max(h["B"], o["B"]) < 1e-5
    for key in ("grad_points", "grad_spheres", "grad_light"):
        assert rel_l2(h[key], o[key]) < 1e-4, key


def test_bitwise_determinism():
    sc = scenegen.scene_random_shell(8, 5000, 100, 8)
    w = sc["grad_radiance"]
    a = run_hip(sc, w)
    b = run_hip(sc, w)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("n,k", [(8, 4), (6, 0), (3, 2)])
def test_exponential_variants_are_bitwise_identical(n, k):
    """One receiver per lane vs each receiver spread over four waves."""
    sc = scenegen.scene_random_shell(21, 3000, 40, n)
    w = sc["grad_radiance"]
    a = run_hip(sc, w, k=k, flags=1)
    b = run_hip(sc, w, k=k, flags=2)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("n,k,P,flags", [(8, 4, 3000, 0), (8, 4, 3000, 1), (6, 0, 777, 2), (4, 3, 70000, 0),
                                          (5, 2, 130, 1)])
def test_render_path_matches_separate_entry_points(n, k, P, flags):
    """sh_render_forward / sh_render_backward are bit-identical to the four
    separate entry points, in both exponential layouts."""
    sc = scenegen.scene_random_shell(31 + n, P, 37, n)
    w = sc["grad_radiance"]
    a = run_hip(sc, w, k=k, flags=flags)
    b = run_render(sc, w, k=k, flags=flags)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_render_path_null_outputs():
    sc = scenegen.scene_random_shell(41, 900, 12, 6)
    w = sc["grad_radiance"]
    full = run_render(sc, w)
    part = run_render(sc, w, null=("grad_points", "grad_normals", "grad_light"))
    for key in ("grad_albedo", "grad_spheres", "V", "B"):
        assert np.array_equal(full[key], part[key]), key
    only_light = run_render(sc, w, null=("grad_points", "grad_normals", "grad_albedo", "grad_spheres"))
    assert np.array_equal(full["grad_light"], only_light["grad_light"])


def test_zero_receivers_is_noop_and_zeroes_reductions():
    L = lib()
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    prm = L.params(4)
    st = torch.cuda.current_stream().cuda_stream
    gL = torch.full((16,), 7.0, device=dev)
    gS = torch.full((3, 4), 7.0, device=dev)
    sph = torch.ones(3, 4, device=dev)
    L.sh_visibility_forward(None, 0, sph, 3, prm, None, None, 0, None, 0, st)
    L.sh_shade_backward(None, None, None, None, None, 0, prm, None, None, None, gL, None, 0, st)
    L.sh_visibility_backward(None, None, None, 0, sph, 3, prm, None, 0, None, gS, None, 0, st)
    torch.cuda.synchronize()
    assert torch.all(gL == 0) and torch.all(gS == 0)


def test_optional_outputs_may_be_null():
    L = lib()
    from paper_2104_00359_amd import ops
    sc = scenegen.scene_random_shell(9, 500, 20, 4)
    full = run_hip(sc, sc["grad_radiance"])
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    prm = L.params(4)
    P, S = 500, 20
    pts, nrm = to_dev(sc["points"].T), to_dev(sc["normals"].T)
    alb, sph, lig = to_dev(sc["albedo"]), to_dev(sc["spheres"]), to_dev(sc["light"])
    gB = to_dev(sc["grad_radiance"])
    vis = torch.empty(16, P, device=dev)
    saved = torch.empty(L.shv_saved_floats(P, prm), device=dev)
    nb = L.shv_workspace_bytes(P, S, prm)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    L.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, L.nbytes(saved), ws, nb, st)
    gV = torch.empty(16, P, device=dev)
    gL = torch.empty(16, device=dev)
    L.sh_shade_backward(gB, vis, nrm, alb, lig, P, prm, gV, None, None, gL, ws, nb, st)
    gS = torch.empty(S, 4, device=dev)
    L.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, L.nbytes(saved), None, gS, ws, nb, st)
    torch.cuda.synchronize()
    assert np.array_equal(gL.cpu().numpy(), full["grad_light"])
    assert np.array_equal(gS.cpu().numpy(), full["grad_spheres"])


def test_invalid_arguments_return_status_codes():
    L = lib()
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    st = torch.cuda.current_stream().cuda_stream
    f = L.raw("sh_visibility_forward")
    pts = torch.zeros(3, 10, device=dev)
    sph = torch.zeros(2, 4, device=dev)
    vis = torch.zeros(16, 10, device=dev)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=dev)
    good = L.params(4)
    assert f(pts.data_ptr(), 10, sph.data_ptr(), 2, ctypes.byref(L.params(9)), vis.data_ptr(), None, 0,
             ws.data_ptr(), ws.numel(), st) == L.SHV_ERR_UNSUPPORTED
    assert f(pts.data_ptr(), -1, sph.data_ptr(), 2, ctypes.byref(good), vis.data_ptr(), None, 0,
             ws.data_ptr(), ws.numel(), st) == L.SHV_ERR_INVALID_ARG
    assert f(None, 10, sph.data_ptr(), 2, ctypes.byref(good), vis.data_ptr(), None, 0,
             ws.data_ptr(), ws.numel(), st) == L.SHV_ERR_INVALID_ARG
    assert f(pts.data_ptr(), 10, sph.data_ptr(), 2, ctypes.byref(good), vis.data_ptr(), None, 0,
             ws.data_ptr(), 16, st) == L.SHV_ERR_WORKSPACE
    assert f(pts.data_ptr(), 10, sph.data_ptr() + 4, 2, ctypes.byref(good), vis.data_ptr(), None, 0,
             ws.data_ptr(), ws.numel(), st) == L.SHV_ERR_INVALID_ARG
    assert "aligned" in L.shv_last_error()
    with pytest.raises(RuntimeError):
        L.sh_visibility_forward(pts, 10, sph, 2, L.params(0), vis, None, 0, ws, ws.numel(), st)


def test_autograd_function_matches_c_abi():
    from paper_2104_00359_amd import shade_sh
    sc = scenegen.scene_random_shell(12, 700, 30, 6)
    w = sc["grad_radiance"]
    ref = run_hip(sc, w)
    dev = "cuda"
    t = {k: to_dev(sc[k]).requires_grad_(True) for k in ("points", "normals", "albedo", "spheres", "light")}
    B = shade_sh(t["points"], t["normals"], t["albedo"], t["spheres"], t["light"], 6)
    (B * to_dev(w)).sum().backward()
    assert np.array_equal(B.detach().cpu().numpy(), ref["B"])
    assert np.array_equal(t["points"].grad.cpu().numpy(), ref["grad_points"])
    assert np.array_equal(t["spheres"].grad.cpu().numpy(), ref["grad_spheres"])
    assert np.array_equal(t["light"].grad.cpu().numpy(), ref["grad_light"])
    assert np.array_equal(t["normals"].grad.cpu().numpy(), ref["grad_normals"])
    assert np.array_equal(t["albedo"].grad.cpu().numpy(), ref["grad_albedo"])


def test_zero_radius_spheres_are_invisible():
    """A sphere of radius 0 subtends no cap (its coefficients are exact
    zeros): results equal the scene without it up to the summation order of
    the other spheres, and its gradients are finite."""
    sc = scenegen.scene_random_shell(12, 500, 12, 8)
    sph = sc["spheres"].copy()
    sph[3, 3] = 0.0
    sph[7, 3] = 0.0
    sc["spheres"] = sph
    keep = np.array([i for i in range(12) if i not in (3, 7)])
    sc2 = dict(sc)
    sc2["spheres"] = np.ascontiguousarray(sph[keep])
    w = sc["grad_radiance"]
    h = run_render(sc, w)
    h2 = run_render(sc2, w)
    assert np.allclose(h["V"], h2["V"], rtol=0, atol=1e-6 * np.abs(h2["V"]).max())
    assert rel_max(h["B"], h2["B"]) < 1e-6
    assert np.all(np.isfinite(h["grad_spheres"]))
    assert np.allclose(h["grad_spheres"][keep], h2["grad_spheres"], rtol=1e-5, atol=1e-6 * np.abs(h2["grad_spheres"]).max())


def _mode_flags(mode):
    L = lib()
    return {"product": L.SHV_FLAG_EXP_PRODUCT, "quadrature": L.SHV_FLAG_EXP_QUADRATURE,
            "taylor2": L.SHV_FLAG_EXP_TAYLOR | L.SHV_FLAG_EXP_TAYLOR_ORDER(2)}[mode]


@pytest.mark.parametrize("mode", ["product", "quadrature", "taylor2"])
def test_exponential_modes_without_spheres(mode):
    """No occluders under every other way of forming V: V is the unoccluded
    sqrt(4 pi) e_0, the point gradients are exactly zero, and the shading and
    lighting gradient equal the oracle's."""
    from oracle import method
    sc = scenegen.scene_random_shell(3, 300, 0, 8)
    sc["spheres"] = np.zeros((0, 4), np.float32)
    w = sc["grad_radiance"]
    h = run_hip(sc, w, flags=_mode_flags(mode))
    o = {k: v.detach().numpy() for k, v in method.run_forward_backward(sc, w, exp_mode=mode).items()}
    e0 = np.zeros(64)
    e0[0] = np.sqrt(4 * np.pi)
    assert np.abs(h["V"] - e0).max() < 1e-5
    assert rel_max(h["B"], o["B"]) < 1e-5
    assert h["grad_spheres"].shape == (0, 4)
    assert np.all(h["grad_points"] == 0)
    assert rel_l2(h["grad_light"], o["grad_light"]) < 1e-4


@pytest.mark.parametrize("mode", ["product", "quadrature", "taylor2"])
def test_exponential_modes_single_receiver_and_sphere(mode):
    """One receiver (a block of 64 lanes with 63 idle) and one sphere under
    every other way of forming V, against the oracle's same mode."""
    from oracle import method
    sc = scenegen.scene_random_shell(4, 1, 1, 5)
    w = sc["grad_radiance"]
    h = run_hip(sc, w, flags=_mode_flags(mode))
    o = {k: v.detach().numpy() for k, v in method.run_forward_backward(sc, w, exp_mode=mode).items()}
    assert rel_l2(h["V"], o["V"]) < 1e-5 and rel_max(h["B"], o["B"]) < 1e-5
    for key in ("grad_points", "grad_spheres", "grad_light", "grad_normals", "grad_albedo"):
        assert rel_l2(h[key], o[key]) < 1e-4, key
