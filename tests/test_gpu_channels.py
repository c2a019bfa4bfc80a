"""Colour channels sharing one visibility (Eq. 8 per channel) and the
environment-map projection of the lighting (Eq. 9), GPU (FP32 HIP kernels)
through the C ABI against the FP64 oracle and against the one-channel entry
points.

Tolerances as in the single-channel parity tests: radiance max |dB| / max |B|
<= 1e-5, gradients ||d grad|| / ||grad|| <= 1e-4 per parameter group.  The
projection is compared per channel, ||dL|| / ||L|| <= 2e-5: each pixel's
direction is formed in FP32 from its azimuth (error a few 1e-7 rad, times
derivatives of y_lm up to about l = 7 per radian), and each row is an FP32
sum of at most a few thousand products.
"""
import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import lib, rel_l2, rel_max, to_dev
from oracle import method, sh

pytestmark = pytest.mark.gpu

TOL_B = 1e-5
TOL_G = 1e-4
TOL_ENV = 2e-5


def _setup(sc):
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    return dev, torch.cuda.current_stream().cuda_stream


def _vis(L, sc, prm, dev, st):
    n = int(sc["n_bands"])
    P, S = sc["points"].shape[0], sc["spheres"].shape[0]
    vis = torch.empty(n * n, P, device=dev)
    nb = L.shv_workspace_bytes(P, S, prm)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    L.sh_visibility_forward(to_dev(sc["points"].T), P, to_dev(sc["spheres"]), S, prm, vis, None, 0, ws, nb, st)
    return vis


@pytest.mark.parametrize("n,C", [(3, 3), (8, 3), (8, 1), (6, 4), (8, 2), (1, 4)])
def test_each_channel_is_the_one_channel_call(n, C):
    """Radiance, albedo and lighting gradients of channel c are bitwise those
    of sh_shade / sh_shade_backward with that channel's albedo and light; the
    V and normal cotangents are the channel sums (bitwise for one channel).
    777 receivers: several 256-receiver blocks and a ragged tail."""
    L = lib()
    sc = scenegen.scene_random_shell(60 + n, 777, 37, n)
    ch = scenegen.colour_channels(sc, C, seed=n)
    dev, st = _setup(sc)
    prm = L.params(n)
    P, N = sc["points"].shape[0], n * n
    vis = _vis(L, sc, prm, dev, st)
    nrm = to_dev(sc["normals"].T)
    alb = to_dev(ch["albedo"].T)          # [C][P]
    lig = to_dev(ch["light"])             # [C][N]
    gB = to_dev(ch["grad_radiance"].T)    # [C][P]
    nb = max(L.shv_workspace_bytes(P, 0, prm), L.shv_channels_workspace_bytes(P, C, prm))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    rad = torch.full((C, P), float("nan"), device=dev)
    L.sh_shade_channels(vis, nrm, alb, lig, C, P, prm, rad, ws, nb, st)
    gV = torch.full((N, P), float("nan"), device=dev)
    gN = torch.full((3, P), float("nan"), device=dev)
    gA = torch.full((C, P), float("nan"), device=dev)
    gL = torch.full((C, N), float("nan"), device=dev)
    L.sh_shade_channels_backward(gB, vis, nrm, alb, lig, C, P, prm, gV, gN, gA, gL, ws, nb, st)
    sV = sN = None
    for c in range(C):
        r1 = torch.empty(P, device=dev)
        L.sh_shade(vis, nrm, alb[c].contiguous(), lig[c].contiguous(), P, prm, r1, ws, nb, st)
        v1, n1 = torch.empty(N, P, device=dev), torch.empty(3, P, device=dev)
        a1, l1 = torch.empty(P, device=dev), torch.empty(N, device=dev)
        L.sh_shade_backward(gB[c].contiguous(), vis, nrm, alb[c].contiguous(), lig[c].contiguous(), P, prm,
                            v1, n1, a1, l1, ws, nb, st)
        torch.cuda.synchronize()
        assert torch.equal(rad[c], r1), f"radiance of channel {c}"
        assert torch.equal(gA[c], a1), f"albedo gradient of channel {c}"
        assert torch.equal(gL[c], l1), f"lighting gradient of channel {c}"
        v1, n1 = v1.double(), n1.double()
        sV = v1 if sV is None else sV + v1
        sN = n1 if sN is None else sN + n1
    torch.cuda.synchronize()
    if C == 1:
        assert torch.equal(gV.double(), sV) and torch.equal(gN.double(), sN)
    else:
        assert rel_l2(gV.cpu().numpy(), sV.cpu().numpy()) <= 1e-6
        assert rel_l2(gN.cpu().numpy(), sN.cpu().numpy()) <= 1e-6


def _check(h, o, idx=None):
    eb = rel_max(h["B"] if idx is None else h["B"][idx], o["B"])
    print(f"B rel max {eb:.2e}")
    assert eb <= TOL_B
    for key in ("grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light"):
        a = h[key] if idx is None or key in ("grad_light", "grad_spheres") else h[key][idx]
        e = rel_l2(a, o[key])
        print(f"{key} rel l2 {e:.2e}")
        assert e <= TOL_G, f"{key} rel l2 {e:.3e}"


def _run_op(sc, ch, grad_B):
    """Forward and backward through ops.shade_sh_channels (visibility, then
    the multi-channel shading entry points, and their adjoints)."""
    from paper_2104_00359_amd import shade_sh_channels
    dev, _ = _setup(sc)
    t = {k: to_dev(sc[k]).requires_grad_(True) for k in ("points", "normals", "spheres")}
    alb = to_dev(ch["albedo"]).requires_grad_(True)
    lig = to_dev(ch["light"]).requires_grad_(True)
    B = shade_sh_channels(t["points"], t["normals"], alb, t["spheres"], lig, int(sc["n_bands"]))
    (B * to_dev(grad_B)).sum().backward()
    torch.cuda.synchronize()
    return {"B": B.detach().cpu().numpy(), "grad_points": t["points"].grad.cpu().numpy(),
            "grad_normals": t["normals"].grad.cpu().numpy(), "grad_albedo": alb.grad.cpu().numpy(),
            "grad_spheres": t["spheres"].grad.cpu().numpy(), "grad_light": lig.grad.cpu().numpy()}


@pytest.mark.parametrize("n,C", [(2, 3), (5, 4), (8, 3), (8, 1)])
def test_channels_parity_with_oracle(n, C):
    sc = scenegen.scene_random_shell(80 + n, 777, 37, n)
    ch = scenegen.colour_channels(sc, C, seed=10 + n)
    h = _run_op(sc, ch, ch["grad_radiance"])
    o = method.run_forward_backward_channels(sc, ch["albedo"], ch["light"], ch["grad_radiance"])
    _check(h, {k: v.detach().double().numpy() for k, v in o.items()})


def test_channels_body_scene_full_size_sampled():
    """RGB on the body-like scene at full size (20,000 receivers, 128 spheres,
    8 bands); the cotangent is nonzero on 384 sampled receivers only, so the
    sphere and lighting gradients are exactly the oracle's sums over them."""
    sc = scenegen.scene_body()
    P = sc["points"].shape[0]
    ch = scenegen.colour_channels(sc, 3, seed=5)
    idx = np.sort(np.random.default_rng(3).choice(P, 384, replace=False))
    w = np.zeros((P, 3), np.float32)
    w[idx] = ch["grad_radiance"][idx]
    h = _run_op(sc, ch, w)
    o = method.run_forward_backward_channels(sc, ch["albedo"], ch["light"], w[idx], idx=idx)
    _check(h, {k: v.detach().double().numpy() for k, v in o.items()}, idx=idx)


@pytest.mark.parametrize("P", [1, 63, 65])
def test_channels_tiny_receiver_sets(P):
    """Fewer receivers than one 64-receiver block, and one more than a block."""
    sc = scenegen.scene_random_shell(90 + P, P, 9, 8)
    ch = scenegen.colour_channels(sc, 2, seed=P)
    h = _run_op(sc, ch, ch["grad_radiance"])
    o = method.run_forward_backward_channels(sc, ch["albedo"], ch["light"], ch["grad_radiance"])
    _check(h, {k: v.detach().double().numpy() for k, v in o.items()})


def test_channels_empty_receiver_set():
    L = lib()
    dev, st = _setup(None)
    prm = L.params(4)
    gL = torch.full((3, 16), float("nan"), device=dev)
    ws = torch.empty(256, dtype=torch.uint8, device=dev)
    L.sh_shade_channels(None, None, None, None, 3, 0, prm, None, None, 0, st)
    L.sh_shade_channels_backward(None, None, None, None, None, 3, 0, prm, None, None, None, gL, ws, 256, st)
    torch.cuda.synchronize()
    assert torch.equal(gL, torch.zeros_like(gL))


def _project(img, n):
    L = lib()
    dev, st = _setup(None)
    C, H, W = img.shape
    prm = L.params(n)
    out = torch.full((C, n * n), float("nan"), device=dev)
    nb = L.shv_envmap_workspace_bytes(C, H, W, prm)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    L.sh_envmap_project(to_dev(img), C, H, W, prm, out, ws, nb, st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("n,H,W", [(8, 96, 300), (4, 37, 64), (1, 5, 7), (8, 512, 1024), (6, 3, 5000)])
def test_envmap_projection_parity(n, H, W):
    """Ragged rows (300 = 256 + 44 columns), odd sizes, one band, a
    512 x 1024 RGB map, and rows wider than one block's pixel budget (one
    row per block)."""
    img = scenegen.envmap_image(seed=H, C=3, H=H, W=W)
    g = _project(img, n)
    o = sh.envmap_to_sh(img, n).numpy()
    for c in range(3):
        e = rel_l2(g[c], o[c])
        print(f"channel {c} rel l2 {e:.2e}")
        assert e <= TOL_ENV


def test_envmap_constant_map_and_single_pixel():
    g = _project(np.full((1, 64, 128), 2.5, np.float32), 8)
    o = sh.envmap_to_sh(np.full((64, 128), 2.5), 8).numpy()
    assert abs(g[0, 0] - 2.5 * np.sqrt(4 * np.pi)) <= 1e-6 * 2.5 * np.sqrt(4 * np.pi)
    assert np.abs(g[0] - o).max() <= 1e-5
    # one pixel covers the whole sphere (weight 4 pi) and is sampled at th = pi/2, ph = pi
    g1 = _project(np.full((2, 1, 1), 3.0, np.float32), 3)
    o1 = sh.envmap_to_sh(np.full((2, 1, 1), 3.0), 3).numpy()
    assert np.abs(g1 - o1).max() <= 1e-5 * np.abs(o1).max()


def test_envmap_empty_map_gives_zero_light():
    L = lib()
    dev, st = _setup(None)
    prm = L.params(6)
    out = torch.full((2, 36), float("nan"), device=dev)
    L.sh_envmap_project(None, 2, 0, 16, prm, out, None, 0, st)
    torch.cuda.synchronize()
    assert torch.equal(out, torch.zeros_like(out))


def test_envmap_op_matches_entry_point():
    from paper_2104_00359_amd import envmap_to_sh
    img = scenegen.envmap_image(seed=1, C=3, H=64, W=128)
    dev, _ = _setup(None)
    a = envmap_to_sh(to_dev(img), 8).cpu().numpy()
    b = envmap_to_sh(to_dev(img[1]), 8).cpu().numpy()
    assert np.array_equal(a, _project(img, 8))
    assert np.array_equal(b, a[1])
