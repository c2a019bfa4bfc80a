"""The ways of forming V through the autograd-level Python API (ops.
visibility_sh and ops.shade_sh_channels with ``mode``), against the FP64
oracle with torch autograd on the same inputs.

Tolerances as for the entry points: V ||dV|| / ||V|| <= 1e-5, B max |dB| /
max |B| <= 1e-5, gradients ||d grad|| / ||grad|| <= 1e-4."""
import math

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import rel_l2, rel_max
from oracle import method, sh

pytestmark = pytest.mark.gpu

DT = torch.float64
MODES = ["squaring", "quadrature", "product", "taylor3"]


def _oracle_V(points, spheres, n, mode, eps=3.0, k=4):
    C = sh.gaunt_tensor(n).to(DT)
    if mode == "product":
        return method.sh_direct_product(points, spheres, n, eps, C)
    F = method.log_visibility(points, spheres, n, eps)
    if mode == "quadrature":
        return method.sh_exponential_quadrature(F, n)
    if mode.startswith("taylor"):
        return method.sh_exponential_taylor(F, C, int(mode[6:]), k)
    return method.sh_exponential(F, C, k)[0]


@pytest.mark.parametrize("mode", MODES)
def test_visibility_sh_forward_and_gradients(mode):
    from paper_2104_00359_amd import visibility_sh
    sc = scenegen.scene_random_shell(61, 333, 23, 6)
    rng = np.random.default_rng(2)
    G = rng.standard_normal((333, 36)).astype(np.float32)
    pts = torch.tensor(sc["points"], device="cuda", requires_grad=True)
    sph = torch.tensor(sc["spheres"], device="cuda", requires_grad=True)
    V = visibility_sh(pts, sph, 6, mode=mode)
    (V * torch.tensor(G, device="cuda")).sum().backward()
    op = torch.tensor(sc["points"], dtype=DT, requires_grad=True)
    os_ = torch.tensor(sc["spheres"], dtype=DT, requires_grad=True)
    oV = _oracle_V(op, os_, 6, mode)
    (oV * torch.tensor(G, dtype=DT)).sum().backward()
    ev = rel_l2(V.detach().cpu().numpy(), oV.detach().numpy())
    ep = rel_l2(pts.grad.cpu().numpy(), op.grad.numpy())
    es = rel_l2(sph.grad.cpu().numpy(), os_.grad.numpy())
    print(f"{mode}: V {ev:.2e}  grad points {ep:.2e}  grad spheres {es:.2e}")
    assert ev <= 1e-5 and ep <= 1e-4 and es <= 1e-4


@pytest.mark.parametrize("mode", ["product", "taylor2"])
def test_shade_sh_channels_with_a_mode(mode):
    """Two colour channels through a non-default V: each channel and every
    gradient against the oracle."""
    from paper_2104_00359_amd import shade_sh_channels
    sc = scenegen.scene_random_shell(62, 300, 17, 4)
    rng = np.random.default_rng(3)
    alb = rng.uniform(0.2, 0.9, (300, 2)).astype(np.float32)
    light = np.stack([sc["light"], rng.standard_normal(16).astype(np.float32)])
    w = rng.standard_normal((300, 2)).astype(np.float32)
    t = {k: torch.tensor(v, device="cuda", requires_grad=True)
         for k, v in (("points", sc["points"]), ("normals", sc["normals"]), ("albedo", alb),
                      ("spheres", sc["spheres"]), ("light", light))}
    B = shade_sh_channels(t["points"], t["normals"], t["albedo"], t["spheres"], t["light"], 4, mode=mode)
    (B * torch.tensor(w, device="cuda")).sum().backward()
    o = {k: torch.tensor(v.detach().cpu().numpy(), dtype=DT, requires_grad=True) for k, v in t.items()}
    Bo = []
    for c in range(2):
        out = method.forward(o["points"], o["normals"], o["albedo"][:, c], o["spheres"], o["light"][c], 4,
                             exp_mode=mode)
        Bo.append(out["B"])
    Bo = torch.stack(Bo, 1)
    (Bo * torch.tensor(w, dtype=DT)).sum().backward()
    assert rel_max(B.detach().cpu().numpy(), Bo.detach().numpy()) <= 1e-5
    for k in t:
        e = rel_l2(t[k].grad.cpu().numpy(), o[k].grad.numpy())
        print(f"{mode} grad {k} {e:.2e}")
        assert e <= 1e-4, k


def test_unknown_mode_is_rejected():
    from paper_2104_00359_amd import ops
    for bad in ("taylor0", "taylor9", "exp", 3):
        with pytest.raises(ValueError):
            ops.mode_flags(bad)
    assert ops.mode_flags("taylor8") == 16 | (8 << 8)
    assert math.isfinite(ops.mode_flags("product"))
