"""The exponential by quadrature projection (SHV_FLAG_EXP_QUADRATURE, on MFMA)
against the FP64 oracle's projection with the same rule.

Tolerances: V ||dV|| / ||V|| <= 1e-5 and B max |dB| / max |B| <= 1e-5 per
scene; gradients ||d grad|| / ||grad|| <= 1e-4 per parameter group, as for the
squaring exponential.  The MFMA products accumulate in FP32 over 64-node tiles.
"""
import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import lib, rel_l2, rel_max, run_hip
from oracle import brute, method

pytestmark = pytest.mark.gpu

QUAD = 4


def _oracle(sc, grad_B=None, idx=None):
    if grad_B is None:
        o = method.run_forward(sc, idx=idx, exp_mode="quadrature")
        return {"V": o["V"].numpy(), "B": o["B"].numpy()}
    o = method.run_forward_backward(sc, grad_B, idx=idx, exp_mode="quadrature")
    return {k: v.detach().numpy() for k, v in o.items()}


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8])
def test_quadrature_forward_and_gradients(n):
    """777 receivers (12 blocks of 64 and a ragged tail), every band count
    class (odd n pads the node count to a multiple of 64)."""
    sc = scenegen.scene_random_shell(70 + n, 777, 37, n)
    w = sc["grad_radiance"]
    h = run_hip(sc, w, flags=QUAD)
    o = _oracle(sc, w)
    ev, eb = rel_l2(h["V"], o["V"]), rel_max(h["B"], o["B"])
    print(f"V {ev:.2e}  B {eb:.2e}")
    assert ev <= 1e-5 and eb <= 1e-5
    for key in ("grad_points", "grad_normals", "grad_albedo", "grad_light", "grad_spheres"):
        e = rel_l2(h[key], o[key])
        print(f"{key} {e:.2e}")
        assert e <= 1e-4, key


def test_quadrature_body_scene_sampled():
    """The body-like scene at full size (heavy cap overlap): outputs on 256
    sampled receivers, sphere gradients from a cotangent nonzero only there."""
    sc = scenegen.scene_body()
    P = sc["points"].shape[0]
    idx = np.sort(np.random.default_rng(1).choice(P, 256, replace=False))
    w = np.zeros(P, np.float32)
    w[idx] = sc["grad_radiance"][idx]
    h = run_hip(sc, w, flags=QUAD)
    o = _oracle(sc, w[idx], idx=idx)
    ev, eb = rel_l2(h["V"][idx], o["V"]), rel_max(h["B"][idx], o["B"])
    print(f"V {ev:.2e}  B {eb:.2e}")
    assert ev <= 1e-5 and eb <= 1e-5
    for key in ("grad_points", "grad_normals"):
        assert rel_l2(h[key][idx], o[key]) <= 1e-4, key
    for key in ("grad_light", "grad_spheres"):
        assert rel_l2(h[key], o[key]) <= 1e-4, key


def test_quadrature_is_closer_to_the_projected_exponential_than_squaring():
    """Accuracy under heavy overlap: against the projected exponential by a
    degree-160 rule (brute force), the quadrature mode is far closer than the
    scaling-and-squaring scheme."""
    sc = scenegen.subset(scenegen.scene_body(), np.arange(0, 20000, 100))
    T = method.scene_tensors(sc)
    F = method.log_visibility(T["points"], T["spheres"], 8, 3.0)
    ref = brute.exact_exponential(F, 8, degree=160).numpy()
    q = run_hip(sc, flags=QUAD)["V"]
    s = run_hip(sc)["V"]
    eq, es = rel_l2(q, ref), rel_l2(s, ref)
    print(f"quadrature {eq:.2e}  squaring {es:.2e}")
    assert eq < 5e-3 and eq < es / 50


def test_quadrature_flag_is_rejected_by_the_fused_and_batched_paths():
    L = lib()
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    import ctypes
    prm = L.params(4, 3.0, 4, QUAD)
    f = L.raw("sh_render_forward")
    assert f(None, None, None, None, None, 10, 1, ctypes.byref(prm), None, None, None, 0, None, 0, None) == \
        L.SHV_ERR_UNSUPPORTED
    assert L.shv_saved_floats(100, prm) == max((1 + 4 * 16) * 100, 16 * 100)
    assert L.shv_saved_floats(100, L.params(4, 3.0, 0, QUAD)) == 16 * 100
