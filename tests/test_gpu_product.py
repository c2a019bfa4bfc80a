"""The direct product chain of Eq. 12 (SHV_FLAG_EXP_PRODUCT) against the FP64
oracle's chain on the same inputs, and the accuracy of every way of forming V
against the projection of the true floored visibility.

Tolerances: V ||dV|| / ||V|| <= 1e-5 and B max |dB| / max |B| <= 1e-5 per
scene; gradients ||d grad|| / ||grad|| <= 1e-4 per parameter group, as for the
log-space path (the chain is S products long, each a few thousand FP32
terms)."""
import ctypes
import math

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import lib, rel_l2, rel_max, run_hip
from oracle import brute, method

pytestmark = pytest.mark.gpu

PROD = 8


def _oracle(sc, grad_B=None, idx=None):
    if grad_B is None:
        o = method.run_forward(sc, idx=idx, exp_mode="product")
        return {"V": o["V"].numpy(), "B": o["B"].numpy()}
    o = method.run_forward_backward(sc, grad_B, idx=idx, exp_mode="product")
    return {k: v.detach().numpy() for k, v in o.items()}


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8])
def test_product_forward_and_gradients(n):
    """777 receivers (12 blocks of 64 and a ragged tail) and 37 spheres, every
    band count class."""
    sc = scenegen.scene_random_shell(80 + n, 777, 37, n)
    w = sc["grad_radiance"]
    h = run_hip(sc, w, flags=PROD)
    o = _oracle(sc, w)
    ev, eb = rel_l2(h["V"], o["V"]), rel_max(h["B"], o["B"])
    print(f"V {ev:.2e}  B {eb:.2e}")
    assert ev <= 1e-5 and eb <= 1e-5
    for key in ("grad_points", "grad_normals", "grad_albedo", "grad_light", "grad_spheres"):
        e = rel_l2(h[key], o[key])
        print(f"{key} {e:.2e}")
        assert e <= 1e-4, key


def test_product_body_scene_sampled():
    """The body-like scene at full size (20,000 receivers, a 128-product chain
    each): outputs on 192 sampled receivers, sphere gradients from a cotangent
    nonzero only there."""
    sc = scenegen.scene_body()
    P = sc["points"].shape[0]
    idx = np.sort(np.random.default_rng(2).choice(P, 192, replace=False))
    w = np.zeros(P, np.float32)
    w[idx] = sc["grad_radiance"][idx]
    h = run_hip(sc, w, flags=PROD)
    o = _oracle(sc, w[idx], idx=idx)
    ev, eb = rel_l2(h["V"][idx], o["V"]), rel_max(h["B"][idx], o["B"])
    print(f"V {ev:.2e}  B {eb:.2e}")
    assert ev <= 1e-5 and eb <= 1e-5
    for key in ("grad_points", "grad_normals"):
        e = rel_l2(h[key][idx], o[key])
        print(f"{key} {e:.2e}")
        assert e <= 1e-4, key
    for key in ("grad_light", "grad_spheres"):
        e = rel_l2(h[key], o[key])
        print(f"{key} {e:.2e}")
        assert e <= 1e-4, key


def test_product_degenerate_receivers():
    """A receiver inside a sphere (hemisphere cap), one exactly at a sphere's
    centre (that sphere blocks nothing), and no spheres at all (V = 1)."""
    n = 5
    sc = scenegen.scene_random_shell(9, 70, 5, n)
    sc["points"] = sc["points"].copy()
    sc["points"][3] = sc["spheres"][1, :3] + np.float32(0.25) * sc["spheres"][1, 3]
    sc["points"][7] = sc["spheres"][2, :3]
    w = sc["grad_radiance"]
    h = run_hip(sc, w, flags=PROD)
    o = _oracle(sc, w)
    assert rel_l2(h["V"], o["V"]) <= 1e-5
    assert rel_l2(h["grad_points"], o["grad_points"]) <= 1e-4
    assert rel_l2(h["grad_spheres"], o["grad_spheres"]) <= 1e-4
    empty = dict(sc)
    empty["spheres"] = np.zeros((0, 4), np.float32)
    h0 = run_hip(empty, w, flags=PROD)
    one = np.zeros(n * n, np.float32)
    one[0] = np.float32(math.sqrt(4 * math.pi))
    assert np.array_equal(h0["V"], np.broadcast_to(one, h0["V"].shape))
    assert not h0["grad_points"].any()


@pytest.mark.parametrize("scene", ["body", "shell"])
def test_accuracy_of_every_way_of_forming_V(scene):
    """Against the SH projection of the true floored visibility (brute force):
    100 receivers of the body scene (heavy cap overlap) or of a 37-sphere
    shell scene.  The log-space schemes share the error of band-limiting the
    logarithm before exponentiating, so the squaring and quadrature
    exponentials land close to each other; the product chain truncates only
    products of the blockers themselves and is several times closer."""
    if scene == "body":
        sc = scenegen.subset(scenegen.scene_body(), np.arange(0, 20000, 200))
    else:
        sc = scenegen.scene_random_shell(81, 100, 37, 8)
    T = method.scene_tensors(sc)
    ref = brute.projected_visibility(T["points"], T["spheres"], 8, 3.0, degree=240).numpy()
    errs = {}
    for name, flags in (("squaring", 0), ("quadrature", 4), ("product", PROD)):
        errs[name] = rel_l2(run_hip(sc, flags=flags)["V"], ref)
    print("  ".join(f"{k} {v:.3e}" for k, v in errs.items()))
    assert errs["product"] < errs["squaring"] / 5
    assert errs["product"] < errs["quadrature"] / 5


def test_product_flag_is_rejected_by_the_fused_and_batched_paths():
    L = lib()
    from paper_2104_00359_amd import ops
    ops.ensure_init(torch.device("cuda", 0))
    prm = L.params(4, 3.0, 4, PROD)
    f = L.raw("sh_render_forward")
    assert f(None, None, None, None, None, 10, 1, ctypes.byref(prm), None, None, None, 0, None, 0, None) == \
        L.SHV_ERR_UNSUPPORTED
    assert L.shv_saved_floats(100, prm) == 0
    assert L.shv_workspace_bytes(100, 7, prm) >= 7 * 16 * 100 * 4
