"""GPU (FP32 HIP kernels) vs FP64 oracle parity, through the C ABI.

Tolerances (FP32 kernels against FP64 on identical FP32 inputs):
  V            ||dV|| / ||V||              <= 1e-5 per scene
  B            max |dB| / max |B|          <= 1e-5
  gradients    ||d grad|| / ||grad||       <= 1e-4 per parameter group
               (1e-3 for receiver / sphere gradients of the G-buffer scene,
                whose contact-adjacent pairs put 1/t ~ 10 into the adjoint)
"""
import numpy as np
import pytest

import scenegen
from gpu_helpers import rel_l2, rel_max, run_hip, run_oracle

pytestmark = pytest.mark.gpu

TOL_V = 1e-5
TOL_B = 1e-5
TOL_G = 1e-4
GRAD_KEYS = ["grad_points", "grad_normals", "grad_albedo", "grad_light", "grad_spheres"]


def check_forward(h, o, tol_v=TOL_V, tol_b=TOL_B):
    ev = rel_l2(h["V"], o["V"])
    eb = rel_max(h["B"], o["B"])
    print(f"V rel l2 {ev:.2e}  B rel max {eb:.2e}")
    assert ev <= tol_v, f"V rel l2 {ev:.3e}"
    assert eb <= tol_b, f"B rel max {eb:.3e}"


def check_grads(h, o, tol=TOL_G, tol_geom=None, idx=None):
    for key in GRAD_KEYS:
        a = h[key] if idx is None or key in ("grad_light", "grad_spheres") else h[key][idx]
        e = rel_l2(a, o[key])
        print(f"{key} rel l2 {e:.2e}")
        t = tol_geom if (tol_geom and key in ("grad_points", "grad_spheres")) else tol
        assert e <= t, f"{key} rel l2 {e:.3e} > {t:.0e}"


def test_icosphere_shell_forward():
    """2,562 icosphere receivers, 32 shell spheres, 4 bands: every output."""
    sc = scenegen.scene_icosphere_shell()
    check_forward(run_hip(sc), run_oracle(sc))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_band_count_forward_and_gradients(n):
    """Ragged receiver count (not a multiple of the 256-lane block) over
    several tiles, every supported n."""
    sc = scenegen.scene_random_shell(40 + n, 777, 37, n)
    w = sc["grad_radiance"]
    h = run_hip(sc, w)
    o = run_oracle(sc, w)
    check_forward(h, o)
    check_grads(h, o)


@pytest.mark.parametrize("k", [0, 1, 2, 6])
def test_squaring_counts(k):
    sc = scenegen.scene_random_shell(5, 300, 24, 6)
    w = sc["grad_radiance"]
    h = run_hip(sc, w, k=k)
    o = run_oracle(sc, w, k=k)
    tol = TOL_V * (2 ** max(k - 4, 0))  # FP32 error grows about 2x per squaring
    check_forward(h, o, tol_v=tol, tol_b=tol)
    check_grads(h, o, tol=TOL_G * (2 ** max(k - 4, 0)))


def test_body_scene_full_size_sampled():
    """Body-like scene at full size (20,000 receivers, 128 spheres, 8 bands)
    in the configuration the benchmark times.  Outputs are compared on 512
    sampled receivers; the cotangent is nonzero only there, so the sphere and
    lighting gradients (sums over receivers) are exactly the oracle's sums
    over the sample."""
    sc = scenegen.scene_body()
    P = sc["points"].shape[0]
    idx = np.sort(np.random.default_rng(0).choice(P, 512, replace=False))
    w = np.zeros(P, np.float32)
    w[idx] = sc["grad_radiance"][idx]
    h = run_hip(sc, w)
    o = run_oracle(sc, w[idx], idx=idx)
    check_forward({"V": h["V"][idx], "B": h["B"][idx]}, o)
    check_grads(h, o, idx=idx)
    mask = np.ones(P, bool)
    mask[idx] = False
    assert np.all(h["grad_points"][mask] == 0) and np.all(h["grad_albedo"][mask] == 0)


def _gbuffer_cotangent(sc, idx):
    """2 (B - T) at receivers idx (0 elsewhere), T the oracle's radiance of
    the target scene (jittered centres, perturbed light)."""
    tgt = dict(scenegen.subset(sc, idx))
    tgt["spheres"], tgt["light"] = sc["target_spheres"], sc["target_light"]
    T = run_oracle(tgt)["B"]
    B = run_oracle(sc, idx=idx)["B"]
    w = np.zeros(sc["points"].shape[0], np.float32)
    w[idx] = (2.0 * (B - T)).astype(np.float32)
    return w


def test_gbuffer_scene_full_size_sampled():
    """512 x 512 G-buffer receivers over 256 spheres, 8 bands, k = 4, at full
    size, compared on 256 sampled receivers away from contact with the
    photometric-loss cotangent restricted to them.  Most of these receivers
    sit under many overlapping caps (|F^| up to ~70), where the truncated
    squarings amplify rounding; the oracle's FP32 twin (same algorithm in
    FP32 arithmetic) is printed beside the GPU error as the inherent floor."""
    import torch
    sc = scenegen.scene_gbuffer()
    ok = np.flatnonzero(~sc["contact"])
    idx = np.sort(np.random.default_rng(2).choice(ok, 256, replace=False))
    w = _gbuffer_cotangent(sc, idx)
    h = run_hip(sc, w)
    o = run_oracle(sc, w[idx], idx=idx)
    t = run_oracle(sc, w[idx], idx=idx, dtype=torch.float32)
    print("fp32 twin: V %.2e B %.2e" % (rel_l2(t["V"], o["V"]), rel_max(t["B"], o["B"])))
    check_forward({"V": h["V"][idx], "B": h["B"][idx]}, o)
    check_grads(h, o, tol_geom=1e-3, idx=idx)


def test_largest_squaring_count():
    """k = 12, the largest supported: FP32 error roughly doubles per squaring."""
    sc = scenegen.scene_random_shell(9, 300, 24, 6)
    w = sc["grad_radiance"]
    h = run_hip(sc, w, k=12)
    o = run_oracle(sc, w, k=12)
    tol = TOL_V * 2 ** 8
    check_forward(h, o, tol_v=tol, tol_b=tol)
    check_grads(h, o, tol=TOL_G * 2 ** 8)


def test_large_request_scene_sampled():
    """The serving workload's large request (262,144 receivers on the unit
    sphere, 512 shell spheres, 8 bands) at full size, compared on 128 sampled
    receivers with the cotangent restricted to them."""
    sc = scenegen.large_request_scene(500)
    P = sc["points"].shape[0]
    idx = np.sort(np.random.default_rng(3).choice(P, 128, replace=False))
    w = np.zeros(P, np.float32)
    w[idx] = sc["grad_radiance"][idx]
    h = run_hip(sc, w)
    o = run_oracle(sc, w[idx], idx=idx)
    check_forward({"V": h["V"][idx], "B": h["B"][idx]}, o)
    check_grads(h, o, idx=idx)
