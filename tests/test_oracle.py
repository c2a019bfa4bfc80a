"""Pins for the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: a library
routine (SciPy spherical harmonics, NumPy Legendre series, adaptive
quadrature), a closed form, an exact integral taken by a different rule, an
invariance, a limit, or central finite differences.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special
import torch

import scenegen
from oracle import brute, method, sh

DT = torch.float64
PI = math.pi


def unit(n, seed=0):
    g = torch.Generator().manual_seed(seed)
    d = torch.randn(n, 3, dtype=DT, generator=g)
    return d / d.norm(dim=1, keepdim=True)


# ------------------------------------------------------------------ basis

def test_basis_matches_scipy():
    d = unit(64)
    Y = sh.real_sh(d, 8).numpy()
    th = np.arccos(np.clip(d[:, 2].numpy(), -1, 1))
    ph = np.arctan2(d[:, 1].numpy(), d[:, 0].numpy())
    for l in range(8):
        for m in range(-l, l + 1):
            Yc = scipy.special.sph_harm_y(l, abs(m), th, ph)
            # SciPy carries the Condon-Shortley phase; the real basis here does not.
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * Yc.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * Yc.imag
            else:
                ref = Yc.real
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13)


def test_basis_low_order_closed_forms():
    d = unit(32, 1)
    x, y, z = d.unbind(1)
    Y = sh.real_sh(d, 3)
    k1 = math.sqrt(3 / (4 * PI))
    ref = [torch.full_like(x, 0.5 / math.sqrt(PI)), k1 * y, k1 * z, k1 * x,
           0.5 * math.sqrt(15 / PI) * x * y, 0.5 * math.sqrt(15 / PI) * y * z,
           0.25 * math.sqrt(5 / PI) * (3 * z * z - 1), 0.5 * math.sqrt(15 / PI) * x * z,
           0.25 * math.sqrt(15 / PI) * (x * x - y * y)]
    torch.testing.assert_close(Y, torch.stack(ref, 1), atol=1e-14, rtol=0)


def test_basis_orthonormal():
    d, w = sh.sphere_quadrature(2 * 7)
    Y = sh.real_sh(d, 8)
    G = (Y.T * w) @ Y
    assert (G - torch.eye(64, dtype=DT)).abs().max() < 1e-13


def test_legendre_matches_numpy():
    z = torch.linspace(-1, 1, 41, dtype=DT)
    for l in range(10):
        ref = np.polynomial.legendre.legval(z.numpy(), [0] * l + [1])
        np.testing.assert_allclose(sh.legendre(l, z).numpy(), ref, atol=1e-14)


# ------------------------------------------------------------------ log-cap zonal coefficients

@pytest.mark.parametrize("alpha", [0.1, 0.7, PI / 2, 2.5])
def test_cap_coefficients_vs_adaptive_quadrature(alpha):
    t = math.cos(alpha)
    g = method.log_cap_zonal(torch.tensor(t, dtype=DT), 8, 3.0)
    for l in range(8):
        val, _ = scipy.integrate.quad(lambda x: scipy.special.eval_legendre(l, x), t, 1.0,
                                      epsabs=1e-15, epsrel=1e-13, limit=200)
        assert abs(g[l].item() - (-3.0 * 2 * PI * val)) < 1e-12


def test_cap_coefficients_legendre_difference_identity():
    # int_t^1 P_l = (P_{l-1}(t) - P_{l+1}(t)) / (2l + 1), with P_{-1} = 1.
    t = torch.linspace(-1, 1, 33, dtype=DT)
    g = method.log_cap_zonal(t, 8, 3.0)
    for l in range(8):
        pm = torch.ones_like(t) if l == 0 else sh.legendre(l - 1, t)
        ref = -3.0 * 2 * PI / (2 * l + 1) * (pm - sh.legendre(l + 1, t))
        torch.testing.assert_close(g[:, l], ref, atol=1e-12, rtol=0)


def test_cap_coefficient_derivative_is_legendre():
    t = torch.linspace(-0.95, 0.95, 17, dtype=DT, requires_grad=True)
    g = method.log_cap_zonal(t, 8, 3.0)
    for l in range(8):
        (dg,) = torch.autograd.grad(g[:, l].sum(), t, retain_graph=True)
        torch.testing.assert_close(dg, 2 * PI * 3.0 * sh.legendre(l, t.detach()), atol=1e-12, rtol=0)


def test_cap_coefficient_limits():
    eps = 3.0
    # tiny cap: every band -> -eps * (solid angle) = -eps * pi s^2
    s = 1e-4
    g = method.log_cap_zonal(torch.tensor(math.sqrt(1 - s * s), dtype=DT), 8, eps)
    torch.testing.assert_close(g, torch.full((8,), -eps * PI * s * s, dtype=DT), rtol=1e-6, atol=0)
    # whole sphere (t = -1): only the DC band survives
    g = method.log_cap_zonal(torch.tensor(-1.0, dtype=DT), 8, eps)
    assert abs(g[0].item() + eps * 4 * PI) < 1e-12 and g[1:].abs().max() < 1e-12
    # hemisphere (t = 0): even bands above 0 vanish (P_odd(0) = 0)
    g = method.log_cap_zonal(torch.tensor(0.0, dtype=DT), 8, eps)
    assert abs(g[0].item() + eps * 2 * PI) < 1e-12
    assert abs(g[1].item() + eps * PI) < 1e-12
    assert g[2].abs() < 1e-12 and g[4].abs() < 1e-12 and g[6].abs() < 1e-12
    assert abs(g[3].item() - (-eps) * 2 * PI / 7 * (-0.5 - 0.375)) < 1e-12  # P_2(0) = -1/2, P_4(0) = 3/8


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rotated_cap_is_projection_of_indicator(seed):
    """Steps 2-3 together: g_l(t) y_lm(s) must equal the SH projection of
    -eps * 1[w . s >= t].  The cap rule about s makes the integral exact."""
    s_hat = unit(1, seed)[0]
    t = [0.93, 0.4, -0.2][seed]
    d, w = sh.cap_quadrature(s_hat.numpy(), t, 1.0, 12, 20)
    ref = -3.0 * torch.einsum("q,qi->i", w, sh.real_sh(d, 8))
    g = method.log_cap_zonal(torch.tensor(t, dtype=DT), 8, 3.0)
    got = g[method.band_of_index(8)] * sh.real_sh(s_hat[None], 8)[0]
    torch.testing.assert_close(got, ref, atol=1e-12, rtol=0)


def test_log_visibility_single_sphere_geometry():
    """F for one sphere is the projection of -eps on the cone it subtends;
    a receiver inside the sphere sees a hemisphere cap; d = 0 contributes 0."""
    p = torch.tensor([[0.1, -0.2, 0.3]], dtype=DT)
    sph = torch.tensor([[0.6, 0.4, 0.9, 0.35]], dtype=DT)
    v = sph[0, :3] - p[0]
    dist = v.norm()
    t = math.sqrt(1 - (0.35 / dist.item()) ** 2)
    d, w = sh.cap_quadrature((v / dist).numpy(), t, 1.0, 12, 20)
    ref = -3.0 * torch.einsum("q,qi->i", w, sh.real_sh(d, 6))
    F = method.log_visibility(p, sph, 6, 3.0)[0]
    torch.testing.assert_close(F, ref, atol=1e-12, rtol=0)
    inside = torch.tensor([[0.6, 0.4, 0.9, 2.0]], dtype=DT)
    d, w = sh.cap_quadrature((v / dist).numpy(), 0.0, 1.0, 12, 20)
    ref = -3.0 * torch.einsum("q,qi->i", w, sh.real_sh(d, 6))
    torch.testing.assert_close(method.log_visibility(p, inside, 6, 3.0)[0], ref, atol=1e-12, rtol=0)
    centred = torch.tensor([[0.1, -0.2, 0.3, 0.5]], dtype=DT)
    assert method.log_visibility(p, centred, 6, 3.0).abs().max() == 0


# ------------------------------------------------------------------ transfer H

def test_clamped_cosine_coefficients():
    ref = [PI, 2 * PI / 3, PI / 4, 0.0, -PI / 24, 0.0, PI / 64, 0.0]
    for l, r in enumerate(ref):
        assert abs(sh.clamped_cosine_coeff(l) - r) < 1e-15
    # Ramamoorthi-Hanrahan closed form for even l >= 2
    for l in range(2, 12, 2):
        rh = 2 * PI * (-1) ** (l // 2 - 1) / ((l + 2) * (l - 1)) * math.factorial(l) / (
            2 ** l * math.factorial(l // 2) ** 2)
        assert abs(sh.clamped_cosine_coeff(l) - rh) < 1e-14


def test_transfer_is_projection_of_clamped_cosine():
    nrm = unit(4, 3) * torch.tensor([[1.0], [2.5], [0.3], [7.0]], dtype=DT)  # non-unit normals
    H = method.transfer(nrm, 8)
    for k in range(4):
        nh = nrm[k] / nrm[k].norm()
        d, w = sh.cap_quadrature(nh.numpy(), 0.0, 1.0, 10, 20)
        ref = torch.einsum("q,q,qi->i", w, d @ nh, sh.real_sh(d, 8))
        torch.testing.assert_close(H[k], ref, atol=1e-12, rtol=0)


# ------------------------------------------------------------------ triple product

@pytest.mark.parametrize("n,nnz", [(4, 353), (6, 2907), (8, 12868)])
def test_gaunt_structure(n, nnz):
    C = sh.gaunt_tensor(n)
    N = n * n
    assert (C - C.permute(1, 0, 2)).abs().max() < 1e-14
    assert (C - C.permute(2, 1, 0)).abs().max() < 1e-14
    torch.testing.assert_close(C[0], torch.eye(N, dtype=DT) / math.sqrt(4 * PI), atol=1e-14, rtol=0)
    assert int((C.abs() > 1e-12).sum()) == nnz
    bands = [int(math.isqrt(i)) for i in range(N)]
    for i in range(N):
        for j in range(N):
            for k in range(N):
                li, lj, lk = bands[i], bands[j], bands[k]
                if (li + lj + lk) % 2 or li > lj + lk or lj > li + lk or lk > li + lj:
                    assert abs(C[i, j, k]) < 1e-13


def test_gaunt_known_value():
    # int y_10 y_10 y_20 = 1 / sqrt(5 pi)  (hand integration of z^2 (3 z^2 - 1))
    C = sh.gaunt_tensor(3)
    assert abs(C[2, 2, 6].item() - 1 / math.sqrt(5 * PI)) < 1e-14


def test_triple_product_is_projection_of_product():
    """a * b = Proj_n[a~ b~], checked with a finer rule of a different size."""
    g = torch.Generator().manual_seed(5)
    a = torch.randn(3, 64, dtype=DT, generator=g)
    b = torch.randn(3, 64, dtype=DT, generator=g)
    got = sh.triple_product(a, b, sh.gaunt_tensor(8))
    d, w = sh.sphere_quadrature(31)
    Y = sh.real_sh(d, 8)
    ref = ((Y @ a.T) * (Y @ b.T) * w[:, None]).T @ Y
    torch.testing.assert_close(got, ref, atol=1e-12, rtol=0)


# ------------------------------------------------------------------ exponential

def test_exp_of_zero_and_of_constant():
    C = sh.gaunt_tensor(8)
    F = torch.zeros(2, 64, dtype=DT)
    F[1, 0] = -2.7
    for k in (0, 1, 4, 6):
        V, c, _ = method.sh_exponential(F, C, k)
        e0 = torch.zeros(64, dtype=DT)
        e0[0] = math.sqrt(4 * PI)
        # roundoff grows about 2x per squaring
        torch.testing.assert_close(V[0], e0, atol=1e-14 * 2 ** (k + 2), rtol=0)
        torch.testing.assert_close(V[1], math.exp(-2.7 / math.sqrt(4 * PI)) * e0, atol=1e-14 * 2 ** (k + 2), rtol=0)


def test_exp_single_band_is_scalar_exponential():
    C = sh.gaunt_tensor(1)
    F = torch.tensor([[0.8], [-5.0]], dtype=DT)
    V, _, _ = method.sh_exponential(F, C, 4)
    torch.testing.assert_close(V[:, 0], math.sqrt(4 * PI) * torch.exp(F[:, 0] / math.sqrt(4 * PI)))


def test_optimal_linear_coefficients():
    """a = b = exp(sigma^2/2) minimises E[(e^g - a - b g)^2] for g ~ N(0, sigma^2)
    (Gauss-Hermite expectation, then the 2x2 normal equations)."""
    x, w = np.polynomial.hermite_e.hermegauss(80)
    w = w / w.sum()
    for sigma in (0.05, 0.3, 1.0):
        g = sigma * x
        A = np.array([[1, (w * g).sum()], [(w * g).sum(), (w * g * g).sum()]])
        rhs = np.array([(w * np.exp(g)).sum(), (w * g * np.exp(g)).sum()])
        a, b = np.linalg.solve(A, rhs)
        assert abs(a - math.exp(sigma ** 2 / 2)) < 1e-12 and abs(b - math.exp(sigma ** 2 / 2)) < 1e-12
    # and the oracle's E_0 uses sigma^2 = |G|^2 / (4 pi), the variance of G~ over the sphere
    G = torch.zeros(1, 16, dtype=DT)
    G[0, 5] = 0.4
    F = G * 2 ** 3
    _, _, Es = method.sh_exponential(F, sh.gaunt_tensor(4), 3)
    a = math.exp(0.4 ** 2 / (8 * PI))
    assert abs(Es[0][0, 0].item() - a * math.sqrt(4 * PI)) < 1e-14
    assert abs(Es[0][0, 5].item() - a * 0.4) < 1e-14


def test_squaring_step_is_projected_square():
    C = sh.gaunt_tensor(6)
    g = torch.Generator().manual_seed(2)
    F = 0.3 * torch.randn(2, 36, dtype=DT, generator=g)
    _, _, Es = method.sh_exponential(F, C, 3)
    d, w = sh.sphere_quadrature(25)
    Y = sh.real_sh(d, 6)
    for m in range(3):
        vals = (Y @ Es[m].T) ** 2
        ref = (vals * w[:, None]).T @ Y
        torch.testing.assert_close(Es[m + 1], ref, atol=1e-12, rtol=0)


def test_exp_second_order_error_term():
    """Expand the scheme for F = delta F0: exact DC split, E_0 = a (1 + G) with
    G = F^/2^k, k truncated squarings.  To second order it gives
    1 + F^ + (1 - 2^-k)/2 F^*F^ + a-correction; the exact projected exponential
    has 1 + F^ + F^*F^/2.  The variance term a = exp(|G|^2/8pi) cancels the DC
    part of the gap exactly, so (V - Proj[exp F~]) / delta^2 must tend to
    -2^-(k+1) (F^*F^ with its DC entry removed), with an O(delta) remainder.
    A wrong scaling, squaring count or linear coefficient breaks this."""
    C = sh.gaunt_tensor(4)
    g = torch.Generator().manual_seed(4)
    F0 = torch.randn(1, 16, dtype=DT, generator=g)
    Fh = F0.clone()
    Fh[:, 0] = 0
    Q = sh.triple_product(Fh, Fh, C)
    Q[:, 0] = 0
    for k in (0, 1, 3, 4):
        lead = -(2.0 ** (-k - 1)) * Q
        rem = []
        for delta in (1e-2, 1e-3):
            V, _, _ = method.sh_exponential(delta * F0, C, k)
            ex = brute.exact_exponential(delta * F0, 4)
            rem.append(((V - ex) / delta ** 2 - lead).norm().item())
        assert rem[0] < 0.05 * lead.norm().item() + 0.03, (k, rem)
        assert 7.0 < rem[0] / rem[1] < 13.0, (k, rem)   # remainder is O(delta)


# ------------------------------------------------------------------ shading

def test_shade_is_triple_integral():
    g = torch.Generator().manual_seed(7)
    V = torch.randn(5, 64, dtype=DT, generator=g)
    H = torch.randn(5, 64, dtype=DT, generator=g)
    L = torch.randn(64, dtype=DT, generator=g)
    a = torch.rand(5, dtype=DT, generator=g)
    B = method.shade(V, H, a, L, sh.gaunt_tensor(8))
    d, w = sh.sphere_quadrature(21)
    Y = sh.real_sh(d, 8)
    ref = a * ((Y @ L)[:, None] * (Y @ V.T) * (Y @ H.T) * w[:, None]).sum(0)
    torch.testing.assert_close(B, ref, atol=1e-12, rtol=0)


@pytest.mark.parametrize("n", [3, 4, 8])
def test_unoccluded_is_irradiance(n):
    """No spheres: V = sqrt(4 pi) e_0 and B = a int L~ max(w . n, 0) dw."""
    sc = scenegen.scene_random_shell(11, 12, 0, n)
    sc["spheres"] = np.zeros((0, 4), np.float32)
    o = method.run_forward(sc)
    T = method.scene_tensors(sc)
    e0 = torch.zeros(n * n, dtype=DT)
    e0[0] = math.sqrt(4 * PI)
    torch.testing.assert_close(o["V"], e0.expand_as(o["V"]), atol=1e-12, rtol=0)
    ref = brute.radiance_unshadowed(T["normals"], T["albedo"], T["light"], n)
    torch.testing.assert_close(o["B"], ref, atol=1e-12, rtol=0)


# ------------------------------------------------------------------ invariances

def _small_scene(seed=0, P=24, S=10, n=6):
    return scenegen.scene_random_shell(seed, P, S, n)


def _rotation(seed):
    g = np.random.default_rng(seed)
    q, r = np.linalg.qr(g.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_rotation_invariance():
    sc = _small_scene()
    R = _rotation(3)
    B0 = method.run_forward(sc)["B"]
    rot = dict(sc)
    rot["points"] = (sc["points"].astype(np.float64) @ R.T)
    rot["normals"] = (sc["normals"].astype(np.float64) @ R.T)
    sp = sc["spheres"].astype(np.float64).copy()
    sp[:, :3] = sp[:, :3] @ R.T
    rot["spheres"] = sp
    M = brute.rotation_matrix(R, 6)
    rot["light"] = (M @ torch.tensor(sc["light"], dtype=DT)).numpy()
    B1 = method.run_forward(rot)["B"]
    torch.testing.assert_close(B1, B0, atol=1e-12, rtol=0)


def test_translation_scale_permutation_invariance():
    sc = _small_scene(1)
    B0 = method.run_forward(sc)["B"]
    tr = dict(sc)
    shift = np.array([0.3, -1.2, 2.0])
    tr["points"] = sc["points"].astype(np.float64) + shift
    sp = sc["spheres"].astype(np.float64).copy()
    sp[:, :3] += shift
    tr["spheres"] = sp
    torch.testing.assert_close(method.run_forward(tr)["B"], B0, atol=1e-12, rtol=0)
    scl = dict(sc)
    scl["points"] = sc["points"].astype(np.float64) * 3.7
    scl["spheres"] = sc["spheres"].astype(np.float64) * 3.7
    torch.testing.assert_close(method.run_forward(scl)["B"], B0, atol=1e-12, rtol=0)
    perm = dict(sc)
    perm["spheres"] = sc["spheres"][np.random.default_rng(0).permutation(len(sc["spheres"]))]
    torch.testing.assert_close(method.run_forward(perm)["B"], B0, atol=1e-12, rtol=0)


def test_far_sphere_limit():
    """A sphere of solid angle ~ pi s^2 far away acts like a point blocker:
    F_lm -> -eps pi s^2 y_lm(s_hat)."""
    p = torch.zeros(1, 3, dtype=DT)
    dirn = unit(1, 9)[0]
    Dist, r = 1e4, 1.0
    sph = torch.cat([dirn * Dist, torch.tensor([r], dtype=DT)])[None]
    F = method.log_visibility(p, sph, 8, 3.0)[0]
    ref = -3.0 * PI * (r / Dist) ** 2 * sh.real_sh(dirn[None], 8)[0]
    torch.testing.assert_close(F, ref, rtol=1e-6, atol=1e-16)


# ------------------------------------------------------------------ against the binary ground truth

def test_against_binary_visibility_bruteforce():
    """Eq. 2 with the binary blocker function (loose: the method is an
    approximation); it must be closer than ignoring shadows altogether."""
    sc = scenegen.scene_icosphere_shell()
    idx = np.arange(0, 2562, 101)
    T = method.scene_tensors(sc)
    Bm = method.run_forward(sc, idx=idx)["B"]
    Bb = brute.radiance_binary(T["points"][idx], T["normals"][idx], T["albedo"][idx],
                               T["spheres"], T["light"], 4)
    Bu = brute.radiance_unshadowed(T["normals"][idx], T["albedo"][idx], T["light"], 4)
    scale = Bb.abs().max()
    e_method = ((Bm - Bb).abs().max() / scale).item()
    e_unshadowed = ((Bu - Bb).abs().max() / scale).item()
    assert e_method < 0.25 and e_method < e_unshadowed, (e_method, e_unshadowed)


# ------------------------------------------------------------------ gradients vs finite differences

def test_gradients_vs_central_differences():
    sc = scenegen.subset(scenegen.scene_body(), np.arange(0, 20000, 625))  # 32 receivers
    sc["spheres"] = sc["spheres"][::4]                                      # 32 spheres
    P = sc["points"].shape[0]
    w = np.random.default_rng(1).standard_normal(P)
    got = method.run_forward_backward(sc, w)
    base = method.scene_tensors(sc)

    def loss(T):
        with torch.no_grad():
            o = method.forward(T["points"], T["normals"], T["albedo"], T["spheres"], T["light"], 8)
            return float((o["B"] * torch.tensor(w, dtype=DT)).sum())

    h = 1e-4
    rng = np.random.default_rng(2)

    def central(key, j=None, u=None):
        """Central differences at h and h/2 combined by Richardson
        extrapolation (truncation O(h^4); small spheres make h^2 visible)."""
        vals = []
        for step in (h, h / 2):
            Tp = {k: v.clone() for k, v in base.items()}
            Tm = {k: v.clone() for k, v in base.items()}
            if u is None:
                Tp[key].view(-1)[j] += step
                Tm[key].view(-1)[j] -= step
            else:
                Tp[key] = Tp[key] + step * u.reshape(base[key].shape)
                Tm[key] = Tm[key] - step * u.reshape(base[key].shape)
            vals.append((loss(Tp) - loss(Tm)) / (2 * step))
        return (4 * vals[1] - vals[0]) / 3

    checks = [("spheres", "grad_spheres"), ("light", "grad_light"), ("albedo", "grad_albedo"),
              ("points", "grad_points"), ("normals", "grad_normals")]
    for key, gkey in checks:
        G = got[gkey]
        flat = base[key].reshape(-1)
        picks = rng.choice(flat.numel(), size=min(12, flat.numel()), replace=False)
        scale = G.abs().max().item()
        for j in picks:
            fd = central(key, j=j)
            assert abs(fd - G.reshape(-1)[j].item()) <= 1e-6 * scale, (key, j, fd, G.reshape(-1)[j].item())
        # a random directional derivative through the whole group
        u = torch.tensor(rng.standard_normal(flat.numel()), dtype=DT)
        fd = central(key, u=u)
        an = (G.reshape(-1) * u).sum().item()
        assert abs(fd - an) <= 1e-6 * max(abs(an), scale), (key, fd, an)


# --------------------------------------------------------------- Eq. 9, channels

def test_envmap_weights_cover_the_sphere_and_constant_map_is_dc():
    d, w = sh.envmap_directions(32, 64)
    assert abs(float(w.sum()) - 4 * np.pi) < 1e-12
    assert torch.allclose(torch.linalg.norm(d, dim=-1), torch.ones(32, 64, dtype=torch.float64))
    L = sh.envmap_to_sh(np.full((32, 64), 2.5), 4)
    assert abs(float(L[0]) - 2.5 * np.sqrt(4 * np.pi)) < 1e-12        # exact: weights sum to 4 pi
    assert float(L[1:].abs().max()) < 1.5e-2   # midpoint-in-theta error of the m = 0 bands at 32 rows


@pytest.mark.parametrize("j", [0, 2, 5, 7, 12, 20, 40, 63])
def test_envmap_of_a_basis_function_recovers_its_coefficient(j):
    """Orthonormality: projecting y_j sampled on the map gives e_j up to the
    quadrature error, which falls as the map is refined."""
    errs = []
    for H in (64, 256):
        d, _ = sh.envmap_directions(H, 2 * H)
        img = sh.real_sh(d, 8)[..., j].numpy()
        L = sh.envmap_to_sh(img, 8)
        e = torch.zeros(64, dtype=torch.float64)
        e[j] = 1.0
        errs.append(float((L - e).abs().max()))
    assert errs[1] < 2e-4 and errs[1] < errs[0] / 8


def test_envmap_channels_are_independent():
    rng = np.random.default_rng(0)
    img = rng.random((3, 16, 32))
    L = sh.envmap_to_sh(img, 5)
    for c in range(3):
        assert torch.allclose(L[c], sh.envmap_to_sh(img[c], 5), rtol=0, atol=1e-14)


def test_shade_channels_is_monochrome_per_channel():
    sc = scenegen.scene_random_shell(21, 40, 8, 6)
    rng = np.random.default_rng(1)
    alb = torch.tensor(rng.uniform(0.2, 0.9, (40, 3)))
    light = torch.tensor(rng.standard_normal((3, 36)))
    T = method.scene_tensors(sc)
    C = sh.gaunt_tensor(6)
    F = method.log_visibility(T["points"], T["spheres"], 6, 3.0)
    V, _, _ = method.sh_exponential(F, C, 4)
    H = method.transfer(T["normals"], 6)
    B = method.shade_channels(V, H, alb, light, C)
    for c in range(3):
        assert torch.allclose(B[:, c], method.shade(V, H, alb[:, c], light[c], C), rtol=1e-14, atol=1e-14)


def test_channel_gradients_are_per_channel_and_summed_where_shared():
    """Per channel, the multi-channel oracle's radiance, albedo and lighting
    gradients are the one-channel oracle's (each pinned above); the receiver,
    normal and sphere gradients, through the shared V and H, are the sums of
    the one-channel ones (linearity of the cotangent)."""
    sc = scenegen.scene_random_shell(4, 60, 10, 5)
    ch = scenegen.colour_channels(sc, 3, seed=2)
    o = method.run_forward_backward_channels(sc, ch["albedo"], ch["light"], ch["grad_radiance"], chunk=25)
    acc = {k: 0.0 for k in ("grad_points", "grad_normals", "grad_spheres")}
    for c in range(3):
        s1 = dict(sc, albedo=ch["albedo"][:, c].copy(), light=ch["light"][c].copy())
        m = method.run_forward_backward(s1, ch["grad_radiance"][:, c])
        assert torch.allclose(o["B"][:, c], m["B"], rtol=1e-13, atol=1e-13)
        assert torch.allclose(o["grad_albedo"][:, c], m["grad_albedo"], rtol=1e-12, atol=1e-13)
        assert torch.allclose(o["grad_light"][c], m["grad_light"], rtol=1e-12, atol=1e-12)
        for k in acc:
            acc[k] = acc[k] + m[k]
    for k in acc:
        assert torch.allclose(o[k], acc[k], rtol=1e-11, atol=1e-11), k


# ------------------------------------------------------- quadrature exponential

def test_quadrature_exponential_exact_cases():
    for n in (1, 3, 8):
        N = n * n
        z = torch.zeros(2, N, dtype=DT)
        V = method.sh_exponential_quadrature(z, n)
        e0 = torch.zeros(N, dtype=DT)
        e0[0] = math.sqrt(4 * PI)
        assert torch.allclose(V, e0.expand(2, N), rtol=0, atol=1e-13)       # exp(0) = 1
        F = torch.zeros(1, N, dtype=DT)
        F[0, 0] = -2.5
        V = method.sh_exponential_quadrature(F, n)
        assert torch.allclose(V[0], math.exp(-2.5 / math.sqrt(4 * PI)) * e0, rtol=1e-13, atol=1e-14)


def test_quadrature_exponential_converges_to_the_projected_exponential():
    """The rule of degree 8n - 1 against a far finer one (brute force, degree
    120): spectral convergence for smooth moderate F."""
    g = torch.Generator().manual_seed(3)
    for n, tol in ((2, 1e-12), (4, 1e-8), (8, 1e-4)):
        F = torch.randn(4, n * n, dtype=DT, generator=g) * 0.5
        F[:, 0] = -3.0
        V = method.sh_exponential_quadrature(F, n)
        ref = brute.exact_exponential(F, n, degree=120)
        assert float((V - ref).norm() / ref.norm()) < tol, n


def test_quadrature_exponential_gradient_matches_central_differences():
    g = torch.Generator().manual_seed(4)
    F = (torch.randn(3, 16, dtype=DT, generator=g) * 0.4).requires_grad_(True)
    W = torch.randn(3, 16, dtype=DT, generator=g)
    f = lambda x: (method.sh_exponential_quadrature(x, 4) * W).sum()  # noqa: E731
    gr = torch.autograd.grad(f(F), F)[0]
    h = 1e-6
    for (a, b) in ((0, 0), (1, 5), (2, 15), (0, 9)):
        e = torch.zeros_like(F)
        e[a, b] = h
        fd = (f(F.detach() + e) - f(F.detach() - e)) / (2 * h)
        assert abs(float(gr[a, b] - fd)) < 1e-7 * max(1.0, abs(float(fd)))
