"""Pins for the oracle's direct product chain (Eq. 12 with the floored
blockers of Eq. 13), CPU only:
  * one blocker: the chain's V is the exact projection of the floored cap
    indicator, computed by Gauss rules split at the cap's edge in the sphere's
    own frame (exact: on each side the integrand is a polynomial in the
    cosine after the azimuthal rule);
  * several blockers: the chain is the left fold of pointwise products of the
    band-limited blocker functions, each projected by a rule exact for the
    product's degree (no Gaunt tensor involved);
  * no spheres, and a sphere centred on the receiver: V = 1;
  * against brute force: one sphere is exact, and heavy overlap keeps the
    chain's error against the projected true visibility at the truncation
    level;
  * large eps gives the binary blocker."""
import math

import numpy as np
import pytest
import torch

import scenegen
from oracle import brute, method, sh

DT = torch.float64


def _exact_blocker(p, c, r, n, eps):
    """Projection of 1 - (1 - e^-eps) 1[w . s >= t] about the sphere's axis,
    by cap rules on [t, 1] and [-1, t] (exact for band-limited y_lm)."""
    v = np.asarray(c) - np.asarray(p)
    d = np.linalg.norm(v)
    s = min(r / d, 1.0)
    t = math.sqrt(max(0.0, 1.0 - s * s))
    out = torch.zeros(n * n, dtype=DT)
    for lo, hi, val in ((t, 1.0, math.exp(-eps)), (-1.0, t, 1.0)):
        dirs, w = sh.cap_quadrature(v / d, lo, hi, n + 2, 2 * n + 2)
        out += val * (w @ sh.real_sh(dirs, n))
    return out


def _rand(seed, P, S, spread=1.5):
    g = torch.Generator().manual_seed(seed)
    pts = torch.randn(P, 3, generator=g, dtype=DT) * 0.3
    cen = torch.randn(S, 3, generator=g, dtype=DT) * spread
    rad = 0.2 + 0.5 * torch.rand(S, 1, generator=g, dtype=DT)
    return pts, torch.cat([cen, rad], 1)


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("eps", [3.0, 0.5, 40.0])
def test_single_blocker_is_its_exact_projection(n, eps):
    pts, sph = _rand(n, 6, 1)
    V = method.sh_direct_product(pts, sph, n, eps, sh.gaunt_tensor(n))
    for j in range(pts.shape[0]):
        ref = _exact_blocker(pts[j].numpy(), sph[0, :3].numpy(), float(sph[0, 3]), n, eps)
        assert torch.abs(V[j] - ref).max() < 1e-12


def test_receiver_inside_a_sphere_sees_a_floored_hemisphere():
    n, eps = 6, 3.0
    pts = torch.zeros(1, 3, dtype=DT)
    sph = torch.tensor([[0.1, -0.2, 0.3, 1.0]], dtype=DT)
    V = method.sh_direct_product(pts, sph, n, eps, sh.gaunt_tensor(n))[0]
    axis = (sph[0, :3] / torch.linalg.norm(sph[0, :3])).numpy()
    ref = torch.zeros(n * n, dtype=DT)
    for lo, hi, val in ((0.0, 1.0, math.exp(-eps)), (-1.0, 0.0, 1.0)):
        dirs, w = sh.cap_quadrature(axis, lo, hi, n + 2, 2 * n + 2)
        ref += val * (w @ sh.real_sh(dirs, n))
    assert torch.abs(V - ref).max() < 1e-12


@pytest.mark.parametrize("n", [2, 3, 5])
def test_chain_is_the_left_fold_of_pointwise_products(n):
    """Proj[Proj[Proj[b1 b2] b3] b4] with every product taken pointwise at the
    nodes of a rule exact to degree 3 (n - 1)."""
    pts, sph = _rand(7 + n, 4, 4, spread=0.8)
    V = method.sh_direct_product(pts, sph, n, 3.0, sh.gaunt_tensor(n))
    d, w = sh.sphere_quadrature(3 * (n - 1))
    Y = sh.real_sh(d, n)
    for j in range(pts.shape[0]):
        acc = None
        for i in range(sph.shape[0]):
            b = _exact_blocker(pts[j].numpy(), sph[i, :3].numpy(), float(sph[i, 3]), n, 3.0)
            acc = b if acc is None else (w * (Y @ acc) * (Y @ b)) @ Y
        assert torch.abs(V[j] - acc).max() < 1e-12


def test_order_matters_and_is_sphere_order():
    """Truncated products are not associative: reversing the spheres changes
    V (the chain is defined in sphere order)."""
    n = 4
    pts, sph = _rand(3, 5, 6, spread=0.6)
    C = sh.gaunt_tensor(n)
    a = method.sh_direct_product(pts, sph, n, 3.0, C)
    b = method.sh_direct_product(pts, sph.flip(0), n, 3.0, C)
    assert torch.abs(a - b).max() > 1e-6


def test_no_blockers_and_centred_sphere_give_one():
    n = 5
    pts = torch.tensor([[0.3, 0.1, -0.2]], dtype=DT)
    C = sh.gaunt_tensor(n)
    one = torch.zeros(n * n, dtype=DT)
    one[0] = math.sqrt(4 * math.pi)
    V0 = method.sh_direct_product(pts, torch.zeros(0, 4, dtype=DT), n, 3.0, C)
    assert torch.equal(V0[0], one)
    sph = torch.tensor([[0.3, 0.1, -0.2, 0.5]], dtype=DT)
    V1 = method.sh_direct_product(pts, sph, n, 3.0, C)
    assert torch.abs(V1[0] - one).max() < 1e-13


def test_large_eps_gives_the_binary_blocker():
    """e^-eps below double resolution relative to 1: the floored blocker is
    the binary one of Eq. 12 (0 on the cone)."""
    n = 4
    pts, sph = _rand(11, 3, 1)
    V = method.sh_direct_product(pts, sph, n, 50.0, sh.gaunt_tensor(n))
    for j in range(3):
        v = (sph[0, :3] - pts[j]).numpy()
        dd = np.linalg.norm(v)
        t = math.sqrt(1 - (float(sph[0, 3]) / dd) ** 2)
        dirs, w = sh.cap_quadrature(v / dd, -1.0, t, n + 2, 2 * n + 2)
        ref = w @ sh.real_sh(dirs, n)
        assert torch.abs(V[j] - ref).max() < 1e-12


def test_chain_against_brute_force_projected_visibility():
    """Two disjoint small caps: the chain's only error is the truncation of
    one product, far below the log-space schemes' band-limit error of the
    logarithm; against the brute-force projection of the true floored
    visibility it is within the quadrature's own accuracy scale."""
    n = 8
    pts = torch.zeros(1, 3, dtype=DT)
    sph = torch.tensor([[0.0, 0.0, 3.0, 0.6], [3.0, 0.0, 0.0, 0.6]], dtype=DT)
    V = method.sh_direct_product(pts, sph, n, 3.0, sh.gaunt_tensor(n))
    ref = brute.projected_visibility(pts, sph, n, 3.0, degree=400)
    assert torch.linalg.norm(V - ref) / torch.linalg.norm(ref) < 5e-3


def test_forward_product_mode_runs_through_the_pipeline():
    sc = scenegen.scene_random_shell(5, 20, 6, 4)
    o = method.run_forward(sc, exp_mode="product")
    T = method.scene_tensors(sc)
    V = method.sh_direct_product(T["points"], T["spheres"], 4, 3.0, sh.gaunt_tensor(4))
    assert torch.allclose(o["V"], V, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- taylor-K

def _band1_F(seed, n, P=5, scale=1.0):
    """Log-visibility vectors with a DC term and band-1 terms only, so every
    truncated power G^{*j} of band <= j stays exact while j < n."""
    g = torch.Generator().manual_seed(seed)
    F = torch.zeros(P, n * n, dtype=DT)
    F[:, 0] = torch.randn(P, generator=g, dtype=DT)
    F[:, 1:4] = torch.randn(P, 3, generator=g, dtype=DT) * scale
    return F


@pytest.mark.parametrize("K,k", [(1, 0), (1, 2), (2, 1), (3, 1), (4, 0), (7, 0), (2, 0)])
def test_taylor_is_exact_when_no_product_truncates(K, k):
    """n = 8 and F in bands <= 1: E_0 has band <= K and E_k band <= K 2^k <= 7,
    so no truncation happens and V is the projection of the pointwise
    exp(c) (sum_{j <= K} (g / 2^k)^j / j!)^(2^k), g the band-1 function."""
    n = 8
    F = _band1_F(K * 10 + k, n)
    V = method.sh_exponential_taylor(F, sh.gaunt_tensor(n), K, k)
    d, w = sh.sphere_quadrature(3 * n)
    Y = sh.real_sh(d, n)
    g = (F[:, 1:4] @ Y[:, 1:4].T) * 2.0 ** -k                  # [P, Q]
    poly = sum(g ** j / math.factorial(j) for j in range(K + 1)) ** (2 ** k)
    ref = torch.exp(F[:, 0] / math.sqrt(4 * math.pi))[:, None] * ((poly * w) @ Y)
    assert torch.abs(V - ref).max() < 1e-12 * max(1.0, float(torch.abs(ref).max()))


def test_taylor_converges_to_the_quadrature_exponential_without_truncation():
    """Still exact band-1 input, high order: sum_j g^j/j! -> exp(g), so V
    approaches Proj_n[exp(F~)] at the rate of the series' remainder."""
    n = 8
    F = _band1_F(3, n, scale=0.3)
    V = method.sh_exponential_taylor(F, sh.gaunt_tensor(n), 7, 0)
    ref = brute.exact_exponential(F, n, degree=80)
    rem = max(float(torch.linalg.norm(F[j, 1:4])) * math.sqrt(3 / (4 * math.pi)) for j in range(F.shape[0]))
    bound = rem ** 8 / math.factorial(8) * math.exp(rem) * 4 * math.pi
    assert float(torch.abs(V - ref).max() / torch.abs(ref).max()) < bound
