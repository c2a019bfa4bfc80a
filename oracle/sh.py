"""Real spherical harmonics and SH algebra in FP64 (oracle; test infrastructure).

Follows Sec. 3.2 of the paper:
  * Eq. 3   SH projection  f_i = integral of f(w) y_i(w) over the sphere
  * index   i = l*l + l + m with -l <= m <= l (0-based, band l < n)
  * Eq. 5   integral of a product of two band-limited functions = dot product
  * Eqs. 6-7 triple product (a * b)_i = sum_jk C_ijk a_j b_k with
            C_ijk = integral of y_i y_j y_k

Basis convention (the paper leaves it open): real, orthonormal, without the
Condon-Shortley phase.  With w = (x, y, z) a unit vector,
  y_l0      = K_l^0 P_l(z)
  y_lm      = sqrt(2) K_l^m Q_l^m(z) Re((x + i y)^m)      m > 0
  y_l,-m    = sqrt(2) K_l^m Q_l^m(z) Im((x + i y)^m)      m > 0
where Q_l^m = d^m P_l / dz^m and K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
This is the textbook definition P_l^m(cos t) cos(m phi) = (1 - z^2)^(m/2)
Q_l^m(z) cos(m phi) written with sin^m(t) e^(i m phi) = (x + i y)^m, which keeps
the basis a polynomial in (x, y, z) and therefore differentiable everywhere.

Legendre polynomials come from their explicit finite sum with exact rational
coefficients; integrals of polynomials are done exactly through
antiderivatives.  Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np
import torch

DT = torch.float64
FOUR_PI = 4.0 * math.pi


def sh_index(l: int, m: int) -> int:
    return l * l + l + m


def lm_of_index(i: int):
    l = int(math.isqrt(i))
    return l, i - l * l - l


# ---------------------------------------------------------------- polynomials

@lru_cache(maxsize=None)
def legendre_coeffs(l: int):
    """Exact coefficients c_j of P_l(z) = sum_j c_j z^j from
    P_l(z) = 2^-l sum_k (-1)^k C(l, k) C(2l - 2k, l) z^(l - 2k)."""
    c = [Fraction(0)] * (l + 1)
    for k in range(l // 2 + 1):
        c[l - 2 * k] += Fraction((-1) ** k * math.comb(l, k) * math.comb(2 * l - 2 * k, l), 2 ** l)
    return tuple(c)


def poly_deriv(c, m=1):
    c = list(c)
    for _ in range(m):
        c = [c[j] * j for j in range(1, len(c))] or [Fraction(0)]
    return tuple(c)


def poly_antideriv(c):
    return (Fraction(0),) + tuple(cj / (j + 1) for j, cj in enumerate(c))


def poly_eval(c, x):
    """Horner evaluation of exact coefficients at a float64 tensor / float."""
    acc = x * 0.0 + float(c[-1]) if isinstance(x, torch.Tensor) else float(c[-1])
    for cj in reversed(c[:-1]):
        acc = acc * x + float(cj)
    return acc


def poly_eval_exact(c, x: Fraction) -> Fraction:
    acc = Fraction(0)
    for cj in reversed(c):
        acc = acc * x + cj
    return acc


def legendre(l: int, z):
    return poly_eval(legendre_coeffs(l), z)


# ---------------------------------------------------------------- SH basis

def norm_K(l: int, m: int) -> float:
    m = abs(m)
    return math.sqrt((2 * l + 1) / FOUR_PI * math.factorial(l - m) / math.factorial(l + m))


def real_sh(dirs: torch.Tensor, n_bands: int) -> torch.Tensor:
    """y_i(w) for i < n_bands^2 at unit vectors ``dirs`` [..., 3] -> [..., n^2]."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    # Re / Im of (x + i y)^m, m = 0 .. n-1
    re = [torch.ones_like(x)]
    im = [torch.zeros_like(x)]
    for m in range(1, n_bands):
        r_prev, i_prev = re[-1], im[-1]
        re.append(r_prev * x - i_prev * y)
        im.append(r_prev * y + i_prev * x)
    out = [None] * (n_bands * n_bands)
    for l in range(n_bands):
        pl = legendre_coeffs(l)
        for m in range(0, l + 1):
            q = poly_eval(poly_deriv(pl, m), z)
            if m == 0:
                out[sh_index(l, 0)] = norm_K(l, 0) * q
            else:
                k = math.sqrt(2.0) * norm_K(l, m)
                out[sh_index(l, m)] = k * q * re[m]
                out[sh_index(l, -m)] = k * q * im[m]
    return torch.stack(out, dim=-1)


# ---------------------------------------------------------------- Funk-Hecke

def funk_hecke_cap(t, l: int):
    """2 pi * integral_t^1 P_l(x) dx: the Funk-Hecke eigenvalue of the
    indicator of the cap {w : w . s >= t}, exact through the antiderivative."""
    A = poly_antideriv(legendre_coeffs(l))
    return 2.0 * math.pi * (float(poly_eval_exact(A, Fraction(1))) - poly_eval(A, t))


@lru_cache(maxsize=None)
def clamped_cosine_coeff(l: int) -> float:
    """A_l = 2 pi * integral_0^1 x P_l(x) dx: the Funk-Hecke eigenvalue of
    max(w . n, 0) (Eq. 10), exact in rational arithmetic."""
    xp = (Fraction(0),) + legendre_coeffs(l)
    A = poly_antideriv(xp)
    return 2.0 * math.pi * float(poly_eval_exact(A, Fraction(1)) - poly_eval_exact(A, Fraction(0)))


# ---------------------------------------------------------------- quadrature

def sphere_quadrature(degree: int):
    """Product rule exact for every polynomial in (x, y, z) of total degree
    <= ``degree`` on the unit sphere: Gauss-Legendre in z with
    ceil((degree+1)/2) nodes times a uniform rule in phi with degree+1 nodes.
    Returns (dirs [Q, 3], weights [Q]) in float64."""
    q = degree // 2 + 1
    M = degree + 1
    z, wz = np.polynomial.legendre.leggauss(q)
    phi = (np.arange(M) + 0.5) * (2.0 * np.pi / M)
    Z, PH = np.meshgrid(z, phi, indexing="ij")
    W = np.repeat(wz[:, None], M, axis=1) * (2.0 * np.pi / M)
    st = np.sqrt(1.0 - Z ** 2)
    d = np.stack([st * np.cos(PH), st * np.sin(PH), Z], axis=-1).reshape(-1, 3)
    return torch.tensor(d, dtype=DT), torch.tensor(W.reshape(-1), dtype=DT)


def cap_quadrature(axis, t_lo: float, t_hi: float, n_z: int, n_phi: int):
    """Quadrature over the band {w : t_lo <= w . axis <= t_hi}: Gauss-Legendre
    in the cosine about ``axis`` and a uniform rule in the azimuth.  Exact for
    polynomials of degree <= 2 n_z - 1 in the cosine and < n_phi in the
    azimuthal frequency."""
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    tmp = np.array([1.0, 0.0, 0.0]) if abs(axis[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(axis, tmp)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    u, wu = np.polynomial.legendre.leggauss(n_z)
    c = 0.5 * (t_hi - t_lo) * u + 0.5 * (t_hi + t_lo)
    wc = 0.5 * (t_hi - t_lo) * wu
    phi = (np.arange(n_phi) + 0.5) * (2.0 * np.pi / n_phi)
    C, PH = np.meshgrid(c, phi, indexing="ij")
    W = np.repeat(wc[:, None], n_phi, axis=1) * (2.0 * np.pi / n_phi)
    st = np.sqrt(np.maximum(0.0, 1.0 - C ** 2))
    d = (st * np.cos(PH))[..., None] * e1 + (st * np.sin(PH))[..., None] * e2 + C[..., None] * axis
    return torch.tensor(d.reshape(-1, 3), dtype=DT), torch.tensor(W.reshape(-1), dtype=DT)


@lru_cache(maxsize=None)
def gaunt_tensor(n_bands: int) -> torch.Tensor:
    """C_ijk = integral of y_i y_j y_k (Eq. 7), i, j, k < n^2, by a rule exact
    to degree 3 (n - 1) (the integrand's degree)."""
    d, w = sphere_quadrature(max(3 * (n_bands - 1), 0))
    Y = real_sh(d, n_bands)
    return torch.einsum("q,qi,qj,qk->ijk", w, Y, Y, Y)


def project(fun, n_bands: int, degree: int) -> torch.Tensor:
    """SH projection (Eq. 3) of a callable f(dirs) by a rule exact to
    ``degree`` (exact when f is a polynomial of at most that degree)."""
    d, w = sphere_quadrature(degree)
    return torch.einsum("q,q,qi->i", w, fun(d), real_sh(d, n_bands))


def triple_product(a: torch.Tensor, b: torch.Tensor, C: torch.Tensor) -> torch.Tensor:
    """(a * b)_i = sum_jk C_ijk a_j b_k over the last axis (Eq. 7)."""
    return torch.einsum("ijk,...j,...k->...i", C, a, b)


# ---------------------------------------------------------------- Eq. 9

def envmap_directions(H: int, W: int):
    """Pixel-centre directions and exact pixel solid angles of an
    equirectangular map: row r spans polar angles [r pi / H, (r + 1) pi / H]
    from +z, column c spans azimuths [c 2 pi / W, (c + 1) 2 pi / W]; the
    weight of a pixel is the area of that patch, (cos th_r - cos th_{r+1})
    2 pi / W, and the weights sum to 4 pi.  Returns dirs [H, W, 3] and
    weights [H, W] (float64)."""
    th_edges = np.arange(H + 1) * (np.pi / H)
    th = (np.arange(H) + 0.5) * (np.pi / H)
    ph = (np.arange(W) + 0.5) * (2.0 * np.pi / W)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1)
    wrow = (np.cos(th_edges[:-1]) - np.cos(th_edges[1:])) * (2.0 * np.pi / W)
    return torch.tensor(d, dtype=DT), torch.tensor(np.repeat(wrow[:, None], W, axis=1), dtype=DT)


def envmap_to_sh(image, n_bands: int) -> torch.Tensor:
    """Eq. 9 by numerical integration over an equirectangular map:
    L_i = sum over pixels of L(w) y_i(w) dw.  ``image`` [H, W] or [C, H, W]
    -> [n^2] or [C, n^2]."""
    img = torch.as_tensor(np.asarray(image), dtype=DT)
    H, W = img.shape[-2:]
    d, w = envmap_directions(H, W)
    Y = real_sh(d, n_bands)                                   # [H, W, N]
    return torch.einsum("...hw,hw,hwi->...i", img, w, Y)
