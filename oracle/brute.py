"""Reference integrals that pin the oracle (test infrastructure).

None of these is the method; they are the quantities the method approximates
or identities it must satisfy:
  * radiance_binary: Eq. 2 with the binary blocker function (the exact
    product of blockers, Eq. 12, evaluated pointwise in direction space)
    integrated by dense quadrature;
  * radiance_unshadowed: Eq. 1 (V = 1) by quadrature exact on the hemisphere;
  * exact_exponential: the SH projection of exp(F~), i.e. what the
    scaling/squaring/linear-approximation scheme stands in for;
  * projected_visibility: the SH projection of the exact product of the
    floored blockers (Eq. 13), the quantity that the log-space scheme's
    exponential variants and the direct product chain of Eq. 12 approximate;
  * rotation_matrix: the SH rotation used for rotation-invariance checks,
    computed as an exact projection integral.
"""
from __future__ import annotations

import math

import torch

from . import sh

DT = torch.float64


def radiance_binary(points, normals, albedo, spheres, light, n_bands, degree=240):
    """B(x) = a int L~(w) prod_i V_i(w, x) max(w . n, 0) dw with the binary
    blocker V_i = 0 on the sphere's cone, 1 elsewhere.  Dense product
    quadrature; the integrand is discontinuous, so accuracy is ~1e-3."""
    d, w = sh.sphere_quadrature(degree)
    Lw = sh.real_sh(d, n_bands) @ light                      # L~ at the nodes
    out = []
    for p, nrm, a in zip(points, normals, albedo):
        vis = torch.ones(d.shape[0], dtype=DT)
        for c in spheres:
            v = c[:3] - p
            dist = torch.linalg.norm(v)
            s = min(float(c[3] / dist), 1.0)
            cos_a = math.sqrt(max(0.0, 1.0 - s * s))
            vis = vis * (d @ (v / dist) < cos_a).to(DT)
        nh = nrm / torch.linalg.norm(nrm)
        cosn = torch.clamp(d @ nh, min=0.0)
        out.append(a * (w * Lw * vis * cosn).sum())
    return torch.stack(out)


def radiance_unshadowed(points_normals, albedo, light, n_bands, n_z=None):
    """B = a int L~(w) max(w . n, 0) dw (Eq. 1, no occluders).  The integrand
    is a polynomial on the hemisphere about n, so a cap rule on [0, 1] in the
    cosine is exact."""
    n_z = n_z or n_bands + 2
    out = []
    for nrm, a in zip(points_normals, albedo):
        nh = nrm / torch.linalg.norm(nrm)
        d, w = sh.cap_quadrature(nh.numpy(), 0.0, 1.0, n_z, 2 * n_bands + 2)
        Lw = sh.real_sh(d, n_bands) @ light
        out.append(a * (w * Lw * (d @ nh)).sum())
    return torch.stack(out)


def exact_exponential(F, n_bands, degree=120):
    """Proj_n[exp(F~)] for F [..., n^2] by a dense product rule (exp(F~) is
    smooth, so the rule converges spectrally)."""
    d, w = sh.sphere_quadrature(degree)
    Y = sh.real_sh(d, n_bands)
    vals = torch.exp(F @ Y.T)
    return (vals * w) @ Y


def projected_visibility(points, spheres, n_bands, eps=3.0, degree=240):
    """Proj_n[prod_i V'_i] for each receiver: the SH projection of the exact
    product of the floored blockers of Eq. 13 (e^-eps on each sphere's cone, 1
    elsewhere), evaluated pointwise in direction space.  This is the visibility
    vector that every variant of step 5 approximates.  The integrand is
    discontinuous, so a dense rule gives about 1e-3."""
    d, w = sh.sphere_quadrature(degree)
    Y = sh.real_sh(d, n_bands)
    floor = math.exp(-eps)
    out = []
    for p in points:
        vis = torch.ones(d.shape[0], dtype=DT)
        for c in spheres:
            v = c[:3] - p
            dist = torch.linalg.norm(v)
            if float(dist) == 0.0:
                continue
            s = min(float(c[3] / dist), 1.0)
            cos_a = math.sqrt(max(0.0, 1.0 - s * s))
            vis = vis * torch.where(d @ (v / dist) >= cos_a, floor, 1.0).to(DT)
        out.append((w * vis) @ Y)
    return torch.stack(out)


def rotation_matrix(R, n_bands):
    """M with (M f)_i = coefficients of w -> f~(R^T w): M_ij = int y_i(w) y_j(R^T w) dw,
    exact by a rule of degree 2 (n - 1)."""
    R = torch.as_tensor(R, dtype=DT)
    d, w = sh.sphere_quadrature(2 * (n_bands - 1))
    Yi = sh.real_sh(d, n_bands)
    Yj = sh.real_sh(d @ R, n_bands)       # rows are (R^T w)^T = w^T R
    return torch.einsum("q,qi,qj->ij", w, Yi, Yj)
