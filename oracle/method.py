"""The shadow method, step by step, in FP64 (oracle; test infrastructure).

Steps, in the paper's order (Sec. 3.3.2 and Sec. 3.2):
  1. pair geometry: for receiver x and sphere (c, r) the sphere blocks the
     cone of directions around s = (c - x)/|c - x| with half-angle
     alpha = asin(r/|c - x|); t = cos(alpha)            (blocker function)
  2. log-cap zonal coefficients: log V'_i equals -eps inside the cap and 0
     outside (Eq. 13, eps = 3); its projection about the z axis is analytic
     in distance and radius
  3. rotation of that zonal vector to s (the SH rotation of Eq. 11 applied
     to a zonal function)
  4. sum over spheres: F = sum_i f_i (the log turns the product of Eq. 12
     into a sum)
  5. SH exponential of F by scaling, squaring and an optimal linear
     approximation (the Ren et al. setting the paper adopts)
  6. clamped-cosine transfer H(x) = rotated z-aligned max(w_z, 0) (Eqs. 10-11)
  7. shading B = a (L . (V * H)) (Eq. 8)
Gradients of B with respect to every input come from torch autograd.

Readings where the paper is silent (each is listed in the design notes):
  * steps 2-3 use the Funk-Hecke theorem: a function h(w . s) has SH
    coefficients lambda_l y_lm(s) with lambda_l = 2 pi int_-1^1 h(x) P_l(x) dx,
    which is exactly "project about z, then rotate to s";
  * step 5: the DC term is split off exactly (exp(c) with c = F_0/sqrt(4 pi)),
    the rest is scaled by 2^-k, approximated by a + b G with
    a = b = exp(|G|^2 / (8 pi)) (the least-squares line through exp(g) when
    g's values over the sphere are Gaussian with variance |G|^2 / (4 pi)),
    then squared k times with the truncated triple product; k is fixed per
    call (default 4).  The paper's own fitted OL tables are not available, so
    agreement with its exponential is parity unpinned; this closed form is
    pinned by the exact cases and the least-squares and second-order tests;
  * a receiver inside a sphere (r >= d) sees a hemisphere cap (t = 0); a
    sphere centred on the receiver (d = 0) contributes nothing;
  * normals are normalised before use; no clamping of V or B anywhere.
"""
from __future__ import annotations

import math

import torch

from . import sh

DT = torch.float64
SQRT_4PI = math.sqrt(4.0 * math.pi)


def _t(a):
    return torch.as_tensor(a).to(DT)


# ---------------------------------------------------------------- step 1

def pair_geometry(points: torch.Tensor, spheres: torch.Tensor):
    """points [P, 3], spheres [S, 4] -> (s_hat [P, S, 3], t [P, S], live [P, S]).

    s_hat is the unit direction from the receiver to the sphere centre,
    t = cos(alpha) = sqrt(1 - (r/d)^2) (0 when the receiver is inside)."""
    v = spheres[None, :, :3] - points[:, None, :]
    d2 = (v * v).sum(-1)
    live = d2 > 0
    d = torch.sqrt(torch.where(live, d2, torch.ones_like(d2)))
    s_hat = v / d[..., None]
    s = spheres[None, :, 3] / d
    u = 1.0 - s * s
    inside = u <= 0
    t = torch.where(inside, torch.zeros_like(u), torch.sqrt(torch.where(inside, torch.ones_like(u), u)))
    return s_hat, t, live


# ---------------------------------------------------------------- step 2

def log_cap_zonal(t: torch.Tensor, n_bands: int, eps: float) -> torch.Tensor:
    """Funk-Hecke eigenvalues of log V' = -eps on {w . s >= t}:
    g_l(t) = -eps * 2 pi * int_t^1 P_l(x) dx, l < n  -> [..., n]."""
    return torch.stack([-eps * sh.funk_hecke_cap(t, l) for l in range(n_bands)], dim=-1)


def band_of_index(n_bands: int):
    return torch.tensor([int(math.isqrt(i)) for i in range(n_bands * n_bands)])


# ---------------------------------------------------------------- steps 3-4

def log_visibility(points, spheres, n_bands: int, eps: float) -> torch.Tensor:
    """F(x) = sum over spheres of g_l(t) y_lm(s_hat)  -> [P, n^2]."""
    if spheres.shape[0] == 0:
        return points.new_zeros(points.shape[0], n_bands * n_bands)
    s_hat, t, live = pair_geometry(points, spheres)
    g = log_cap_zonal(t, n_bands, eps)                       # [P, S, n]
    Y = sh.real_sh(s_hat, n_bands)                            # [P, S, n^2]
    f = g[..., band_of_index(n_bands)] * Y                    # rotate (step 3)
    f = torch.where(live[..., None], f, torch.zeros_like(f))
    return f.sum(dim=1)                                       # sum (step 4)


# ---------------------------------------------------------------- step 5

def sh_exponential(F: torch.Tensor, C: torch.Tensor, n_squarings: int):
    """V = exp*(F) by DC isolation, scaling, optimal linear approximation and
    truncated squaring.  Returns (V, c, [E_0, ..., E_k])."""
    N = F.shape[-1]
    e0 = torch.zeros(N, dtype=F.dtype)
    e0[0] = 1.0
    c = F[..., 0] / SQRT_4PI                       # constant value of the DC part
    G = torch.cat([torch.zeros_like(F[..., :1]), F[..., 1:]], dim=-1) * (2.0 ** -n_squarings)
    a = torch.exp((G * G).sum(-1) / (8.0 * math.pi))
    E = a[..., None] * (SQRT_4PI * e0 + G)          # a * 1 + b * G with a = b
    Es = [E]
    for _ in range(n_squarings):
        E = sh.triple_product(E, E, C)
        Es.append(E)
    V = torch.exp(c)[..., None] * E
    return V, c, Es


def sh_exponential_taylor(F: torch.Tensor, C: torch.Tensor, order: int, n_squarings: int):
    """The scaling-and-squaring exponential with the linear approximation
    replaced by the Taylor series of exp truncated after the term of degree
    ``order`` (K): E_0 = sum_{j <= K} G^{*j} / j!, each power the truncated
    product of the previous one with G (G^{*0} the constant 1), then the same
    k truncated squarings.  The DC term is split off exactly and the rest is
    scaled by 2^-k, as in sh_exponential; K = 1 is the linear approximation
    with a = b = 1."""
    N = F.shape[-1]
    c = F[..., 0] / SQRT_4PI
    G = torch.cat([torch.zeros_like(F[..., :1]), F[..., 1:]], dim=-1) * (2.0 ** -n_squarings)
    one = torch.zeros(N, dtype=F.dtype)
    one[0] = SQRT_4PI
    E = one.expand_as(F).clone()
    power = None
    for j in range(1, order + 1):
        power = G if j == 1 else sh.triple_product(power, G, C)
        E = E + power / math.factorial(j)
    for _ in range(n_squarings):
        E = sh.triple_product(E, E, C)
    return torch.exp(c)[..., None] * E


def sh_exponential_quadrature(F: torch.Tensor, n_bands: int, degree: int | None = None):
    """The exponential as the projection Proj_n[exp(F~)] of the pointwise
    exponential (the function-space quantity the scaling and squaring scheme
    stands in for), taken with the product rule of degree 8n - 1 (4n
    Gauss-Legendre nodes in z times 8n azimuths).  The DC term is split off
    exactly as in sh_exponential: V = exp(c) sum_q w_q exp(F^~(w_q)) y(w_q)
    with c = F_0 / sqrt(4 pi) and F^ = F without its DC coefficient."""
    degree = 8 * n_bands - 1 if degree is None else degree
    d, w = sh.sphere_quadrature(degree)
    Y = sh.real_sh(d, n_bands).to(F.dtype)
    c = F[..., 0] / SQRT_4PI
    Fh = torch.cat([torch.zeros_like(F[..., :1]), F[..., 1:]], dim=-1)
    V = torch.exp(c)[..., None] * ((torch.exp(Fh @ Y.T) * w.to(F.dtype)) @ Y)
    return V


def projected_blocker(points, spheres, n_bands: int, eps: float) -> torch.Tensor:
    """SH vectors of the floored blocker functions V'_i (Eq. 13: e^-eps inside
    the sphere's cone, 1 elsewhere), one per (receiver, sphere) -> [P, S, n^2].

    V'_i = 1 - (1 - e^-eps) 1[w . s >= t]; by Funk-Hecke its coefficients
    about s are (4 pi delta_l0 - (1 - e^-eps) 2 pi int_t^1 P_l) y_lm(s), the
    constant 1 having coefficient sqrt(4 pi) on y_00.  A sphere centred on the
    receiver blocks nothing (the constant 1)."""
    s_hat, t, live = pair_geometry(points, spheres)
    beta = -math.expm1(-eps)
    lam = torch.stack([(4.0 * math.pi if l == 0 else 0.0) - beta * sh.funk_hecke_cap(t, l)
                       for l in range(n_bands)], dim=-1)              # [P, S, n]
    b = lam[..., band_of_index(n_bands)] * sh.real_sh(s_hat, n_bands)
    one = torch.zeros(n_bands * n_bands, dtype=points.dtype)
    one[0] = SQRT_4PI
    return torch.where(live[..., None], b, one)


def sh_direct_product(points, spheres, n_bands: int, eps: float, C: torch.Tensor) -> torch.Tensor:
    """V = V'_1 * V'_2 * ... * V'_S (Eq. 12): the chain of truncated SH
    products (Eqs. 6-7) of the projected blockers, taken left to right in
    sphere order (truncated products are commutative but not associative, so
    the order is part of the definition).  The chain starts from the constant
    1, so no spheres give V = 1.  The blockers are the floored ones of Eq. 13,
    the same functions whose logarithms the log-space scheme sums; a large eps
    (e^-eps below FP32 resolution) gives Eq. 12's binary blockers."""
    P = points.shape[0]
    V = torch.zeros(P, n_bands * n_bands, dtype=points.dtype)
    V[:, 0] = SQRT_4PI
    if spheres.shape[0] == 0:
        return V
    b = projected_blocker(points, spheres, n_bands, eps)
    for i in range(spheres.shape[0]):
        V = sh.triple_product(V, b[:, i], C)
    return V


# ---------------------------------------------------------------- step 6

def transfer(normals: torch.Tensor, n_bands: int) -> torch.Tensor:
    """H(x)_lm = A_l y_lm(n / |n|), A_l the clamped-cosine Funk-Hecke
    eigenvalues (Eqs. 10-11)  -> [P, n^2]."""
    nh = normals / torch.linalg.norm(normals, dim=-1, keepdim=True)
    A = torch.tensor([sh.clamped_cosine_coeff(l) for l in range(n_bands)], dtype=normals.dtype)
    return A[band_of_index(n_bands)] * sh.real_sh(nh, n_bands)


# ---------------------------------------------------------------- step 7

def shade(V, H, albedo, light, C):
    """B = a * (L . (V * H)) (Eq. 8)."""
    return albedo * (light * sh.triple_product(V, H, C)).sum(-1)


def shade_channels(V, H, albedo, light, C):
    """Several colour channels sharing one visibility: B_c = a_c (L_c . (V * H))
    per channel (Eq. 8 for each channel; albedo [P, Ch], light [Ch, N] ->
    [P, Ch])."""
    T = sh.triple_product(V, H, C)                              # [P, N]
    return albedo * (T @ light.T)


# ---------------------------------------------------------------- pipeline

def forward(points, normals, albedo, spheres, light, n_bands: int, eps: float = 3.0,
            n_squarings: int = 4, keep=False, exp_mode: str = "squaring"):
    """Whole forward path on one chunk of receivers (FP64 tensors; FP32
    tensors give the oracle's FP32 twin, used only to measure how much error
    FP32 arithmetic alone introduces).  ``exp_mode`` "quadrature" takes the
    exponential by sh_exponential_quadrature instead; "taylorK" (K = 1..8) by
    sh_exponential_taylor of order K; "product" forms V by the direct product
    chain of Eq. 12 (sh_direct_product) instead of the log-space scheme."""
    C = sh.gaunt_tensor(n_bands).to(points.dtype)
    F = log_visibility(points, spheres, n_bands, eps)
    if exp_mode == "quadrature":
        V, c, Es = sh_exponential_quadrature(F, n_bands), F[..., 0] / SQRT_4PI, []
    elif exp_mode == "product":
        V, c, Es = sh_direct_product(points, spheres, n_bands, eps, C), F[..., 0] / SQRT_4PI, []
    elif exp_mode.startswith("taylor"):
        V, c, Es = sh_exponential_taylor(F, C, int(exp_mode[6:]), n_squarings), F[..., 0] / SQRT_4PI, []
    else:
        V, c, Es = sh_exponential(F, C, n_squarings)
    H = transfer(normals, n_bands)
    B = shade(V, H, albedo, light, C)
    out = dict(F=F, V=V, B=B, H=H, c=c)
    if keep:
        out["E"] = Es
    return out


def scene_tensors(scene, dtype=DT):
    """FP32 scene arrays -> FP64 tensors (bit-identical inputs)."""
    return {k: torch.as_tensor(scene[k]).to(dtype) for k in ("points", "normals", "albedo", "spheres", "light")}


def run_forward(scene, eps=3.0, n_squarings=4, chunk=1024, idx=None, dtype=DT, exp_mode="squaring"):
    """Forward over a scene (optionally a subset of receivers), chunked."""
    T = scene_tensors(scene, dtype)
    n = int(scene["n_bands"])
    P = T["points"].shape[0]
    sel = torch.arange(P) if idx is None else torch.as_tensor(idx)
    outs = {"F": [], "V": [], "B": []}
    with torch.no_grad():
        for s in range(0, len(sel), chunk):
            j = sel[s:s + chunk]
            o = forward(T["points"][j], T["normals"][j], T["albedo"][j], T["spheres"],
                        T["light"], n, eps, n_squarings, exp_mode=exp_mode)
            for k in outs:
                outs[k].append(o[k])
    N = n * n
    return {k: (torch.cat(v) if v else torch.zeros((0, N) if k != "B" else (0,), dtype=dtype))
            for k, v in outs.items()}


def run_forward_backward(scene, grad_B, eps=3.0, n_squarings=4, chunk=512, idx=None, dtype=DT,
                         exp_mode="squaring"):
    """Forward plus gradients of sum_p grad_B[p] * B[p].

    ``idx`` restricts the receivers to a subset (grad_B then has that
    subset's length); sphere and light gradients are the sums over that
    subset only.  Returns numpy-free FP64 tensors:
    B [P'], V [P', N], grad_points [P', 3], grad_normals [P', 3],
    grad_albedo [P'], grad_spheres [S, 4], grad_light [N]."""
    T = scene_tensors(scene, dtype)
    n = int(scene["n_bands"])
    P = T["points"].shape[0]
    sel = torch.arange(P) if idx is None else torch.as_tensor(idx)
    gB = torch.as_tensor(grad_B).to(dtype)
    spheres = T["spheres"].clone().requires_grad_(True)
    light = T["light"].clone().requires_grad_(True)
    gs = torch.zeros_like(spheres)
    gl = torch.zeros_like(light)
    res = {k: [] for k in ("B", "V", "grad_points", "grad_normals", "grad_albedo")}
    for s in range(0, len(sel), chunk):
        j = sel[s:s + chunk]
        p = T["points"][j].clone().requires_grad_(True)
        nrm = T["normals"][j].clone().requires_grad_(True)
        a = T["albedo"][j].clone().requires_grad_(True)
        o = forward(p, nrm, a, spheres, light, n, eps, n_squarings, exp_mode=exp_mode)
        loss = (o["B"] * gB[s:s + chunk]).sum()
        ins = [p, nrm, a, spheres, light]
        g = torch.autograd.grad(loss, ins, allow_unused=True)
        g = [torch.zeros_like(x) if gx is None else gx for gx, x in zip(g, ins)]  # unused: zero
        res["B"].append(o["B"].detach())
        res["V"].append(o["V"].detach())
        res["grad_points"].append(g[0])
        res["grad_normals"].append(g[1])
        res["grad_albedo"].append(g[2])
        gs += g[3]
        gl += g[4]
    out = {k: torch.cat(v) for k, v in res.items()}
    out["grad_spheres"] = gs
    out["grad_light"] = gl
    return out


def run_forward_backward_channels(scene, albedo, light, grad_B, eps=3.0, n_squarings=4, chunk=512, idx=None,
                                  dtype=DT):
    """Colour channels sharing one visibility (Eq. 8 per channel):
    albedo [P, Ch], light [Ch, N], grad_B [P', Ch] the cotangent of the
    radiance [P', Ch] on receivers ``idx`` (all when None).  Returns B,
    grad_points, grad_normals, grad_albedo [P', Ch] (or [P', 3]),
    grad_spheres [S, 4] and grad_light [Ch, N], the last two summed over the
    selected receivers."""
    T = scene_tensors(scene, dtype)
    n = int(scene["n_bands"])
    C = sh.gaunt_tensor(n).to(dtype)
    P = T["points"].shape[0]
    sel = torch.arange(P) if idx is None else torch.as_tensor(idx)
    alb_all = torch.as_tensor(albedo).to(dtype)
    gB = torch.as_tensor(grad_B).to(dtype)
    spheres = T["spheres"].clone().requires_grad_(True)
    lights = torch.as_tensor(light).to(dtype).clone().requires_grad_(True)
    gs = torch.zeros_like(spheres)
    gl = torch.zeros_like(lights)
    res = {k: [] for k in ("B", "grad_points", "grad_normals", "grad_albedo")}
    for s in range(0, len(sel), chunk):
        j = sel[s:s + chunk]
        p = T["points"][j].clone().requires_grad_(True)
        nrm = T["normals"][j].clone().requires_grad_(True)
        a = alb_all[j].clone().requires_grad_(True)
        F = log_visibility(p, spheres, n, eps)
        V, _, _ = sh_exponential(F, C, n_squarings)
        B = shade_channels(V, transfer(nrm, n), a, lights, C)
        ins = [p, nrm, a, spheres, lights]
        g = torch.autograd.grad((B * gB[s:s + chunk]).sum(), ins, allow_unused=True)
        g = [torch.zeros_like(x) if gx is None else gx for gx, x in zip(g, ins)]
        res["B"].append(B.detach())
        res["grad_points"].append(g[0])
        res["grad_normals"].append(g[1])
        res["grad_albedo"].append(g[2])
        gs += g[3]
        gl += g[4]
    out = {k: torch.cat(v) for k, v in res.items()}
    out["grad_spheres"] = gs
    out["grad_light"] = gl
    return out
