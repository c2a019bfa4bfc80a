"""Scene parameterisation upstream of the spheres, in FP64 (oracle; test
infrastructure only).

Sec. 3.3.1 drives the geometry by the spheres: their centres are the nodes of
an embedded deformation graph (Sumner et al. 2007), each sphere attached to
its K nearest template vertices, and the deformation is parameterised by a
rotation and a translation per sphere.  Sec. 3.5 adds a global rigid pose of
the object and optimises all of it by gradient descent on the rendering loss
(step 1e-2, 200-1000 iterations).

Readings where the paper is silent (each is listed in the design notes):
  * rotations are axis-angle vectors a (rotation by |a| about a / |a|),
    turned into matrices by Rodrigues' formula;
  * attachment: sphere k is attached to the K template vertices nearest to
    its centre g_k (squared Euclidean distance, ties to the lower vertex
    index); vertex j is driven by the spheres attached to it;
  * weights follow Sumner et al.: u_jk = (1 - |v_j - g_k| / d_k)^2 with d_k
    the distance from g_k to its (K+1)-th nearest vertex (its K-th when
    K = P), normalised over the spheres attached to vertex j; a vertex with
    no attached sphere, or whose raw weights are all zero, keeps its template
    position and normal before the global pose;
  * deformed vertex  x_j = R_0 y_j + t_0,
      y_j = sum_k w_jk (R_k (v_j - g_k) + g_k + t_k) + (1 - sum_k w_jk) v_j;
    deformed normal  n_j = R_0 (sum_k w_jk R_k m_j + (1 - sum_k w_jk) m_j)
    (not renormalised: the shading normalises normals itself);
    deformed sphere  c_k = R_0 (g_k + t_k) + t_0 with the template radius.
Gradients come from torch autograd.
"""
from __future__ import annotations

import numpy as np
import torch

DT = torch.float64


def skew(a: torch.Tensor) -> torch.Tensor:
    """[..., 3] -> [..., 3, 3] with skew(a) b = a x b."""
    z = torch.zeros_like(a[..., 0])
    return torch.stack([torch.stack([z, -a[..., 2], a[..., 1]], -1),
                        torch.stack([a[..., 2], z, -a[..., 0]], -1),
                        torch.stack([-a[..., 1], a[..., 0], z], -1)], -2)


def rodrigues(a: torch.Tensor) -> torch.Tensor:
    """Rotation matrices R = I + (sin t / t) K + ((1 - cos t) / t^2) K^2,
    K = skew(a), t = |a|; below t = 1e-3 the two coefficients take their
    Taylor series (exact to FP64 there).  a [..., 3] -> [..., 3, 3]."""
    t2 = (a * a).sum(-1)
    small = t2 < 1e-6
    t2s = torch.where(small, torch.ones_like(t2), t2)
    t = torch.sqrt(t2s)
    A = torch.where(small, 1.0 - t2 / 6.0 + t2 * t2 / 120.0, torch.sin(t) / t)
    B = torch.where(small, 0.5 - t2 / 24.0 + t2 * t2 / 720.0, (1.0 - torch.cos(t)) / t2s)
    K = skew(a)
    eye = torch.eye(3, dtype=a.dtype).expand(K.shape)
    return eye + A[..., None, None] * K + B[..., None, None] * (K @ K)


def attach(vertices: np.ndarray, centres: np.ndarray, K: int):
    """Brute-force attachment: for every sphere its K nearest vertices (by
    squared distance dx*dx + dy*dy + dz*dz in FP64 from the FP32 inputs, ties
    to the lower index) and the raw weights u_jk.
    vertices [P, 3], centres [S, 3] -> (idx [S, K] int64, u [S, K] float64)."""
    v = np.asarray(vertices, np.float64)
    g = np.asarray(centres, np.float64)
    P = v.shape[0]
    idx = np.zeros((g.shape[0], K), np.int64)
    u = np.zeros((g.shape[0], K))
    for k in range(g.shape[0]):
        dx = v[:, 0] - g[k, 0]
        dy = v[:, 1] - g[k, 1]
        dz = v[:, 2] - g[k, 2]
        d2 = dx * dx + dy * dy + dz * dz
        order = np.lexsort((np.arange(P), d2))        # by distance, then by index
        idx[k] = order[:K]
        dmax = np.sqrt(d2[order[K]] if K < P else d2[order[K - 1]])
        d = np.sqrt(d2[order[:K]])
        u[k] = (1.0 - d / dmax) ** 2 if dmax > 0 else 0.0
    return idx, u


def normalised_weights(idx: np.ndarray, u: np.ndarray, P: int):
    """w_jk = u_jk / sum over the spheres attached to j (0 where that sum is
    0).  Returns w [S, K] float64."""
    tot = np.zeros(P)
    np.add.at(tot, idx.ravel(), u.ravel())
    den = tot[idx]
    return np.where(den > 0, u / np.where(den > 0, den, 1.0), 0.0)


def deform(params: torch.Tensor, vertices: torch.Tensor, normals: torch.Tensor, spheres: torch.Tensor,
           idx: torch.Tensor, w: torch.Tensor):
    """params [S + 1, 6]: rows k < S are (a_k, t_k) of sphere k, row S the
    global pose (a_0, t_0).  vertices, normals [P, 3]; spheres [S, 4];
    idx [S, K] attached vertices, w [S, K] normalised weights.
    Returns (points [P, 3], normals [P, 3], spheres [S, 4])."""
    S = spheres.shape[0]
    R = rodrigues(params[:, :3])                 # [S + 1, 3, 3]
    Rk, R0 = R[:S], R[S]
    tk, t0 = params[:S, 3:], params[S, 3:]
    g = spheres[:, :3]
    P = vertices.shape[0]
    vj = vertices[idx]                           # [S, K, 3]
    mj = normals[idx]
    local = torch.einsum("skab,skb->ska", Rk[:, None].expand(-1, idx.shape[1], -1, -1).contiguous(),
                         vj - g[:, None]) + g[:, None] + tk[:, None]
    nloc = torch.einsum("skab,skb->ska", Rk[:, None].expand(-1, idx.shape[1], -1, -1).contiguous(), mj)
    wsum = torch.zeros(P, dtype=vertices.dtype).index_add(0, idx.reshape(-1), w.reshape(-1))
    y = (1.0 - wsum)[:, None] * vertices
    y = y.index_add(0, idx.reshape(-1), (w[..., None] * local).reshape(-1, 3))
    z = (1.0 - wsum)[:, None] * normals
    z = z.index_add(0, idx.reshape(-1), (w[..., None] * nloc).reshape(-1, 3))
    x = y @ R0.T + t0
    n = z @ R0.T
    c = (g + tk) @ R0.T + t0
    return x, n, torch.cat([c, spheres[:, 3:]], dim=1)


def render_loss(params, scene, idx, w, target, n_bands: int, eps: float = 3.0, n_squarings: int = 4):
    """The inverse problem of Sec. 3.5 on receivers instead of an image:
    L(theta) = mean_j (B_j(theta) - target_j)^2, with B the shading of
    method.forward at the deformed points, normals and spheres (albedo and
    light from ``scene``).  Returns (loss, d loss / d params) in FP64."""
    from . import method
    v, m, s = (torch.as_tensor(scene[k]).to(DT) for k in ("points", "normals", "spheres"))
    p = torch.as_tensor(params).to(DT).clone().requires_grad_(True)
    x, n, c = deform(p, v, m, s, torch.as_tensor(idx), torch.as_tensor(w).to(DT))
    out = method.forward(x, n, torch.as_tensor(scene["albedo"]).to(DT), c, torch.as_tensor(scene["light"]).to(DT),
                         n_bands, eps, n_squarings)
    r = out["B"] - torch.as_tensor(target).to(DT)
    loss = (r * r).mean()
    return loss.detach(), torch.autograd.grad(loss, p)[0]


def image_loss(params, scene, idx, w, target_image, n_bands: int, eps: float = 3.0, n_squarings: int = 4,
               raster_positions: bool = True, face_id=None):
    """The inverse problem of Sec. 3.5 on the image (Eqs. 14-16): the
    deformed mesh's vertex radiance (method.forward) is rasterised
    (raster.render's rules; ``scene`` holds faces, camera, width, height) and
    L(theta) = mean over pixels of (I_R - target)^2.  The face of each pixel
    is decided from the deformed vertices rounded to FP32, or taken from
    ``face_id`` when given (the map held fixed, which makes the loss smooth in
    the parameters).  With ``raster_positions`` False the rasteriser's
    dependence on the vertex positions is cut (gradients through the radiance
    only).  Returns (loss, d loss / d params, face ids) in FP64."""
    import numpy as np

    from . import method, raster
    v, m, s = (torch.as_tensor(scene[k]).to(DT) for k in ("points", "normals", "spheres"))
    p = torch.as_tensor(params).to(DT).clone().requires_grad_(True)
    x, n, c = deform(p, v, m, s, torch.as_tensor(idx), torch.as_tensor(w).to(DT))
    B = method.forward(x, n, torch.as_tensor(scene["albedo"]).to(DT), c, torch.as_tensor(scene["light"]).to(DT),
                       n_bands, eps, n_squarings)["B"]
    cam = np.asarray(scene["camera"], np.float32)
    fid = face_id if face_id is not None else raster.rasterize_ids(
        x.detach().numpy().astype(np.float32), scene["faces"], cam, scene["width"], scene["height"])
    xr = x if raster_positions else x.detach()
    img = raster.shade_pixels(xr, scene["faces"], B, torch.as_tensor(cam).to(DT), fid)
    r = img - torch.as_tensor(target_image).to(DT)
    loss = (r * r).mean()
    return loss.detach(), torch.autograd.grad(loss, p)[0], fid
