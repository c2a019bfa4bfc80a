"""Rasterisation of the shaded mesh (Sec. 3.4, Eq. 14) and its gradients, as a
plain CPU reference (oracle; test infrastructure only).

The image is I_R = R(B(x_0), ..., B(x_n), P) (Eq. 14): the mesh's vertices are
projected by the 3 x 4 camera matrix P, each pixel centre takes the nearest
triangle that covers it, and the pixel's intensity interpolates the vertices'
radiance B with perspective-correct barycentric weights.  Readings (the paper
names a differentiable rasteriser without fixing it):
  * P maps a homogeneous world point X to (u, v, w); the pixel coordinates are
    (u / w, v / w) and w is the depth.  Pixel (i, j) (column i, row j) has its
    centre at (i + 0.5, j + 0.5);
  * a triangle covers a pixel centre when all three edge functions, divided by
    the triangle's doubled signed area, are >= 0 (edges inclusive, either
    orientation, no culling); triangles with a vertex at w <= 1e-6 or zero
    area are not drawn;
  * the depth at the pixel is 1 / sum_k (lambda_k / w_k); the nearest covering
    triangle wins, ties going to the lower face index;
  * uncovered pixels are 0;
  * gradients flow through the winning triangle's weights (with respect to
    the vertices' radiance and positions); which triangle wins is piecewise
    constant and contributes nothing, as in a hard rasteriser.

The coverage and depth decisions pick integers (the face of each pixel) from
floating-point values, so they are taken here in FP32 with one rounding per
operation, in the order the formulas are written below; the image and the
gradients are computed in FP64 from the FP32 inputs, with autograd.
"""
from __future__ import annotations

import numpy as np
import torch

DT = torch.float64
W_MIN = np.float32(1e-6)


def project_f32(vertices, P):
    """vertices [V, 3] float32, P [3, 4] float32 -> (sx, sy, w) float32, each
    coordinate ((P_r0 x + P_r1 y) + P_r2 z) + P_r3 and then u / w, v / w."""
    x, y, z = (vertices[:, i].astype(np.float32) for i in range(3))
    P = P.astype(np.float32)

    def row(r):
        return ((P[r, 0] * x + P[r, 1] * y) + P[r, 2] * z) + P[r, 3]

    u, v, w = row(0), row(1), row(2)
    with np.errstate(divide="ignore", invalid="ignore"):
        return (u / w).astype(np.float32), (v / w).astype(np.float32), w


def edge_f32(ax, ay, bx, by, px, py):
    """(b - p) x (c - p) style edge function: (ax - px) (by - py) - (bx - px) (ay - py)."""
    return (ax - px) * (by - py) - (bx - px) * (ay - py)


def rasterize_ids(vertices, faces, P, width, height):
    """Face index per pixel ([H, W] int32, -1 where nothing covers the centre):
    the FP32 coverage and depth decisions described above."""
    sx, sy, w = project_f32(vertices, P)
    H, W = height, width
    best_z = np.full((H, W), np.inf, np.float32)
    best_f = np.full((H, W), -1, np.int32)
    for f, (a, b, c) in enumerate(faces):
        if not (w[a] > W_MIN and w[b] > W_MIN and w[c] > W_MIN):
            continue
        x0, y0, x1, y1, x2, y2 = sx[a], sy[a], sx[b], sy[b], sx[c], sy[c]
        area = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
        if not (area != 0) or not np.isfinite(area):
            continue
        i0 = max(int(np.floor(min(x0, x1, x2) - 0.5)), 0)
        i1 = min(int(np.ceil(max(x0, x1, x2) - 0.5)), W - 1)
        j0 = max(int(np.floor(min(y0, y1, y2) - 0.5)), 0)
        j1 = min(int(np.ceil(max(y0, y1, y2) - 0.5)), H - 1)
        if i0 > i1 or j0 > j1:
            continue
        px = (np.arange(i0, i1 + 1, dtype=np.float32) + np.float32(0.5))[None, :]
        py = (np.arange(j0, j1 + 1, dtype=np.float32) + np.float32(0.5))[:, None]
        l0 = edge_f32(x1, y1, x2, y2, px, py) / area
        l1 = edge_f32(x2, y2, x0, y0, px, py) / area
        l2 = edge_f32(x0, y0, x1, y1, px, py) / area
        inside = (l0 >= 0) & (l1 >= 0) & (l2 >= 0)
        z = np.float32(1.0) / ((l0 / w[a] + l1 / w[b]) + l2 / w[c])
        blk_z = best_z[j0:j1 + 1, i0:i1 + 1]
        blk_f = best_f[j0:j1 + 1, i0:i1 + 1]
        win = inside & (z < blk_z)          # faces in increasing index: ties keep the lower
        blk_z[win] = z[win]
        blk_f[win] = f
    return best_f


def shade_pixels(vertices, faces, radiance, P, face_id):
    """The image (Eq. 14) from a face index map: I = sum_k b_k B_k with the
    perspective-correct weights b_k = (lambda_k / w_k) / sum_j (lambda_j / w_j)
    of the pixel centre, in the precision of the tensors given (FP64 tensors
    with requires_grad give the gradients by autograd)."""
    H, W = face_id.shape
    Pm = P if torch.is_tensor(P) else torch.as_tensor(P, dtype=vertices.dtype)
    hom = torch.cat([vertices, torch.ones_like(vertices[:, :1])], 1) @ Pm.T   # [V, 3]
    w = hom[:, 2]
    sx, sy = hom[:, 0] / w, hom[:, 1] / w
    js, is_ = np.nonzero(face_id >= 0)
    img = torch.zeros(H * W, dtype=vertices.dtype)
    if len(js) == 0:
        return img.reshape(H, W)
    f = torch.as_tensor(faces[face_id[js, is_]].astype(np.int64))
    px = torch.as_tensor(is_, dtype=vertices.dtype) + 0.5
    py = torch.as_tensor(js, dtype=vertices.dtype) + 0.5
    X = [sx[f[:, k]] for k in range(3)]
    Y = [sy[f[:, k]] for k in range(3)]
    area = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0])
    lam = [((X[1] - px) * (Y[2] - py) - (X[2] - px) * (Y[1] - py)) / area,
           ((X[2] - px) * (Y[0] - py) - (X[0] - px) * (Y[2] - py)) / area,
           ((X[0] - px) * (Y[1] - py) - (X[1] - px) * (Y[0] - py)) / area]
    q = [lam[k] / w[f[:, k]] for k in range(3)]
    Q = q[0] + q[1] + q[2]
    val = sum(q[k] / Q * radiance[f[:, k]] for k in range(3))
    idx = torch.as_tensor(js * W + is_)
    img = img.index_put((idx,), val)
    return img.reshape(H, W)


def render(vertices, faces, radiance, P, width, height):
    """Forward: (face_id [H, W] int32, image [H, W] FP64) from FP32 arrays."""
    fid = rasterize_ids(np.asarray(vertices, np.float32), faces, np.asarray(P, np.float32), width, height)
    img = shade_pixels(torch.as_tensor(np.asarray(vertices, np.float32)).to(DT), faces,
                       torch.as_tensor(np.asarray(radiance, np.float32)).to(DT),
                       torch.as_tensor(np.asarray(P, np.float32)).to(DT), fid)
    return fid, img


def render_backward(vertices, faces, radiance, P, face_id, grad_image):
    """Gradients of sum(grad_image * I) with respect to the vertices' radiance
    [V] and positions [V, 3], for the given face index map (FP64)."""
    v = torch.as_tensor(np.asarray(vertices, np.float32)).to(DT).requires_grad_(True)
    B = torch.as_tensor(np.asarray(radiance, np.float32)).to(DT).requires_grad_(True)
    img = shade_pixels(v, faces, B, torch.as_tensor(np.asarray(P, np.float32)).to(DT), face_id)
    loss = (img * torch.as_tensor(np.asarray(grad_image, np.float32)).to(DT)).sum()
    gv, gB = torch.autograd.grad(loss, [v, B], allow_unused=True)
    gv = torch.zeros_like(v) if gv is None else gv
    gB = torch.zeros_like(B) if gB is None else gB
    return gB.detach(), gv.detach()
