"""Scene parameterisation upstream of the spheres and the inverse problem
(Sec. 3.3.1, Sec. 3.5), over the HIP library.

``DeformGraph`` attaches every sphere of a template scene to its K nearest
template vertices (``shv_deform_graph_build``, once, on the host) and keeps
the template and the attachment in device memory.  ``deform_scene`` is the
differentiable deformation (``sh_deform_forward`` / ``sh_deform_backward``).
``InverseProblem`` runs the paper's optimisation, gradient descent on the
squared difference between the rendered receiver radiance and a target, with
every step in the library: deformation, visibility and shading, the loss and
its cotangent, their adjoints and the parameter update.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from .ops import _stream, ensure_init

RENDER_PARAMS = dict(eps=3.0, n_squarings=4)


class DeformGraph:
    """Template vertices [P, 3], normals [P, 3] and spheres [S, 4] (host or
    device tensors / arrays) with each sphere attached to its K nearest
    vertices.  Row k < S of a parameter tensor [S + 1, 6] is sphere k's
    (axis-angle, translation), row S the global pose."""

    def __init__(self, vertices, normals, spheres, K: int, device=None):
        device = torch.device(device) if device is not None else torch.device("cuda", 0)
        ensure_init(device)
        v = np.ascontiguousarray(np.asarray(torch.as_tensor(vertices).cpu(), np.float32).T)
        m = np.ascontiguousarray(np.asarray(torch.as_tensor(normals).cpu(), np.float32).T)
        s = np.ascontiguousarray(np.asarray(torch.as_tensor(spheres).cpu(), np.float32).reshape(-1, 4))
        P, S = v.shape[1], s.shape[0]
        self.P, self.S, self.K = P, S, int(K)
        vert_ptr = np.zeros(P + 1, np.int32)
        vert_sph = np.zeros(S * K, np.int32)
        vert_w = np.zeros(S * K, np.float32)
        sph_vert = np.zeros(S * K, np.int32)
        sph_w = np.zeros(S * K, np.float32)
        _lib.shv_deform_graph_build(v, P, s, S, K, vert_ptr, vert_sph, vert_w, sph_vert, sph_w)
        self.host = dict(vert_ptr=vert_ptr, vert_sph=vert_sph, vert_w=vert_w, sph_vert=sph_vert, sph_w=sph_w)
        dev = lambda a: torch.from_numpy(a).to(device)  # noqa: E731
        self.dev = dict(vertices=dev(v), normals=dev(m), spheres=dev(s), **{k: dev(a) for k, a in self.host.items()})
        d = self.dev
        self.c = _lib.shv_deform_graph(d["vertices"].data_ptr(), d["normals"].data_ptr(), d["spheres"].data_ptr(),
                                       d["vert_ptr"].data_ptr(), d["vert_sph"].data_ptr(), d["vert_w"].data_ptr(),
                                       d["sph_vert"].data_ptr(), d["sph_w"].data_ptr(), P, S, self.K)
        self.device = device
        self.ws = torch.empty(_lib.shv_deform_workspace_bytes(P, S), dtype=torch.uint8, device=device)

    def forward(self, params):
        """params [S + 1, 6] (device, float32) -> points [3][P], normals
        [3][P], spheres [S][4]."""
        P, S, dev = self.P, self.S, self.device
        pts = torch.empty(3, P, device=dev)
        nrm = torch.empty(3, P, device=dev)
        sph = torch.empty(S, 4, device=dev)
        _lib.sh_deform_forward(self.c, params, pts, nrm, sph, self.ws, self.ws.numel(), _stream())
        return pts, nrm, sph

    def backward(self, params, grad_points=None, grad_normals=None, grad_spheres=None):
        """Cotangents in the layouts of ``forward`` (any may be None) ->
        grad params [S + 1, 6]."""
        gp = torch.empty(self.S + 1, 6, device=self.device)
        _lib.sh_deform_backward(self.c, params, grad_points, grad_normals, grad_spheres, gp, self.ws,
                                self.ws.numel(), _stream())
        return gp


class DeformScene(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, graph):
        p = params.detach().to(torch.float32).contiguous()
        pts, nrm, sph = graph.forward(p)
        ctx.graph = graph
        ctx.save_for_backward(p)
        return pts.t(), nrm.t(), sph

    @staticmethod
    def backward(ctx, gx, gn, gs):
        (p,) = ctx.saved_tensors
        soa = lambda g: None if g is None else g.detach().to(torch.float32).t().contiguous()  # noqa: E731
        gs = None if gs is None else gs.detach().to(torch.float32).contiguous()
        return ctx.graph.backward(p, soa(gx), soa(gn), gs), None


def deform_scene(params, graph: DeformGraph):
    """Differentiable deformation: params [S + 1, 6] -> (points [P, 3],
    normals [P, 3], spheres [S, 4]) ready for ``shade_sh``."""
    return DeformScene.apply(params, graph)


class InverseProblem:
    """Gradient descent on L(theta) = mean_j (B_j(theta) - target_j)^2 with B
    the rendered radiance of the deformed scene (Sec. 3.5; the paper's step is
    1e-2).  ``albedo`` [P], ``light`` [n_bands^2] and ``target`` [P] are fixed;
    ``params`` [S + 1, 6] starts at ``init`` (zeros: the template).

    With ``faces`` [T, 3] (the template's triangles over its P vertices) and
    ``camera`` = (P 3 x 4, width, height), the loss is taken on the image
    instead (Eqs. 14-16): the vertices' radiance is rasterised and L is the
    mean over pixels of (I_R - target)^2, ``target`` then being the
    [height, width] reference image."""

    def __init__(self, graph: DeformGraph, albedo, light, target, n_bands: int, lr: float = 1e-2, init=None,
                 eps: float = 3.0, n_squarings: int = 4, faces=None, camera=None):
        dev = graph.device
        P, S = graph.P, graph.S
        self.graph, self.lr, self.P, self.S = graph, float(lr), P, S
        f = lambda a: torch.as_tensor(np.asarray(torch.as_tensor(a).cpu(), np.float32)).to(dev).contiguous()  # noqa: E731
        self.albedo, self.light, self.target = f(albedo), f(light), f(target)
        self.prm = _lib.params(n_bands, eps, n_squarings)
        N = n_bands * n_bands
        self.params = f(init) if init is not None else torch.zeros(S + 1, 6, device=dev)
        self.grad = torch.empty(S + 1, 6, device=dev)
        self.pts, self.nrm, self.sph = (torch.empty(3, P, device=dev), torch.empty(3, P, device=dev),
                                        torch.empty(S, 4, device=dev))
        self.vis = torch.empty(N, P, device=dev)
        self.rad = torch.empty(P, device=dev)
        self.saved = torch.empty(_lib.shv_render_saved_floats(P, self.prm), device=dev)
        self.gB = torch.empty(P, device=dev)
        self.gP, self.gN, self.gS = torch.empty(3, P, device=dev), torch.empty(3, P, device=dev), torch.empty(S, 4,
                                                                                                               device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.ws_r = torch.empty(_lib.shv_workspace_bytes(P, S, self.prm), dtype=torch.uint8, device=dev)
        self.raster = None
        n_loss = P
        if faces is not None:
            faces = np.ascontiguousarray(np.asarray(faces, np.int32))
            Pm, width, height = camera
            T = len(faces)
            inc_ptr, inc_idx = np.zeros(P + 1, np.int32), np.zeros(max(3 * T, 1), np.int32)
            _lib.shv_raster_incidence_build(faces, T, P, inc_ptr, inc_idx)
            nb = _lib.shv_raster_workspace_bytes(P, T, width, height)
            self.raster = dict(
                T=T, cam=_lib.camera(np.asarray(Pm, np.float32), width, height),
                faces=torch.as_tensor(faces).to(dev), inc_ptr=torch.as_tensor(inc_ptr).to(dev),
                inc_idx=torch.as_tensor(inc_idx).to(dev), image=torch.empty(height, width, device=dev),
                face_id=torch.empty(height, width, dtype=torch.int32, device=dev),
                gI=torch.empty(height, width, device=dev), gPr=torch.empty(3, P, device=dev),
                ws=torch.empty(max(nb, 256), dtype=torch.uint8, device=dev))
            n_loss = width * height
        self.ws_l = torch.empty(max(_lib.shv_l2_workspace_bytes(n_loss), 256), dtype=torch.uint8, device=dev)

    def step(self):
        """One iteration: loss at the current parameters, then the update.
        Enqueued on the current stream; returns nothing (read ``loss``)."""
        g, st, P, S = self.graph, _stream(), self.P, self.S
        _lib.sh_deform_forward(g.c, self.params, self.pts, self.nrm, self.sph, g.ws, g.ws.numel(), st)
        _lib.sh_render_forward(self.pts, self.nrm, self.albedo, self.sph, self.light, P, S, self.prm, self.vis,
                               self.rad, self.saved, _lib.nbytes(self.saved), self.ws_r, self.ws_r.numel(), st)
        r = self.raster
        if r is None:
            _lib.sh_l2_loss(self.rad, self.target, P, self.gB, self.loss, self.ws_l, self.ws_l.numel(), st)
        else:
            _lib.sh_raster_forward(self.pts, P, r["faces"], r["T"], self.rad, r["cam"], r["image"], r["face_id"],
                                   r["ws"], r["ws"].numel(), st)
            _lib.sh_l2_loss(r["image"], self.target, r["image"].numel(), r["gI"], self.loss, self.ws_l,
                            self.ws_l.numel(), st)
            _lib.sh_raster_backward(r["gI"], self.pts, P, r["faces"], r["T"], self.rad, r["cam"], r["face_id"],
                                    r["inc_ptr"], r["inc_idx"], self.gB, r["gPr"], r["ws"], r["ws"].numel(), st)
        _lib.sh_render_backward(self.gB, self.pts, self.nrm, self.albedo, self.sph, P, S, self.prm, self.vis,
                                self.saved, _lib.nbytes(self.saved), self.gP, self.gN, None, self.gS, None, self.ws_r,
                                self.ws_r.numel(), st)
        if r is not None:
            # the vertices' positions reach the loss through the shading and
            # through the rasteriser: gP <- gP - (-1) gPr
            _lib.sh_sgd_step(self.gP, r["gPr"], 3 * P, -1.0, st)
        _lib.sh_deform_backward(g.c, self.params, self.gP, self.gN, self.gS, self.grad, g.ws, g.ws.numel(), st)
        _lib.sh_sgd_step(self.params, self.grad, self.params.numel(), self.lr, st)

    def run(self, iters: int):
        """``iters`` steps; returns the loss before each step (host floats)."""
        hist = torch.empty(iters, device=self.graph.device)
        for i in range(iters):
            self.step()
            hist[i:i + 1].copy_(self.loss)
        return hist.cpu().tolist()
