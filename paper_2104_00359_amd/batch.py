"""Batched render path: many independent scenes through one work table.

``RenderBatch`` holds the device buffers of a list of scenes (inputs in the C
layout, outputs, saved state and per-scene workspace), packs the work table on
the host with ``shv_batch_table_build``, uploads it, and runs the batched
forward / backward entry points.  Argument marshalling only: every step runs
in the library's kernels, and every scene's results are bit-identical to a
single-scene ``sh_render_forward`` / ``sh_render_backward`` call.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .ops import ensure_init

GRAD_NAMES = ("grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light")


@dataclass
class SceneBuffers:
    """Device buffers of one scene in the C layout (SoA [3][P] geometry)."""
    points: torch.Tensor
    normals: torch.Tensor
    albedo: torch.Tensor
    spheres: torch.Tensor
    light: torch.Tensor
    grad_radiance: torch.Tensor | None
    n_bands: int
    eps: float = 3.0
    n_squarings: int = 4
    flags: int = 0
    grads: tuple = GRAD_NAMES
    out: dict = field(default_factory=dict)

    @property
    def P(self) -> int:
        return int(self.points.shape[1])

    @property
    def S(self) -> int:
        return int(self.spheres.shape[0])

    def params(self):
        return _lib.params(self.n_bands, self.eps, self.n_squarings, self.flags)


def scene_buffers(scene: dict, device, eps=3.0, n_squarings=4, flags=0, grads=GRAD_NAMES) -> SceneBuffers:
    """Upload a scene dictionary (arrays points [P,3], normals [P,3], albedo
    [P], spheres [S,4], light [N], n_bands, optional grad_radiance [P])."""
    def t(a):
        return torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32))).to(device)

    S = np.asarray(scene["spheres"]).reshape(-1, 4).shape[0]
    gB = scene.get("grad_radiance")
    return SceneBuffers(points=t(np.asarray(scene["points"]).reshape(-1, 3).T),
                        normals=t(np.asarray(scene["normals"]).reshape(-1, 3).T),
                        albedo=t(scene["albedo"]), spheres=t(np.asarray(scene["spheres"]).reshape(S, 4)),
                        light=t(scene["light"]), grad_radiance=None if gB is None else t(gB),
                        n_bands=int(scene["n_bands"]), eps=eps, n_squarings=n_squarings, flags=flags,
                        grads=tuple(grads))


class RenderBatch:
    """One batch of scenes: outputs are allocated here, the table is built
    and uploaded once; ``forward`` and ``backward`` enqueue the batched calls
    on ``stream`` (default: the current stream)."""

    def __init__(self, scenes: list[SceneBuffers], device=None):
        self.scenes = list(scenes)
        dev = torch.device(device) if device is not None else (
            self.scenes[0].points.device if self.scenes else torch.device("cuda", torch.cuda.current_device()))
        self.device = dev
        ensure_init(dev)
        recs = []
        for sc in self.scenes:
            recs.append(self._allocate(sc))
        nbytes = _lib.shv_batch_table_bytes(len(recs))
        self.table_host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        _lib.shv_batch_table_build(recs, self.table_host)
        self.grid = _lib.shv_batch_table_grid(self.table_host)
        self.table = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.table.copy_(self.table_host, non_blocking=True)
        self._uploaded = torch.cuda.Event()
        self._uploaded.record(torch.cuda.current_stream(dev))
        self._recs = recs

    def _allocate(self, sc: SceneBuffers):
        dev = self.device
        P, S, N = sc.P, sc.S, sc.n_bands * sc.n_bands
        prm = sc.params()
        o = sc.out
        o["vis"] = torch.empty(N, P, device=dev)
        o["radiance"] = torch.empty(P, device=dev)
        o["saved"] = torch.empty(max(_lib.shv_render_saved_floats(P, prm), 1), device=dev)
        ws_bytes = _lib.shv_workspace_bytes(P, S, prm)
        o["ws"] = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
        shapes = {"grad_points": (3, P), "grad_normals": (3, P), "grad_albedo": (P,), "grad_spheres": (max(S, 1), 4),
                  "grad_light": (N,)}
        for g in GRAD_NAMES:
            o[g] = torch.empty(*shapes[g], device=dev) if g in sc.grads else None
        r = _lib.shv_scene()
        r.points, r.normals, r.albedo = _lib.ptr(sc.points), _lib.ptr(sc.normals), _lib.ptr(sc.albedo)
        r.spheres, r.light = _lib.ptr(sc.spheres), _lib.ptr(sc.light)
        r.grad_radiance = _lib.ptr(sc.grad_radiance)
        r.vis, r.radiance, r.saved = _lib.ptr(o["vis"]), _lib.ptr(o["radiance"]), _lib.ptr(o["saved"])
        r.grad_points, r.grad_normals = _lib.ptr(o["grad_points"]), _lib.ptr(o["grad_normals"])
        r.grad_albedo, r.grad_spheres = _lib.ptr(o["grad_albedo"]), _lib.ptr(o["grad_spheres"])
        r.grad_light = _lib.ptr(o["grad_light"])
        r.ws, r.ws_bytes = _lib.ptr(o["ws"]), ws_bytes
        r.P, r.S, r.params = P, S, prm
        return r

    def _stream(self, stream):
        """Raw handle of the launch stream, ordered after the table upload."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        if not torch.cuda.is_current_stream_capturing():   # a captured graph orders itself at replay
            s.wait_event(self._uploaded)
        return s.cuda_stream

    def forward(self, stream=None):
        _lib.sh_render_batched_forward(self.table, self.grid, self._stream(stream))

    def backward(self, stream=None):
        _lib.sh_render_batched_backward(self.table, self.grid, self._stream(stream))

    @property
    def pairs(self) -> int:
        return sum(sc.P * sc.S for sc in self.scenes)


class ShadeSHBatched(torch.autograd.Function):
    """Radiance of many scenes through one batched forward / backward.
    Inputs: a tuple of per-scene settings (n_bands, eps, n_squarings), then
    five tensors per scene (points [P,3], normals [P,3], albedo [P], spheres
    [S,4], light [n_bands^2])."""

    @staticmethod
    def forward(ctx, cfg, *flat):
        if len(flat) != 5 * len(cfg):
            raise ValueError("expected five tensors per scene")
        dev = flat[0].device if flat else torch.device("cuda", torch.cuda.current_device())
        if dev.type != "cuda":
            raise RuntimeError("shade_sh_batched runs on the GPU only; move the inputs to a HIP device")
        bufs = []
        for i, (n, eps, k) in enumerate(cfg):
            pts, nrm, alb, sph, L = flat[5 * i:5 * i + 5]
            if L.numel() != n * n:
                raise ValueError(f"scene {i}: light has {L.numel()} coefficients, expected {n * n}")
            need = ctx.needs_input_grad[1 + 5 * i:6 + 5 * i]
            grads = tuple(g for g, w in zip(("grad_points", "grad_normals", "grad_albedo", "grad_spheres",
                                              "grad_light"), need) if w)
            P = pts.shape[0]
            f32 = lambda x: x.detach().to(torch.float32).contiguous()  # noqa: E731
            bufs.append(SceneBuffers(points=f32(pts).t().contiguous(), normals=f32(nrm).t().contiguous(),
                                     albedo=f32(alb), spheres=f32(sph).reshape(-1, 4), light=f32(L),
                                     grad_radiance=torch.zeros(max(P, 1), device=dev),
                                     n_bands=int(n), eps=float(eps), n_squarings=int(k), grads=grads))
        rb = RenderBatch(bufs, dev)
        rb.forward()
        ctx.rb = rb
        return tuple(b.out["radiance"] for b in bufs)

    @staticmethod
    def backward(ctx, *grad_outputs):
        rb = ctx.rb
        for b, g in zip(rb.scenes, grad_outputs):
            if g is None:
                b.grad_radiance.zero_()
            elif b.P > 0:
                b.grad_radiance[:b.P].copy_(g.detach().to(torch.float32))
        rb.backward()
        out = [None]
        for b in rb.scenes:
            o = b.out
            for name in GRAD_NAMES:
                t = o.get(name)
                if t is None:
                    out.append(None)
                elif name in ("grad_points", "grad_normals"):
                    out.append(t.t())
                elif name == "grad_spheres":
                    out.append(t[:b.S])
                else:
                    out.append(t)
        ctx.rb = None
        return tuple(out)


def shade_sh_batched(points, normals, albedo, spheres, light, n_bands, eps: float = 3.0, n_squarings: int = 4):
    """Per-scene radiance [P_b] for lists of scene tensors (layouts as in
    ``ops.shade_sh``); ``n_bands`` is an int or a list of per-scene ints.
    Differentiable with respect to every tensor input; each scene's results
    are bit-identical to ``ops.shade_sh`` on that scene alone."""
    m = len(points)
    nb = list(n_bands) if isinstance(n_bands, (list, tuple)) else [int(n_bands)] * m
    cfg = tuple((nb[i], eps, n_squarings) for i in range(m))
    flat = []
    for i in range(m):
        flat += [points[i], normals[i], albedo[i], spheres[i], light[i]]
    return list(ShadeSHBatched.apply(cfg, *flat))
