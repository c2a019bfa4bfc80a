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
        return (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream

    def forward(self, stream=None):
        _lib.sh_render_batched_forward(self.table, self.grid, self._stream(stream))

    def backward(self, stream=None):
        _lib.sh_render_batched_backward(self.table, self.grid, self._stream(stream))

    @property
    def pairs(self) -> int:
        return sum(sc.P * sc.S for sc in self.scenes)
