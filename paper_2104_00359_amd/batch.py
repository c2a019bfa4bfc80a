"""Batched render path: many independent scenes through one work table.

``RenderBatch`` holds the device buffers of a list of scenes (inputs in the C
layout, outputs, saved state and per-scene workspace), packs the work table on
the host with ``shv_batch_table_build``, uploads it, and runs the batched
forward / backward entry points.  Argument marshalling only: every step runs
in the library's kernels, and every scene's results are bit-identical to a
single-scene ``sh_render_forward`` / ``sh_render_backward`` call.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .ops import ensure_init

GRAD_NAMES = ("grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light")


_ALIGN = 256


def _aligned(n: int) -> int:
    return (int(n) + _ALIGN - 1) // _ALIGN * _ALIGN


@dataclass(eq=False)
class SceneBuffers:
    """Device buffers of one scene in the C layout (SoA [3][P] geometry).
    ``allocate`` carves the outputs, saved state and workspace out of one
    device allocation and prepares the scene's C record."""
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
    rec: object = None

    @property
    def P(self) -> int:
        return int(self.points.shape[1])

    @property
    def S(self) -> int:
        return int(self.spheres.shape[0])

    def params(self):
        return _lib.params(self.n_bands, self.eps, self.n_squarings, self.flags)

    def _layout(self):
        """(name, shape or byte count) of every buffer the scene needs."""
        P, S, N = self.P, self.S, self.n_bands * self.n_bands
        prm = self.params()
        lay = [("vis", (N, P)), ("radiance", (P,)), ("saved", (max(_lib.shv_render_saved_floats(P, prm), 1),)),
               ("ws", max(_lib.shv_workspace_bytes(P, S, prm), _ALIGN))]
        shapes = {"grad_points": (3, P), "grad_normals": (3, P), "grad_albedo": (P,), "grad_spheres": (max(S, 1), 4),
                  "grad_light": (N,)}
        lay += [(g, shapes[g]) for g in GRAD_NAMES if g in self.grads]
        return lay

    @staticmethod
    def _nbytes(spec) -> int:
        if isinstance(spec, int):
            return spec
        n = 1
        for d in spec:
            n *= d
        return 4 * n

    def device_bytes(self, include_inputs: bool = True) -> int:
        """Device memory this scene occupies once allocated (HBM footprint)."""
        total = sum(_aligned(self._nbytes(spec)) for _, spec in self._layout())
        if include_inputs:
            ins = [self.points, self.normals, self.albedo, self.spheres, self.light, self.grad_radiance]
            total += sum(_aligned(t.numel() * t.element_size()) for t in ins if t is not None)
        return total

    def allocate(self, device=None) -> None:
        dev = device if device is not None else self.points.device
        lay = self._layout()
        offs, total = [], 0
        for _, spec in lay:
            offs.append(total)
            total += _aligned(self._nbytes(spec))
        arena = torch.empty(max(total, _ALIGN), dtype=torch.uint8, device=dev)
        o = {"arena": arena}
        for (name, spec), off in zip(lay, offs):
            nb = self._nbytes(spec)
            if name == "ws":
                o[name] = arena[off:off + nb]
            else:
                o[name] = arena[off:off + nb].view(torch.float32).view(*spec)
        for g in GRAD_NAMES:
            o.setdefault(g, None)
        self.out = o
        r = _lib.shv_scene()
        r.points, r.normals, r.albedo = _lib.ptr(self.points), _lib.ptr(self.normals), _lib.ptr(self.albedo)
        r.spheres, r.light = _lib.ptr(self.spheres), _lib.ptr(self.light)
        r.grad_radiance = _lib.ptr(self.grad_radiance)
        r.vis, r.radiance, r.saved = _lib.ptr(o["vis"]), _lib.ptr(o["radiance"]), _lib.ptr(o["saved"])
        r.saved_bytes = _lib.nbytes(o["saved"])
        r.grad_points, r.grad_normals = _lib.ptr(o["grad_points"]), _lib.ptr(o["grad_normals"])
        r.grad_albedo, r.grad_spheres = _lib.ptr(o["grad_albedo"]), _lib.ptr(o["grad_spheres"])
        r.grad_light = _lib.ptr(o["grad_light"])
        r.ws, r.ws_bytes = _lib.ptr(o["ws"]), o["ws"].numel()
        r.P, r.S, r.params = self.P, self.S, self.params()
        self.rec = r

    def record(self, begin: int = 0, end: int = 0, defer: bool = False):
        """The scene's C record for receivers [begin, end) (0, 0: all)."""
        r = _lib.shv_scene()
        ctypes.pointer(r)[0] = self.rec
        r.range_begin, r.range_end, r.defer_reductions = int(begin), int(end), 1 if defer else 0
        return r


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


class Table:
    """A packed work table (host copy in pinned memory, device copy) and its
    launch grid.  ``records``: C scene records (SceneBuffers.record())."""

    def __init__(self, records, device, stream=None):
        n = len(records)
        nbytes = _lib.shv_batch_table_bytes(n)
        self.host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
        _lib.shv_batch_table_build(records, self.host)
        self.grid = _lib.shv_batch_table_grid(self.host)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.device = torch.empty(nbytes, dtype=torch.uint8, device=device)
        with torch.cuda.stream(s):
            self.device.copy_(self.host, non_blocking=True)
        self.uploaded = torch.cuda.Event()
        self.uploaded.record(s)

    def _handle(self, stream):
        if not torch.cuda.is_current_stream_capturing():   # a captured graph orders itself at replay
            stream.wait_event(self.uploaded)
        return stream.cuda_stream

    def forward(self, stream):
        _lib.sh_render_batched_forward(self.device, self.grid, self._handle(stream))

    def backward(self, stream):
        _lib.sh_render_batched_backward(self.device, self.grid, self._handle(stream))


class RenderBatch:
    """Whole scenes in one batch: buffers are allocated and the table is
    built and uploaded once; ``forward`` and ``backward`` enqueue the batched
    calls on ``stream`` (default: the current stream)."""

    def __init__(self, scenes: list[SceneBuffers], device=None):
        self.scenes = list(scenes)
        dev = torch.device(device) if device is not None else (
            self.scenes[0].points.device if self.scenes else torch.device("cuda", torch.cuda.current_device()))
        self.device = dev
        ensure_init(dev)
        for sc in self.scenes:
            sc.allocate(dev)
        self.tab = Table([sc.record() for sc in self.scenes], dev)

    @property
    def table(self) -> torch.Tensor:
        return self.tab.device

    @property
    def grid(self):
        return self.tab.grid

    def _s(self, stream):
        return stream if stream is not None else torch.cuda.current_stream(self.device)

    def forward(self, stream=None):
        self.tab.forward(self._s(stream))

    def backward(self, stream=None):
        self.tab.backward(self._s(stream))

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
