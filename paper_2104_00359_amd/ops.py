"""PyTorch-facing operations over the HIP library.

``shade_sh`` renders per-receiver radiance with soft shadows from sphere
occluders (Eq. 8 with the visibility of Sec. 3.3.2) and is differentiable with
respect to receiver positions and normals, albedo, sphere centres and radii,
and the lighting SH vector, through hand-written adjoint kernels.  PyTorch
only supplies device memory and the current HIP stream; every step of the
computation runs in the library's kernels.
"""
from __future__ import annotations

import threading

import torch

from . import _lib

_ws_lock = threading.Lock()
_ws_cache: dict = {}
_initialised: set = set()


def ensure_init(device: torch.device) -> None:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _initialised:
        _lib.shv_init(idx)
        _initialised.add(idx)


def workspace(device: torch.device, nbytes: int) -> torch.Tensor:
    """A grow-only scratch buffer per (device, current stream).  Calls on one
    stream run in stream order, so they can share it; calls on different
    streams get different buffers.  The buffer is allocated on the stream
    that uses it, so when it grows the caching allocator reuses the old block
    only after the work already queued on that stream."""
    stream = torch.cuda.current_stream(device)
    key = (device.type, device.index, stream.cuda_stream)
    with _ws_lock:
        buf = _ws_cache.get(key)
        if buf is None or buf.numel() < nbytes:
            with torch.cuda.stream(stream):
                buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            _ws_cache[key] = buf
        return buf


def _shape_error(op: str, name: str, t, want) -> ValueError:
    got = tuple(t.shape) if isinstance(t, torch.Tensor) else type(t).__name__
    return ValueError(f"{op}: {name} must be {want}, got {got}")


def check_inputs(op: str, specs) -> None:
    """Argument checks before anything reaches the library, which sees bare
    pointers and cannot check them: every input is a floating-point tensor of
    the stated shape (``specs``: (name, tensor, shape) with ints or None for
    any size), and all live on one HIP device."""
    dev = None
    for name, t, shape in specs:
        if not isinstance(t, torch.Tensor):
            raise _shape_error(op, name, t, "a tensor")
        if not t.is_floating_point():
            raise ValueError(f"{op}: {name} must be a floating-point tensor, got {t.dtype}")
        if t.dim() != len(shape) or any(w is not None and g != w for g, w in zip(t.shape, shape)):
            raise _shape_error(op, name, t, "[" + ", ".join("*" if w is None else str(w) for w in shape) + "]")
    for name, t, _ in specs:
        if t.device.type != "cuda":
            raise RuntimeError(f"{op} runs on the GPU only; {name} is on {t.device} (move the inputs to a HIP "
                               "device)")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise RuntimeError(f"{op}: {name} is on {t.device}, the other inputs on {dev}")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _soa(x: torch.Tensor) -> torch.Tensor:
    """[P, 3] -> [3, P] FP32 contiguous (layout marshalling)."""
    return x.detach().to(torch.float32).t().contiguous()


def _f32(x: torch.Tensor) -> torch.Tensor:
    return x.detach().to(torch.float32).contiguous()


class ShadeSH(torch.autograd.Function):
    """Radiance with soft shadows through the fused render entry points
    (sh_render_forward / sh_render_backward)."""

    @staticmethod
    def forward(ctx, points, normals, albedo, spheres, light, n_bands, eps, n_squarings):
        P = points.shape[0] if isinstance(points, torch.Tensor) and points.dim() == 2 else None
        S = spheres.shape[0] if isinstance(spheres, torch.Tensor) and spheres.dim() == 2 else None
        N = int(n_bands) * int(n_bands)
        check_inputs("shade_sh", [("points", points, (P, 3)), ("normals", normals, (P, 3)),
                                  ("albedo", albedo, (P,)), ("spheres", spheres, (S, 4)), ("light", light, (N,))])
        dev = points.device
        ensure_init(dev)
        prm = _lib.params(n_bands, eps, n_squarings)
        pts, nrm = _soa(points), _soa(normals)
        alb, sph, L = _f32(albedo), _f32(spheres), _f32(light)
        vis = torch.empty(N, P, dtype=torch.float32, device=dev)
        saved = torch.empty(max(_lib.shv_render_saved_floats(P, prm), 1), dtype=torch.float32, device=dev)
        rad = torch.empty(P, dtype=torch.float32, device=dev)
        ws = workspace(dev, _lib.shv_workspace_bytes(P, S, prm))
        _lib.sh_render_forward(pts, nrm, alb, sph, L, P, S, prm, vis, rad, saved, _lib.nbytes(saved), ws, ws.numel(),
                               _stream())
        ctx.save_for_backward(pts, nrm, alb, sph, vis, saved)
        ctx.cfg = (n_bands, eps, n_squarings)
        return rad

    @staticmethod
    def backward(ctx, grad_rad):
        pts, nrm, alb, sph, vis, saved = ctx.saved_tensors
        n_bands, eps, n_squarings = ctx.cfg
        prm = _lib.params(n_bands, eps, n_squarings)
        dev = pts.device
        P, S, N = pts.shape[1], sph.shape[0], n_bands * n_bands
        gB = _f32(grad_rad)
        need_p, need_n, need_a, need_s, need_l = ctx.needs_input_grad[:5]
        gP = torch.empty(3, P, dtype=torch.float32, device=dev) if need_p else None
        gN = torch.empty(3, P, dtype=torch.float32, device=dev) if need_n else None
        gA = torch.empty(P, dtype=torch.float32, device=dev) if need_a else None
        gS = torch.empty(S, 4, dtype=torch.float32, device=dev) if need_s else None
        gL = torch.empty(N, dtype=torch.float32, device=dev) if need_l else None
        ws = workspace(dev, _lib.shv_workspace_bytes(P, S, prm))
        _lib.sh_render_backward(gB, pts, nrm, alb, sph, P, S, prm, vis, saved, _lib.nbytes(saved), gP, gN, gA, gS, gL,
                                ws, ws.numel(), _stream())
        return (gP.t() if gP is not None else None, gN.t() if gN is not None else None, gA, gS, gL,
                None, None, None)


def shade_sh(points, normals, albedo, spheres, light, n_bands: int, eps: float = 3.0, n_squarings: int = 4):
    """Radiance [P] at receivers ``points`` [P, 3] with ``normals`` [P, 3] and
    ``albedo`` [P], occluded by ``spheres`` [S, 4] = (cx, cy, cz, r), lit by the
    SH vector ``light`` [n_bands^2] (index l*l + l + m, real orthonormal basis
    without Condon-Shortley phase)."""
    return ShadeSH.apply(points, normals, albedo, spheres, light, n_bands, eps, n_squarings)


def mode_flags(mode) -> int:
    """shv_params flags of a way of forming V: "squaring" (the default:
    scaling, squaring and the linear approximation), "quadrature" (the
    projected pointwise exponential), "product" (the direct product chain of
    Eq. 12) or "taylorK" for K = 1..8 (a Taylor series of order K in place of
    the linear approximation)."""
    if mode in (None, "squaring"):
        return 0
    if mode == "quadrature":
        return _lib.SHV_FLAG_EXP_QUADRATURE
    if mode == "product":
        return _lib.SHV_FLAG_EXP_PRODUCT
    if isinstance(mode, str) and mode.startswith("taylor") and mode[6:].isdigit():
        K = int(mode[6:])
        if 1 <= K <= _lib.SHV_MAX_TAYLOR_ORDER:
            return _lib.SHV_FLAG_EXP_TAYLOR | _lib.SHV_FLAG_EXP_TAYLOR_ORDER(K)
    raise ValueError(f"unknown visibility mode {mode!r}")


class VisibilitySH(torch.autograd.Function):
    """Visibility SH vectors through sh_visibility_forward; backward through
    sh_visibility_backward (gradients for receiver positions and spheres)."""

    @staticmethod
    def forward(ctx, points, spheres, n_bands, eps, n_squarings, flags):
        check_inputs("visibility_sh", [("points", points, (None, 3)), ("spheres", spheres, (None, 4))])
        dev = points.device
        ensure_init(dev)
        prm = _lib.params(n_bands, eps, n_squarings, flags)
        P, S, N = points.shape[0], spheres.shape[0], n_bands * n_bands
        pts, sph = _soa(points), _f32(spheres)
        vis = torch.empty(N, P, dtype=torch.float32, device=dev)
        saved = torch.empty(max(_lib.shv_saved_floats(P, prm), 1), dtype=torch.float32, device=dev)
        ws = workspace(dev, _lib.shv_workspace_bytes(P, S, prm))
        _lib.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, _lib.nbytes(saved), ws, ws.numel(), _stream())
        ctx.save_for_backward(pts, sph, vis, saved)
        ctx.cfg = (n_bands, eps, n_squarings, flags)
        return vis.t()

    @staticmethod
    def backward(ctx, grad_vis):
        pts, sph, vis, saved = ctx.saved_tensors
        prm = _lib.params(*ctx.cfg)
        dev = pts.device
        P, S = pts.shape[1], sph.shape[0]
        need_p, need_s = ctx.needs_input_grad[:2]
        if not (need_p or need_s):
            return None, None, None, None, None, None
        gP = torch.empty(3, P, dtype=torch.float32, device=dev) if need_p else None
        gS = torch.empty(max(S, 1), 4, dtype=torch.float32, device=dev) if need_s else None
        ws = workspace(dev, _lib.shv_workspace_bytes(P, S, prm))
        _lib.sh_visibility_backward(_soa(grad_vis), vis, pts, P, sph, S, prm, saved, _lib.nbytes(saved), gP, gS, ws,
                                    ws.numel(), _stream())
        return (gP.t() if gP is not None else None, gS[:S] if gS is not None else None, None, None, None, None)


def visibility_sh(points, spheres, n_bands: int, eps: float = 3.0, n_squarings: int = 4, mode: str = "squaring"):
    """Visibility SH vectors [P, n_bands^2] of receivers ``points`` [P, 3]
    occluded by ``spheres`` [S, 4], differentiable with respect to both;
    ``mode`` selects how V is formed (see mode_flags)."""
    return VisibilitySH.apply(points, spheres, n_bands, eps, n_squarings, mode_flags(mode))


class ShadeSHChannels(torch.autograd.Function):
    """Radiance of several colour channels that share one visibility
    (sh_visibility_forward, then sh_shade_channels; backward through
    sh_shade_channels_backward and sh_visibility_backward)."""

    @staticmethod
    def forward(ctx, points, normals, albedo, spheres, light, n_bands, eps, n_squarings, flags=0):
        P = points.shape[0] if isinstance(points, torch.Tensor) and points.dim() == 2 else None
        S = spheres.shape[0] if isinstance(spheres, torch.Tensor) and spheres.dim() == 2 else None
        C = light.shape[0] if isinstance(light, torch.Tensor) and light.dim() == 2 else None
        N = int(n_bands) * int(n_bands)
        check_inputs("shade_sh_channels", [("points", points, (P, 3)), ("normals", normals, (P, 3)),
                                           ("albedo", albedo, (P, C)), ("spheres", spheres, (S, 4)),
                                           ("light", light, (C, N))])
        dev = points.device
        ensure_init(dev)
        prm = _lib.params(n_bands, eps, n_squarings, flags)
        pts, nrm = _soa(points), _soa(normals)
        alb, sph, L = _soa(albedo), _f32(spheres), _f32(light)
        vis = torch.empty(N, P, dtype=torch.float32, device=dev)
        saved = torch.empty(max(_lib.shv_saved_floats(P, prm), 1), dtype=torch.float32, device=dev)
        rad = torch.empty(C, P, dtype=torch.float32, device=dev)
        ws = workspace(dev, max(_lib.shv_workspace_bytes(P, S, prm), _lib.shv_channels_workspace_bytes(P, C, prm)))
        _lib.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, _lib.nbytes(saved), ws, ws.numel(), _stream())
        _lib.sh_shade_channels(vis, nrm, alb, L, C, P, prm, rad, ws, ws.numel(), _stream())
        ctx.save_for_backward(pts, nrm, alb, sph, L, vis, saved)
        ctx.cfg = (n_bands, eps, n_squarings, flags)
        return rad.t()

    @staticmethod
    def backward(ctx, grad_rad):
        pts, nrm, alb, sph, L, vis, saved = ctx.saved_tensors
        n_bands, eps, n_squarings, flags = ctx.cfg
        prm = _lib.params(n_bands, eps, n_squarings, flags)
        dev = pts.device
        P, S, N, C = pts.shape[1], sph.shape[0], n_bands * n_bands, L.shape[0]
        gB = _soa(grad_rad)
        need_p, need_n, need_a, need_s, need_l = ctx.needs_input_grad[:5]
        need_v = need_p or need_s
        gV = torch.empty(N, P, dtype=torch.float32, device=dev) if need_v else None
        gN = torch.empty(3, P, dtype=torch.float32, device=dev) if need_n else None
        gA = torch.empty(C, P, dtype=torch.float32, device=dev) if need_a else None
        gL = torch.empty(C, N, dtype=torch.float32, device=dev) if need_l else None
        gP = torch.empty(3, P, dtype=torch.float32, device=dev) if need_p else None
        gS = torch.empty(S, 4, dtype=torch.float32, device=dev) if need_s else None
        ws = workspace(dev, max(_lib.shv_workspace_bytes(P, S, prm), _lib.shv_channels_workspace_bytes(P, C, prm)))
        _lib.sh_shade_channels_backward(gB, vis, nrm, alb, L, C, P, prm, gV, gN, gA, gL, ws, ws.numel(), _stream())
        if need_v:
            _lib.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, _lib.nbytes(saved), gP, gS, ws, ws.numel(),
                                        _stream())
        return (gP.t() if gP is not None else None, gN.t() if gN is not None else None,
                gA.t() if gA is not None else None, gS, gL, None, None, None, None)


def shade_sh_channels(points, normals, albedo, spheres, light, n_bands: int, eps: float = 3.0,
                      n_squarings: int = 4, mode: str = "squaring"):
    """Radiance [P, C] of C colour channels (e.g. RGB) at receivers ``points``
    [P, 3] with ``normals`` [P, 3] and ``albedo`` [P, C], under one shared
    visibility from ``spheres`` [S, 4], lit by ``light`` [C, n_bands^2] (one
    SH vector per channel; Eq. 8 per channel).  Differentiable with respect to
    every tensor input; ``mode`` selects how V is formed (see mode_flags)."""
    return ShadeSHChannels.apply(points, normals, albedo, spheres, light, n_bands, eps, n_squarings,
                                 mode_flags(mode))


def envmap_to_sh(image, n_bands: int):
    """SH lighting coefficients of an equirectangular environment map (Eq. 9):
    ``image`` [H, W] or [C, H, W] (row r covers polar angles [r, r+1] pi/H from
    +z, column x azimuths [x, x+1] 2 pi/W from +x towards +y) -> [N] or
    [C, N] with N = n_bands^2.  Forward only."""
    if not isinstance(image, torch.Tensor) or image.dim() not in (2, 3):
        raise _shape_error("envmap_to_sh", "image", image, "[H, W] or [C, H, W]")
    check_inputs("envmap_to_sh", [("image", image, (None,) * image.dim())])
    dev = image.device
    ensure_init(dev)
    mono = image.dim() == 2
    img = _f32(image[None] if mono else image)
    C, H, W = img.shape
    prm = _lib.params(n_bands)
    out = torch.empty(C, n_bands * n_bands, dtype=torch.float32, device=dev)
    ws = workspace(dev, _lib.shv_envmap_workspace_bytes(C, H, W, prm))
    _lib.sh_envmap_project(img, C, H, W, prm, out, ws, ws.numel(), _stream())
    return out[0] if mono else out
