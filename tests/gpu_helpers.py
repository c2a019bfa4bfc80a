"""Shared helpers for the GPU parity tests: run the HIP path through its C ABI
and the FP64 oracle on the same FP32 inputs, and compare."""
import numpy as np
import torch

from oracle import method


def cuda_available():
    return torch.cuda.is_available()


def lib():
    from paper_2104_00359_amd import _lib
    return _lib


def to_dev(a, dev="cuda"):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dev)


def run_hip(scene, grad_B=None, eps=3.0, k=4, want_grads=True, flags=0):
    """Forward (+ backward when grad_B is given) through the C ABI.
    Returns numpy arrays: V [P, N], B [P], and the gradients."""
    L = lib()
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    n = int(scene["n_bands"])
    N = n * n
    P = scene["points"].shape[0]
    S = scene["spheres"].shape[0]
    prm = L.params(n, eps, k, flags)
    pts = to_dev(scene["points"].T)
    nrm = to_dev(scene["normals"].T)
    alb = to_dev(scene["albedo"])
    sph = to_dev(scene["spheres"]).reshape(S, 4)
    lig = to_dev(scene["light"])
    vis = torch.empty(N, P, device=dev)
    saved = torch.empty(max(L.shv_saved_floats(P, prm), 1), device=dev)
    rad = torch.empty(P, device=dev)
    nb = L.shv_workspace_bytes(P, S, prm)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    L.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, L.nbytes(saved), ws, nb, st)
    L.sh_shade(vis, nrm, alb, lig, P, prm, rad, ws, nb, st)
    out = {"V": vis.t().cpu().numpy(), "B": rad.cpu().numpy()}
    if grad_B is not None:
        gB = to_dev(np.asarray(grad_B, np.float32))
        gV = torch.empty(N, P, device=dev)
        gN = torch.empty(3, P, device=dev)
        gA = torch.empty(P, device=dev)
        gL = torch.empty(N, device=dev)
        gP = torch.empty(3, P, device=dev)
        gS = torch.empty(max(S, 1), 4, device=dev)
        L.sh_shade_backward(gB, vis, nrm, alb, lig, P, prm, gV, gN, gA, gL, ws, nb, st)
        L.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, L.nbytes(saved), gP, gS, ws, nb, st)
        out.update(grad_points=gP.t().cpu().numpy(), grad_normals=gN.t().cpu().numpy(),
                   grad_albedo=gA.cpu().numpy(), grad_light=gL.cpu().numpy(),
                   grad_spheres=gS[:S].cpu().numpy())
    torch.cuda.synchronize()
    return out


def run_render(scene, grad_B, eps=3.0, k=4, flags=0, null=()):
    """Fused path (sh_render_forward / sh_render_backward) through the C ABI;
    outputs named in ``null`` are passed as NULL."""
    L = lib()
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    n = int(scene["n_bands"])
    N = n * n
    P = scene["points"].shape[0]
    S = scene["spheres"].shape[0]
    prm = L.params(n, eps, k, flags)
    pts = to_dev(scene["points"].T)
    nrm = to_dev(scene["normals"].T)
    alb = to_dev(scene["albedo"])
    sph = to_dev(scene["spheres"]).reshape(S, 4)
    lig = to_dev(scene["light"])
    vis = torch.empty(N, P, device=dev)
    saved = torch.empty(max(L.shv_render_saved_floats(P, prm), 1), device=dev)
    rad = torch.empty(P, device=dev)
    nb = L.shv_workspace_bytes(P, S, prm)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    L.sh_render_forward(pts, nrm, alb, sph, lig, P, S, prm, vis, rad, saved, L.nbytes(saved), ws, nb, st)
    out = {"V": vis.t().cpu().numpy(), "B": rad.cpu().numpy()}
    gB = to_dev(np.asarray(grad_B, np.float32))
    g = {"grad_points": torch.empty(3, P, device=dev), "grad_normals": torch.empty(3, P, device=dev),
         "grad_albedo": torch.empty(P, device=dev), "grad_spheres": torch.empty(max(S, 1), 4, device=dev),
         "grad_light": torch.empty(N, device=dev)}
    a = {k2: (None if k2 in null else v) for k2, v in g.items()}
    L.sh_render_backward(gB, pts, nrm, alb, sph, P, S, prm, vis, saved, L.nbytes(saved), a["grad_points"],
                         a["grad_normals"],
                         a["grad_albedo"], a["grad_spheres"], a["grad_light"], ws, nb, st)
    torch.cuda.synchronize()
    if "grad_points" not in null:
        out["grad_points"] = g["grad_points"].t().cpu().numpy()
    if "grad_normals" not in null:
        out["grad_normals"] = g["grad_normals"].t().cpu().numpy()
    if "grad_albedo" not in null:
        out["grad_albedo"] = g["grad_albedo"].cpu().numpy()
    if "grad_spheres" not in null:
        out["grad_spheres"] = g["grad_spheres"][:S].cpu().numpy()
    if "grad_light" not in null:
        out["grad_light"] = g["grad_light"].cpu().numpy()
    return out


def run_oracle(scene, grad_B=None, eps=3.0, k=4, idx=None, dtype=torch.float64):
    """FP64 oracle (dtype=float32 gives its FP32 twin, which only measures the
    error FP32 arithmetic alone introduces)."""
    if grad_B is None:
        o = method.run_forward(scene, eps=eps, n_squarings=k, idx=idx, dtype=dtype)
        return {"V": o["V"].double().numpy(), "B": o["B"].double().numpy()}
    o = method.run_forward_backward(scene, grad_B, eps=eps, n_squarings=k, idx=idx, dtype=dtype)
    return {k2: v.detach().double().numpy() for k2, v in o.items()}


def rel_max(a, b):
    """max |a - b| / max |b|."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def run_batched(scenes, cfgs=None, eps=3.0, graph_replays=0):
    """Every scene through one RenderBatch (batched forward then backward).
    ``cfgs[i]`` may set k, flags and null (outputs passed as NULL) per scene;
    a scene without "grad_radiance" is packed without a cotangent.  Returns
    one dict per scene in the format of run_render."""
    from paper_2104_00359_amd import batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    cfgs = cfgs or [{} for _ in scenes]
    bufs = []
    for sc, c in zip(scenes, cfgs):
        grads = tuple(g for g in batch.GRAD_NAMES if g not in c.get("null", ()))
        bufs.append(batch.scene_buffers(sc, dev, eps=eps, n_squarings=c.get("k", 4), flags=c.get("flags", 0),
                                        grads=grads))
    rb = batch.RenderBatch(bufs, dev)
    rb.forward()
    rb.backward()
    torch.cuda.synchronize()
    return [collect(b) for b in bufs]


def collect(b):
    """Host copies of a SceneBuffers' outputs (format of run_render)."""
    o = b.out
    out = {"V": o["vis"].t().cpu().numpy(), "B": o["radiance"].cpu().numpy()}
    for g in b.grads:
        t = o[g]
        if g in ("grad_points", "grad_normals"):
            out[g] = t.t().cpu().numpy()
        elif g == "grad_spheres":
            out[g] = t[:b.S].cpu().numpy()
        else:
            out[g] = t.cpu().numpy()
    return out
