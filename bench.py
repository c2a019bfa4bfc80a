"""Benchmark: point-sphere pair evaluations per second, forward + backward.

One step = the whole differentiable path on one scene resident in HBM: the
fused sh_render_forward (visibility + shading) and sh_render_backward
(gradients for receivers, normals, albedo, spheres and lighting), through the
C ABI (``--path separate`` uses the four separate entry points instead; the
results are bit-identical).  Default workload: the body-like scene (20,000
receivers on 24 capsules, 128 spheres, 8 bands, k = 4), synthetic and seeded.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (its average launch time from HIP events recorded around every launch
on the launch stream during the timed steps) and the FP64 oracle timed on a
bounded sample on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak: 256 CU x 2.4 GHz x 256 flop/clk (packed FMA)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="body", choices=["body", "gbuffer", "icosphere"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle CPU baseline sample (0 disables it)")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--path", default="render", choices=["render", "separate"])
    ap.add_argument("--flags", type=int, default=0, help="shv_params.flags (kernel-variant selection)")
    return ap.parse_args()


def make_scene(name):
    import scenegen
    if name == "body":
        sc = scenegen.scene_body()
        desc = "body-like scene: 20000 receivers on 24 capsules x 128 spheres, 8 bands, k=4, fwd+bwd"
    elif name == "gbuffer":
        sc = scenegen.scene_gbuffer()
        desc = "G-buffer scene: 512x512 receivers x 256 spheres, 8 bands, k=4, fwd+bwd"
    else:
        sc = scenegen.scene_icosphere_shell()
        sc["grad_radiance"] = scenegen.np.random.default_rng(1).standard_normal(
            sc["points"].shape[0]).astype("float32")
        desc = "icosphere scene: 2562 receivers x 32 spheres, 4 bands, k=4, fwd+bwd"
    return sc, desc


def cpu_baseline(sc, k, seconds):
    """The FP64 oracle (autograd for the backward) on a seeded sample of
    receivers of the same scene, all spheres, grown in chunks of 256 until
    ``seconds`` have elapsed."""
    import numpy as np
    import torch

    from oracle import method
    P = sc["points"].shape[0]
    S = sc["spheres"].shape[0]
    order = np.random.default_rng(123).permutation(P)
    done = 0
    t0 = time.perf_counter()
    while done < P:
        idx = np.sort(order[done:done + 256])
        method.run_forward_backward(sc, sc["grad_radiance"][idx], n_squarings=k, idx=idx)
        done += len(idx)
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": done * S / dt, "unit": "pairs/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{done} of {P} receivers (seeded permutation) x all {S} spheres, FP64 forward + "
                      f"autograd backward, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the single-GPU figure is whole-job throughput).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2104_00359_amd import _lib, ops, workmodel

    sc, desc = make_scene(args.workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    n = int(sc["n_bands"])
    N = n * n
    P = sc["points"].shape[0]
    S = sc["spheres"].shape[0]
    k = args.k
    prm = _lib.params(n, 3.0, k, args.flags)

    def t(a):
        return torch.as_tensor(np.ascontiguousarray(a)).to(dev)

    pts, nrm = t(sc["points"].T), t(sc["normals"].T)
    alb, sph, lig = t(sc["albedo"]), t(sc["spheres"]), t(sc["light"])
    gB = t(sc["grad_radiance"])
    vis = torch.empty(N, P, device=dev)
    saved = torch.empty(_lib.shv_render_saved_floats(P, prm), device=dev)
    rad = torch.empty(P, device=dev)
    gV = torch.empty(N, P, device=dev)
    gN = torch.empty(3, P, device=dev)
    gA = torch.empty(P, device=dev)
    gL = torch.empty(N, device=dev)
    gP = torch.empty(3, P, device=dev)
    gS = torch.empty(S, 4, device=dev)
    nb = _lib.shv_workspace_bytes(P, S, prm)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)   # default priority
    st = stream.cuda_stream

    if args.path == "render":
        def step():
            _lib.sh_render_forward(pts, nrm, alb, sph, lig, P, S, prm, vis, rad, saved, ws, nb, st)
            _lib.sh_render_backward(gB, pts, nrm, alb, sph, P, S, prm, vis, saved, gP, gN, gA, gS, gL, ws, nb, st)
    else:
        def step():
            _lib.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, ws, nb, st)
            _lib.sh_shade(vis, nrm, alb, lig, P, prm, rad, ws, nb, st)
            _lib.sh_shade_backward(gB, vis, nrm, alb, lig, P, prm, gV, gN, gA, gL, ws, nb, st)
            _lib.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, gP, gS, ws, nb, st)

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        _lib.shv_profile_enable(True, capacity=16 * args.steps + 64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _lib.shv_profile_enable(False)
    prof = _lib.shv_profile_report()
    ms = (t1 - t0) * 1e3 / args.steps
    value = P * S / (ms * 1e-3)

    kernels = {}
    for name, (cnt, tot) in prof.items():
        if cnt:
            kernels[name] = {"launches": cnt, "avg_us": 1e3 * tot / cnt}
    dom = max(kernels, key=lambda kname: kernels[kname]["avg_us"] * kernels[kname]["launches"])
    flops, units = workmodel.kernel_work(dom, n, k, P, S)
    avg_s = kernels[dom]["avg_us"] * 1e-6
    roof = None
    if flops is not None:
        ach = flops / avg_s / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": None,
                "flops_per_launch": flops, "avg_launch_us": round(kernels[dom]["avg_us"], 2)}
    for name, kv in kernels.items():
        f, _ = workmodel.kernel_work(name, n, k, P, S)
        if f is not None:
            kv["tflops"] = round(f / (kv["avg_us"] * 1e-6) / 1e12, 3)
        kv["avg_us"] = round(kv["avg_us"], 2)

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(sc, k, args.cpu_seconds)

    out = {
        "metric": "point-sphere pair evals/s fwd+bwd",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "receivers": P, "spheres": S, "n_bands": n, "n_squarings": k, "eps": 3.0,
                   "entry_points": args.path},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
