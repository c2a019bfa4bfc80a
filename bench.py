"""Benchmark: point-sphere pair evaluations per second, forward + backward.

Default workload (one step = the whole differentiable path on one scene
resident in HBM): the body-like scene (20,000 receivers on 24 capsules, 128
spheres, 8 bands, k = 4), synthetic and seeded, through the fused
sh_render_forward (visibility + shading) and sh_render_backward (gradients
for receivers, normals, albedo, spheres and lighting) of the C ABI
(``--path separate`` uses the four separate entry points instead; the results
are bit-identical; ``--path separate --flags 4`` takes the exponential by
quadrature projection on MFMA instead of scaling and squaring, and
``--path separate --flags 8`` forms V by the direct product chain of Eq. 12).

``--workload serve``: Poisson arrivals of forward + backward requests (90%
from the 64-scene distribution, 10% at 262,144 receivers x 512 spheres)
against the continuous-batching server and against one request at a time,
per arrival rate; prints throughput and p50 / p99 latency.

``--workload rgb``: the body-like scene with three colour channels (albedo
and lighting per channel, one shared visibility, Eq. 8 per channel); one step
= sh_visibility_forward, sh_shade_channels, sh_shade_channels_backward and
sh_visibility_backward.  ``--workload envmap``: the lighting of a synthetic
3 x 512 x 1024 equirectangular map projected onto 8 bands (Eq. 9) through
sh_envmap_project; throughput in map pixels per second.

``--workload inverse``: one gradient-descent iteration of the inverse problem
on the body-like scene, every step in the library: the embedded deformation
driven by the spheres (each attached to its 625 nearest receivers) and a global
pose, visibility and shading, the mean-squared loss against a target rendered
from a perturbed scene, their adjoints, and the parameter update.

``--workload batched64``: 64 independent scenes (P ~ U{5k..50k}, S ~
U{32..256}, n ~ U{4, 6, 8}, seeds 100 + b); one step = the batched forward +
backward over all 64, replayed from one captured graph; the same 64 scenes
through 64 sequential single-scene forward + backward calls are timed beside
it.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (its average launch time from HIP events recorded around every launch
on the launch stream, during eager steps) and the FP64 oracle timed on a
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
METRIC = "point-sphere pair evals/s fwd+bwd"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="body",
                    choices=["body", "gbuffer", "icosphere", "batched64", "serve", "rgb", "envmap", "inverse",
                             "image"])
    ap.add_argument("--channels", type=int, default=3, help="rgb / envmap: colour channels")
    ap.add_argument("--map", default="512x1024", help="envmap: H x W of the equirectangular map")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle CPU baseline sample (0 disables it)")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--path", default="render", choices=["render", "separate"])
    ap.add_argument("--flags", type=int, default=0,
                    help="shv_params.flags: 1 / 2 select the exponential's kernel layout; 4 selects the "
                         "quadrature exponential, 8 the direct product chain of Eq. 12, 16 | (K << 8) the "
                         "Taylor series of order K (different approximations; separate entry points only)")
    ap.add_argument("--no-graph", action="store_true",
                    help="batched64: time eager batched calls instead of graph replays")
    ap.add_argument("--rates", default="100,200,500,1000,2000,5000",
                    help="serve: Poisson arrival rates (requests/s)")
    ap.add_argument("--duration", type=float, default=4.0, help="serve: seconds of arrivals per rate")
    ap.add_argument("--chunk-pairs", type=int, default=32 << 20, help="serve: pair bound of a request range")
    ap.add_argument("--step-pairs", type=int, default=128 << 20, help="serve: pair bound of a step")
    ap.add_argument("--modes", default="continuous,one_at_a_time", help="serve: scheduler modes to sweep")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device-to-device once (a plain copy kernel "
                         "of known size, to calibrate HBM byte counters)")
    return ap.parse_args()


def make_scene(name):
    import scenegen
    if name == "body":
        sc = scenegen.scene_body()
        desc = "body-like scene: 20000 receivers on 24 capsules x 128 spheres, 8 bands, k=4, fwd+bwd"
    elif name == "gbuffer":
        sc = scenegen.scene_gbuffer()
        sc["grad_radiance"] = scenegen.np.random.default_rng(1).standard_normal(
            sc["points"].shape[0]).astype("float32")
        desc = "G-buffer scene: 512x512 receivers x 256 spheres, 8 bands, k=4, fwd+bwd (cotangent w ~ N(0,1))"
    else:
        sc = scenegen.scene_icosphere_shell()
        sc["grad_radiance"] = scenegen.np.random.default_rng(1).standard_normal(
            sc["points"].shape[0]).astype("float32")
        desc = "icosphere scene: 2562 receivers x 32 spheres, 4 bands, k=4, fwd+bwd"
    return sc, desc


def saved_buffer_floats(lib, P, prm):
    """Floats of a state buffer that serves both the fused render entry points
    and the separate visibility ones (whose state grows with the Taylor
    order), so either path of bench_single can use it."""
    return max(lib.shv_render_saved_floats(P, prm), lib.shv_saved_floats(P, prm), 1)


def cpu_baseline(scenes, k, seconds, exp_mode="squaring"):
    """The FP64 oracle (autograd for the backward) on seeded samples of
    receivers (chunks of 256, all spheres), cycling over ``scenes`` until
    ``seconds`` have elapsed or every receiver is done."""
    import numpy as np
    import torch

    from oracle import method
    perms = [np.random.default_rng(123 + i).permutation(sc["points"].shape[0]) for i, sc in enumerate(scenes)]
    done = [0] * len(scenes)
    pairs = 0
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < seconds:
        j = i % len(scenes)
        sc = scenes[j]
        if done[j] < sc["points"].shape[0]:
            idx = np.sort(perms[j][done[j]:done[j] + 256])
            method.run_forward_backward(sc, sc["grad_radiance"][idx], n_squarings=k, idx=idx, exp_mode=exp_mode)
            done[j] += len(idx)
            pairs += len(idx) * sc["spheres"].shape[0]
        elif all(d >= s["points"].shape[0] for d, s in zip(done, scenes)):
            break
        i += 1
    dt = time.perf_counter() - t0
    tot = sum(s["points"].shape[0] for s in scenes)
    where = (f"{done[0]} of {tot} receivers (seeded permutation)" if len(scenes) == 1 else
             f"{sum(done)} of {tot} receivers over {sum(1 for d in done if d)} of {len(scenes)} scenes "
             "(seeded permutations, 256 per scene in turn)")
    return {"value": pairs / dt, "unit": "pairs/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{where} x all spheres, FP64 forward + autograd backward"
                      f"{'' if exp_mode == 'squaring' else f' ({exp_mode} mode)'}, {dt:.1f} s"}


def kernel_table(prof):
    kernels = {}
    for name, (cnt, tot) in prof.items():
        if cnt:
            kernels[name] = {"launches": cnt, "avg_us": 1e3 * tot / cnt, "total_ms": tot}
    return kernels


def roofline(kernels, steps, work):
    """Roofline entry of the kernel with the largest total time; ``work(name)``
    gives its algorithmic flops per step and ``steps`` is the number of steps
    whose launches were timed.  achieved = flops per launch / average launch
    time."""
    dom = max(kernels, key=lambda kname: kernels[kname]["total_ms"])
    flops_step, _ = work(dom)
    unmodelled = None
    if flops_step is None:
        # the largest launch has no flop model (the rasteriser's, which is bound by latency and launches):
        # report the largest modelled kernel and name the other
        modelled = [kname for kname in kernels if work(kname)[0] is not None]
        if modelled:
            unmodelled = dom
            dom = max(modelled, key=lambda kname: kernels[kname]["total_ms"])
            flops_step, _ = work(dom)
    for name, kv in kernels.items():
        f, _ = work(name)
        if f is not None:
            kv["tflops"] = round(f * steps / (kv["total_ms"] * 1e-3) / 1e12, 3)
        kv["avg_us"] = round(kv["avg_us"], 2)
    if flops_step is None:
        return None
    per_launch = flops_step * steps / kernels[dom]["launches"]
    ach = per_launch / (kernels[dom]["avg_us"] * 1e-6) / 1e12
    bound = "mfma" if dom.startswith("exp_quad") else "alu"   # FP32 MFMA and FP32 vector share the peak
    out = {"bound": bound, "kernel": dom, "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
           "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": None,
           "flops_per_launch": int(per_launch), "avg_launch_us": kernels[dom]["avg_us"]}
    if unmodelled is not None:
        out["largest_unmodelled"] = unmodelled
    return out


def kernel_source_hash():
    """SHA-256 over the kernel sources and the C header: measured counter data
    is only quoted for the build it was taken on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2104_00359_amd", "csrc")
    for f in sorted(x for x in os.listdir(d) if x.endswith((".h", ".hip")) or x == "gen_tables.py"):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "shvis.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of ``kernel`` from rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (scaled by a plain copy of known size), recorded in
    profiles/traffic.json; None when not measured or when the kernel sources
    changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            entries = json.load(fh)["entries"]
    except (OSError, ValueError, KeyError):
        return None
    digest = kernel_source_hash()
    for e in entries:
        if e.get("workload") == workload and e.get("kernel") == kernel and e.get("source_sha256") == digest:
            return int(e["bytes_per_launch"])
    return None


def timed(step, stream, warmup, steps, profile, every=10):
    """Average milliseconds per step over ``steps`` steps after ``warmup``.
    With ``profile``, one step in ``every`` of the timed steps also records a
    HIP event pair around each of its launches (on the launch stream), and
    the library's per-kernel report over those sampled steps is returned.
    Events around every launch would add about 4 us per launch to the timed
    steps; sampling keeps that to a tenth."""
    import torch

    from paper_2104_00359_amd import _lib
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if profile:
            _lib.shv_profile_enable(True, capacity=40 * (steps // every + 1) + 64)
            _lib.shv_profile_enable(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            sample = profile and i % every == 0
            if sample:
                _lib.shv_profile_enable(True, resume=True)
            step()
            if sample:
                _lib.shv_profile_enable(False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, (_lib.shv_profile_report() if profile else None)


def sampled_steps(steps, every=10):
    return (steps + every - 1) // every


def copy_calibration(args, dev, stream):
    if args.copy_mib <= 0:
        return
    import torch
    n = args.copy_mib << 18   # floats
    src = torch.ones(n, device=dev)
    dst = torch.empty(n, device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        dst.copy_(src)
    torch.cuda.synchronize()


def finish_kernels(kernels):
    for kv in kernels.values():
        kv.pop("total_ms", None)
    return kernels


def bench_single(args):
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
    saved = torch.empty(saved_buffer_floats(_lib, P, prm), device=dev)
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

    ms, prof = timed(step, stream, args.warmup, args.steps, True)
    copy_calibration(args, dev, stream)
    kernels = kernel_table(prof)
    order = (args.flags >> 8) & 15 if args.flags & _lib.SHV_FLAG_EXP_TAYLOR else 0
    roof = roofline(kernels, sampled_steps(args.steps),
                    lambda name: workmodel.kernel_work(name, n, k, P, S, order=order))
    if roof is not None:
        roof["traffic"] = measured_traffic(args.workload, roof["kernel"])
    mode = {4: "quadrature", 8: "product"}.get(args.flags, f"taylor{order}" if order else "squaring")
    cpu = cpu_baseline([sc], k, args.cpu_seconds, mode) if args.cpu_seconds > 0 else None
    return {
        "metric": METRIC, "value": P * S / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "receivers": P, "spheres": S, "n_bands": n, "n_squarings": k, "eps": 3.0,
                   "entry_points": args.path, "visibility": mode},
        "roofline": roof, "cpu_baseline": cpu, "kernels": finish_kernels(kernels),
    }


def bench_batched(args):
    import torch

    import scenegen
    from paper_2104_00359_amd import _lib, batch, ops, workmodel

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    k = args.k
    scenes = [scenegen.scene_batched(b) for b in range(64)]
    bufs = [batch.scene_buffers(sc, dev, n_squarings=k) for sc in scenes]
    rb = batch.RenderBatch(bufs, dev)
    pairs = rb.pairs
    stream = torch.cuda.Stream(device=dev)   # default priority
    st = stream.cuda_stream

    def batched():
        rb.forward(stream)
        rb.backward(stream)

    def sequential():
        for b in bufs:
            o, prm = b.out, b.params()
            ws_bytes = o["ws"].numel()
            _lib.sh_render_forward(b.points, b.normals, b.albedo, b.spheres, b.light, b.P, b.S, prm, o["vis"],
                                   o["radiance"], o["saved"], o["ws"], ws_bytes, st)
            _lib.sh_render_backward(b.grad_radiance, b.points, b.normals, b.albedo, b.spheres, b.P, b.S, prm,
                                    o["vis"], o["saved"], o["grad_points"], o["grad_normals"], o["grad_albedo"],
                                    o["grad_spheres"], o["grad_light"], o["ws"], ws_bytes, st)

    # per-kernel times from eager batched steps
    steps_prof = max(args.steps // 4, 5)
    ms_eager, prof = timed(batched, stream, args.warmup, steps_prof, True, every=1)
    ms_seq, _ = timed(sequential, stream, max(args.warmup // 4, 2), max(args.steps // 4, 5), False)
    if args.no_graph:
        ms, mode = ms_eager, "eager batched calls"
    else:
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            batched()
        torch.cuda.synchronize()
        ms, _ = timed(g.replay, stream, args.warmup, args.steps, False)
        mode = "one captured graph (all batched phases) per step"
    kernels = kernel_table(prof)
    desc = [(b.n_bands, k, b.P, b.S) for b in bufs]
    roof = roofline(kernels, steps_prof, lambda name: workmodel.batch_work(name, desc))
    cpu = cpu_baseline(scenes, k, args.cpu_seconds) if args.cpu_seconds > 0 else None
    return {
        "metric": METRIC, "value": pairs / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 independent scenes: P ~ U{5000..50000}, S ~ U{32..256}, n ~ U{4,6,8} "
                               "(seeds 100+b), k=4, fwd+bwd, batched",
                   "scenes": 64, "pairs_per_step": pairs, "receivers": sum(b.P for b in bufs),
                   "n_squarings": k, "eps": 3.0, "launch": mode},
        "batched_eager": {"ms_per_step": ms_eager, "value": pairs / (ms_eager * 1e-3)},
        "sequential": {"ms_per_step": ms_seq, "value": pairs / (ms_seq * 1e-3),
                       "what": "64 x (sh_render_forward + sh_render_backward), eager"},
        "speedup_vs_sequential": ms_seq / ms,
        "roofline": roof, "cpu_baseline": cpu, "kernels": finish_kernels(kernels),
    }


def bench_serve(args):
    """Poisson load against the continuous-batching server and against one
    request at a time (single-scene calls), per arrival rate."""
    import dataclasses

    import numpy as np
    import torch

    import scenegen
    from paper_2104_00359_amd import batch, serve

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    small = [batch.scene_buffers(scenegen.scene_batched(b), dev) for b in range(64)]
    large = [batch.scene_buffers(scenegen.large_request_scene(500 + i), dev) for i in range(4)]
    free, _ = torch.cuda.mem_get_info(dev)
    budget = int(free - (16 << 30))
    rates = [float(r) for r in args.rates.split(",")]
    pick_rng = np.random.default_rng(7)
    n_max = int(max(rates) * args.duration * 1.5 + 100)
    is_large = pick_rng.random(n_max) < 0.1
    which = np.where(is_large, pick_rng.integers(0, 4, n_max), pick_rng.integers(0, 64, n_max))

    def make_request(i):
        src = large[which[i]] if is_large[i] else small[which[i]]
        return dataclasses.replace(src, out={}, rec=None), src.P, src.S

    mean_pairs = float(np.mean([(large[w] if l else small[w]).P * (large[w] if l else small[w]).S
                                for l, w in zip(is_large[:2000], which[:2000])]))
    results = {m: [] for m in args.modes.split(",")}
    for mode in results:
        for rate in rates:
            if mode in ("continuous", "continuous_graph"):
                ex = serve.GpuExecutor(dev, graphs=mode == "continuous_graph")
                sched = serve.Scheduler(ex, budget, chunk_pairs=args.chunk_pairs, step_pairs=args.step_pairs,
                                        max_inflight=2, keep_results=False, admit_ahead=4 * args.step_pairs)
            else:
                ex = serve.GpuExecutor(dev, single_scene=True)
                sched = serve.Scheduler(ex, budget, chunk_pairs=None, max_active=1, max_inflight=1,
                                        keep_results=False)
            sched.start()
            r = serve.run_load(sched, make_request, rate, args.duration, warmup=0.5, seed=7, drain=15.0)
            sched.stop(timeout=30)
            torch.cuda.synchronize()
            print(f"[serve] {mode} rate {rate:g}: {json.dumps(r)}", file=sys.stderr, flush=True)
            results[mode].append(r)
    best = max((r for r in results.get("continuous", []) if r["p99_ms"] is not None and r["unfinished"] == 0),
               key=lambda r: r["throughput_rps"] or 0, default=None)
    return {
        "metric": "served fwd+bwd requests/s (continuous batching, Poisson arrivals)",
        "value": best["throughput_rps"] if best else None, "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "90% requests from the 64-scene distribution (P 5k..50k, S 32..256, n 4/6/8), "
                               "10% large (P 262144, S 512, n 8); Poisson arrivals, seed 7",
                   "duration_s": args.duration, "warmup_s": 0.5, "chunk_pairs": args.chunk_pairs,
                   "step_pairs": args.step_pairs, "memory_budget_gb": round(budget / 2**30, 1),
                   "mean_pairs_per_request": mean_pairs},
        "p50_ms": best["p50_ms"] if best else None, "p99_ms": best["p99_ms"] if best else None,
        "sweep": results,
    }


def bench_rgb(args):
    """Three colour channels sharing one visibility, body-like scene."""
    import numpy as np
    import torch

    import scenegen
    from paper_2104_00359_amd import _lib, ops, workmodel

    sc = scenegen.scene_body()
    C = args.channels
    ch = scenegen.colour_channels(sc, C, seed=5)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    n, k = int(sc["n_bands"]), args.k
    N, P, S = n * n, sc["points"].shape[0], sc["spheres"].shape[0]
    prm = _lib.params(n, 3.0, k, args.flags)

    def t(a):
        return torch.as_tensor(np.ascontiguousarray(a)).to(dev)

    pts, nrm, sph = t(sc["points"].T), t(sc["normals"].T), t(sc["spheres"])
    alb, lig, gB = t(ch["albedo"].T), t(ch["light"]), t(ch["grad_radiance"].T)
    vis = torch.empty(N, P, device=dev)
    saved = torch.empty(_lib.shv_saved_floats(P, prm), device=dev)
    rad = torch.empty(C, P, device=dev)
    gV, gN, gA = torch.empty(N, P, device=dev), torch.empty(3, P, device=dev), torch.empty(C, P, device=dev)
    gL, gP, gS = torch.empty(C, N, device=dev), torch.empty(3, P, device=dev), torch.empty(S, 4, device=dev)
    nb = max(_lib.shv_workspace_bytes(P, S, prm), _lib.shv_channels_workspace_bytes(P, C, prm))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    st = stream.cuda_stream

    def step():
        _lib.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, ws, nb, st)
        _lib.sh_shade_channels(vis, nrm, alb, lig, C, P, prm, rad, ws, nb, st)
        _lib.sh_shade_channels_backward(gB, vis, nrm, alb, lig, C, P, prm, gV, gN, gA, gL, ws, nb, st)
        _lib.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, gP, gS, ws, nb, st)

    ms, prof = timed(step, stream, args.warmup, args.steps, True)
    kernels = kernel_table(prof)
    roof = roofline(kernels, sampled_steps(args.steps),
                    lambda name: workmodel.kernel_work(name, n, k, P, S, channels=C))
    if roof is not None:
        roof["traffic"] = measured_traffic("rgb", roof["kernel"])
    return {
        "metric": METRIC, "value": P * S / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"body-like scene, {C} colour channels sharing one visibility: 20000 receivers x "
                               "128 spheres, 8 bands, k=4, fwd+bwd", "receivers": P, "spheres": S, "n_bands": n,
                   "n_squarings": k, "channels": C},
        "roofline": roof, "cpu_baseline": None, "kernels": finish_kernels(kernels),
    }


def bench_envmap(args):
    """Eq. 9 on a synthetic equirectangular HDR map."""
    import torch

    import scenegen
    from paper_2104_00359_amd import _lib, ops, workmodel

    H, W = (int(v) for v in args.map.lower().split("x"))
    C, n = args.channels, 8
    img_h = scenegen.envmap_image(seed=0, C=C, H=H, W=W)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    prm = _lib.params(n)
    img = torch.as_tensor(img_h).to(dev)
    out = torch.empty(C, n * n, device=dev)
    nb = _lib.shv_envmap_workspace_bytes(C, H, W, prm)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    st = stream.cuda_stream

    def step():
        _lib.sh_envmap_project(img, C, H, W, prm, out, ws, nb, st)

    ms, prof = timed(step, stream, args.warmup, args.steps, True)
    kernels = kernel_table(prof)
    pixels = C * H * W
    roof = roofline(kernels, sampled_steps(args.steps),
                    lambda name: workmodel.kernel_work(name, n, 0, 0, 0, pixels=pixels))
    cpu = None
    if args.cpu_seconds > 0:
        from oracle import sh
        t0 = time.perf_counter()
        reps = 0
        small = img_h[:, :H // 4]          # a quarter of the rows per repetition
        while time.perf_counter() - t0 < min(args.cpu_seconds, 10.0):
            sh.envmap_to_sh(small, n)
            reps += 1
        dt = time.perf_counter() - t0
        cpu = {"value": reps * small.size / dt, "unit": "pixels/s", "cores": torch.get_num_threads(),
               "kind": "oracle", "sample": f"{reps} projections of the map's first {H // 4} rows "
                                           f"({small.size} pixels), FP64, {dt:.1f} s"}
    return {
        "metric": "environment-map pixels projected/s", "value": pixels / (ms * 1e-3), "unit": "pixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"equirectangular map {C} x {H} x {W} -> {n} bands (Eq. 9)", "channels": C,
                   "rows": H, "cols": W, "n_bands": n},
        "roofline": roof, "cpu_baseline": cpu, "kernels": finish_kernels(kernels),
    }


def bench_inverse(args):
    """One gradient-descent iteration of the inverse problem, body-like scene."""
    import numpy as np
    import torch

    import scenegen
    from paper_2104_00359_amd import inverse, ops, workmodel

    sc = scenegen.scene_body()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    n, k = int(sc["n_bands"]), args.k
    P, S = sc["points"].shape[0], sc["spheres"].shape[0]
    K = int(np.ceil(4 * P / S))
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        graph = inverse.DeformGraph(sc["points"], sc["normals"], sc["spheres"], K, dev)
        rng = np.random.default_rng(0)
        true = np.zeros((S + 1, 6), np.float32)
        true[:S, :3] = rng.standard_normal((S, 3)) * 0.1
        true[:S, 3:] = rng.standard_normal((S, 3)) * 0.01
        make = inverse.InverseProblem(graph, sc["albedo"], sc["light"], np.zeros(P, np.float32), n, lr=0.0, init=true,
                                      n_squarings=k)
        make.step()
        target = make.rad.clone()
        ip = inverse.InverseProblem(graph, sc["albedo"], sc["light"], target, n, lr=1e-2, n_squarings=k)
    torch.cuda.synchronize()
    ms, prof = timed(ip.step, stream, args.warmup, args.steps, True)
    kernels = kernel_table(prof)
    roof = roofline(kernels, sampled_steps(args.steps), lambda name: workmodel.kernel_work(name, n, k, P, S))
    if roof is not None:
        roof["traffic"] = measured_traffic("inverse", roof["kernel"])
    return {
        "metric": METRIC, "value": P * S / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"inverse problem on the body-like scene: {P} receivers x {S} spheres, 8 bands, k={k}; "
                               f"one gradient-descent iteration (deformation with K={K}, render, loss, adjoints, "
                               "update)", "receivers": P, "spheres": S, "n_bands": n, "n_squarings": k, "K": K,
                   "iterations_per_s": 1e3 / ms, "lr": 1e-2},
        "roofline": roof, "cpu_baseline": None, "kernels": finish_kernels(kernels),
    }


IMAGE_LR = 1e-5


def bench_image(args):
    """One gradient-descent iteration of the image-space inverse problem
    (Eqs. 14-16): the mesh body scene rendered and rasterised at 512 x 512."""
    import numpy as np
    import torch

    import scenegen
    from paper_2104_00359_amd import inverse, ops, workmodel

    sc = scenegen.scene_mesh_body()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    n, k = int(sc["n_bands"]), args.k
    P, S = sc["points"].shape[0], sc["spheres"].shape[0]
    W, H, T = sc["width"], sc["height"], len(sc["faces"])
    K = int(np.ceil(4 * P / S))
    cam = (sc["camera"], W, H)
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        graph = inverse.DeformGraph(sc["points"], sc["normals"], sc["spheres"], K, dev)
        rng = np.random.default_rng(0)
        true = np.zeros((S + 1, 6), np.float32)
        true[:S, :3] = rng.standard_normal((S, 3)) * 0.1
        true[:S, 3:] = rng.standard_normal((S, 3)) * 0.01
        make = inverse.InverseProblem(graph, sc["albedo"], sc["light"], np.zeros((H, W), np.float32), n, lr=0.0,
                                      init=true, n_squarings=k, faces=sc["faces"], camera=cam)
        make.step()
        target = make.raster["image"].clone()
        # A small step: the image loss on this scene is stiff (receivers sit next to spheres of 0.9 R, where
        # the cap's t(s) is steep), and at 1e-2 the descent stretches the mesh within a few steps, which
        # would make the timed work drift with the trajectory; the work per iteration does not depend on
        # the step.
        ip = inverse.InverseProblem(graph, sc["albedo"], sc["light"], target, n, lr=IMAGE_LR, n_squarings=k,
                                    faces=sc["faces"], camera=cam)
    torch.cuda.synchronize()
    ms, prof = timed(ip.step, stream, args.warmup, args.steps, True)
    kernels = kernel_table(prof)
    roof = roofline(kernels, sampled_steps(args.steps), lambda name: workmodel.kernel_work(name, n, k, P, S))
    if roof is not None:
        roof["traffic"] = measured_traffic("image", roof["kernel"])
    return {
        "metric": METRIC, "value": P * S / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"image-space inverse problem on the mesh body scene: {P} vertices ({T} triangles) x "
                               f"{S} spheres, 8 bands, k={k}, {W} x {H} image; one gradient-descent iteration "
                               f"(deformation with K={K}, render, rasterise, image loss, adjoints, update)",
                   "receivers": P, "spheres": S, "triangles": T, "image": [H, W], "n_bands": n, "n_squarings": k,
                   "K": K, "iterations_per_s": 1e3 / ms, "lr": IMAGE_LR},
        "roofline": roof, "cpu_baseline": None, "kernels": finish_kernels(kernels),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this benchmark runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the single-GPU figure is whole-job throughput).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched64":
        out = bench_batched(args)
    elif args.workload == "serve":
        out = bench_serve(args)
    elif args.workload == "rgb":
        out = bench_rgb(args)
    elif args.workload == "envmap":
        out = bench_envmap(args)
    elif args.workload == "inverse":
        out = bench_inverse(args)
    elif args.workload == "image":
        out = bench_image(args)
    else:
        out = bench_single(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
