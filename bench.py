"""Benchmark: point-sphere pair evaluations per second, forward + backward.

Default workload (``--workload batched64``): 64 independent scenes (P ~
U{5k..50k}, S ~ U{32..256}, n ~ U{4, 6, 8}, seeds 100 + b; 270,399,872
pairs), resident in HBM.  One step = the batched forward + backward of all 64
(sh_solve_batched's launches) replayed from the library's HIP graph
(shv_graph_launch: table copy + one graph launch).  The timed steps carry no
profiling; per-kernel durations come from HIP events around every launch of
a separate window of eager sh_solve_batched steps on the same stream, after
the timed region.  The same line carries, as extra keys:

* ``sequential``: the 64 scenes through 64 single-scene sh_render_forward +
  sh_render_backward calls, eager;
* ``serve``: Poisson arrivals at 2,000 requests/s (90% from the 64-scene
  distribution, 10% at 262,144 receivers x 512 spheres) against the
  continuous-batching server (graph mode) and one request at a time, with
  throughput and p50 / p99 latency;
* ``body``: the body-like scene (20,000 receivers x 128 spheres, n = 8)
  through sh_render_forward / sh_render_backward;
* ``cpu_baseline``: the FP64 oracle on the host's cores, a process pool over
  receiver chunks (all cores and single core, forward and forward +
  backward), on a bounded seeded sample.

Other workloads (``--workload``): body, gbuffer (512 x 512 receivers x 256
spheres), icosphere, serve (a sweep of arrival rates), rgb, envmap, inverse,
image; ``--path separate`` and ``--flags`` select the separate entry points
and the other ways of forming V on the single-scene workloads.
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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched64",
                    choices=["batched64", "body", "gbuffer", "icosphere", "serve", "rgb", "envmap", "inverse",
                             "image"])
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="steps of the separate per-kernel timing window (0: steps / 4, at least 5)")
    ap.add_argument("--channels", type=int, default=3, help="rgb / envmap: colour channels")
    ap.add_argument("--map", default="512x1024", help="envmap: H x W of the equirectangular map")
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="total duration of the oracle CPU baseline's four timed legs (0 disables it)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-core CPU baseline (0: the CPUs this process may run on, at most 16)")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--path", default="render", choices=["render", "separate"])
    ap.add_argument("--flags", type=int, default=0,
                    help="shv_params.flags: 1 / 2 select the exponential's kernel layout; 4 selects the "
                         "quadrature exponential, 8 the direct product chain of Eq. 12, 16 | (K << 8) the "
                         "Taylor series of order K (different approximations; separate entry points only)")
    ap.add_argument("--no-graph", action="store_true",
                    help="batched64: time eager sh_solve_batched calls instead of graph launches")
    ap.add_argument("--no-extras", action="store_true",
                    help="batched64: leave out the serve, sequential and body legs (profiling runs)")
    ap.add_argument("--rates", default="100,200,500,1000,2000,5000",
                    help="serve: Poisson arrival rates (requests/s)")
    ap.add_argument("--duration", type=float, default=4.0, help="serve: seconds of arrivals per rate")
    ap.add_argument("--seed", type=int, default=7, help="serve: seed of the arrivals and the request mix")
    ap.add_argument("--chunk-pairs", type=int, default=32 << 20, help="serve: pair bound of a request range")
    ap.add_argument("--step-pairs", type=int, default=128 << 20, help="serve: pair bound of a step")
    ap.add_argument("--modes", default="continuous,one_at_a_time",
                    help="serve: scheduler modes to sweep (continuous = graph steps, continuous_eager, "
                         "one_at_a_time)")
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


def workload_scenes(name):
    """Host scenes of a workload (the CPU baseline's workers rebuild them from
    the same seeds)."""
    import scenegen
    if name == "batched64":
        return [scenegen.scene_batched(b) for b in range(64)]
    return [make_scene(name)[0]]


def saved_buffer_floats(lib, P, prm):
    """Floats of a state buffer that serves both the fused render entry points
    and the separate visibility ones (whose state grows with the Taylor
    order), so either path of bench_single can use it."""
    return max(lib.shv_render_saved_floats(P, prm), lib.shv_saved_floats(P, prm), 1)


# ---------------------------------------------------------------- CPU baseline
# The FP64 oracle timed on the host's cores: a pool of processes, one thread
# each, over chunks of 256 receivers (all spheres of the scene), cycling over
# the scenes; each scene contributes a fixed seeded subset of at most 8,192
# receivers (pairs/s is linear in the receiver count).

CPU_CHUNK = 256
CPU_SUBSET = 8192
_CPU = {}


def _cpu_init(workload, k, exp_mode):
    import torch
    torch.set_num_threads(1)
    _CPU.update(scenes=workload_scenes(workload), k=k, mode=exp_mode)


def _cpu_task(task):
    import numpy as np

    from oracle import method
    j, idx, backward = task
    sc = _CPU["scenes"][j]
    idx = np.asarray(idx)
    if backward:
        method.run_forward_backward(sc, sc["grad_radiance"][idx], n_squarings=_CPU["k"], idx=idx,
                                    exp_mode=_CPU["mode"])
    else:
        method.run_forward(sc, n_squarings=_CPU["k"], idx=idx, exp_mode=_CPU["mode"])
    return len(idx) * int(sc["spheres"].shape[0])


def _cpu_tasks(scenes, backward):
    """Chunks of each scene's seeded subset, scenes taken in turn."""
    import numpy as np
    per = []
    for i, sc in enumerate(scenes):
        P = sc["points"].shape[0]
        sub = np.sort(np.random.default_rng(123 + i).permutation(P)[:CPU_SUBSET])
        per.append([sub[a:a + CPU_CHUNK] for a in range(0, len(sub), CPU_CHUNK)])
    out = []
    for r in range(max(len(c) for c in per)):
        for j, chunks in enumerate(per):
            if r < len(chunks):
                out.append((j, chunks[r].tolist(), backward))
    return out


def _cpu_leg(pool, procs, tasks, seconds):
    """Pairs/s of the chunks completed: tasks are submitted while ``seconds``
    have not passed, at most two per process in flight, and the ones in flight
    at the deadline are finished and counted with the time they took."""
    import collections
    t0 = time.perf_counter()
    it = iter(tasks)
    inflight = collections.deque()

    def submit():
        task = next(it, None)
        if task is not None:
            inflight.append(pool.apply_async(_cpu_task, (task,)))

    for _ in range(2 * procs):
        submit()
    pairs, n = 0, 0
    while inflight:
        pairs += inflight.popleft().get()
        n += 1
        if time.perf_counter() - t0 < seconds:
            submit()
    dt = time.perf_counter() - t0
    return pairs / dt, n, dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, k, seconds, workers=0, exp_mode="squaring"):
    """The oracle's pairs/s on the host: forward + backward (autograd) on all
    cores is the reported value; single-core and forward-only figures are kept
    beside it."""
    import multiprocessing as mp

    scenes = workload_scenes(workload)
    avail = len(os.sched_getaffinity(0))
    nw = workers if workers > 0 else min(avail, 16)
    ctx = mp.get_context("spawn")
    legs = {}
    share = {"fwd_1": 0.15, "fwdbwd_1": 0.25, "fwd_all": 0.25, "fwdbwd_all": 0.35}
    for name, procs in (("1", 1), ("all", nw)):
        with ctx.Pool(procs, initializer=_cpu_init, initargs=(workload, k, exp_mode)) as pool:
            pool.map(_cpu_task, [(0, [0], False)] * procs)        # start-up (imports, scenes) not timed
            for kind, backward in (("fwd", False), ("fwdbwd", True)):
                tasks = _cpu_tasks(scenes, backward)
                rate, n, dt = _cpu_leg(pool, procs, tasks, seconds * share[f"{kind}_{name}"])
                legs[f"{kind}_{name}"] = {"pairs_per_s": rate, "chunks": n, "seconds": round(dt, 2)}
            pool.terminate()
    total = sum(s["points"].shape[0] for s in scenes)
    sub = sum(min(s["points"].shape[0], CPU_SUBSET) for s in scenes)
    return {"value": legs["fwdbwd_all"]["pairs_per_s"], "unit": "pairs/s", "cores": nw, "kind": "oracle",
            "sample": f"FP64 forward + autograd backward{'' if exp_mode == 'squaring' else f' ({exp_mode} mode)'}, "
                      f"{nw} processes x 1 thread over chunks of {CPU_CHUNK} receivers x all spheres, from a seeded "
                      f"subset of <= {CPU_SUBSET} receivers per scene ({sub} of {total} receivers over "
                      f"{len(scenes)} scene(s)), {legs['fwdbwd_all']['chunks']} chunks in "
                      f"{legs['fwdbwd_all']['seconds']} s",
            "cpu_model": cpu_model(), "cpus_available": avail,
            "forward_all_cores": legs["fwd_all"]["pairs_per_s"],
            "forward_single_core": legs["fwd_1"]["pairs_per_s"],
            "fwd_bwd_single_core": legs["fwdbwd_1"]["pairs_per_s"], "legs": legs}


# ---------------------------------------------------------------- timing

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
    """SHA-256 over the library's kernel sources and the C header: measured
    counter data is only quoted for the build it was taken on.  The probes
    (``*_probe.hip``) are measurement tools outside the library and are left
    out."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2104_00359_amd", "csrc")
    for f in sorted(x for x in os.listdir(d)
                    if (x.endswith((".h", ".hip")) and not x.endswith("_probe.hip")) or x == "gen_tables.py"):
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


LAST_STEPS = {}


def timed(step, stream, warmup, steps):
    """Average milliseconds per step over ``steps`` steps after ``warmup``
    (host clock, synchronised on both sides).  Nothing else runs in the timed
    region except one HIP event record per step on the stream (events created
    beforehand), whose spacing gives the per-step GPU times kept in
    LAST_STEPS (median, 10th / 90th percentile, min, max)."""
    import numpy as np
    import torch
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record(stream)
        for i in range(steps):
            step()
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(steps)])
    LAST_STEPS.clear()
    LAST_STEPS.update({"median": float(np.median(per)), "p10": float(np.percentile(per, 10)),
                       "p90": float(np.percentile(per, 90)), "min": float(per.min()), "max": float(per.max())})
    return (t1 - t0) * 1e3 / steps


def untimed_steps(step, stream, min_steps, min_seconds):
    """Steps for an untimed leg: at least ``min_steps``, and enough for about
    ``min_seconds`` of GPU work (measured on one step)."""
    import torch
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    return max(int(min_steps), int(min_seconds / max(dt, 1e-6)) + 1)


def profile_window(step, stream, steps):
    """Per-kernel report ({name: (launches, total ms)}) of ``steps`` further
    steps with a HIP event pair recorded around each launch on the launch
    stream (the event pool is created before the window)."""
    import torch

    from paper_2104_00359_amd import _lib
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        _lib.shv_profile_enable(True, capacity=1024)      # one step first, to count its launches
        step()
        _lib.shv_profile_enable(False)
        torch.cuda.synchronize()
        per_step = sum(c for c, _ in _lib.shv_profile_report().values())
        _lib.shv_profile_enable(True, capacity=per_step * steps + 64)
        for _ in range(steps):
            step()
        _lib.shv_profile_enable(False)
        torch.cuda.synchronize()
    return _lib.shv_profile_report()


PROFILE_SECONDS = 0.75   # GPU work of the per-kernel window (it also takes the GPU past its clock transients)


def timed_and_profiled(step, stream, args):
    """(ms per step of the unprofiled timed steps, per-kernel report of the
    separate window, steps in that window).  The window runs first, untimed,
    for at least PROFILE_SECONDS of GPU work."""
    n = args.profile_steps or untimed_steps(step, stream, max(args.steps // 4, 5), PROFILE_SECONDS)
    prof = profile_window(step, stream, n)
    return timed(step, stream, args.warmup, args.steps), prof, n


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


def bench_single(args, workload=None, with_cpu=True):
    import numpy as np
    import torch

    from paper_2104_00359_amd import _lib, ops, workmodel

    workload = workload or args.workload
    sc, desc = make_scene(workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    n = int(sc["n_bands"])
    N = n * n
    P = sc["points"].shape[0]
    S = sc["spheres"].shape[0]
    k = args.k
    flags = args.flags if workload == args.workload else 0
    path = args.path if workload == args.workload else "render"
    prm = _lib.params(n, 3.0, k, flags)

    def t(a):
        return torch.as_tensor(np.ascontiguousarray(a)).to(dev)

    pts, nrm = t(sc["points"].T), t(sc["normals"].T)
    alb, sph, lig = t(sc["albedo"]), t(sc["spheres"]), t(sc["light"])
    gB = t(sc["grad_radiance"])
    vis = torch.empty(N, P, device=dev)
    saved = torch.empty(saved_buffer_floats(_lib, P, prm), device=dev)
    sb = _lib.nbytes(saved)
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

    if path == "render":
        def step():
            _lib.sh_render_forward(pts, nrm, alb, sph, lig, P, S, prm, vis, rad, saved, sb, ws, nb, st)
            _lib.sh_render_backward(gB, pts, nrm, alb, sph, P, S, prm, vis, saved, sb, gP, gN, gA, gS, gL, ws, nb, st)
    else:
        def step():
            _lib.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, sb, ws, nb, st)
            _lib.sh_shade(vis, nrm, alb, lig, P, prm, rad, ws, nb, st)
            _lib.sh_shade_backward(gB, vis, nrm, alb, lig, P, prm, gV, gN, gA, gL, ws, nb, st)
            _lib.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, sb, gP, gS, ws, nb, st)

    ms, prof, nprof = timed_and_profiled(step, stream, args)
    step_ms = dict(LAST_STEPS)
    copy_calibration(args, dev, stream)
    kernels = kernel_table(prof)
    order = (flags >> 8) & 15 if flags & _lib.SHV_FLAG_EXP_TAYLOR else 0
    roof = roofline(kernels, nprof, lambda name: workmodel.kernel_work(name, n, k, P, S, order=order))
    if roof is not None:
        roof["traffic"] = measured_traffic(workload, roof["kernel"])
    mode = {4: "quadrature", 8: "product"}.get(flags, f"taylor{order}" if order else "squaring")
    cpu = (cpu_baseline(workload, k, args.cpu_seconds, args.cpu_workers, mode)
           if with_cpu and args.cpu_seconds > 0 else None)
    return {
        "metric": METRIC, "value": P * S / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "receivers": P, "spheres": S, "n_bands": n, "n_squarings": k, "eps": 3.0,
                   "entry_points": path, "visibility": mode},
        "roofline": roof, "cpu_baseline": cpu, "kernels": finish_kernels(kernels), "profiled_steps": nprof,
        "step_ms": step_ms,
    }


def serve_leg(args, rate, duration, modes):
    """Poisson arrivals at ``rate`` for ``duration`` seconds per scheduler mode;
    one result dict per mode."""
    import dataclasses

    import numpy as np
    import torch

    import scenegen
    from paper_2104_00359_amd import batch, serve

    dev = torch.device("cuda", 0)
    small = [batch.scene_buffers(scenegen.scene_batched(b), dev) for b in range(64)]
    large = [batch.scene_buffers(scenegen.large_request_scene(500 + i), dev) for i in range(4)]
    free, _ = torch.cuda.mem_get_info(dev)
    budget = int(free - (16 << 30))
    seed = getattr(args, "seed", 7)
    pick_rng = np.random.default_rng(seed)
    n_max = int(rate * duration * 1.5 + 100)
    is_large = pick_rng.random(n_max) < 0.1
    which = np.where(is_large, pick_rng.integers(0, 4, n_max), pick_rng.integers(0, 64, n_max))

    def make_request(i):
        src = large[which[i]] if is_large[i] else small[which[i]]
        return dataclasses.replace(src, out={}, rec=None), src.P, src.S

    mean_pairs = float(np.mean([(large[w] if l else small[w]).P * (large[w] if l else small[w]).S
                                for l, w in zip(is_large[:2000], which[:2000])]))
    out = {}
    for mode in modes:
        if mode in ("continuous", "continuous_eager"):
            ex = serve.GpuExecutor(dev, graphs=mode == "continuous")
            sched = serve.Scheduler(ex, budget, chunk_pairs=args.chunk_pairs, step_pairs=args.step_pairs,
                                    max_inflight=2, keep_results=False, admit_ahead=4 * args.step_pairs)
        else:
            ex = serve.GpuExecutor(dev, single_scene=True, graphs=False)
            sched = serve.Scheduler(ex, budget, chunk_pairs=None, max_active=1, max_inflight=1, keep_results=False)
        sched.start()
        r = serve.run_load(sched, make_request, rate, duration, warmup=0.5, seed=seed, drain=15.0)
        sched.stop(timeout=30)
        torch.cuda.synchronize()
        if ex.graph is not None:
            r["graph_steps"], r["eager_steps"] = ex.graph.graph_steps, ex.graph.eager_steps
        ex.close()
        print(f"[serve] {mode} rate {rate:g}: {json.dumps(r)}", file=sys.stderr, flush=True)
        out[mode] = r
    return out, budget, mean_pairs


def bench_batched(args):
    import torch

    import scenegen
    from paper_2104_00359_amd import _lib, batch, ops, workmodel

    # the host baseline first: its worker processes start before this one holds the GPU busy
    cpu = cpu_baseline("batched64", args.k, args.cpu_seconds, args.cpu_workers) if args.cpu_seconds > 0 else None
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ops.ensure_init(dev)
    k = args.k
    scenes = [scenegen.scene_batched(b) for b in range(64)]
    bufs = [batch.scene_buffers(sc, dev, n_squarings=k) for sc in scenes]
    rb = batch.RenderBatch(bufs, dev)
    records = [b.record() for b in bufs]
    pairs = rb.pairs
    stream = torch.cuda.Stream(device=dev)   # default priority
    st = stream.cuda_stream

    def eager():
        _lib.sh_solve_batched(rb.table, rb.grid, rb.tab._handle(stream))

    graph = None
    if args.no_graph:
        step, mode = eager, "eager sh_solve_batched calls"
    else:
        graph = _lib.shv_graph_create(rb.grid, len(records))

        def step():
            _lib.shv_graph_launch(graph, records, st)
        mode = "shv_graph_launch: table copy + one graph of all batched phases per step"
    # The untimed legs run first, for at least PROFILE_SECONDS of GPU work
    # (they also take the GPU past the clock transients of its first second
    # under load); then the warm-up and the timed steps.
    nprof = args.profile_steps or untimed_steps(eager, stream, max(args.steps // 4, 5), PROFILE_SECONDS)
    prof = profile_window(eager, stream, nprof)
    extras = {}
    if not args.no_extras:
        def sequential():
            for b in bufs:
                o, prm = b.out, b.params()
                wsb = o["ws"].numel()
                _lib.sh_render_forward(b.points, b.normals, b.albedo, b.spheres, b.light, b.P, b.S, prm, o["vis"],
                                       o["radiance"], o["saved"], _lib.nbytes(o["saved"]), o["ws"], wsb, st)
                _lib.sh_render_backward(b.grad_radiance, b.points, b.normals, b.albedo, b.spheres, b.P, b.S, prm,
                                        o["vis"], o["saved"], _lib.nbytes(o["saved"]), o["grad_points"],
                                        o["grad_normals"], o["grad_albedo"], o["grad_spheres"], o["grad_light"],
                                        o["ws"], wsb, st)
        nseq = max(args.steps // 5, 10)
        ms_seq = timed(sequential, stream, 2, nseq)
        ms_eager = timed(eager, stream, 2, max(args.steps // 5, 10))
        extras["sequential"] = {"ms_per_step": ms_seq, "value": pairs / (ms_seq * 1e-3), "steps": nseq,
                                "what": "64 x (sh_render_forward + sh_render_backward), eager"}
        extras["batched_eager"] = {"ms_per_step": ms_eager, "value": pairs / (ms_eager * 1e-3),
                                   "what": "sh_solve_batched, eager launches"}
    if graph is not None:
        # A new graph's first few launches are slower now and then (a few ms
        # each, measured); the steady state is what a serving loop sees, so an
        # untimed leg of graph launches comes before the warm-up.
        ngl = untimed_steps(step, stream, 30, 0.25)
        extras["graph_first_launches"] = {"steps": ngl, "ms_per_step": timed(step, stream, 0, ngl),
                                       "step_ms": dict(LAST_STEPS)}
    ms = timed(step, stream, args.warmup, args.steps)
    step_ms = dict(LAST_STEPS)
    copy_calibration(args, dev, stream)
    kernels = kernel_table(prof)
    desc = [(b.n_bands, k, b.P, b.S) for b in bufs]
    roof = roofline(kernels, nprof, lambda name: workmodel.batch_work(name, desc))
    if roof is not None:
        roof["traffic"] = measured_traffic("batched64", roof["kernel"])
    out = {
        "metric": METRIC, "value": pairs / (ms * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 independent scenes: P ~ U{5000..50000}, S ~ U{32..256}, n ~ U{4,6,8} "
                               "(seeds 100+b), k=4, eps=3, fwd+bwd with all five gradients, batched",
                   "scenes": 64, "pairs_per_step": pairs, "receivers": sum(b.P for b in bufs),
                   "n_squarings": k, "eps": 3.0, "launch": mode},
        "roofline": roof, "cpu_baseline": cpu, "kernels": finish_kernels(kernels), "profiled_steps": nprof,
        "step_ms": step_ms,
    }
    out.update(extras)
    if "sequential" in out:
        out["speedup_vs_sequential"] = out["sequential"]["ms_per_step"] / ms
    if graph is not None:
        torch.cuda.synchronize()
        _lib.shv_graph_destroy(graph)
    if not args.no_extras:
        res, budget, mean_pairs = serve_leg(args, 2000.0, 2.5, ["continuous", "one_at_a_time"])
        out["serve"] = {"rate_rps": 2000.0, "duration_s": 2.5, "warmup_s": 0.5, "memory_budget_gb":
                        round(budget / 2**30, 1), "mean_pairs_per_request": mean_pairs,
                        "requests": "90% from the 64-scene distribution, 10% at 262144 x 512 (n 8); Poisson, seed 7",
                        **{m: {key: r[key] for key in ("throughput_rps", "pairs_per_s", "p50_ms", "p99_ms",
                                                      "completed", "unfinished", "failed")} for m, r in res.items()}}
        body = bench_single(args, "body", with_cpu=False)
        out["body"] = {key: body[key] for key in ("value", "ms_per_step", "step_ms", "roofline", "kernels")}
        out["body"]["workload"] = body["config"]["workload"]
    return out


def bench_serve(args):
    """Poisson load against the continuous-batching server (graph steps, and
    eager steps with ``continuous_eager``) and against one request at a time
    (single-scene calls), per arrival rate."""
    import torch
    torch.cuda.set_device(0)
    rates = [float(r) for r in args.rates.split(",")]
    modes = args.modes.split(",")
    results = {m: [] for m in modes}
    budget = mean_pairs = None
    for rate in rates:
        res, budget, mean_pairs = serve_leg(args, rate, args.duration, modes)
        for m in modes:
            results[m].append(res[m])
    best = max((r for r in results.get("continuous", []) if r["p99_ms"] is not None and r["unfinished"] == 0),
               key=lambda r: r["throughput_rps"] or 0, default=None)
    return {
        "metric": "served fwd+bwd requests/s (continuous batching, Poisson arrivals)",
        "value": best["throughput_rps"] if best else None, "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "90% requests from the 64-scene distribution (P 5k..50k, S 32..256, n 4/6/8), "
                               f"10% large (P 262144, S 512, n 8); Poisson arrivals, seed {args.seed}",
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
    sb = _lib.nbytes(saved)
    rad = torch.empty(C, P, device=dev)
    gV, gN, gA = torch.empty(N, P, device=dev), torch.empty(3, P, device=dev), torch.empty(C, P, device=dev)
    gL, gP, gS = torch.empty(C, N, device=dev), torch.empty(3, P, device=dev), torch.empty(S, 4, device=dev)
    nb = max(_lib.shv_workspace_bytes(P, S, prm), _lib.shv_channels_workspace_bytes(P, C, prm))
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    st = stream.cuda_stream

    def step():
        _lib.sh_visibility_forward(pts, P, sph, S, prm, vis, saved, sb, ws, nb, st)
        _lib.sh_shade_channels(vis, nrm, alb, lig, C, P, prm, rad, ws, nb, st)
        _lib.sh_shade_channels_backward(gB, vis, nrm, alb, lig, C, P, prm, gV, gN, gA, gL, ws, nb, st)
        _lib.sh_visibility_backward(gV, vis, pts, P, sph, S, prm, saved, sb, gP, gS, ws, nb, st)

    ms, prof, nprof = timed_and_profiled(step, stream, args)
    kernels = kernel_table(prof)
    roof = roofline(kernels, nprof, lambda name: workmodel.kernel_work(name, n, k, P, S, channels=C))
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

    ms, prof, nprof = timed_and_profiled(step, stream, args)
    kernels = kernel_table(prof)
    pixels = C * H * W
    roof = roofline(kernels, nprof, lambda name: workmodel.kernel_work(name, n, 0, 0, 0, pixels=pixels))
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
    ms, prof, nprof = timed_and_profiled(ip.step, stream, args)
    kernels = kernel_table(prof)
    roof = roofline(kernels, nprof, lambda name: workmodel.kernel_work(name, n, k, P, S))
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
    ms, prof, nprof = timed_and_profiled(ip.step, stream, args)
    kernels = kernel_table(prof)
    roof = roofline(kernels, nprof, lambda name: workmodel.kernel_work(name, n, k, P, S))
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
