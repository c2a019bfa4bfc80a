"""Continuous-batching server for forward + backward shadow solves.

Clients submit requests (a scene whose inputs are resident in device memory,
with the cotangent of its radiance) from any thread and get a future.  A
scheduler thread

* admits waiting requests in arrival order while their HBM footprint (inputs,
  outputs, saved state and workspace) fits the memory budget;
* packs one step from every admitted request with work left: its next
  receiver range, bounded by ``chunk_pairs`` receiver-sphere pairs, so a
  large request is spread over several steps and newcomers join at the next
  step boundary;
* launches the step (batched forward then backward of all its ranges) on the
  server stream, keeping up to ``max_inflight`` steps queued on the device so
  the host packs step t + 1 while step t runs;
* resolves a request's future once the step that holds its last range has
  completed, and returns its footprint to the budget.

Each request's results are bit-identical to the same request processed alone
(batched calls and receiver ranges reproduce a single-scene call exactly), so
the mix a request lands in never changes its answer.

The scheduler only talks to an ``Executor`` (footprint / admit / launch /
done / release); ``GpuExecutor`` drives the library, and tests substitute a
host-side fake.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

from . import _lib

RANGE_ALIGN = _lib.SHV_RANGE_ALIGN


@dataclass(eq=False)
class Request:
    scene: object                  # batch.SceneBuffers (inputs on the device) or an executor-specific object
    P: int
    S: int
    rid: int = 0
    arrival: float = 0.0           # time.perf_counter() at submission
    admitted: float = 0.0
    done: float = 0.0
    footprint: int = 0
    future: Future = field(default_factory=Future)

    @property
    def pairs(self) -> int:
        return self.P * self.S


def ranges_for(P: int, S: int, chunk_pairs: int | None) -> list:
    """Receiver ranges a request is processed in: the whole scene when it has
    at most ``chunk_pairs`` pairs (or chunking is off), else ranges of a
    multiple of RANGE_ALIGN receivers holding at most ``chunk_pairs`` pairs
    (at least RANGE_ALIGN receivers)."""
    if P == 0 or chunk_pairs is None or P * S <= chunk_pairs:
        return [(0, P)]
    step = max(RANGE_ALIGN, (chunk_pairs // max(S, 1)) // RANGE_ALIGN * RANGE_ALIGN)
    return [(a, min(a + step, P)) for a in range(0, P, step)]


class Executor:
    """Interface the scheduler drives."""

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def admit(self, req: Request) -> None:
        raise NotImplementedError

    def launch(self, items: list) -> object:
        """Enqueue one step; items = [(request, begin, end, defer_reductions)].
        Returns a token for ``done``."""
        raise NotImplementedError

    def done(self, token) -> bool:
        raise NotImplementedError

    def release(self, req: Request) -> None:
        pass


class StepGraph:
    """The batched forward + backward of a serving step replayed from one HIP
    graph of the library (shv_graph_create), captured once when the executor
    starts, never on the serving path.

    The graph holds the pair launches and the exponential launches of the
    band counts in ``bands`` (in the layout batched launches take by default:
    one receiver per lane up to 6 bands, four waves per 64 receivers above)
    and the closing reductions; each launch sets every node to the exact
    block count its step needs, so one graph serves steps of any size.  A
    step the graph does not hold (another band count or layout, more than
    ``max_scenes`` ranges) is launched eagerly instead and counted in
    ``eager_steps``."""

    def __init__(self, device, bands=(4, 6, 8), max_scenes: int = 1024):
        self.device = device
        self.max_scenes = int(max_scenes)
        groups = _lib.shv_batch_grid()
        for n in bands:
            groups.pair_fwd[int(n)] = 1
            groups.pair_bwd[int(n)] = 1
            groups.exp[0 if int(n) <= 6 else 1][int(n)] = 1
        groups.finalize = 1
        self.handle = _lib.shv_graph_create(groups, self.max_scenes)
        self.graph_steps = 0
        self.eager_steps = 0

    def run(self, records, stream_handle) -> bool:
        """Enqueue one step; False when the graph does not hold it (nothing
        was enqueued, the caller launches it eagerly)."""
        if len(records) > self.max_scenes:
            self.eager_steps += 1
            return False
        ok = _lib.shv_graph_launch(self.handle, records, stream_handle, unsupported_ok=True)
        if ok:
            self.graph_steps += 1
        else:
            self.eager_steps += 1
        return ok

    def close(self):
        if self.handle:
            _lib.shv_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # noqa: BLE001 - interpreter shutdown
            pass


class _Markers:
    """roctx ranges around serving steps (visible in rocprofv3 --marker-trace)
    when the ROCm tracer library is present; otherwise nothing is recorded."""

    def __init__(self):
        import ctypes
        import os
        self.lib = None
        for path in ("/opt/rocm/lib/libroctx64.so", "libroctx64.so"):
            if path.startswith("/") and not os.path.exists(path):
                continue
            try:
                lib = ctypes.CDLL(path)
                lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
                lib.roctxRangePushA.restype = ctypes.c_int
                lib.roctxRangePop.restype = ctypes.c_int
                self.lib = lib
                break
            except OSError:
                continue

    def push(self, text: str):
        if self.lib is not None:
            self.lib.roctxRangePushA(text.encode())

    def pop(self):
        if self.lib is not None:
            self.lib.roctxRangePop()


class GpuExecutor(Executor):
    """Steps as batched library calls on one stream (default priority).
    With ``graphs`` (the default) each step replays the library's HIP graph of
    the batched forward + backward (StepGraph, captured at construction for
    the band counts in ``bands``).  With ``single_scene`` a step holding one
    whole request goes through the single-scene entry points instead (the
    one-request-at-a-time baseline)."""

    def __init__(self, device, stream=None, single_scene: bool = False, graphs: bool = True, bands=(4, 6, 8),
                 max_scenes: int = 1024):
        import torch

        from .ops import ensure_init
        self.torch = torch
        self.device = torch.device(device)
        ensure_init(self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.single_scene = single_scene
        self.graph = StepGraph(self.device, bands, max_scenes) if graphs and not single_scene else None
        self.markers = _Markers()

    def footprint(self, req):
        return req.scene.device_bytes()

    def admit(self, req):
        req.scene.allocate(self.device)

    def launch(self, items):
        from .batch import Table
        torch = self.torch
        st = self.stream
        h = st.cuda_stream
        pairs = sum((e - a) * req.S for req, a, e, _ in items)
        self.markers.push(f"shv_step ranges={len(items)} pairs={pairs}")
        try:
            if self.single_scene and len(items) == 1 and items[0][1] == 0 and items[0][2] == items[0][0].P:
                b = items[0][0].scene
                o, prm = b.out, b.params()
                _lib.sh_render_forward(b.points, b.normals, b.albedo, b.spheres, b.light, b.P, b.S, prm, o["vis"],
                                       o["radiance"], o["saved"], _lib.nbytes(o["saved"]), o["ws"], o["ws"].numel(),
                                       h)
                _lib.sh_render_backward(b.grad_radiance, b.points, b.normals, b.albedo, b.spheres, b.P, b.S, prm,
                                        o["vis"], o["saved"], _lib.nbytes(o["saved"]), o["grad_points"],
                                        o["grad_normals"], o["grad_albedo"], o["grad_spheres"], o["grad_light"],
                                        o["ws"], o["ws"].numel(), h)
                tab = None
            else:
                recs = [req.scene.record(a, e, defer) for req, a, e, defer in items]
                tab = None
                if self.graph is None or not self.graph.run(recs, h):
                    tab = Table(recs, self.device, st)
                    _lib.sh_solve_batched(tab.device, tab.grid, tab._handle(st))
            ev = torch.cuda.Event()
            ev.record(st)
        finally:
            self.markers.pop()
        return ev, tab

    def done(self, token):
        return token[0].query()

    def close(self):
        if self.graph is not None:
            self.torch.cuda.synchronize(self.device)
            self.graph.close()


class Scheduler:
    """Continuous-batching scheduler (one host thread).

    memory_budget: bytes of device memory requests may occupy together.
    chunk_pairs:   pair bound of one request's range per step (None: whole
                   requests).
    step_pairs:    pair bound of a step (None: every admitted request with
                   work left contributes a range to every step).
    admit_ahead:   admit only while the admitted, not yet issued work is
                   below this many pairs (None: memory is the only bound);
                   keeps an overloaded server from holding memory for
                   requests many steps away.
    max_active:    bound on admitted requests (1 with chunk_pairs None is the
                   one-request-at-a-time baseline).
    keep_results:  False drops a request's device buffers when it completes
                   (load tests); the future then carries timings only.
    record_steps:  keep [(request id, begin, end, defer)] per launched step
                   in ``step_log``.
    """

    def __init__(self, executor: Executor, memory_budget: int, chunk_pairs: int | None = 8 << 20,
                 step_pairs: int | None = None, max_inflight: int = 2, max_active: int | None = None,
                 keep_results: bool = True, record_steps: bool = False, admit_ahead: int | None = None):
        self.ex = executor
        self.budget = int(memory_budget)
        self.chunk_pairs = chunk_pairs
        self.step_pairs = step_pairs
        self.max_inflight = max(1, int(max_inflight))
        self.max_active = max_active
        self.keep_results = keep_results
        self.admit_ahead = admit_ahead
        self._pending_pairs = 0                # admitted pairs not yet issued
        self.step_log = [] if record_steps else None
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._incoming = collections.deque()
        self._waiting = collections.deque()
        self._active = collections.deque()     # admitted, ranges left to issue
        self._inflight = collections.deque()   # (token, [requests finishing in that step], all requests)
        self._ranges = {}
        self.used = 0
        self.peak_used = 0
        self.steps = 0
        self._stop = False
        self._next_id = 0
        self._thread = None
        self.error = None

    # -- client side -------------------------------------------------------
    def submit(self, scene, P: int, S: int) -> Future:
        with self._lock:
            req = Request(scene=scene, P=int(P), S=int(S), rid=self._next_id, arrival=time.perf_counter())
            self._next_id += 1
            self._incoming.append(req)
            self._wake.notify()
        return req.future

    def start(self):
        self._thread = threading.Thread(target=self._run, name="shv-scheduler", daemon=True)
        self._thread.start()
        return self

    def stop(self, timeout: float | None = None):
        """Stop after the work already submitted has been completed (or
        ``timeout`` seconds have passed)."""
        with self._lock:
            self._stop = True
            self._wake.notify()
        if self._thread is not None:
            self._thread.join(timeout)

    def idle(self) -> bool:
        with self._lock:
            return not (self._incoming or self._waiting or self._active or self._inflight)

    # -- scheduler thread --------------------------------------------------
    def _fail(self, req: Request, exc: BaseException, release: bool):
        if release:
            self.used -= req.footprint
            try:
                self.ex.release(req)
            except Exception:   # noqa: BLE001 - the original failure is what the client needs
                pass
        if not req.future.done():
            req.future.set_exception(exc)

    def _admit(self):
        while self._waiting:
            if self.max_active is not None and len(self._active) + self._n_unfinished_inflight() >= self.max_active:
                return
            if self.admit_ahead is not None and self._active and self._pending_pairs >= self.admit_ahead:
                return
            req = self._waiting[0]
            if not req.footprint:
                try:
                    req.footprint = int(self.ex.footprint(req))
                except Exception as e:   # noqa: BLE001
                    self._waiting.popleft()
                    self._fail(req, e, release=False)
                    continue
            if req.footprint > self.budget:
                self._waiting.popleft()
                self._fail(req, MemoryError(f"request {req.rid} needs {req.footprint} bytes, "
                                            f"more than the whole budget of {self.budget}"), release=False)
                continue
            if self.used + req.footprint > self.budget:
                return   # arrival order: wait for memory
            self._waiting.popleft()
            try:
                self.ex.admit(req)
            except Exception as e:   # noqa: BLE001
                self._fail(req, e, release=False)
                continue
            self.used += req.footprint
            self.peak_used = max(self.peak_used, self.used)
            req.admitted = time.perf_counter()
            self._ranges[req.rid] = collections.deque(ranges_for(req.P, req.S, self.chunk_pairs))
            self._pending_pairs += req.pairs
            self._active.append(req)

    def _n_unfinished_inflight(self):
        return sum(len(fin) for _, fin, _ in self._inflight)

    def _plan(self):
        """One range from each admitted request with work left (arrival order,
        within the step bound); then, while the bound leaves room, requests
        extend their range over their next consecutive ranges (a merged range
        gives the same bits as its parts)."""
        picked, pairs = [], 0
        for req in self._active:
            rq = self._ranges[req.rid]
            a, e = rq[0]
            p = (e - a) * req.S
            if picked and self.step_pairs is not None and pairs + p > self.step_pairs:
                break
            rq.popleft()
            picked.append([req, a, e])
            pairs += p
            self._pending_pairs -= p
        if self.step_pairs is not None:
            for it in picked:
                req = it[0]
                rq = self._ranges[req.rid]
                while rq and rq[0][0] == it[2] and pairs + (rq[0][1] - rq[0][0]) * req.S <= self.step_pairs:
                    a, e = rq.popleft()
                    p = (e - a) * req.S
                    it[2] = e
                    pairs += p
                    self._pending_pairs -= p
        items, finishing = [], []
        for req, a, e in picked:
            last = not self._ranges[req.rid]
            items.append((req, a, e, not last))
            if last:
                finishing.append(req)
                self._active.remove(req)
                del self._ranges[req.rid]
        return items, finishing

    def _complete(self):
        progressed = False
        while self._inflight:
            token, finishing, everyone = self._inflight[0]
            if not self.ex.done(token):
                break
            self._inflight.popleft()
            now = time.perf_counter()
            for req in finishing:
                req.done = now
                self.used -= req.footprint
                self.ex.release(req)
                if not self.keep_results:
                    req.scene = None
                req.future.set_result(req)
            progressed = True
        return progressed

    def _run(self):
        try:
            while True:
                with self._lock:
                    while self._incoming:
                        self._waiting.append(self._incoming.popleft())
                    stop = self._stop
                    if stop and not (self._waiting or self._active or self._inflight):
                        return
                    if not (self._waiting or self._active or self._inflight):
                        self._wake.wait(0.05)
                        continue
                progressed = self._complete()
                self._admit()
                if self._active and len(self._inflight) < self.max_inflight:
                    items, finishing = self._plan()
                    try:
                        token = self.ex.launch(items)
                    except Exception as e:   # noqa: BLE001 - fail this step's requests, keep serving
                        failed = {id(r): r for r, *_ in items}
                        for req in failed.values():
                            if req in self._active:
                                self._active.remove(req)
                            left = self._ranges.pop(req.rid, None)
                            if left:
                                self._pending_pairs -= sum((b - a) * req.S for a, b in left)
                            self._fail(req, e, release=True)
                        continue
                    self.steps += 1
                    if self.step_log is not None:
                        self.step_log.append([(r.rid, a, e, d) for r, a, e, d in items])
                    self._inflight.append((token, finishing, [r for r, *_ in items]))
                    progressed = True
                if not progressed:
                    time.sleep(20e-6)
        except BaseException as e:   # noqa: BLE001 - surface scheduler crashes to every client
            self.error = e
            for q in (self._incoming, self._waiting, self._active):
                for req in q:
                    if not req.future.done():
                        req.future.set_exception(e)
            for _, _, everyone in self._inflight:
                for req in everyone:
                    if not req.future.done():
                        req.future.set_exception(e)
            raise


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from the start) of a Poisson process."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration * 1.5 + 50)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, n))])
    return t[t < duration]


def run_load(sched: Scheduler, make_request, rate: float, duration: float, warmup: float = 0.0, seed: int = 7,
             drain: float = 10.0) -> dict:
    """Submit requests at Poisson times for ``duration`` seconds; latency is
    arrival -> completion.  ``make_request(i)`` returns (scene, P, S).  Only
    requests arriving after ``warmup`` are measured; requests still
    unfinished ``drain`` seconds after the last arrival count as unfinished
    (their latency is infinite in the percentiles)."""
    times = poisson_arrivals(rate, duration, seed)
    futs = []
    t0 = time.perf_counter()
    for i, ta in enumerate(times):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        scene, P, S = make_request(i)
        futs.append((ta, P * S, sched.submit(scene, P, S)))
    deadline = time.perf_counter() + drain
    lat, pairs, unfinished, failed = [], 0, 0, 0
    first = last = None
    for ta, pq, f in futs:
        left = deadline - time.perf_counter()
        try:
            req = f.result(timeout=max(left, 0.0))
        except TimeoutError:
            if ta >= warmup:
                unfinished += 1
                lat.append(np.inf)
            continue
        except Exception:   # noqa: BLE001
            failed += 1
            continue
        if ta < warmup:
            continue
        lat.append(req.done - req.arrival)
        pairs += pq
        d = req.done - t0
        last = d if last is None else max(last, d)
        first = req.arrival - t0 if first is None else min(first, req.arrival - t0)
    lat = np.asarray(lat)
    done = int(np.isfinite(lat).sum())
    span = (last - first) if (first is not None and last is not None and last > first) else float("nan")

    def pct(q):
        if lat.size == 0:
            return None
        v = float(np.percentile(lat, q))
        return round(v * 1e3, 3) if np.isfinite(v) else None

    return {"rate": rate, "offered": int((times >= warmup).sum()), "completed": done, "unfinished": unfinished,
            "failed": failed, "throughput_rps": done / span if span == span else None,
            "pairs_per_s": pairs / span if span == span else None, "p50_ms": pct(50), "p99_ms": pct(99),
            "steps": sched.steps, "peak_mem_gb": round(sched.peak_used / 2**30, 3)}
