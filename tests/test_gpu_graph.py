"""Batched forward + backward as one library call (sh_solve_batched) and as a
HIP graph behind the C ABI (shv_graph_create / _launch / _destroy): every
launch equals the eager batched calls bit for bit, over several launches with
eager work between them, for batches larger and smaller than the one the
graph was captured with, for batches without some of its band counts (their
nodes disabled, then enabled again), on two streams, and with fixed captured
grids."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import collect, run_batched

pytestmark = pytest.mark.gpu

KEYS = ["V", "B", "grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light"]

# (seed, P, S, n): band counts 4, 6 and 8, ragged sizes
FIRST = [(40, 6000, 80, 8), (41, 2500, 40, 6), (42, 900, 200, 4), (43, 7000, 16, 4)]
BIGGER = [(60, 9000, 120, 8), (61, 5000, 60, 6), (62, 3100, 210, 4), (63, 20000, 32, 8), (64, 300, 5, 6)]
SMALLER = [(70, 700, 30, 8), (71, 256, 64, 4)]
ONLY8 = [(75, 3000, 50, 8), (76, 1100, 90, 8), (77, 20000, 128, 8)]  # the last: 2 forward, 4 adjoint chunks


def _scenes(spec):
    for s, P, S, n in spec:
        print(f"scene seed={s} P={P} S={S} n={n}", flush=True)
    return [scenegen.scene_random_shell(s, P, S, n) for s, P, S, n in spec]


def _buffers(scenes):
    from paper_2104_00359_amd import batch
    dev = torch.device("cuda", 0)
    bufs = [batch.scene_buffers(sc, dev) for sc in scenes]
    for b in bufs:
        b.allocate(dev)
    return bufs


def _clobber(bufs):
    for b in bufs:
        for t in b.out.values():
            if t is not None and t.dtype == torch.float32:
                t.fill_(float("nan"))


def _same(bufs, refs, what):
    for b, ref in zip(bufs, refs):
        got = collect(b)
        for key in KEYS:
            assert np.array_equal(got[key], ref[key]), f"{what}: {key} (P={b.P} S={b.S} n={b.n_bands})"


def _groups(*grids):
    """Groups present in any of the grids, each with its largest count."""
    from paper_2104_00359_amd import _lib
    g = _lib.shv_batch_grid()
    for gr in grids:
        for n in range(9):
            g.pair_fwd[n] = max(g.pair_fwd[n], gr.pair_fwd[n])
            g.pair_bwd[n] = max(g.pair_bwd[n], gr.pair_bwd[n])
            g.exp[0][n] = max(g.exp[0][n], gr.exp[0][n])
            g.exp[1][n] = max(g.exp[1][n], gr.exp[1][n])
        g.finalize = max(g.finalize, gr.finalize)
    return g


def test_solve_batched_equals_forward_then_backward():
    from paper_2104_00359_amd import _lib, batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    scenes = _scenes(FIRST)
    ref = run_batched(scenes)
    bufs = _buffers(scenes)
    tab = batch.Table([b.record() for b in bufs], dev)
    s = torch.cuda.current_stream()
    _lib.sh_solve_batched(tab.device, tab.grid, tab._handle(s))
    torch.cuda.synchronize()
    _same(bufs, ref, "sh_solve_batched")


@pytest.mark.parametrize("fixed", [False, True], ids=["exact-grids", "fixed-grids"])
def test_graph_launches_equal_eager_bitwise(fixed):
    from paper_2104_00359_amd import _lib, batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    batches = {name: _scenes(spec) for name, spec in (("first", FIRST), ("bigger", BIGGER), ("smaller", SMALLER),
                                                       ("only8", ONLY8))}
    refs = {name: run_batched(sc) for name, sc in batches.items()}
    bufs = {name: _buffers(sc) for name, sc in batches.items()}
    grids = {name: batch.Table([b.record() for b in bufs[name]], dev).grid for name in bufs}
    # exact grids: captured from the first batch's counts, larger batches fit by the per-launch update;
    # fixed grids: captured with room for every batch below
    groups = _groups(grids["first"]) if not fixed else _groups(*grids.values())
    if not fixed:
        assert any(grids["bigger"].pair_bwd[n] > grids["first"].pair_bwd[n] for n in range(9))
    flags = _lib.SHV_GRAPH_FIXED_GRID if fixed else 0
    g = _lib.shv_graph_create(groups, 16, flags)
    try:
        s1 = torch.cuda.Stream(device=dev)
        s2 = torch.cuda.Stream(device=dev)
        order = ["first", "first", "bigger", "smaller", "only8", "first", "only8", "bigger"]
        for i, name in enumerate(order):
            _clobber(bufs[name])
            st = s1 if i % 2 == 0 else s2        # consecutive launches alternate streams
            with torch.cuda.stream(st):
                _lib.shv_graph_launch(g, [b.record() for b in bufs[name]], st.cuda_stream)
                torch.zeros(1000, device=dev).add_(1.0)   # eager work between launches
            torch.cuda.synchronize()
            print(f"launch {i}: batch {name} on stream {1 + i % 2}", flush=True)
            _same(bufs[name], refs[name], f"launch {i} ({name})")
    finally:
        torch.cuda.synchronize()
        _lib.shv_graph_destroy(g)


def test_graph_refuses_a_batch_it_does_not_hold():
    """A batch that needs a group the graph was not captured with (here: 5
    bands), or with fixed grids more blocks than captured, is refused with
    SHV_ERR_UNSUPPORTED before anything is enqueued: the outputs keep their
    previous contents."""
    from paper_2104_00359_amd import _lib, batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    small = _buffers(_scenes(SMALLER))
    groups = batch.Table([b.record() for b in small], dev).grid
    other = _buffers(_scenes([(80, 1000, 20, 5)]))
    big = _buffers(_scenes(BIGGER[:1]))
    launch = _lib.raw("shv_graph_launch")
    for flags in (0, _lib.SHV_GRAPH_FIXED_GRID):
        g = _lib.shv_graph_create(groups, 8, flags)
        try:
            cases = [other] + ([big] if flags else [])
            for bufs in cases:
                _clobber(bufs)
                recs = [b.record() for b in bufs]
                arr = (_lib.shv_scene * len(recs))(*recs)
                st = launch(g, arr, len(recs), torch.cuda.current_stream().cuda_stream)
                assert st == _lib.SHV_ERR_UNSUPPORTED, _lib.shv_last_error()
                torch.cuda.synchronize()
                assert torch.isnan(bufs[0].out["radiance"]).all()
            assert _lib.raw("shv_graph_launch")(g, arr, 9, None) == _lib.SHV_ERR_INVALID_ARG   # > max_scenes
        finally:
            _lib.shv_graph_destroy(g)


def test_graph_launch_of_an_empty_batch_enqueues_nothing():
    """An empty batch disables every node and enqueues nothing (no error, no
    output touched); the next batch enables its groups again and matches the
    eager calls bit for bit."""
    from paper_2104_00359_amd import _lib, batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    scenes = _scenes(SMALLER)
    ref = run_batched(scenes)
    bufs = _buffers(scenes)
    g = _lib.shv_graph_create(batch.Table([b.record() for b in bufs], dev).grid, 8)
    try:
        st = torch.cuda.current_stream().cuda_stream
        _clobber(bufs)
        _lib.shv_graph_launch(g, [], st)
        torch.cuda.synchronize()
        assert torch.isnan(bufs[0].out["radiance"]).all()
        _lib.shv_graph_launch(g, [b.record() for b in bufs], st)
        torch.cuda.synchronize()
        _same(bufs, ref, "after an empty batch")
    finally:
        torch.cuda.synchronize()
        _lib.shv_graph_destroy(g)
