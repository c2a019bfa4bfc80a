"""Batched render path (one work table over many scenes) on the GPU:
bit-identical to single-scene calls, parity with the oracle on the 64-scene
workload, and replay of a captured graph for a new batch."""
import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import collect, rel_l2, rel_max, run_batched, run_oracle, run_render

pytestmark = pytest.mark.gpu

KEYS = ["V", "B", "grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light"]

# (seed, P, S, n, k, flags, outputs passed as NULL): mixed band counts, both
# exponential layouts (flags 1 forces the one-wave layout, 2 the four-wave one),
# empty scenes, ragged sizes and partial gradient requests.
MIX = [
    (11, 3000, 40, 8, 4, 0, ()),
    (12, 70000, 20, 4, 4, 1, ()),
    (13, 777, 37, 6, 2, 0, ()),
    (14, 0, 5, 5, 4, 0, ()),
    (15, 130, 0, 3, 4, 0, ()),
    (16, 5000, 100, 8, 4, 1, ()),
    (17, 1, 1, 1, 4, 0, ()),
    (18, 2000, 64, 7, 3, 2, ("grad_points", "grad_spheres", "grad_normals")),
    (19, 1000, 10, 2, 0, 0, ("grad_light",)),
    (20, 4100, 300, 8, 4, 0, ()),
    (21, 20000, 128, 8, 4, 0, ()),   # 2 forward and 4 adjoint sphere chunks
]


def _mix_scenes():
    scenes, cfgs = [], []
    for seed, P, S, n, k, flags, null in MIX:
        scenes.append(scenegen.scene_random_shell(seed, P, S, n))
        cfgs.append({"k": k, "flags": flags, "null": null})
    return scenes, cfgs


def _assert_same(a, b, what):
    for key in KEYS:
        if key in a or key in b:
            assert key in a and key in b, (what, key)
            assert a[key].shape == b[key].shape, (what, key)
            assert np.array_equal(a[key], b[key]), f"{what}: {key} differs (max {np.abs(a[key] - b[key]).max()})"


def test_batched_equals_single_scene_bitwise():
    scenes, cfgs = _mix_scenes()
    for seed, P, S, n, k, flags, null in MIX:
        print(f"scene seed={seed} P={P} S={S} n={n} k={k} flags={flags} null={null}", flush=True)
    got = run_batched(scenes, cfgs)
    for sc, c, g in zip(scenes, cfgs, got):
        ref = run_render(sc, sc["grad_radiance"], k=c["k"], flags=c["flags"], null=c["null"])
        _assert_same(g, ref, f"P={sc['points'].shape[0]} n={sc['n_bands']}")


def test_scene_without_cotangent_is_skipped_by_backward():
    a = scenegen.scene_random_shell(30, 900, 30, 6)
    b = scenegen.scene_random_shell(31, 500, 20, 4)
    b = dict(b)
    del b["grad_radiance"]
    got = run_batched([a, b])
    ref = run_render(a, a["grad_radiance"])
    _assert_same(got[0], ref, "scene with cotangent")
    fwd = run_render(dict(b, grad_radiance=np.zeros(500, np.float32)), np.zeros(500, np.float32))
    assert np.array_equal(got[1]["V"], fwd["V"]) and np.array_equal(got[1]["B"], fwd["B"])


def test_batched_64_scene_workload_vs_oracle_sampled():
    """The 64-scene workload (P 5k..50k, S 32..256, n in {4, 6, 8}) at full
    size; every scene is compared with the oracle on 24 sampled receivers,
    with the cotangent restricted to them (so sphere and lighting gradients
    are the oracle's sums over the sample)."""
    scenes, idxs = [], []
    for b in range(64):
        sc = dict(scenegen.scene_batched(b))
        P = sc["points"].shape[0]
        idx = np.sort(np.random.default_rng(1000 + b).choice(P, 24, replace=False))
        w = np.zeros(P, np.float32)
        w[idx] = sc["grad_radiance"][idx]
        sc["grad_radiance"] = w
        scenes.append(sc)
        idxs.append(idx)
    got = run_batched(scenes)
    worst = {}
    for b, (sc, idx, g) in enumerate(zip(scenes, idxs, got)):
        o = run_oracle(sc, sc["grad_radiance"][idx], idx=idx)
        errs = {"V": rel_l2(g["V"][idx], o["V"]), "B": rel_max(g["B"][idx], o["B"])}
        for key in ("grad_points", "grad_normals", "grad_albedo"):
            errs[key] = rel_l2(g[key][idx], o[key])
        for key in ("grad_spheres", "grad_light"):
            errs[key] = rel_l2(g[key], o[key])
        for key, e in errs.items():
            worst[key] = max(worst.get(key, 0.0), e)
            tol = 1e-5 if key in ("V", "B") else 1e-4
            assert e <= tol, f"scene {b} (P={sc['points'].shape[0]} S={sc['spheres'].shape[0]} " \
                             f"n={sc['n_bands']}): {key} {e:.3e}"
    print("worst over 64 scenes: " + " ".join(f"{k} {v:.2e}" for k, v in worst.items()))


def test_graph_replay_and_new_batch_in_same_table():
    """Batched forward + backward captured in one graph: every replay (with
    eager work between replays) equals the eager result bitwise; writing a
    new, smaller batch into the same device table and replaying the same
    graph gives that batch's eager results."""
    from paper_2104_00359_amd import batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    first = [scenegen.scene_random_shell(40 + i, P, S, n) for i, (P, S, n) in
             enumerate([(6000, 80, 8), (2500, 40, 6), (900, 200, 4), (70000, 16, 4)])]
    eager = run_batched(first)
    bufs = [batch.scene_buffers(sc, dev) for sc in first]
    rb = batch.RenderBatch(bufs, dev)
    torch.cuda.synchronize()
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up outside capture
        rb.forward(s)
        rb.backward(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rb.forward()
        rb.backward()
    for rep in range(3):
        for b in bufs:   # clobber outputs between replays
            for t in b.out.values():
                if t is not None and t.dtype == torch.float32:
                    t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for b, ref in zip(bufs, eager):
            _assert_same(collect(b), ref, f"replay {rep}")
    # a new batch with no more work per group, written into the same table
    second = [scenegen.scene_random_shell(60 + i, P, S, n) for i, (P, S, n) in
              enumerate([(5000, 60, 8), (2000, 40, 6), (800, 100, 4)])]
    eager2 = run_batched(second)
    bufs2 = [batch.scene_buffers(sc, dev) for sc in second]
    rb2 = batch.RenderBatch(bufs2, dev)
    for name in ("pair_fwd", "pair_bwd", "exp"):
        a, b = np.ctypeslib.as_array(getattr(rb2.grid, name)), np.ctypeslib.as_array(getattr(rb.grid, name))
        assert np.all(a <= b), name
    assert rb2.grid.finalize <= rb.grid.finalize
    assert rb2.table.numel() <= rb.table.numel()
    torch.cuda.synchronize()
    rb.table[:rb2.table.numel()].copy_(rb2.table)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for b, ref in zip(bufs2, eager2):
        _assert_same(collect(b), ref, "new batch")


def test_autograd_batched_matches_single_scene_autograd():
    from paper_2104_00359_amd import batch, ops
    dev = torch.device("cuda", 0)
    cases = [(70, 1500, 30, 8), (71, 900, 50, 4), (72, 2100, 12, 6)]
    scenes = [scenegen.scene_random_shell(s, P, S, n) for s, P, S, n in cases]

    def leaves(sc):
        return [torch.tensor(sc[key], device=dev, requires_grad=True)
                for key in ("points", "normals", "albedo", "spheres", "light")]
    batched_in = [leaves(sc) for sc in scenes]
    outs = batch.shade_sh_batched(*[[x[i] for x in batched_in] for i in range(5)],
                                  n_bands=[sc["n_bands"] for sc in scenes])
    loss = sum((o * torch.tensor(sc["grad_radiance"], device=dev)).sum() for o, sc in zip(outs, scenes))
    loss.backward()
    for sc, xs, o in zip(scenes, batched_in, outs):
        ys = leaves(sc)
        r = ops.shade_sh(*ys, n_bands=sc["n_bands"])
        (r * torch.tensor(sc["grad_radiance"], device=dev)).sum().backward()
        assert torch.equal(o.detach(), r.detach())
        for x, y in zip(xs, ys):
            assert torch.equal(x.grad, y.grad)


def test_receiver_ranges_reproduce_whole_scene_bitwise():
    """Scenes split into receiver ranges over several batched calls (ranges of
    different scenes mixed in one table, reductions deferred to each scene's
    last range) give the whole-scene results bit for bit."""
    from paper_2104_00359_amd import batch, ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    # scene 3 has 2 forward and 4 adjoint sphere chunks
    cases = [(80, 70000, 30, 6), (81, 5000, 100, 8), (82, 1000, 20, 4), (83, 20000, 128, 8)]
    scenes = [scenegen.scene_random_shell(s, P, S, n) for s, P, S, n in cases]
    refs = [run_render(sc, sc["grad_radiance"]) for sc in scenes]
    bufs = [batch.scene_buffers(sc, dev) for sc in scenes]
    for b in bufs:
        b.allocate(dev)
    cuts = {0: [0, 256, 20480, 40960, 70000], 1: [0, 2048, 2304, 5000], 2: [0, 1000], 3: [0, 4096, 12288, 20000]}
    calls = [[(0, 0), (1, 0), (3, 0)], [(0, 1), (2, 0)], [(0, 2), (1, 1), (3, 1)], [(1, 2), (0, 3), (3, 2)]]
    stream = torch.cuda.current_stream()
    for call in calls:
        recs = []
        for sc, j in call:
            c = cuts[sc]
            recs.append(bufs[sc].record(c[j], c[j + 1], defer=(j + 2 < len(c))))
            print(f"call: scene {sc} receivers [{c[j]}, {c[j + 1]}) defer={j + 2 < len(c)}", flush=True)
        tab = batch.Table(recs, dev)
        tab.forward(stream)
        tab.backward(stream)
    torch.cuda.synchronize()
    for b, ref in zip(bufs, refs):
        _assert_same(collect(b), ref, f"ranges P={b.P}")
