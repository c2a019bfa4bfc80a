"""Continuous-batching server on the GPU: requests served in a mix (batched
with others, large ones split into receiver ranges over several steps) give
exactly the results of the same request processed alone."""
import dataclasses
import time

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import collect, run_render

pytestmark = pytest.mark.gpu

KEYS = ["V", "B", "grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light"]


@pytest.mark.parametrize("graphs", [False, True], ids=["eager", "graphs"])
def test_served_in_mix_equals_alone_bitwise(graphs):
    from paper_2104_00359_amd import batch, serve
    dev = torch.device("cuda", 0)
    specs = [(90, 20000, 64, 8), (91, 70000, 16, 4), (92, 3000, 40, 6), (93, 800, 100, 8), (94, 5000, 32, 5),
             (95, 256, 7, 3)]
    pool = [scenegen.scene_random_shell(s, P, S, n) for s, P, S, n in specs]
    inputs = [batch.scene_buffers(sc, dev) for sc in pool]
    ex = serve.GpuExecutor(dev, graphs=graphs, bands=(3, 4, 5, 6, 8))
    sched = serve.Scheduler(ex, memory_budget=16 << 30, chunk_pairs=300_000, step_pairs=1_500_000, max_inflight=2,
                            record_steps=True)
    rng = np.random.default_rng(5)
    picks = rng.integers(0, len(pool), 40)
    futs = []
    # half the requests are queued before the loop starts (so steps are shared),
    # the rest arrive while it runs (newcomers join at step boundaries)
    for n, j in enumerate(picks):
        if n == 20:
            sched.start()
        futs.append(sched.submit(dataclasses.replace(inputs[j], out={}, rec=None), inputs[j].P, inputs[j].S))
        if n >= 20:
            time.sleep(rng.exponential(0.0005))
    reqs = [f.result(timeout=120) for f in futs]
    sched.stop(timeout=30)
    print(f"{sched.steps} steps; widest step {max(len(s) for s in sched.step_log)} ranges"
          + (f"; {ex.graph.graph_steps} from the graph, {ex.graph.eager_steps} eager" if graphs else ""),
          flush=True)
    if graphs:
        assert ex.graph.graph_steps > 0 and ex.graph.eager_steps == 0
    ex.close()
    assert any(len(step) > 1 for step in sched.step_log)                   # requests shared steps
    assert any(d for step in sched.step_log for *_, d in step)              # some were split into ranges
    alone = {}
    for i in rng.choice(len(picks), 32, replace=False):
        j = int(picks[i])
        if j not in alone:
            alone[j] = run_render(pool[j], pool[j]["grad_radiance"])
        got = collect(reqs[i].scene)
        for key in KEYS:
            assert np.array_equal(got[key], alone[j][key]), f"request {i} (scene {j}): {key}"
