"""sh_render_forward_noalloc (scratch in a static device array, for callers
that cannot allocate) against sh_render_forward with a caller's workspace:
bit-identical outputs on two calls in a row, the second smaller than the
first (the array keeps the first call's contents), and sizes beyond the
array refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import lib, to_dev

pytestmark = pytest.mark.gpu


def _inputs(sc, dev):
    return (to_dev(np.ascontiguousarray(sc["points"].T)), to_dev(np.ascontiguousarray(sc["normals"].T)),
            to_dev(sc["albedo"]), to_dev(sc["spheres"]), to_dev(sc["light"]))


def _forward(L, sc, noalloc, with_saved=True):
    dev = torch.device("cuda", 0)
    P, S, n = sc["points"].shape[0], sc["spheres"].shape[0], int(sc["n_bands"])
    prm = L.params(n)
    pts, nrm, alb, sph, lig = _inputs(sc, dev)
    vis = torch.full((n * n, P), float("nan"), device=dev)
    rad = torch.full((P,), float("nan"), device=dev)
    saved = torch.full((L.shv_render_saved_floats(P, prm),), float("nan"), device=dev) if with_saved else None
    st = torch.cuda.current_stream().cuda_stream
    if noalloc:
        L.sh_render_forward_noalloc(pts, nrm, alb, sph, lig, P, S, prm, vis, rad, saved, L.nbytes(saved), st)
    else:
        nb = L.shv_workspace_bytes(P, S, prm)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        L.sh_render_forward(pts, nrm, alb, sph, lig, P, S, prm, vis, rad, saved, L.nbytes(saved), ws, nb, st)
    torch.cuda.synchronize()
    out = {"V": vis.cpu().numpy(), "B": rad.cpu().numpy()}
    if with_saved:
        out["saved"] = saved.cpu().numpy()
    return out


def test_noalloc_forward_equals_workspace_forward_on_two_calls():
    L = lib()
    from paper_2104_00359_amd import ops
    ops.ensure_init(torch.device("cuda", 0))
    big = scenegen.scene_random_shell(901, 30000, 96, 8)       # 2 sphere chunks: partials over most of the array
    small = scenegen.scene_random_shell(902, 1000, 40, 6)      # then a smaller call over the leftover contents
    for name, sc, with_saved in (("first (30000 x 96, n 8)", big, True), ("second (1000 x 40, n 6)", small, True),
                                 ("third (1000 x 40, n 6, no saved state)", small, False)):
        print(f"call {name}", flush=True)
        a = _forward(L, sc, True, with_saved)
        b = _forward(L, sc, False, with_saved)
        for key in a:   # bit patterns: the state's row padding is never written and keeps the NaN fill
            assert np.array_equal(a[key].view(np.uint32), b[key].view(np.uint32)), f"{name}: {key}"
        assert np.isfinite(a["B"]).all()


def test_noalloc_forward_refuses_sizes_beyond_its_scratch():
    L = lib()
    from paper_2104_00359_amd import ops
    ops.ensure_init(torch.device("cuda", 0))
    f = L.raw("sh_render_forward_noalloc")
    prm = L.params(8)
    ptr = 1 << 40                                            # never dereferenced: refused first
    P = 500_000                                              # 64 * 500000 * 4 bytes of partials > 96 MiB
    assert f(ptr, ptr, ptr, ptr, ptr, P, 100, ctypes.byref(prm), ptr, ptr, None, 0, None) == L.SHV_ERR_WORKSPACE
    assert "static scratch" in L.shv_last_error()
