"""Host-side checks of the C ABI library that need no GPU: it loads, exports
every entry point its header declares, sizes its buffers consistently and
rejects invalid parameters before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shvis.h")


@pytest.fixture(scope="module")
def L():
    from paper_2104_00359_amd import _lib
    return _lib


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sh[v]?_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("sh_visibility_forward", "sh_visibility_backward", "sh_shade", "sh_shade_backward", "shv_init"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(L.EXPORTED)


def test_status_strings(L):
    assert L.shv_status_string(0) == "ok"
    assert "workspace" in L.shv_status_string(-3)
    assert L.shv_status_string(12345) == "unknown status"


def test_saved_and_workspace_sizes(L):
    for n, k in ((4, 4), (8, 4), (8, 0), (6, 7)):
        prm = L.params(n, 3.0, k)
        assert L.shv_saved_floats(1000, prm) == (1 + k * n * n) * 1000
    prm = L.params(8)
    a = L.shv_workspace_bytes(20000, 128, prm)
    b = L.shv_workspace_bytes(20000, 256, prm)
    c = L.shv_workspace_bytes(40000, 128, prm)
    assert 0 < a <= b and a <= c and a % 256 == 0
    # V-sized scratch at least (the adjoint's weights live there)
    assert a >= 64 * 20000 * 4
    # exactly the render backward's carving at 20,000 x 128: the forward's
    # chunk partials (2 chunks x N x P), then the receiver-gradient partials
    # (4 adjoint chunks x 3 x P), the per-tile sphere partials (313 tiles x S
    # float4) and lighting partials (313 tiles x N), each region 256-aligned
    tiles = (20000 + 63) // 64
    assert a == 2 * 64 * 20000 * 4 + 4 * 3 * 20000 * 4 + tiles * 128 * 16 + tiles * 64 * 4
    assert L.shv_workspace_bytes(10, 10, L.params(9)) == 0
    assert L.shv_workspace_bytes(0, 0, prm) >= 0


def test_invalid_parameters_rejected_before_any_device_call(L):
    f = L.raw("sh_visibility_forward")
    st = None
    bad_bands = L.params(9)
    assert f(None, 10, None, 0, ctypes.byref(bad_bands), None, None, 0, None, 0, st) == L.SHV_ERR_UNSUPPORTED
    assert "n_bands" in L.shv_last_error()
    bad_k = L.params(4, 3.0, 13)
    assert f(None, 10, None, 0, ctypes.byref(bad_k), None, None, 0, None, 0, st) == L.SHV_ERR_UNSUPPORTED
    neg = L.params(4)
    assert f(None, -5, None, 0, ctypes.byref(neg), None, None, 0, None, 0, st) == L.SHV_ERR_INVALID_ARG
    bad_eps = L.params(4, -1.0)
    assert f(None, 10, None, 0, ctypes.byref(bad_eps), None, None, 0, None, 0, st) == L.SHV_ERR_INVALID_ARG
    # unknown bit; both layouts; quadrature or product with another flag; Taylor without an order, with
    # order 9, with a layout flag; an order without the Taylor flag
    for bad_flags in (32, 3, 5, 6, 9, 12, 16, 16 | (9 << 8), 16 | (2 << 8) | 1, 2 << 8):
        flags = L.shv_params(4, 4, 3.0, bad_flags)
        assert f(None, 10, None, 0, ctypes.byref(flags), None, None, 0, None, 0, st) == L.SHV_ERR_INVALID_ARG
    g = L.raw("sh_shade")
    assert g(None, None, None, None, 5, None, None, None, 0, st) == L.SHV_ERR_INVALID_ARG


def test_channel_and_envmap_workspace_sizes(L):
    prm = L.params(8)
    one = L.shv_channels_workspace_bytes(20000, 1, prm)
    three = L.shv_channels_workspace_bytes(20000, 3, prm)
    # per channel: M(L) (N^2 floats) and the tile partials of the lighting gradient
    assert one >= 64 * 64 * 4 + ((20000 + 63) // 64) * 64 * 4
    assert three >= 3 * 64 * 64 * 4 + 3 * ((20000 + 63) // 64) * 64 * 4 and three % 256 == 0
    for bad in (0, L.SHV_MAX_CHANNELS + 1, -1):
        assert L.shv_channels_workspace_bytes(100, bad, prm) == 0
    assert L.shv_channels_workspace_bytes(100, 1, L.params(9)) == 0
    e = L.shv_envmap_workspace_bytes(3, 256, 512, prm)
    assert e >= 3 * 256 * 64 * 4 and e % 256 == 0
    assert L.shv_envmap_workspace_bytes(3, L.SHV_MAX_ENVMAP_ROWS + 1, 8, prm) == 0
    assert L.shv_envmap_workspace_bytes(3, 8, L.SHV_MAX_ENVMAP_COLS + 1, prm) == 0
    assert L.shv_envmap_workspace_bytes(L.SHV_MAX_CHANNELS + 1, 8, 8, prm) == 0


def test_channel_and_envmap_arguments_rejected_before_any_device_call(L):
    st = None
    prm = L.params(4)
    f = L.raw("sh_shade_channels")
    for bad in (0, L.SHV_MAX_CHANNELS + 1):
        assert f(None, None, None, None, bad, 10, ctypes.byref(prm), None, None, 0, st) == L.SHV_ERR_INVALID_ARG
        assert "channels" in L.shv_last_error()
    b = L.raw("sh_shade_channels_backward")
    assert b(None, None, None, None, None, 0, 10, ctypes.byref(prm), None, None, None, None, None, 0,
             st) == L.SHV_ERR_INVALID_ARG
    assert b(None, None, None, None, None, 2, -1, ctypes.byref(prm), None, None, None, None, None, 0,
             st) == L.SHV_ERR_INVALID_ARG
    e = L.raw("sh_envmap_project")
    assert e(None, 1, -1, 8, ctypes.byref(prm), None, None, 0, st) == L.SHV_ERR_INVALID_ARG
    assert e(None, 1, 8, L.SHV_MAX_ENVMAP_COLS + 1, ctypes.byref(prm), None, None, 0, st) == L.SHV_ERR_INVALID_ARG
    assert "too large" in L.shv_last_error()
    assert e(None, 0, 8, 8, ctypes.byref(prm), None, None, 0, st) == L.SHV_ERR_INVALID_ARG
    assert e(None, 1, 8, 8, ctypes.byref(L.params(9)), None, None, 0, st) == L.SHV_ERR_UNSUPPORTED


def _fake_scene(L, P, S, n, k=4, flags=0, base=1 << 40):
    """A scene record with distinct, aligned fake device addresses (the table
    is packed on the host; nothing is dereferenced)."""
    r = L.shv_scene()
    addr = [base]

    def nxt():
        addr[0] += 1 << 24
        return addr[0]
    for name in ("points", "normals", "albedo", "spheres", "light", "grad_radiance", "vis", "radiance", "saved",
                 "grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light", "ws"):
        setattr(r, name, nxt())
    prm = L.params(n, 3.0, k, flags)
    r.ws_bytes = L.shv_workspace_bytes(P, S, prm)
    r.saved_bytes = 4 * L.shv_render_saved_floats(P, prm)
    r.P, r.S, r.params = P, S, prm
    return r


def test_batch_table_packing_and_grid(L):
    """Host-side packing: block counts per group (exponential: 64 receivers
    per block in the four-wave layout, the default at 7 and 8 bands, and 256
    in the one-wave layout, the default up to 6 bands or selected by flags)."""
    scenes = [_fake_scene(L, 3000, 40, 8), _fake_scene(L, 70000, 20, 4, flags=L.SHV_FLAG_EXP_ONE_WAVE),
              _fake_scene(L, 777, 37, 8),
              _fake_scene(L, 0, 5, 5), _fake_scene(L, 5000, 100, 8, flags=L.SHV_FLAG_EXP_ONE_WAVE)]
    n = len(scenes)
    buf = (ctypes.c_uint8 * L.shv_batch_table_bytes(n))()
    L.shv_batch_table_build(scenes, buf)
    g = L.shv_batch_table_grid(buf)
    exp_four = np.ctypeslib.as_array(g.exp)[1]
    exp_one = np.ctypeslib.as_array(g.exp)[0]
    assert exp_four[8] == (3000 + 63) // 64 + (777 + 63) // 64
    assert exp_one[8] == (5000 + 255) // 256
    assert exp_one[4] == (70000 + 255) // 256 and exp_four[4] == 0
    assert exp_four[5] == 0 and exp_one[5] == 0 and np.ctypeslib.as_array(g.pair_fwd)[5] == 0
    six = [_fake_scene(L, 3000, 40, 6), _fake_scene(L, 3000, 40, 6, flags=L.SHV_FLAG_EXP_FOUR_WAVES)]
    buf6 = (ctypes.c_uint8 * L.shv_batch_table_bytes(2))()
    L.shv_batch_table_build(six, buf6)
    g6 = L.shv_batch_table_grid(buf6)
    assert np.ctypeslib.as_array(g6.exp)[0][6] == (3000 + 255) // 256
    assert np.ctypeslib.as_array(g6.exp)[1][6] == (3000 + 63) // 64
    # pair items: receiver tiles x sphere chunks, the forward aiming at 2,048
    # waves and the adjoint at 4,096 (4 waves per tile), at least 8 spheres
    # per wave and at most 512 spheres per chunk
    def chunks(P, S, target):
        waves = 4 * ((P + 63) // 64)
        c = min(-(-target // waves), -(-S // 32))
        c = max(c, -(-S // 512), 1)
        return -(-S // -(-S // c))
    eight = [(3000, 40), (777, 37), (5000, 100)]
    pf, pb = np.ctypeslib.as_array(g.pair_fwd), np.ctypeslib.as_array(g.pair_bwd)
    assert pf[0] == 0 and pb[0] == 0
    assert pf[8] == sum((P + 63) // 64 * chunks(P, S, 2048) for P, S in eight)
    assert pb[8] == sum((P + 63) // 64 * chunks(P, S, 4096) for P, S in eight)
    assert pf[4] == (70000 + 63) // 64 and pb[4] == (70000 + 63) // 64
    # a 20,000 x 128 scene: 2 forward chunks, 4 adjoint chunks
    body = (ctypes.c_uint8 * L.shv_batch_table_bytes(1))()
    L.shv_batch_table_build([_fake_scene(L, 20000, 128, 8)], body)
    gb = L.shv_batch_table_grid(body)
    assert chunks(20000, 128, 2048) == 2 and chunks(20000, 128, 4096) == 4
    assert gb.pair_fwd[8] == 313 * 2 and gb.pair_bwd[8] == 313 * 4
    assert g.finalize > 0
    assert L.shv_batch_table_bytes(-1) == 0


def test_batch_table_validation_names_the_scene(L):
    good = _fake_scene(L, 100, 10, 4)
    bad = _fake_scene(L, 100, 10, 4)
    bad.ws_bytes = 16
    buf = (ctypes.c_uint8 * L.shv_batch_table_bytes(2))()
    with pytest.raises(RuntimeError, match="scene 1"):
        L.shv_batch_table_build([good, bad], buf)
    bad = _fake_scene(L, 100, 10, 9)
    with pytest.raises(RuntimeError, match="scene 0"):
        L.shv_batch_table_build([bad, good], buf)
    small = (ctypes.c_uint8 * 8)()
    with pytest.raises(RuntimeError, match="table has"):
        L.shv_batch_table_build([good], small)


def test_batch_receiver_range_validation(L):
    buf = (ctypes.c_uint8 * L.shv_batch_table_bytes(1))()
    for begin, end in ((100, 512), (0, 300), (512, 256), (0, 1100), (-256, 0)):
        r = _fake_scene(L, 1000, 10, 4)
        r.range_begin, r.range_end = begin, end
        with pytest.raises(RuntimeError, match="receiver range"):
            L.shv_batch_table_build([r], buf)
    for begin, end in ((0, 256), (256, 1000), (512, 512)):
        r = _fake_scene(L, 1000, 10, 4)
        r.range_begin, r.range_end = begin, end
        L.shv_batch_table_build([r], buf)
    r = _fake_scene(L, 1000, 10, 4, flags=L.SHV_FLAG_EXP_FOUR_WAVES)
    r.range_begin, r.range_end, r.defer_reductions = 256, 1000, 1
    L.shv_batch_table_build([r], buf)
    g = L.shv_batch_table_grid(buf)
    assert g.finalize == 0
    assert np.ctypeslib.as_array(g.exp)[1][4] == (1000 + 63) // 64 - 256 // 64
    r = _fake_scene(L, 1000, 10, 4)                   # 4 bands, batched: one receiver per lane by default
    r.range_begin, r.range_end = 256, 1000
    L.shv_batch_table_build([r], buf)
    g = L.shv_batch_table_grid(buf)
    assert np.ctypeslib.as_array(g.exp)[0][4] == (1000 + 255) // 256 - 256 // 256
    assert np.ctypeslib.as_array(g.exp)[1][4] == 0


def _attach_host(L, sc, K):
    P, S = sc["points"].shape[0], sc["spheres"].shape[0]
    v = np.ascontiguousarray(sc["points"].T.astype(np.float32))
    s = np.ascontiguousarray(sc["spheres"].astype(np.float32))
    out = dict(vert_ptr=np.zeros(P + 1, np.int32), vert_sph=np.zeros(S * K, np.int32),
               vert_w=np.zeros(S * K, np.float32), sph_vert=np.zeros(S * K, np.int32),
               sph_w=np.zeros(S * K, np.float32))
    L.shv_deform_graph_build(v, P, s, S, K, out["vert_ptr"], out["vert_sph"], out["vert_w"], out["sph_vert"],
                             out["sph_w"])
    return out


@pytest.mark.parametrize("P,S,K", [(300, 12, 40), (500, 7, 500), (64, 20, 3)])
def test_attachment_graph_matches_the_oracle_bit_for_bit(L, P, S, K):
    """The host builder's attachment (index work) equals the oracle's exactly;
    its FP32 weights are the oracle's FP64 weights rounded once."""
    import scenegen
    from oracle import deform
    sc = scenegen.scene_random_shell(P + S, P, S, 4)
    g = _attach_host(L, sc, K)
    idx, u = deform.attach(sc["points"], sc["spheres"][:, :3], K)
    w = deform.normalised_weights(idx, u, P)
    assert np.array_equal(g["sph_vert"].reshape(S, K), idx)
    assert np.array_equal(g["sph_w"].reshape(S, K), w.astype(np.float32))
    # the vertex-major view lists the same attachments, spheres ascending
    ptr = g["vert_ptr"]
    assert ptr[0] == 0 and ptr[-1] == S * K
    for j in range(P):
        ks = g["vert_sph"][ptr[j]:ptr[j + 1]]
        assert list(ks) == sorted(ks)
        for k, wj in zip(ks, g["vert_w"][ptr[j]:ptr[j + 1]]):
            q = list(idx[k]).index(j)
            assert wj == np.float32(w[k, q])


def test_deform_arguments_rejected_before_any_device_call(L):
    st = None
    z = np.zeros(16, np.float32)
    zi = np.zeros(16, np.int32)
    hp = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    f = L.raw("shv_deform_graph_build")
    assert f(hp(z), 4, hp(z), 1, 5, hp(zi), hp(zi), hp(z), hp(zi), hp(z)) == L.SHV_ERR_INVALID_ARG   # K > P
    assert f(hp(z), 4, hp(z), 0, 1, hp(zi), hp(zi), hp(z), hp(zi), hp(z)) == L.SHV_ERR_INVALID_ARG   # S = 0
    assert f(None, 4, hp(z), 1, 1, hp(zi), hp(zi), hp(z), hp(zi), hp(z)) == L.SHV_ERR_INVALID_ARG
    g = L.shv_deform_graph(1, 1, 1, 1, 1, 1, 1, 1, 10, 2, 11)                                          # K > P
    assert L.raw("sh_deform_forward")(ctypes.byref(g), None, None, None, None, None, 0, st) == L.SHV_ERR_INVALID_ARG
    assert "graph" in L.shv_last_error()
    assert L.raw("sh_deform_backward")(None, None, None, None, None, None, None, 0, st) == L.SHV_ERR_INVALID_ARG
    assert L.raw("sh_l2_loss")(None, None, 0, None, None, None, 0, st) == L.SHV_ERR_INVALID_ARG
    assert L.raw("sh_sgd_step")(None, None, -1, ctypes.c_float(0.1), st) == L.SHV_ERR_INVALID_ARG
    assert L.shv_deform_workspace_bytes(0, 5) == 0 and L.shv_deform_workspace_bytes(100, 5) > 0
    assert L.shv_l2_workspace_bytes(0) == 0 and L.shv_l2_workspace_bytes(1000) >= 4 * 4


def test_taylor_flags_and_saved_sizes(L):
    for K in (1, 3, 8):
        prm = L.params(4, 3.0, 2, L.SHV_FLAG_EXP_TAYLOR | L.SHV_FLAG_EXP_TAYLOR_ORDER(K))
        assert L.shv_saved_floats(100, prm) == (1 + (2 + K) * 16) * 100
        assert L.shv_workspace_bytes(100, 7, prm) == L.shv_workspace_bytes(100, 7, L.params(4, 3.0, 2))
    assert L.shv_saved_floats(100, L.params(4, 3.0, 2, L.SHV_FLAG_EXP_PRODUCT)) == 0


def test_raster_incidence_and_argument_checks(L):
    import ctypes
    import numpy as np
    rng = np.random.default_rng(0)
    V, T = 50, 80
    faces = rng.integers(0, V, size=(T, 3)).astype(np.int32)
    ptr = np.zeros(V + 1, np.int32)
    idx = np.zeros(3 * T, np.int32)
    L.shv_raster_incidence_build(faces, T, V, ptr, idx)
    flat = faces.reshape(-1)
    order = np.argsort(flat, kind="stable")                 # corners grouped by vertex, in corner order
    assert np.array_equal(idx, order.astype(np.int32))
    assert np.array_equal(ptr, np.concatenate([[0], np.cumsum(np.bincount(flat, minlength=V))]).astype(np.int32))
    bad = faces.copy()
    bad[7, 1] = V
    with pytest.raises(RuntimeError):
        L.shv_raster_incidence_build(bad, T, V, ptr, idx)
    assert L.shv_raster_workspace_bytes(V, T, 64, 48) >= T * (64 + 17 * 4)
    # the forward's scratch: 64-byte face records, then an 8-byte depth key per
    # pixel, 64-bit chunk offsets and 32-bit counts and offsets per tile (plus
    # one), the shared-list count and a pad word, 16 slots and 16 list
    # entries per face and the shared list
    for (v, t, w, h) in [(V, T, 64, 48), (100, 1, 1, 1), (5000, 9000, 1024, 600), (3, 1, 16384, 16384)]:
        tiles = ((w + 7) // 8) * ((h + 7) // 8)
        layout = 8 * w * h + 8 * (tiles + 1) + 4 * (2 * (tiles + 1) + 2 + 33 * t)
        assert L.shv_raster_workspace_bytes(v, t, w, h) >= 64 * t + layout, (v, t, w, h)
    assert L.shv_raster_workspace_bytes(-1, T, 64, 48) == 0
    assert L.shv_raster_workspace_bytes(V, T, 0, 48) == 0
    assert L.shv_raster_workspace_bytes(V, 1 << 26, 64, 48) == 0
    assert L.shv_raster_workspace_bytes(V, (1 << 26) - 1, 64, 48) > 0
    f = L.raw("sh_raster_forward")
    cam = L.camera(np.zeros((3, 4)), 0, 10)
    assert f(None, 3, None, 1, None, ctypes.byref(cam), None, None, None, 0, None) == L.SHV_ERR_INVALID_ARG
    cam = L.camera(np.full((3, 4), np.nan), 8, 8)
    assert f(None, 3, None, 1, None, ctypes.byref(cam), None, None, None, 0, None) == L.SHV_ERR_INVALID_ARG


def test_bench_state_buffer_covers_every_mode(L):
    """The benchmark's state buffer must hold what either path writes, for
    every flag combination it is run with (the Taylor state grows with K)."""
    import bench
    for P in (1, 777, 20000):
        for flags in (0, 1, 2, 4, 8, 16 | (1 << 8), 16 | (2 << 8), 16 | (8 << 8)):
            for k in (0, 4, 12):
                prm = L.params(8, 3.0, k, flags)
                n = bench.saved_buffer_floats(L, P, prm)
                assert n >= L.shv_saved_floats(P, prm) and n >= L.shv_render_saved_floats(P, prm)


# Modes of forming V and the state each one's forward keeps for the backward.
SAVED_MODES = {"squaring": 0, "quadrature": 4, "product": 8, "taylor2": 16 | (2 << 8)}


@pytest.mark.parametrize("mode", sorted(SAVED_MODES))
def test_undersized_saved_state_is_refused_before_any_device_call(L, mode):
    """Every entry point that writes or reads the forward's state takes its
    size and refuses a buffer one float short with SHV_ERR_WORKSPACE; the
    refusal comes before the device is queried (there is none here), so a
    wrong caller gets an error instead of an overrun on the GPU.  The product
    chain keeps no state (its buffer may be NULL); for it the undersized
    workspace is what is refused."""
    P, S = 1000, 20
    prm = L.params(4, 3.0, 4, SAVED_MODES[mode])
    ptr = 1 << 40                                   # aligned fake device addresses, never dereferenced
    floats = L.shv_saved_floats(P, prm)
    ws_bytes = L.shv_workspace_bytes(P, S, prm)
    fwd, bwd = L.raw("sh_visibility_forward"), L.raw("sh_visibility_backward")
    if mode == "product":
        assert floats == 0
        assert fwd(ptr, P, ptr, S, ctypes.byref(prm), ptr, None, 0, ptr, 0, None) in (L.SHV_ERR_NOT_INITIALIZED,
                                                                                      L.SHV_ERR_HIP)
        assert bwd(ptr, ptr, ptr, P, ptr, S, ctypes.byref(prm), None, 0, ptr, ptr, ptr, ws_bytes - 256,
                   None) == L.SHV_ERR_WORKSPACE
        return
    short = 4 * floats - 4
    assert fwd(ptr, P, ptr, S, ctypes.byref(prm), ptr, ptr, short, ptr, ws_bytes, None) == L.SHV_ERR_WORKSPACE
    assert "saved has" in L.shv_last_error()
    assert bwd(ptr, ptr, ptr, P, ptr, S, ctypes.byref(prm), ptr, short, ptr, ptr, ptr, ws_bytes,
               None) == L.SHV_ERR_WORKSPACE
    assert bwd(ptr, ptr, ptr, P, ptr, S, ctypes.byref(prm), None, 0, ptr, ptr, ptr, ws_bytes,
               None) == L.SHV_ERR_INVALID_ARG          # the backward needs the state
    # exactly the size passes the check (the call then stops at the missing device)
    assert fwd(ptr, P, ptr, S, ctypes.byref(prm), ptr, ptr, 4 * floats, ptr, ws_bytes, None) in (
        L.SHV_ERR_NOT_INITIALIZED, L.SHV_ERR_HIP)


def test_undersized_render_state_is_refused_before_any_device_call(L):
    P, S = 777, 33
    prm = L.params(8)
    ptr = 1 << 40
    floats = L.shv_render_saved_floats(P, prm)
    assert floats == (1 + 4 * 64) * P + 64 * 64
    ws_bytes = L.shv_workspace_bytes(P, S, prm)
    f, b = L.raw("sh_render_forward"), L.raw("sh_render_backward")
    short = 4 * floats - 4
    assert f(ptr, ptr, ptr, ptr, ptr, P, S, ctypes.byref(prm), ptr, ptr, ptr, short, ptr, ws_bytes,
             None) == L.SHV_ERR_WORKSPACE
    assert b(ptr, ptr, ptr, ptr, ptr, P, S, ctypes.byref(prm), ptr, ptr, short, ptr, ptr, ptr, ptr, ptr, ptr,
             ws_bytes, None) == L.SHV_ERR_WORKSPACE
    assert f(ptr, ptr, ptr, ptr, ptr, P, S, ctypes.byref(prm), ptr, ptr, ptr + 2, 4 * floats, ptr, ws_bytes,
             None) == L.SHV_ERR_INVALID_ARG             # misaligned state
    # the batch table checks each scene's state size too, and names the scene
    good = _fake_scene(L, 100, 10, 4)
    bad = _fake_scene(L, 100, 10, 4, base=1 << 41)
    bad.saved_bytes = good.saved_bytes - 4
    buf = (ctypes.c_uint8 * L.shv_batch_table_bytes(2))()
    L.shv_batch_table_build([good], buf)
    with pytest.raises(RuntimeError, match="scene 1: saved has"):
        L.shv_batch_table_build([good, bad], buf)


def test_graph_arguments_rejected_before_any_device_call(L):
    f = L.raw("shv_graph_create")
    out = ctypes.c_void_p()
    empty = L.shv_batch_grid()
    assert f(ctypes.byref(empty), 16, 0, ctypes.byref(out)) == L.SHV_ERR_INVALID_ARG      # no launch selected
    assert "no launch" in L.shv_last_error()
    g = L.shv_batch_grid()
    g.pair_fwd[8] = 4
    assert f(ctypes.byref(g), 0, 0, ctypes.byref(out)) == L.SHV_ERR_INVALID_ARG           # max_scenes
    assert f(ctypes.byref(g), 16, 6, ctypes.byref(out)) == L.SHV_ERR_INVALID_ARG          # unknown flags
    assert f(ctypes.byref(g), 16, 0, None) == L.SHV_ERR_INVALID_ARG
    g.pair_bwd[0] = 1
    assert f(ctypes.byref(g), 16, 0, ctypes.byref(out)) == L.SHV_ERR_INVALID_ARG          # 0 bands
    assert out.value is None
    assert L.raw("shv_graph_launch")(None, None, 0, None) == L.SHV_ERR_INVALID_ARG
    assert L.raw("shv_graph_destroy")(None) == L.SHV_OK
    s = L.raw("sh_solve_batched")
    assert s(None, ctypes.byref(g), None) == L.SHV_ERR_INVALID_ARG


def test_autograd_inputs_are_checked_before_the_library():
    """The autograd functions check shapes, dtypes and devices of every input
    themselves (the library sees bare pointers): a mismatch raises before any
    device call, naming the input."""
    import torch

    from paper_2104_00359_amd import ops
    P, S, n = 10, 3, 4
    ok = dict(points=torch.zeros(P, 3), normals=torch.ones(P, 3), albedo=torch.ones(P),
              spheres=torch.ones(S, 4), light=torch.zeros(n * n))
    bad = {"normals": torch.ones(P - 1, 3), "albedo": torch.ones(P, 1), "spheres": torch.ones(S, 3),
           "light": torch.zeros(n * n + 1), "points": torch.zeros(P, 4)}
    for name, t in bad.items():
        args = dict(ok, **{name: t})
        with pytest.raises(ValueError, match=name):
            ops.shade_sh(args["points"], args["normals"], args["albedo"], args["spheres"], args["light"], n)
    with pytest.raises(ValueError, match="floating-point"):
        ops.shade_sh(ok["points"], ok["normals"], torch.ones(P, dtype=torch.int32), ok["spheres"], ok["light"], n)
    with pytest.raises(RuntimeError, match="GPU only"):
        ops.shade_sh(ok["points"], ok["normals"], ok["albedo"], ok["spheres"], ok["light"], n)
    with pytest.raises(ValueError, match="spheres"):
        ops.visibility_sh(ok["points"], torch.ones(S, 3), n)
    with pytest.raises(ValueError, match="points"):
        ops.visibility_sh(torch.zeros(P, 2), ok["spheres"], n)
    C = 3
    with pytest.raises(ValueError, match="albedo"):
        ops.shade_sh_channels(ok["points"], ok["normals"], torch.ones(P, C - 1), ok["spheres"],
                              torch.zeros(C, n * n), n)
    with pytest.raises(ValueError, match="light"):
        ops.shade_sh_channels(ok["points"], ok["normals"], torch.ones(P, C), ok["spheres"],
                              torch.zeros(C, n * n - 1), n)
    with pytest.raises(ValueError, match="image"):
        ops.envmap_to_sh(torch.zeros(8), n)


def test_noalloc_forward_refuses_sizes_beyond_its_scratch_before_any_device_call(L):
    f = L.raw("sh_render_forward_noalloc")
    prm = L.params(8)
    ptr = 1 << 40
    # 500,000 receivers at 8 bands: 128 MB of partials, more than the static scratch holds
    assert f(ptr, ptr, ptr, ptr, ptr, 500_000, 100, ctypes.byref(prm), ptr, ptr, None, 0, None) == L.SHV_ERR_WORKSPACE
    assert "static scratch" in L.shv_last_error()
    assert L.SHV_NOALLOC_SCRATCH_BYTES == 96 << 20
    # a size that fits passes the check and stops at the missing device
    assert f(ptr, ptr, ptr, ptr, ptr, 300_000, 100, ctypes.byref(prm), ptr, ptr, None, 0, None) in (
        L.SHV_ERR_NOT_INITIALIZED, L.SHV_ERR_HIP)
