"""ctypes binding of libshvis.so: argument marshalling only.

Every function here has the name of the C entry point it calls (see
include/shvis.h for the contract).  Tensor arguments are passed as device
pointers; a non-zero status raises ``RuntimeError`` with the library's error
text.  There is no fallback: if the shared library is missing the import
fails.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SHV_LIBRARY selects another build of the same library (the host-sanitized
# one of build_sanitized.py, for CPU tests); by default the in-tree product
# build is loaded.
LIB_PATH = os.environ.get("SHV_LIBRARY") or os.path.join(HERE, "libshvis.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_2104_00359_amd/build.py` (there is no non-HIP fallback)")

_lib = ctypes.CDLL(LIB_PATH)

SHV_OK = 0
SHV_ERR_INVALID_ARG = -1
SHV_ERR_UNSUPPORTED = -2
SHV_ERR_WORKSPACE = -3
SHV_ERR_NOT_INITIALIZED = -4
SHV_ERR_HIP = -5

EXPORTED = [
    "shv_init", "shv_status_string", "shv_last_error", "shv_saved_floats", "shv_workspace_bytes",
    "sh_visibility_forward", "sh_shade", "sh_shade_backward", "sh_visibility_backward",
    "shv_channels_workspace_bytes", "sh_shade_channels", "sh_shade_channels_backward",
    "shv_envmap_workspace_bytes", "sh_envmap_project",
    "shv_deform_graph_build", "shv_deform_workspace_bytes", "sh_deform_forward", "sh_deform_backward",
    "shv_raster_incidence_build", "shv_raster_workspace_bytes", "sh_raster_forward", "sh_raster_backward",
    "shv_l2_workspace_bytes", "sh_l2_loss", "sh_sgd_step",
    "shv_render_saved_floats", "sh_render_forward", "sh_render_forward_noalloc", "sh_render_backward",
    "shv_batch_table_bytes", "shv_batch_table_build", "shv_batch_table_grid",
    "sh_render_batched_forward", "sh_render_batched_backward", "sh_solve_batched",
    "shv_graph_create", "shv_graph_launch", "shv_graph_destroy",
    "shv_profile_enable", "shv_profile_report",
]

SHV_RANGE_ALIGN = 256
SHV_MAX_CHANNELS = 4
SHV_MAX_ENVMAP_ROWS = 65536
SHV_MAX_ENVMAP_COLS = 1048576
SHV_FLAG_EXP_ONE_WAVE = 1
SHV_FLAG_EXP_FOUR_WAVES = 2
SHV_FLAG_EXP_QUADRATURE = 4
SHV_FLAG_EXP_PRODUCT = 8
SHV_FLAG_EXP_TAYLOR = 16
SHV_MAX_TAYLOR_ORDER = 8
SHV_GRAPH_FIXED_GRID = 1
SHV_NOALLOC_SCRATCH_BYTES = 96 << 20


def SHV_FLAG_EXP_TAYLOR_ORDER(K):
    """Bits that carry the Taylor order K of SHV_FLAG_EXP_TAYLOR."""
    return (int(K) & 15) << 8


class shv_params(ctypes.Structure):
    _fields_ = [("n_bands", ctypes.c_int32), ("n_squarings", ctypes.c_int32),
                ("eps", ctypes.c_float), ("flags", ctypes.c_uint32)]


class shv_scene(ctypes.Structure):
    """One scene of a batched render (field order and types as in the C struct)."""
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "points", "normals", "albedo", "spheres", "light", "grad_radiance", "vis", "radiance", "saved")] + [
        ("saved_bytes", ctypes.c_size_t)] + [(name, ctypes.c_void_p) for name in (
        "grad_points", "grad_normals", "grad_albedo", "grad_spheres", "grad_light", "ws")] + [
        ("ws_bytes", ctypes.c_size_t), ("P", ctypes.c_int64), ("S", ctypes.c_int64), ("params", shv_params),
        ("range_begin", ctypes.c_int64), ("range_end", ctypes.c_int64), ("defer_reductions", ctypes.c_int32)]


class shv_deform_graph(ctypes.Structure):
    """Device pointers of an attachment graph (field order as in the C struct)."""
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "vertices", "normals", "spheres", "vert_ptr", "vert_sph", "vert_w", "sph_vert", "sph_w")] + [
        ("P", ctypes.c_int64), ("S", ctypes.c_int64), ("K", ctypes.c_int32)]


class shv_camera(ctypes.Structure):
    """Row-major 3 x 4 projection and the image size (as in the C struct)."""
    _fields_ = [("P", ctypes.c_float * 12), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


def camera(P, width, height):
    c = shv_camera()
    flat = [float(x) for row in P for x in row]
    if len(flat) != 12:
        raise ValueError("camera matrix must be 3 x 4")
    c.P[:] = flat
    c.width, c.height = int(width), int(height)
    return c


class shv_batch_grid(ctypes.Structure):
    """Block counts of the batched launches (see the C header)."""
    _fields_ = [("pair_fwd", ctypes.c_int64 * 9), ("pair_bwd", ctypes.c_int64 * 9), ("exp", (ctypes.c_int64 * 9) * 2),
                ("finalize", ctypes.c_int64)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_PRM = ctypes.POINTER(shv_params)

_sig = {
    "shv_init": (ctypes.c_int32, [ctypes.c_int]),
    "shv_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
    "shv_last_error": (ctypes.c_char_p, []),
    "shv_saved_floats": (_I64, [_I64, _PRM]),
    "shv_workspace_bytes": (_SZ, [_I64, _I64, _PRM]),
    "sh_visibility_forward": (ctypes.c_int32, [_P, _I64, _P, _I64, _PRM, _P, _P, _SZ, _P, _SZ, _P]),
    "sh_shade": (ctypes.c_int32, [_P, _P, _P, _P, _I64, _PRM, _P, _P, _SZ, _P]),
    "sh_shade_backward": (ctypes.c_int32, [_P, _P, _P, _P, _P, _I64, _PRM, _P, _P, _P, _P, _P, _SZ, _P]),
    "sh_visibility_backward": (ctypes.c_int32, [_P, _P, _P, _I64, _P, _I64, _PRM, _P, _SZ, _P, _P, _P, _SZ, _P]),
    "shv_channels_workspace_bytes": (_SZ, [_I64, ctypes.c_int, _PRM]),
    "sh_shade_channels": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_int, _I64, _PRM, _P, _P, _SZ, _P]),
    "sh_shade_channels_backward": (ctypes.c_int32, [_P, _P, _P, _P, _P, ctypes.c_int, _I64, _PRM, _P, _P, _P, _P,
                                                    _P, _SZ, _P]),
    "shv_envmap_workspace_bytes": (_SZ, [ctypes.c_int, _I64, _I64, _PRM]),
    "sh_envmap_project": (ctypes.c_int32, [_P, ctypes.c_int, _I64, _I64, _PRM, _P, _P, _SZ, _P]),
    "shv_deform_graph_build": (ctypes.c_int32, [_P, _I64, _P, _I64, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "shv_deform_workspace_bytes": (_SZ, [_I64, _I64]),
    "shv_raster_incidence_build": (ctypes.c_int32, [_P, _I64, _I64, _P, _P]),
    "shv_raster_workspace_bytes": (_SZ, [_I64, _I64, ctypes.c_int32, ctypes.c_int32]),
    "sh_raster_forward": (ctypes.c_int32, [_P, _I64, _P, _I64, _P, ctypes.POINTER(shv_camera), _P, _P, _P, _SZ, _P]),
    "sh_raster_backward": (ctypes.c_int32, [_P, _P, _I64, _P, _I64, _P, ctypes.POINTER(shv_camera), _P, _P, _P, _P,
                                            _P, _P, _SZ, _P]),
    "sh_deform_forward": (ctypes.c_int32, [ctypes.POINTER(shv_deform_graph), _P, _P, _P, _P, _P, _SZ, _P]),
    "sh_deform_backward": (ctypes.c_int32, [ctypes.POINTER(shv_deform_graph), _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "shv_l2_workspace_bytes": (_SZ, [_I64]),
    "sh_l2_loss": (ctypes.c_int32, [_P, _P, _I64, _P, _P, _P, _SZ, _P]),
    "sh_sgd_step": (ctypes.c_int32, [_P, _P, _I64, ctypes.c_float, _P]),
    "shv_render_saved_floats": (_I64, [_I64, _PRM]),
    "sh_render_forward": (ctypes.c_int32, [_P, _P, _P, _P, _P, _I64, _I64, _PRM, _P, _P, _P, _SZ, _P, _SZ, _P]),
    "sh_render_forward_noalloc": (ctypes.c_int32, [_P, _P, _P, _P, _P, _I64, _I64, _PRM, _P, _P, _P, _SZ, _P]),
    "sh_render_backward": (ctypes.c_int32, [_P, _P, _P, _P, _P, _I64, _I64, _PRM, _P, _P, _SZ, _P, _P, _P, _P, _P,
                                            _P, _SZ, _P]),
    "shv_batch_table_bytes": (_SZ, [ctypes.c_int32]),
    "shv_batch_table_build": (ctypes.c_int32, [ctypes.POINTER(shv_scene), ctypes.c_int32, _P, _SZ]),
    "shv_batch_table_grid": (ctypes.c_int32, [_P, ctypes.POINTER(shv_batch_grid)]),
    "sh_render_batched_forward": (ctypes.c_int32, [_P, ctypes.POINTER(shv_batch_grid), _P]),
    "sh_render_batched_backward": (ctypes.c_int32, [_P, ctypes.POINTER(shv_batch_grid), _P]),
    "sh_solve_batched": (ctypes.c_int32, [_P, ctypes.POINTER(shv_batch_grid), _P]),
    "shv_graph_create": (ctypes.c_int32, [ctypes.POINTER(shv_batch_grid), ctypes.c_int32, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "shv_graph_launch": (ctypes.c_int32, [_P, ctypes.POINTER(shv_scene), ctypes.c_int32, _P]),
    "shv_graph_destroy": (ctypes.c_int32, [_P]),
    "shv_profile_enable": (ctypes.c_int32, [ctypes.c_int, ctypes.c_int32]),
    "shv_profile_report": (_I64, [ctypes.c_char_p, _I64]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def params(n_bands: int, eps: float = 3.0, n_squarings: int = 4, flags: int = 0) -> shv_params:
    return shv_params(int(n_bands), int(n_squarings), float(eps), int(flags))


def ptr(t) -> int | None:
    """Device pointer of a tensor (None for None); ints pass through."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _check(status: int, what: str):
    if status != SHV_OK:
        msg = _lib.shv_last_error().decode()
        name = _lib.shv_status_string(status).decode()
        raise RuntimeError(f"{what}: {name} ({status}): {msg}")


def shv_status_string(status: int) -> str:
    return _lib.shv_status_string(int(status)).decode()


def shv_last_error() -> str:
    return _lib.shv_last_error().decode()


def shv_init(device: int) -> None:
    _check(_lib.shv_init(int(device)), "shv_init")


def shv_saved_floats(P: int, prm: shv_params) -> int:
    return int(_lib.shv_saved_floats(int(P), ctypes.byref(prm)))


def shv_workspace_bytes(P: int, S: int, prm: shv_params) -> int:
    return int(_lib.shv_workspace_bytes(int(P), int(S), ctypes.byref(prm)))


def raw(name: str):
    """The raw ctypes function (returns the status; used by error-path tests)."""
    return getattr(_lib, name)


def nbytes(t) -> int:
    """Size in bytes of a buffer argument (0 for None)."""
    if t is None:
        return 0
    return int(t.numel()) * int(t.element_size())


def sh_visibility_forward(points, P, spheres, S, prm, vis, saved, saved_bytes, ws, ws_bytes, stream):
    _check(_lib.sh_visibility_forward(ptr(points), int(P), ptr(spheres), int(S), ctypes.byref(prm), ptr(vis),
                                      ptr(saved), int(saved_bytes), ptr(ws), int(ws_bytes), stream),
           "sh_visibility_forward")


def sh_shade(vis, normals, albedo, light, P, prm, radiance, ws, ws_bytes, stream):
    _check(_lib.sh_shade(ptr(vis), ptr(normals), ptr(albedo), ptr(light), int(P), ctypes.byref(prm),
                         ptr(radiance), ptr(ws), int(ws_bytes), stream), "sh_shade")


def sh_shade_backward(grad_radiance, vis, normals, albedo, light, P, prm, grad_vis, grad_normals, grad_albedo,
                      grad_light, ws, ws_bytes, stream):
    _check(_lib.sh_shade_backward(ptr(grad_radiance), ptr(vis), ptr(normals), ptr(albedo), ptr(light), int(P),
                                  ctypes.byref(prm), ptr(grad_vis), ptr(grad_normals), ptr(grad_albedo),
                                  ptr(grad_light), ptr(ws), int(ws_bytes), stream), "sh_shade_backward")


def shv_channels_workspace_bytes(P: int, channels: int, prm: shv_params) -> int:
    return int(_lib.shv_channels_workspace_bytes(int(P), int(channels), ctypes.byref(prm)))


def sh_shade_channels(vis, normals, albedo, light, channels, P, prm, radiance, ws, ws_bytes, stream):
    _check(_lib.sh_shade_channels(ptr(vis), ptr(normals), ptr(albedo), ptr(light), int(channels), int(P),
                                  ctypes.byref(prm), ptr(radiance), ptr(ws), int(ws_bytes), stream),
           "sh_shade_channels")


def sh_shade_channels_backward(grad_radiance, vis, normals, albedo, light, channels, P, prm, grad_vis,
                               grad_normals, grad_albedo, grad_light, ws, ws_bytes, stream):
    _check(_lib.sh_shade_channels_backward(ptr(grad_radiance), ptr(vis), ptr(normals), ptr(albedo), ptr(light),
                                           int(channels), int(P), ctypes.byref(prm), ptr(grad_vis),
                                           ptr(grad_normals), ptr(grad_albedo), ptr(grad_light), ptr(ws),
                                           int(ws_bytes), stream), "sh_shade_channels_backward")


def shv_envmap_workspace_bytes(channels: int, H: int, W: int, prm: shv_params) -> int:
    return int(_lib.shv_envmap_workspace_bytes(int(channels), int(H), int(W), ctypes.byref(prm)))


def sh_envmap_project(image, channels, H, W, prm, light, ws, ws_bytes, stream):
    _check(_lib.sh_envmap_project(ptr(image), int(channels), int(H), int(W), ctypes.byref(prm), ptr(light),
                                  ptr(ws), int(ws_bytes), stream), "sh_envmap_project")


def shv_deform_graph_build(vertices, P, spheres, S, K, vert_ptr, vert_sph, vert_w, sph_vert, sph_w):
    """Host arrays (numpy, C-contiguous): vertices float32 [3][P], spheres
    float32 [S][4]; outputs int32 / float32 arrays of the documented sizes."""
    def hp(a):
        return ctypes.c_void_p(a.ctypes.data)
    _check(_lib.shv_deform_graph_build(hp(vertices), int(P), hp(spheres), int(S), int(K), hp(vert_ptr),
                                       hp(vert_sph), hp(vert_w), hp(sph_vert), hp(sph_w)), "shv_deform_graph_build")


def shv_raster_incidence_build(faces, T, V, inc_ptr, inc_idx):
    """Host arrays (numpy, C-contiguous): faces int32 [T][3]; outputs int32
    inc_ptr [V + 1] and inc_idx [3 T]."""
    def hp(a):
        return ctypes.c_void_p(a.ctypes.data)
    _check(_lib.shv_raster_incidence_build(hp(faces), int(T), int(V), hp(inc_ptr), hp(inc_idx)),
           "shv_raster_incidence_build")


def shv_raster_workspace_bytes(V: int, T: int, width: int, height: int) -> int:
    return int(_lib.shv_raster_workspace_bytes(int(V), int(T), int(width), int(height)))


def sh_raster_forward(vertices, V, faces, T, radiance, cam, image, face_id, ws, ws_bytes, stream):
    _check(_lib.sh_raster_forward(ptr(vertices), int(V), ptr(faces), int(T), ptr(radiance), ctypes.byref(cam),
                                  ptr(image), ptr(face_id), ptr(ws), int(ws_bytes), stream), "sh_raster_forward")


def sh_raster_backward(grad_image, vertices, V, faces, T, radiance, cam, face_id, inc_ptr, inc_idx, grad_radiance,
                       grad_vertices, ws, ws_bytes, stream):
    _check(_lib.sh_raster_backward(ptr(grad_image), ptr(vertices), int(V), ptr(faces), int(T), ptr(radiance),
                                   ctypes.byref(cam), ptr(face_id), ptr(inc_ptr), ptr(inc_idx), ptr(grad_radiance),
                                   ptr(grad_vertices), ptr(ws), int(ws_bytes), stream), "sh_raster_backward")


def shv_deform_workspace_bytes(P: int, S: int) -> int:
    return int(_lib.shv_deform_workspace_bytes(int(P), int(S)))


def sh_deform_forward(graph, params, points, normals, spheres, ws, ws_bytes, stream):
    _check(_lib.sh_deform_forward(ctypes.byref(graph), ptr(params), ptr(points), ptr(normals), ptr(spheres),
                                  ptr(ws), int(ws_bytes), stream), "sh_deform_forward")


def sh_deform_backward(graph, params, grad_points, grad_normals, grad_spheres, grad_params, ws, ws_bytes, stream):
    _check(_lib.sh_deform_backward(ctypes.byref(graph), ptr(params), ptr(grad_points), ptr(grad_normals),
                                   ptr(grad_spheres), ptr(grad_params), ptr(ws), int(ws_bytes), stream),
           "sh_deform_backward")


def shv_l2_workspace_bytes(n: int) -> int:
    return int(_lib.shv_l2_workspace_bytes(int(n)))


def sh_l2_loss(value, target, n, grad, loss, ws, ws_bytes, stream):
    _check(_lib.sh_l2_loss(ptr(value), ptr(target), int(n), ptr(grad), ptr(loss), ptr(ws), int(ws_bytes), stream),
           "sh_l2_loss")


def sh_sgd_step(x, grad, n, lr, stream):
    _check(_lib.sh_sgd_step(ptr(x), ptr(grad), int(n), float(lr), stream), "sh_sgd_step")


def sh_visibility_backward(grad_vis, vis, points, P, spheres, S, prm, saved, saved_bytes, grad_points, grad_spheres,
                           ws, ws_bytes, stream):
    _check(_lib.sh_visibility_backward(ptr(grad_vis), ptr(vis), ptr(points), int(P), ptr(spheres), int(S),
                                       ctypes.byref(prm), ptr(saved), int(saved_bytes), ptr(grad_points),
                                       ptr(grad_spheres), ptr(ws), int(ws_bytes), stream), "sh_visibility_backward")


def shv_render_saved_floats(P: int, prm: shv_params) -> int:
    return int(_lib.shv_render_saved_floats(int(P), ctypes.byref(prm)))


def sh_render_forward(points, normals, albedo, spheres, light, P, S, prm, vis, radiance, saved, saved_bytes, ws,
                      ws_bytes, stream):
    _check(_lib.sh_render_forward(ptr(points), ptr(normals), ptr(albedo), ptr(spheres), ptr(light), int(P), int(S),
                                  ctypes.byref(prm), ptr(vis), ptr(radiance), ptr(saved), int(saved_bytes), ptr(ws),
                                  int(ws_bytes), stream), "sh_render_forward")


def sh_render_forward_noalloc(points, normals, albedo, spheres, light, P, S, prm, vis, radiance, saved, saved_bytes,
                              stream):
    _check(_lib.sh_render_forward_noalloc(ptr(points), ptr(normals), ptr(albedo), ptr(spheres), ptr(light), int(P),
                                          int(S), ctypes.byref(prm), ptr(vis), ptr(radiance), ptr(saved),
                                          int(saved_bytes), stream), "sh_render_forward_noalloc")


def sh_render_backward(grad_radiance, points, normals, albedo, spheres, P, S, prm, vis, saved, saved_bytes,
                       grad_points, grad_normals, grad_albedo, grad_spheres, grad_light, ws, ws_bytes, stream):
    _check(_lib.sh_render_backward(ptr(grad_radiance), ptr(points), ptr(normals), ptr(albedo), ptr(spheres), int(P),
                                   int(S), ctypes.byref(prm), ptr(vis), ptr(saved), int(saved_bytes),
                                   ptr(grad_points), ptr(grad_normals), ptr(grad_albedo), ptr(grad_spheres),
                                   ptr(grad_light), ptr(ws), int(ws_bytes), stream), "sh_render_backward")


def shv_batch_table_bytes(n_scenes: int) -> int:
    return int(_lib.shv_batch_table_bytes(int(n_scenes)))


def shv_batch_table_build(scenes, table_host) -> None:
    """Pack the work table of ``scenes`` (a sequence of shv_scene) into the
    host buffer ``table_host`` (a writable ctypes buffer or bytearray-backed
    object exposing the buffer protocol, or a CPU tensor of uint8)."""
    n = len(scenes)
    arr = (shv_scene * max(n, 1))(*scenes)
    if hasattr(table_host, "data_ptr"):
        addr, size = table_host.data_ptr(), table_host.numel() * table_host.element_size()
    else:
        addr, size = ctypes.addressof(table_host), ctypes.sizeof(table_host)
    _check(_lib.shv_batch_table_build(arr, n, addr, size), "shv_batch_table_build")


def shv_batch_table_grid(table_host) -> shv_batch_grid:
    addr = table_host.data_ptr() if hasattr(table_host, "data_ptr") else ctypes.addressof(table_host)
    g = shv_batch_grid()
    _check(_lib.shv_batch_table_grid(addr, ctypes.byref(g)), "shv_batch_table_grid")
    return g


def sh_render_batched_forward(table_device, grid, stream):
    _check(_lib.sh_render_batched_forward(ptr(table_device), ctypes.byref(grid), stream),
           "sh_render_batched_forward")


def sh_render_batched_backward(table_device, grid, stream):
    _check(_lib.sh_render_batched_backward(ptr(table_device), ctypes.byref(grid), stream),
           "sh_render_batched_backward")


def sh_solve_batched(table_device, grid, stream):
    _check(_lib.sh_solve_batched(ptr(table_device), ctypes.byref(grid), stream), "sh_solve_batched")


def shv_graph_create(groups, max_scenes: int, flags: int = 0) -> int:
    """Handle (an opaque address) of a new graph of sh_solve_batched."""
    h = ctypes.c_void_p()
    _check(_lib.shv_graph_create(ctypes.byref(groups), int(max_scenes), int(flags), ctypes.byref(h)),
           "shv_graph_create")
    return h.value


def shv_graph_launch(graph: int, scenes, stream, unsupported_ok: bool = False) -> bool:
    """scenes: a sequence of shv_scene (host records).  With ``unsupported_ok``
    a batch the graph does not hold (SHV_ERR_UNSUPPORTED: nothing was
    enqueued) returns False instead of raising."""
    n = len(scenes)
    arr = (shv_scene * max(n, 1))(*scenes)
    st = _lib.shv_graph_launch(graph, arr, n, stream)
    if unsupported_ok and st == SHV_ERR_UNSUPPORTED:
        return False
    _check(st, "shv_graph_launch")
    return True


def shv_graph_destroy(graph: int) -> None:
    _check(_lib.shv_graph_destroy(graph), "shv_graph_destroy")


def shv_profile_enable(enable: bool, capacity: int = 4096, resume: bool = False) -> None:
    """Start (or with ``resume`` continue, without growing the event pool)
    recording per-launch events; False pauses."""
    mode = (2 if resume else 1) if enable else 0
    _check(_lib.shv_profile_enable(mode, 0 if resume else int(capacity)), "shv_profile_enable")


def shv_profile_report() -> dict:
    """{kernel name: (launches, total milliseconds)} after the stream drained."""
    need = _lib.shv_profile_report(None, 0)
    buf = ctypes.create_string_buffer(int(need))
    _lib.shv_profile_report(buf, int(need))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out
