"""The rasteriser (Eq. 14) and its adjoint through the C ABI against the
oracle's (oracle/raster.py) on the same inputs.

Bars: the face of every pixel is bit-exact (both sides take the coverage and
depth decisions in FP32 with one rounding per operation in the same order).
The values have fixed bars on every case: image max |dI| / max |I| <= 6e-4,
radiance gradient ||d|| / ||g|| <= 1e-4, vertex gradient <= 1.5e-3.

Grazing faces are excluded from the value bars, counted and reported, the
way contact pixels are on the G-buffer scene.  The projected pixel
coordinates (a few hundred pixels) carry about delta = 2e-5 px of FP32
rounding, which moves a face's barycentric weights by about delta * kappa,
kappa = (longest projected edge) / (projected area) in 1 / px.  The body
mesh's faces have kappa of about 1; a face seen almost edge-on has kappa in
the hundreds and weights that FP32 cannot hold to 1e-3.  Pixels whose face has
kappa > 32 / px (FP64 projection) are left out of the image metric and get a
zero cotangent on both sides for the gradient metrics: 7, 10 and 8 pixels of
the 100 x 90, 512 x 512 and 1024 x 600 body images, none of the stress scene.
The oracle's formulas in FP32 (its FP32 twin) against FP64 then give, on
those three images: image 1.8e-5 / 8.8e-5 / 2.0e-4, radiance gradient
1.3e-5 / 1.5e-5 / 2.2e-5, vertex gradient 3.0e-5 / 1.3e-4 / 2.7e-4: the bars
sit at 3x or more above the worst of them, and a kept face's weight error is
at most delta * 32 = 6.4e-4 of its value."""
import numpy as np
import pytest
import torch

import scenegen
from gpu_helpers import lib, rel_l2, rel_max, to_dev
from oracle import raster

pytestmark = pytest.mark.gpu


def run_raster(verts, faces, B, P, width, height, gI, inc_faces=None):
    L = lib()
    from paper_2104_00359_amd import ops
    dev = torch.device("cuda", 0)
    ops.ensure_init(dev)
    V, T = len(verts), len(faces)
    cam = L.camera(P, width, height)
    vt = to_dev(np.ascontiguousarray(verts.T))
    ft = to_dev(np.ascontiguousarray(faces, np.int32))
    bt = to_dev(B)
    img = torch.empty(height, width, device=dev)
    fid = torch.empty(height, width, dtype=torch.int32, device=dev)
    nb = L.shv_raster_workspace_bytes(V, T, width, height)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream().cuda_stream
    L.sh_raster_forward(vt, V, ft, T, bt, cam, img, fid, ws, nb, st)
    ptr = np.zeros(V + 1, np.int32)
    idx = np.zeros(max(3 * T, 1), np.int32)
    inc_faces = faces if inc_faces is None else inc_faces
    L.shv_raster_incidence_build(np.ascontiguousarray(inc_faces, np.int32), T, V, ptr, idx)
    gB = torch.empty(V, device=dev)
    gv = torch.empty(3, V, device=dev)
    L.sh_raster_backward(to_dev(gI), vt, V, ft, T, bt, cam, fid, to_dev(ptr), to_dev(idx), gB, gv, ws, nb, st)
    torch.cuda.synchronize()
    return fid.cpu().numpy(), img.cpu().numpy(), gB.cpu().numpy(), gv.t().cpu().numpy()


def twin_floor(verts, faces, B, P, fid, gI, oimg, ogB, ogv, keep):
    """The oracle's shading and its gradients evaluated in FP32 (the same
    formulas, FP32 tensors) against its FP64 values: the error that FP32
    arithmetic alone makes on this case (reported beside the GPU's)."""
    v = torch.as_tensor(np.asarray(verts, np.float32)).requires_grad_(True)
    b = torch.as_tensor(np.asarray(B, np.float32)).requires_grad_(True)
    img = raster.shade_pixels(v, faces, b, torch.as_tensor(np.asarray(P, np.float32)), fid)
    gv, gb = torch.autograd.grad((img * torch.as_tensor(np.asarray(gI, np.float32))).sum(), [v, b])
    return (rel_max(np.where(keep, img.detach().numpy(), 0), np.where(keep, oimg.numpy(), 0)),
            rel_l2(gb.numpy(), ogB.numpy()), rel_l2(gv.numpy(), ogv.numpy()))


KAPPA_MAX = 32.0     # 1 / px: faces above it are grazing
BAR_IMAGE, BAR_GRAD_RADIANCE, BAR_GRAD_VERTICES = 6e-4, 1e-4, 1.5e-3


def face_kappa(verts, faces, P):
    """Longest projected edge over projected area (1 / px) of every face, from
    the FP64 projection of the FP32 inputs (inf for a zero-area face)."""
    v = np.asarray(verts, np.float64)
    hom = np.concatenate([v, np.ones((len(v), 1))], 1) @ np.asarray(P, np.float32).astype(np.float64).T
    sx, sy = hom[:, 0] / hom[:, 2], hom[:, 1] / hom[:, 2]
    a, b, c = (np.asarray(faces)[:, i] for i in range(3))
    area = 0.5 * np.abs((sx[b] - sx[a]) * (sy[c] - sy[a]) - (sx[c] - sx[a]) * (sy[b] - sy[a]))
    edge = np.max(np.stack([np.hypot(sx[b] - sx[a], sy[b] - sy[a]), np.hypot(sx[c] - sx[b], sy[c] - sy[b]),
                            np.hypot(sx[a] - sx[c], sy[a] - sy[c])]), 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(area > 0, edge / area, np.inf)


def check(verts, faces, B, P, width, height, gI, max_grazing=0.01):
    ofid, oimg = raster.render(verts, faces, B, P, width, height)
    kappa = face_kappa(verts, faces, P) if len(faces) else np.zeros(0)
    grazing = (ofid >= 0) & (kappa[np.maximum(ofid, 0)] > KAPPA_MAX) if len(faces) else ofid < -1
    gI = np.where(grazing, 0, gI).astype(np.float32)   # grazing pixels: no cotangent on either side
    fid, img, gB, gv = run_raster(verts, faces, B, P, width, height, gI)
    assert np.array_equal(fid, ofid), f"{(fid != ofid).sum()} pixels differ"
    assert (fid >= 0).sum() > 0
    keep = ~grazing
    eI = rel_max(np.where(keep, img, 0), np.where(keep, oimg.numpy(), 0))
    ogB, ogv = raster.render_backward(verts, faces, B, P, ofid, gI)
    eB, ev = rel_l2(gB, ogB.numpy()), rel_l2(gv, ogv.numpy())
    tI, tB, tv = twin_floor(verts, faces, B, P, ofid, gI, oimg, ogB, ogv, keep)
    print(f"covered {(fid >= 0).sum()}  grazing (excluded) {grazing.sum()}  image {eI:.2e}  grad_radiance "
          f"{eB:.2e}  grad_vertices {ev:.2e}  (FP32 twin {tI:.2e} {tB:.2e} {tv:.2e})")
    assert grazing.sum() <= max_grazing * (fid >= 0).sum() + 1   # the rule leaves out a few pixels, not a region
    assert eI <= BAR_IMAGE and eB <= BAR_GRAD_RADIANCE and ev <= BAR_GRAD_VERTICES


def test_raster_small_image_with_ragged_tiles():
    """100 x 90 pixels (ragged 16 x 16 tiles) of the mesh body scene."""
    sc = scenegen.scene_mesh_body(width=100, height=90)
    rng = np.random.default_rng(4)
    B = rng.uniform(0.0, 2.0, len(sc["points"])).astype(np.float32)
    gI = rng.standard_normal((90, 100)).astype(np.float32)
    check(sc["points"], sc["faces"], B, sc["camera"], 100, 90, gI)


def test_raster_full_size_body():
    """The mesh body scene at 512 x 512: every pixel's face and value, both
    gradients."""
    sc = scenegen.scene_mesh_body()
    rng = np.random.default_rng(5)
    B = rng.uniform(0.0, 2.0, len(sc["points"])).astype(np.float32)
    check(sc["points"], sc["faces"], B, sc["camera"], sc["width"], sc["height"], sc["grad_image"])


def test_raster_wide_image_scans_in_several_segments():
    """1024 x 600 pixels: 9,600 tiles, so the tile-count scan runs three
    4,096-entry segments (the last partial) with a carry between them."""
    sc = scenegen.scene_mesh_body(width=1024, height=600)
    rng = np.random.default_rng(7)
    B = rng.uniform(0.0, 2.0, len(sc["points"])).astype(np.float32)
    check(sc["points"], sc["faces"], B, sc["camera"], sc["width"], sc["height"], sc["grad_image"])


@pytest.mark.parametrize("width,height", [(1, 1), (7, 3)])
def test_raster_tiny_images(width, height):
    """The whole body inside one tile smaller than 8 x 8: most of the 42,480
    faces miss every pixel centre or have an empty box, and a pixel's
    nearest face is found among thousands of candidates.  Every face is far
    below a pixel here (kappa well above 32 / px), so all covered pixels are
    grazing: the case checks the face map (bit-exact), not the values."""
    sc = scenegen.scene_mesh_body(width=width, height=height)
    rng = np.random.default_rng(9)
    B = rng.uniform(0.0, 2.0, len(sc["points"])).astype(np.float32)
    check(sc["points"], sc["faces"], B, sc["camera"], width, height, sc["grad_image"], max_grazing=1.0)


def test_raster_degenerate_faces():
    """A face behind the camera, a face with one corner behind it (its
    projection flips across the image), a zero-area face and a face with an
    index outside [0, V) are not drawn; the rest is unchanged (the oracle sees
    the invalid face as a zero-area one)."""
    sc = scenegen.scene_mesh_body(width=64, height=64)
    verts = sc["points"].copy()
    faces = sc["faces"].copy()
    eye_y = float(np.mean(sc["points"][:, 1])) + 4.0
    behind = np.array([[0.0, 10.0, 1.0], [0.2, 10.0, 1.0], [0.0, 10.0, 1.2]], np.float32)
    straddle = np.array([[-0.3, 0.0, 0.9], [0.3, 0.0, 0.9], [0.0, eye_y + 1.0, 1.1]], np.float32)
    verts = np.concatenate([verts, behind, straddle])
    n0 = len(verts) - 6
    extra = np.array([[n0, n0 + 1, n0 + 2], [5, 5, 7], [0, 1, 2], [n0 + 3, n0 + 4, n0 + 5]], np.int32)
    faces = np.concatenate([extra, faces])
    rng = np.random.default_rng(6)
    B = rng.uniform(0.0, 2.0, len(verts)).astype(np.float32)
    gI = rng.standard_normal((64, 64)).astype(np.float32)
    bad = faces.copy()
    bad[2] = [0, 1, len(verts) + 5]                    # index out of range: the kernel skips the face
    ref = faces.copy()
    ref[2] = [0, 0, 0]                                 # zero area: the oracle skips it
    fid, img, gB, gv = run_raster(verts, bad, B, sc["camera"], 64, 64, gI, inc_faces=ref)
    ofid, oimg = raster.render(verts, ref, B, sc["camera"], 64, 64)
    assert np.array_equal(fid, ofid)
    assert not np.isin(fid, [0, 1, 2, 3]).any()
    assert rel_max(img, oimg.numpy()) <= 3e-4
    ogB, ogv = raster.render_backward(verts, ref, B, sc["camera"], ofid, gI)
    assert rel_l2(gB, ogB.numpy()) <= 1e-4 and rel_l2(gv, ogv.numpy()) <= 1.5e-3


def test_raster_empty_mesh_gives_a_black_image():
    verts = np.zeros((3, 3), np.float32)
    fid, img, gB, gv = run_raster(verts, np.zeros((0, 3), np.int32), np.ones(3, np.float32),
                                  scenegen.look_at_camera((0, 4, 0), (0, 0, 0), (0, 0, 1), 50, 32, 16), 32, 16,
                                  np.ones((16, 32), np.float32))
    assert (fid == -1).all() and not img.any() and not gB.any() and not gv.any()


def test_raster_stress_binning_and_depth_ties():
    """Faces spanning more than 16 tiles (the shared list, scanned by every
    tile), a tile list of more than eight 64-entry chunks, and exact depth
    ties with later twins of the same faces (the lower index wins): every
    pixel's face bit-exact, image and gradients to the usual bars."""
    sc = scenegen.scene_raster_stress()
    check(sc["points"], sc["faces"], sc["radiance"], sc["camera"], sc["width"], sc["height"], sc["grad_image"])
