"""Seeded synthetic scene generators.

This module only builds inputs: receiver points, normals, albedo, sphere
occluders, lighting SH vectors and output cotangents.  It holds none of the
shadow method's arithmetic, so both the FP64 oracle tests and the GPU path can
consume the same arrays.

Every generator draws from ``numpy.random.default_rng(seed)`` (PCG64) in a
fixed, documented order, works in FP64 and returns FP32 arrays (the precision
the GPU path consumes).  The oracle promotes those FP32 arrays to FP64, so both
sides see bit-identical inputs.

Shapes of the returned scene dict:
  points  [P, 3]  receiver positions
  normals [P, 3]  unit outward normals
  albedo  [P]     diffuse albedo
  spheres [S, 4]  (cx, cy, cz, r)
  light   [n*n]   lighting SH vector, coefficient index l*l + l + m
  n_bands int
The scenes stand in for the paper's mesh / environment-map workloads (its
assets are not available); sizes follow the paper's setting of n = 8 bands and
tens to hundreds of spheres (Sec. 3.2, Sec. 4 ablation table).
"""
from __future__ import annotations

import math

import numpy as np

SHADOW_BIAS = 1e-3  # receivers on a surface are lifted this far along the normal


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def draw_light(rng, n_bands, dc=3.0):
    """Lighting SH: coefficient 0 set to ``dc``, the rest i.i.d. N(0, 1)."""
    L = rng.standard_normal(n_bands * n_bands)
    L[0] = dc
    return L


def draw_albedo(rng, P):
    return rng.uniform(0.2, 0.9, size=P)


# --------------------------------------------------------------------------
# receiver sets
# --------------------------------------------------------------------------

def icosphere(subdiv):
    """Vertices of an icosphere: 12-vertex icosahedron, ``subdiv`` midpoint
    splits, every vertex projected to the unit sphere.  subdiv = 4 gives 2,562."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
             (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
             (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = v[a] + v[b]
                v.append(m / np.linalg.norm(m))
                cache[key] = len(v) - 1
            return cache[key]

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    return np.stack(v)


def uniform_sphere_points(rng, P):
    d = rng.standard_normal((P, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def shell_spheres(rng, S, r_lo=0.05, r_hi=0.3, outer=2.0, margin=0.05):
    """Occluders around the unit receiver sphere: radii U[r_lo, r_hi], unit
    directions from normalised N(0, I3), centre distance rho with
    rho^3 ~ U[(1 + r + margin)^3, outer^3] (uniform in volume within the
    shell between the receiver surface plus a margin and ``outer``).
    Draw order: radii, directions, then the volume variate."""
    r = rng.uniform(r_lo, r_hi, size=S)
    d = rng.standard_normal((S, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u = rng.uniform(0.0, 1.0, size=S)
    lo = (1.0 + r + margin) ** 3
    rho = np.cbrt(lo + u * (outer ** 3 - lo))
    return np.concatenate([d * rho[:, None], r[:, None]], axis=1)


# --------------------------------------------------------------------------
# configuration scenes
# --------------------------------------------------------------------------

def scene_icosphere_shell(seed=0, subdiv=4, S=32, n_bands=4):
    """Parity scene: icosphere receivers (2,562 at subdiv 4, radius 1,
    outward normals) inside a shell of S spheres.  Draw order (one rng):
    sphere radii, directions, volume variates, light, albedo."""
    rng = np.random.default_rng(seed)
    pts = icosphere(subdiv)
    spheres = shell_spheres(rng, S)
    light = draw_light(rng, n_bands)
    albedo = draw_albedo(rng, pts.shape[0])
    return dict(points=_f32(pts), normals=_f32(pts), albedo=_f32(albedo),
                spheres=_f32(spheres), light=_f32(light), n_bands=n_bands)


def scene_random_shell(seed, P, S, n_bands):
    """Receivers uniform on the unit sphere (normals = positions) and S shell
    spheres.  Draw order: points, sphere radii, directions, volume variates,
    light, albedo, output cotangent w ~ N(0, 1) per point."""
    rng = np.random.default_rng(seed)
    pts = uniform_sphere_points(rng, P)
    spheres = shell_spheres(rng, S)
    light = draw_light(rng, n_bands)
    albedo = draw_albedo(rng, P)
    w = rng.standard_normal(P)
    return dict(points=_f32(pts), normals=_f32(pts), albedo=_f32(albedo),
                spheres=_f32(spheres), light=_f32(light), n_bands=n_bands,
                grad_radiance=_f32(w))


# Stick-figure capsules (metres, z up, facing +y): (name, A, B, R).
_BODY_CENTRE = [
    ("head", (0, 0, 1.60), (0, 0, 1.72), 0.10),
    ("neck", (0, 0, 1.47), (0, 0, 1.56), 0.05),
    ("chest", (-.12, 0, 1.36), (.12, 0, 1.36), 0.12),
    ("spine", (0, 0, 1.10), (0, 0, 1.32), 0.13),
    ("abdomen", (0, .04, 1.02), (0, .04, 1.12), 0.10),
    ("pelvis", (-.09, 0, .98), (.09, 0, .98), 0.11),
]
_BODY_MIRRORED = [
    ("clavicle", (.03, 0, 1.45), (.18, 0, 1.44), 0.045),
    ("upper_arm", (.20, 0, 1.42), (.24, 0, 1.16), 0.045),
    ("forearm", (.24, 0, 1.14), (.26, .06, .90), 0.035),
    ("hand", (.26, .07, .87), (.27, .09, .78), 0.03),
    ("buttock", (.07, -.06, .93), (.07, -.06, .85), 0.08),
    ("thigh", (.09, 0, .93), (.10, .02, .53), 0.075),
    ("shin", (.10, .02, .50), (.10, 0, .10), 0.05),
    ("foot", (.10, -.03, .05), (.11, .15, .04), 0.035),
    ("toes", (.11, .16, .035), (.11, .22, .03), 0.025),
]


def body_capsules():
    caps = [(n, np.array(a, float), np.array(b, float), r) for n, a, b, r in _BODY_CENTRE]
    for n, a, b, r in _BODY_MIRRORED:
        for sgn, side in ((-1.0, "l"), (1.0, "r")):
            a2 = np.array(a, float) * np.array([sgn, 1, 1])
            b2 = np.array(b, float) * np.array([sgn, 1, 1])
            caps.append((f"{n}_{side}", a2, b2, r))
    return caps


def _largest_remainder(weights, total, minimum=1):
    w = np.asarray(weights, float)
    base = np.full(len(w), minimum, dtype=np.int64)
    rest = total - base.sum()
    share = w / w.sum() * rest
    extra = np.floor(share).astype(np.int64)
    rem = share - extra
    left = rest - extra.sum()
    order = np.argsort(-rem, kind="stable")
    extra[order[:left]] += 1
    return base + extra


def _dist_to_segment(p, a, b):
    ab = b - a
    tt = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
    q = a + tt[:, None] * ab
    return np.linalg.norm(p - q, axis=1)


def scene_body(seed=0, P=20000, S=128, n_bands=8):
    """Body-like scene: receivers on a union of 24 capsules, spheres of radius
    0.9 R filling them (count per capsule proportional to (length + 2R)/R by
    largest remainder, at least one, centres evenly spaced from A to B).

    Receivers: capsule chosen with probability proportional to its area;
    uniform on its cylinder (prob. proportional to cylinder area) or its two
    end caps; a sample strictly inside another capsule is rejected; outward
    normal; lifted by the shadow bias.  Draw order (one rng): receivers in
    batches, light, albedo, output cotangent w ~ N(0, 1)."""
    caps = body_capsules()
    lens = np.array([np.linalg.norm(b - a) for _, a, b, _ in caps])
    radii = np.array([r for *_, r in caps])
    counts = _largest_remainder((lens + 2 * radii) / radii, S)
    sph = []
    for (_, a, b, R), cnt in zip(caps, counts):
        if cnt == 1:
            cs = [(a + b) / 2]
        else:
            cs = [a + (b - a) * i / (cnt - 1) for i in range(cnt)]
        for c in cs:
            sph.append([c[0], c[1], c[2], 0.9 * R])
    spheres = np.array(sph)

    rng = np.random.default_rng(seed)
    area_cyl = 2 * np.pi * radii * lens
    area_cap = 4 * np.pi * radii ** 2
    area = area_cyl + area_cap
    prob = area / area.sum()
    pts_out, nrm_out = [], []
    have = 0
    while have < P:
        B = 4096
        ci = rng.choice(len(caps), size=B, p=prob)
        u_part = rng.uniform(size=B)
        u1 = rng.uniform(size=B)
        u2 = rng.uniform(size=B)
        g = rng.standard_normal((B, 3))
        pts = np.empty((B, 3))
        nrm = np.empty((B, 3))
        for k in range(B):
            _, a, b, R = caps[ci[k]]
            axis = b - a
            ln = np.linalg.norm(axis)
            ez = axis / ln
            tmp = np.array([1.0, 0, 0]) if abs(ez[0]) < 0.9 else np.array([0, 1.0, 0])
            ex = np.cross(ez, tmp)
            ex /= np.linalg.norm(ex)
            ey = np.cross(ez, ex)
            if u_part[k] < area_cyl[ci[k]] / area[ci[k]]:
                ang = 2 * np.pi * u1[k]
                n = np.cos(ang) * ex + np.sin(ang) * ey
                p = a + u2[k] * axis + R * n
            else:
                n = g[k] / np.linalg.norm(g[k])
                end = b if n @ ez > 0 else a
                p = end + R * n
            pts[k], nrm[k] = p, n
        keep = np.ones(B, bool)
        for j, (_, a, b, R) in enumerate(caps):
            inside = _dist_to_segment(pts, a, b) < R - 1e-9
            keep &= ~(inside & (ci != j))
        pts, nrm = pts[keep], nrm[keep]
        pts_out.append(pts)
        nrm_out.append(nrm)
        have += len(pts)
    pts = np.concatenate(pts_out)[:P]
    nrm = np.concatenate(nrm_out)[:P]
    pts = pts + SHADOW_BIAS * nrm
    light = draw_light(rng, n_bands)
    albedo = draw_albedo(rng, P)
    w = rng.standard_normal(P)
    return dict(points=_f32(pts), normals=_f32(nrm), albedo=_f32(albedo),
                spheres=_f32(spheres), light=_f32(light), n_bands=n_bands,
                grad_radiance=_f32(w))


def gbuffer_spheres(rng, S=256):
    r = rng.uniform(0.05, 0.25, size=S)
    xy = rng.uniform(-1.0, 1.0, size=(S, 2))
    return np.concatenate([xy, r[:, None], r[:, None]], axis=1)


def raycast_gbuffer(spheres, res):
    """Orthographic top-down camera over [-1, 1]^2 with rays along -z: the
    nearest analytic hit among the spheres and the plane z = 0 gives the
    receiver position and normal per pixel centre."""
    c = (np.arange(res) + 0.5) / res * 2.0 - 1.0
    X, Y = np.meshgrid(c, c, indexing="xy")
    X, Y = X.ravel(), Y.ravel()
    best_z = np.zeros_like(X)
    best_i = np.full(X.shape, -1, dtype=np.int64)
    for i, (cx, cy, cz, r) in enumerate(spheres):
        h2 = r * r - (X - cx) ** 2 - (Y - cy) ** 2
        hit = h2 >= 0
        z = np.where(hit, cz + np.sqrt(np.where(hit, h2, 0.0)), -np.inf)
        better = z > best_z
        best_z = np.where(better, z, best_z)
        best_i = np.where(better, i, best_i)
    P = np.stack([X, Y, best_z], axis=1)
    N = np.tile(np.array([0.0, 0.0, 1.0]), (X.size, 1))
    on = best_i >= 0
    cs = spheres[best_i[on]]
    N[on] = (P[on] - cs[:, :3]) / cs[:, 3:4]
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return P, N


def contact_flags(points, spheres, s_max=0.996):
    """True where some sphere has r / |c - p| > s_max (receivers touching an
    occluder; kept in timed workloads, left out of parity metrics)."""
    flag = np.zeros(points.shape[0], bool)
    for cx, cy, cz, r in spheres:
        d = np.linalg.norm(points - np.array([cx, cy, cz]), axis=1)
        flag |= r > s_max * d
    return flag


def scene_gbuffer(seed=0, res=512, S=256, n_bands=8):
    """Image-space G-buffer scene: ``res`` x ``res`` receivers from ray casting
    S spheres resting on the ground plane (r ~ U[0.05, 0.25], (x, y) ~
    U[-1, 1]^2, z = r).  Draw order (one rng): sphere radii, xy, albedo,
    light; then rng(2) jitters the centres by N(0, 0.02^2) in xy and rng(3)
    perturbs the light by 0.1 N(0, 1) for the target scene."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.05, 0.25, size=S)
    xy = rng.uniform(-1.0, 1.0, size=(S, 2))
    spheres = np.concatenate([xy, r[:, None], r[:, None]], axis=1)
    P, N = raycast_gbuffer(spheres, res)
    P = P + SHADOW_BIAS * N
    albedo = draw_albedo(rng, P.shape[0])
    light = draw_light(rng, n_bands)
    rng2 = np.random.default_rng(2)
    tgt_spheres = spheres.copy()
    tgt_spheres[:, :2] += rng2.normal(0.0, 0.02, size=(S, 2))
    rng3 = np.random.default_rng(3)
    tgt_light = light + 0.1 * rng3.standard_normal(light.shape)
    pts32 = _f32(P)
    sph32 = _f32(spheres)
    return dict(points=pts32, normals=_f32(N), albedo=_f32(albedo),
                spheres=sph32, light=_f32(light), n_bands=n_bands,
                target_spheres=_f32(tgt_spheres), target_light=_f32(tgt_light),
                contact=contact_flags(pts32.astype(np.float64), sph32.astype(np.float64)))


def batched_scene_sizes(b):
    """Sizes of scene ``b`` of the 64-scene batched workload (seed 100 + b):
    P ~ U{5000..50000}, S ~ U{32..256}, n ~ U{4, 6, 8}."""
    rng = np.random.default_rng(100 + b)
    P = int(rng.integers(5000, 50001))
    S = int(rng.integers(32, 257))
    n = int(rng.choice([4, 6, 8]))
    return P, S, n, rng.integers(0, 2**31 - 1)


def scene_batched(b):
    P, S, n, sub = batched_scene_sizes(b)
    return scene_random_shell(int(sub), P, S, n)


def large_request_scene(seed, P=262144, S=512, n_bands=8):
    return scene_random_shell(seed, P, S, n_bands)


def subset(scene, idx):
    """A scene restricted to receiver indices ``idx`` (spheres and light kept)."""
    out = dict(scene)
    for key in ("points", "normals", "albedo", "grad_radiance", "contact"):
        if key in scene:
            out[key] = np.ascontiguousarray(scene[key][idx])
    return out


# --------------------------------------------------------------------------
# colour channels and environment maps
# --------------------------------------------------------------------------


def colour_channels(scene, C=3, seed=0):
    """Per-channel albedo [P, C], lighting [C, n*n] and output cotangent
    [P, C] for ``scene`` (RGB-like when C = 3).  Draw order: per channel the
    light (DC 3 plus N(0, 1), as draw_light), then albedo uniform in
    [0.2, 0.9], then the cotangent N(0, 1)."""
    rng = np.random.default_rng(seed)
    P = scene["points"].shape[0]
    n = int(scene["n_bands"])
    light = np.stack([draw_light(rng, n) for _ in range(C)])
    albedo = rng.uniform(0.2, 0.9, size=(P, C))
    w = rng.standard_normal((P, C))
    return dict(albedo=_f32(albedo), light=_f32(light), grad_radiance=_f32(w))


def envmap_image(seed=0, C=3, H=256, W=512, suns=3):
    """A synthetic equirectangular HDR environment map [C, H, W] (row r covers
    polar angles [r, r + 1] pi / H from +z, column x azimuths
    [x, x + 1] 2 pi / W): a sky-to-ground gradient, a slowly varying
    azimuthal pattern and ``suns`` small bright Gaussian spots (the dynamic
    range of captured sky maps).  Draw order: per-channel sky and ground
    levels, pattern amplitudes and phases, then per sun its direction, width
    (radians) and per-channel intensity."""
    rng = np.random.default_rng(seed)
    th = (np.arange(H) + 0.5) * (np.pi / H)
    ph = (np.arange(W) + 0.5) * (2.0 * np.pi / W)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1)
    sky = rng.uniform(0.5, 1.5, size=C)
    ground = rng.uniform(0.05, 0.3, size=C)
    amp = rng.uniform(0.0, 0.3, size=(C, 3))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(C, 3))
    img = np.empty((C, H, W))
    up = np.clip(d[..., 2], 0.0, 1.0)
    for c in range(C):
        img[c] = ground[c] + (sky[c] - ground[c]) * up
        for j in range(3):
            img[c] *= 1.0 + amp[c, j] * np.cos((j + 1) * PH + phase[c, j]) * np.sin(TH)
    for _ in range(suns):
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        width = rng.uniform(0.03, 0.1)
        power = rng.uniform(20.0, 200.0, size=C)
        ang2 = np.arccos(np.clip(d @ v, -1.0, 1.0)) ** 2
        for c in range(C):
            img[c] += power[c] * np.exp(-ang2 / (2.0 * width * width))
    return _f32(img)


def capsule_mesh(a, b, R, segments, spacing):
    """Triangulated capsule around the segment a-b: two hemispherical caps
    and a cylinder, rings of ``segments`` vertices about every ``spacing`` of
    arc length, a vertex at each pole.  Returns (vertices, outward normals,
    faces), faces wound counter-clockwise seen from outside."""
    a, b = np.asarray(a, float), np.asarray(b, float)
    axis = b - a
    ln = np.linalg.norm(axis)
    ez = axis / ln
    tmp = np.array([1.0, 0, 0]) if abs(ez[0]) < 0.9 else np.array([0, 1.0, 0])
    ex = np.cross(ez, tmp)
    ex /= np.linalg.norm(ex)
    ey = np.cross(ez, ex)
    n_cap = max(2, int(round(0.5 * np.pi * R / spacing)))
    n_cyl = max(1, int(round(ln / spacing)))
    # rings from the pole at a to the pole at b: (centre, polar angle from -ez)
    rings = []
    for k in range(1, n_cap + 1):
        th = 0.5 * np.pi * k / n_cap                      # 0 at the pole of a, pi/2 at the equator
        rings.append((a, th))
    for k in range(1, n_cyl):
        rings.append((a + axis * k / n_cyl, 0.5 * np.pi))
    for k in range(n_cap, 0, -1):
        rings.append((b, np.pi - 0.5 * np.pi * k / n_cap))
    phi = 2 * np.pi * np.arange(segments) / segments
    ring_dir = np.cos(phi)[:, None] * ex + np.sin(phi)[:, None] * ey
    verts, nrms = [a - R * ez], [-ez]
    for c, th in rings:
        n = -np.cos(th) * ez + np.sin(th) * ring_dir
        verts.extend(c + R * n)
        nrms.extend(n)
    verts.append(b + R * ez)
    nrms.append(ez)
    faces = []
    first = 1
    for s in range(segments):
        faces.append((0, first + (s + 1) % segments, first + s))
    for r in range(len(rings) - 1):
        o0, o1 = 1 + r * segments, 1 + (r + 1) * segments
        for s in range(segments):
            s1 = (s + 1) % segments
            faces.append((o0 + s, o0 + s1, o1 + s1))
            faces.append((o0 + s, o1 + s1, o1 + s))
    top, last = len(verts) - 1, 1 + (len(rings) - 1) * segments
    for s in range(segments):
        faces.append((last + s, last + (s + 1) % segments, top))
    return np.array(verts), np.array(nrms), np.array(faces, np.int64)


def look_at_camera(eye, target, up, f, width, height):
    """3 x 4 pinhole projection: pixel x to the right, y down, depth along
    the view direction; principal point at the image centre."""
    eye, target, up = (np.asarray(v, float) for v in (eye, target, up))
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    Rm = np.stack([right, down, fwd])
    K = np.array([[f, 0, width / 2.0], [0, f, height / 2.0], [0, 0, 1.0]])
    return K @ np.concatenate([Rm, (-Rm @ eye)[:, None]], 1)


def scene_mesh_body(seed=0, segments=24, spacing=None, n_bands=8, width=512, height=512):
    """The body scene as a triangle mesh: every capsule tessellated
    (capsule_mesh, 24 azimuths, rings about 1 cm of arc apart: 21,288
    vertices and 42,480 triangles), the same 128 spheres; the vertices are the
    receivers (lifted by the shadow bias).  A camera 4 m in front of the body
    looking at its middle frames it in a width x height image.  Draw order
    (one rng): light, albedo, image cotangent."""
    caps = body_capsules()
    spacing = 0.0102 if spacing is None else spacing
    V, N, F = [], [], []
    for _, a, b, R in caps:
        v, n, f = capsule_mesh(a, b, R, segments, spacing)
        F.append(f + sum(len(x) for x in V))
        V.append(v)
        N.append(n)
    verts, nrm, faces = np.concatenate(V), np.concatenate(N), np.concatenate(F)
    verts = verts + SHADOW_BIAS * nrm
    spheres = scene_body(seed, P=1, n_bands=n_bands)["spheres"]
    rng = np.random.default_rng(seed)
    light = draw_light(rng, n_bands)
    albedo = draw_albedo(rng, len(verts))
    lo, hi = verts.min(0), verts.max(0)
    mid = (lo + hi) / 2
    f = 0.9 * height * 4.0 / (hi[2] - lo[2])
    P = look_at_camera(mid + np.array([0.0, 4.0, 0.0]), mid, (0, 0, 1), f, width, height)
    gI = rng.standard_normal((height, width))
    return dict(points=_f32(verts), normals=_f32(nrm), albedo=_f32(albedo), spheres=_f32(spheres),
                light=_f32(light), n_bands=n_bands, faces=faces.astype(np.int32), camera=_f32(P),
                width=width, height=height, grad_image=_f32(gI))


def scene_raster_stress(seed=8, width=100, height=90, n_big=160, n_small=2400, n_dup=40):
    """Unconnected triangles that load the rasteriser's binning: n_big large
    ones (0.8 to 2.5 m across, many spanning more than 16 of the 8 x 8 pixel
    tiles) spread over and past the frame, n_small small ones (4 to 12 cm)
    packed in front of them in a patch of a few tiles, and the first n_dup
    large ones repeated at the end of the face list (equal depths: ties).
    Each triangle's corners sit at angles 120 degrees apart (jittered) around
    its centre, so none is a sliver.  Camera 4 m away, focal length 50 px."""
    rng = np.random.default_rng(seed)

    def triangles(c, r):
        n = len(c)
        th = (rng.uniform(0, 2 * np.pi, n)[:, None] + 2 * np.pi * np.arange(3)[None, :] / 3
              + rng.uniform(-0.3, 0.3, (n, 3)))
        v = np.stack([c[:, 0:1] + r[:, None] * np.cos(th), c[:, 1:2] + rng.uniform(-0.2, 0.2, (n, 3)) * r[:, None],
                      c[:, 2:3] + r[:, None] * np.sin(th)], -1)
        return v.reshape(-1, 3)

    cb = np.stack([rng.uniform(-2.5, 2.5, n_big), rng.uniform(-1.0, 1.0, n_big), rng.uniform(-2.5, 2.5, n_big)], 1)
    vb = triangles(cb, rng.uniform(0.8, 2.5, n_big))
    cs = np.stack([rng.uniform(0.1, 0.5, n_small), rng.uniform(1.0, 1.4, n_small), rng.uniform(-0.4, 0.0, n_small)], 1)
    vs = triangles(cs, rng.uniform(0.04, 0.12, n_small))
    verts = np.concatenate([vb, vs])
    faces = np.arange(len(verts)).reshape(-1, 3)
    faces = np.concatenate([faces, faces[:n_dup]])
    P = look_at_camera((0, 4, 0), (0, 0, 0), (0, 0, 1), 50, width, height)
    radiance = rng.uniform(0.0, 2.0, len(verts))
    gI = rng.standard_normal((height, width))
    return dict(points=_f32(verts), faces=faces.astype(np.int32), camera=_f32(P), width=width, height=height,
                radiance=_f32(radiance), grad_image=_f32(gI), n_dup=n_dup)
