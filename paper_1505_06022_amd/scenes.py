"""Seeded synthetic inputs: triangle scenes, materials, cameras and ray batches.

This module only *describes* inputs (geometry, material tables, camera poses,
ray origins/directions drawn with numpy's PCG64).  It holds none of the
renderer's arithmetic: no intersection, no sampling of the renderer's random
streams, no photon or density-estimation math.  Both the GPU path and the CPU
oracle consume exactly these arrays.

The paper's own scenes (the metal Cornell box used by its released code, the
teaser scenes with a scanned model, the scenes behind its ray-casting plot)
are not available; the generators below are synthetic stand-ins of the same
kinds of structure (room-with-boxes, random triangle soup, procedural
heightfield + spheres inside a room).

Conventions
-----------
* ``verts``     float32 [T, 3, 3]  triangle vertices; winding defines the
                geometric normal n = normalize((v1 - v0) x (v2 - v0)).
* ``tri_mat``   uint32  [T]        material index per triangle.
* materials     ``mat_type`` int32 (0 diffuse, 1 mirror, 2 glass),
                ``mat_rho`` float32 diffuse albedo (throughput),
                ``mat_q``   float32 Russian-roulette survival probability
                            (the nominal albedo, held fixed),
                ``mat_Le``  float32 emitted radiance (front side, along n),
                ``mat_ior`` float32 index of refraction (glass only).
* camera        pinhole: position, look-at point, up vector, tan(fov_y / 2),
                width, height.
* rays          float32 [N, 8] = (o.x, o.y, o.z, tmin, d.x, d.y, d.z, tmax).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DIFFUSE = 0
MIRROR = 1
GLASS = 2


@dataclasses.dataclass
class Camera:
    pos: tuple
    look: tuple
    up: tuple
    tan_half_fov: float
    width: int
    height: int


@dataclasses.dataclass
class Scene:
    verts: np.ndarray          # float32 [T,3,3]
    tri_mat: np.ndarray        # uint32 [T]
    mat_type: np.ndarray       # int32 [M]
    mat_rho: np.ndarray        # float32 [M]
    mat_q: np.ndarray          # float32 [M]
    mat_Le: np.ndarray         # float32 [M]
    mat_ior: np.ndarray        # float32 [M]
    camera: Camera
    name: str = ""
    # indices of the diffuse materials that are free parameters (adjoint)
    albedo_params: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros(0, np.int32))

    @property
    def n_tri(self) -> int:
        return int(self.verts.shape[0])

    def with_rho(self, rho: np.ndarray) -> "Scene":
        """Copy with a new albedo table (RR probabilities stay nominal)."""
        s = dataclasses.replace(self)
        s.mat_rho = np.ascontiguousarray(rho, dtype=np.float32)
        return s

    def with_Le(self, scale: float) -> "Scene":
        s = dataclasses.replace(self)
        s.mat_Le = (self.mat_Le * np.float32(scale)).astype(np.float32)
        return s


class _Builder:
    def __init__(self):
        self.tris = []
        self.mats = []
        self.mat_type = []
        self.mat_rho = []
        self.mat_Le = []
        self.mat_ior = []

    def material(self, kind=DIFFUSE, rho=0.0, Le=0.0, ior=1.0) -> int:
        self.mat_type.append(kind)
        self.mat_rho.append(rho)
        self.mat_Le.append(Le)
        self.mat_ior.append(ior)
        return len(self.mat_type) - 1

    def add(self, tris, mat: int):
        tris = np.asarray(tris, dtype=np.float64).reshape(-1, 3, 3)
        self.tris.append(tris)
        self.mats.append(np.full(len(tris), mat, np.uint32))

    def quad(self, p0, p1, p2, p3, mat: int):
        """Two triangles (p0,p1,p2), (p0,p2,p3); normal along (p1-p0)x(p2-p0)."""
        self.add([[p0, p1, p2], [p0, p2, p3]], mat)

    def finish(self, camera: Camera, name: str, params=None) -> Scene:
        rho = np.asarray(self.mat_rho, np.float32)
        tris = np.concatenate(self.tris) if self.tris else np.zeros((0, 3, 3))
        mats = np.concatenate(self.mats) if self.mats else np.zeros(0, np.uint32)
        return Scene(
            verts=np.ascontiguousarray(tris.astype(np.float32)),
            tri_mat=np.ascontiguousarray(mats),
            mat_type=np.asarray(self.mat_type, np.int32),
            mat_rho=rho.copy(),
            mat_q=rho.copy(),
            mat_Le=np.asarray(self.mat_Le, np.float32),
            mat_ior=np.asarray(self.mat_ior, np.float32),
            camera=camera,
            name=name,
            albedo_params=np.asarray(params if params is not None else [], np.int32),
        )


def _box(lo, hi):
    """12 triangles of an axis-aligned box with outward normals."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    c = [(x0, y0, z0), (x1, y0, z0), (x1, y1, z0), (x0, y1, z0),
         (x0, y0, z1), (x1, y0, z1), (x1, y1, z1), (x0, y1, z1)]
    faces = [(0, 3, 2, 1),  # -z
             (4, 5, 6, 7),  # +z
             (0, 4, 7, 3),  # -x
             (1, 2, 6, 5),  # +x
             (0, 1, 5, 4),  # -y
             (3, 7, 6, 2)]  # +y
    out = []
    for a, b, cc, d in faces:
        out.append([c[a], c[b], c[cc]])
        out.append([c[a], c[cc], c[d]])
    return np.asarray(out, np.float64)


def _room_walls(b: _Builder, rhos):
    """Floor, ceiling, back, left, right of [0,1]^3 (front z=0 open), inward normals."""
    m = [b.material(DIFFUSE, r) for r in rhos]
    b.quad((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 0, 0), m[0])      # floor  (+y)
    b.quad((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1), m[1])      # ceiling (-y)
    b.quad((0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 0, 1), m[2])      # back (-z)
    b.quad((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1), m[3])      # left (+x)
    b.quad((1, 0, 0), (1, 0, 1), (1, 1, 1), (1, 1, 0), m[4])      # right (-x)
    return m


def _ceiling_light(b: _Builder, Le=10.0, y=0.999, x=(0.4, 0.6), z=(0.4, 0.6)):
    """Square emitter facing -y (black, one-sided)."""
    m = b.material(DIFFUSE, 0.0, Le=Le)
    b.quad((x[0], y, z[0]), (x[1], y, z[0]), (x[1], y, z[1]), (x[0], y, z[1]), m)
    return m


def box_scene(width=64, height=64) -> Scene:
    """Room with two boxes and a ceiling quad light (34 diffuse + 2 light triangles)."""
    b = _Builder()
    walls = _room_walls(b, (0.8, 0.8, 0.8, 0.5, 0.3))
    m1 = b.material(DIFFUSE, 0.6)
    m2 = b.material(DIFFUSE, 0.7)
    b.add(_box((0.15, 0.0, 0.5), (0.45, 0.3, 0.8)), m1)
    b.add(_box((0.55, 0.0, 0.2), (0.85, 0.6, 0.5)), m2)
    _ceiling_light(b, 10.0)
    cam = Camera((0.5, 0.5, -1.2), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 0.45, width, height)
    return b.finish(cam, "box", params=walls + [m1, m2])


def _icosphere(level: int):
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = np.asarray(v, np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.asarray(f, np.int64)
    for _ in range(level):
        a, bb, c = F[:, 0], F[:, 1], F[:, 2]
        edges = np.concatenate([np.stack([a, bb], 1), np.stack([bb, c], 1), np.stack([c, a], 1)])
        key = np.sort(edges, axis=1)
        uniq, inv = np.unique(key, axis=0, return_inverse=True)
        mid = V[uniq[:, 0]] + V[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(V)
        V = np.concatenate([V, mid])
        nF = len(F)
        ab = base + inv[:nF]
        bc = base + inv[nF:2 * nF]
        ca = base + inv[2 * nF:]
        F = np.concatenate([np.stack([a, ab, ca], 1), np.stack([bb, bc, ab], 1),
                            np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)])
    return V[F]  # [F,3,3], outward winding


def _value_noise_fbm(rng, n_samples: int, octaves=4):
    """fBm of bilinear-smoothstep value noise sampled on an (n+1)^2 vertex grid."""
    xs = np.linspace(0.0, 1.0, n_samples)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    h = np.zeros_like(X)
    amp, freq = 1.0, 4
    for _ in range(octaves):
        lat = rng.random((freq + 2, freq + 2))
        fx, fz = X * freq, Z * freq
        ix, iz = np.floor(fx).astype(int), np.floor(fz).astype(int)
        tx, tz = fx - ix, fz - iz
        sx, sz = tx * tx * (3 - 2 * tx), tz * tz * (3 - 2 * tz)
        v00, v10 = lat[ix, iz], lat[ix + 1, iz]
        v01, v11 = lat[ix, iz + 1], lat[ix + 1, iz + 1]
        h += amp * ((v00 * (1 - sx) + v10 * sx) * (1 - sz) + (v01 * (1 - sx) + v11 * sx) * sz)
        amp *= 0.5
        freq *= 2
    h -= h.min()
    h /= max(h.max(), 1e-12)
    return h


def procedural_scene(width=1280, height=720, hf_cells=231, sphere_level=5,
                     glass_level=6, seed=3, Le=10.0) -> Scene:
    """Room + noise heightfield (3x3 material tiles) + 2 diffuse, 1 mirror, 1 glass sphere.

    With the defaults: 10 + 2*231^2 + 3*20*4^5 + 20*4^6 + 2 = 250,094 triangles and
    16 diffuse materials (5 walls, 9 heightfield tiles, 2 spheres) with albedo
    drawn U[0.3, 0.8].
    """
    rng = np.random.default_rng(seed)
    rhos = rng.uniform(0.3, 0.8, 16)
    b = _Builder()
    walls = _room_walls(b, rhos[:5])
    tiles = [b.material(DIFFUSE, float(r)) for r in rhos[5:14]]
    sA = b.material(DIFFUSE, float(rhos[14]))
    sB = b.material(DIFFUSE, float(rhos[15]))
    mir = b.material(MIRROR, 0.0)
    gl = b.material(GLASS, 0.0, ior=1.5)
    # heightfield
    n = hf_cells
    H = 0.01 + 0.15 * _value_noise_fbm(rng, n + 1)
    xs = np.linspace(0.0, 1.0, n + 1)
    P = np.stack(np.meshgrid(xs, xs, indexing="ij"), -1)  # [n+1,n+1,2] (x,z)
    V = np.stack([P[..., 0], H, P[..., 1]], -1)
    v00, v10, v01, v11 = V[:-1, :-1], V[1:, :-1], V[:-1, 1:], V[1:, 1:]
    # upward-facing: (v01 - v00) x (v10 - v00) points +y
    t1 = np.stack([v00, v01, v11], 2).reshape(-1, 3, 3)
    t2 = np.stack([v00, v11, v10], 2).reshape(-1, 3, 3)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    tile = ((ii * 3) // n) * 3 + (jj * 3) // n
    tile = tile.reshape(-1)
    hf = np.stack([t1, t2], 1).reshape(-1, 3, 3)
    hf_mat = np.repeat(tile, 2)
    for t in range(9):
        b.add(hf[hf_mat == t], tiles[t])
    ico = _icosphere(sphere_level)
    ico_g = ico if glass_level == sphere_level else _icosphere(glass_level)
    b.add(np.asarray((0.22, 0.32, 0.72)) + 0.12 * ico, sA)
    b.add(np.asarray((0.78, 0.30, 0.70)) + 0.11 * ico, sB)
    b.add(np.asarray((0.30, 0.45, 0.30)) + 0.10 * ico, mir)
    b.add(np.asarray((0.68, 0.42, 0.32)) + 0.13 * ico_g, gl)
    _ceiling_light(b, Le)
    cam = Camera((0.5, 0.5, -1.2), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 0.45, width, height)
    return b.finish(cam, "procedural", params=walls + tiles + [sA, sB])


def furnace_scene(rho=0.5, Le=1.0, width=32, height=32) -> Scene:
    """Closed unit cube; every face is diffuse with albedo rho and emits Le inward.

    Radiance everywhere inside equals Le / (1 - rho).
    """
    b = _Builder()
    m = b.material(DIFFUSE, rho, Le=Le)
    tris = _box((0, 0, 0), (1, 1, 1))
    tris = tris[:, [0, 2, 1]]  # flip winding: normals point inward
    b.add(tris, m)
    cam = Camera((0.5, 0.5, 0.5), (0.5, 0.5, 1.0), (0.0, 1.0, 0.0), 0.5, width, height)
    return b.finish(cam, "furnace", params=[m])


def polygon_light_scene(rho=0.5, Le=1.0, half=0.25, height=1.0, floor_half=40.0,
                        width=48, height_px=48) -> Scene:
    """Square emitter (side 2*half) at y=height facing down over a large diffuse floor.

    Nothing can carry light back to the floor, so the floor radiance is
    (rho/pi) * E(x) with E the irradiance from the polygon source.
    """
    b = _Builder()
    mf = b.material(DIFFUSE, rho)
    f = floor_half
    b.quad((-f, 0, -f), (-f, 0, f), (f, 0, f), (f, 0, -f), mf)   # +y
    _ceiling_light(b, Le, y=height, x=(-half, half), z=(-half, half))
    cam = Camera((0.0, 0.9, -0.9), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.35, width, height_px)
    return b.finish(cam, "polygon_light", params=[mf])


def two_light_scene(Le=(10.0, 10.0), half=(0.1, 0.05), width=16, height=16) -> Scene:
    """Two square emitters facing down over a diffuse floor, with their own
    materials: light i has side 2*half[i] and radiance Le[i].  Emission by
    power picks light i with probability A_i Le_i / sum_j A_j Le_j."""
    b = _Builder()
    mf = b.material(DIFFUSE, 0.5)
    f = 4.0
    b.quad((-f, 0, -f), (-f, 0, f), (f, 0, f), (f, 0, -f), mf)   # +y
    _ceiling_light(b, Le[0], y=1.0, x=(-0.5 - half[0], -0.5 + half[0]), z=(-half[0], half[0]))
    _ceiling_light(b, Le[1], y=1.0, x=(0.5 - half[1], 0.5 + half[1]), z=(-half[1], half[1]))
    cam = Camera((0.0, 0.9, -1.4), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.5, width, height)
    return b.finish(cam, "two_lights", params=[mf])


def mirror_floor_scene(width=24, height=16, rho=0.5) -> Scene:
    """A diffuse floor (y = 0, z <= 2) in front of a vertical mirror (z = 2,
    facing -z, spanning y in [0.3, 4]); the camera looks at the mirror, so
    most eye paths reflect once and end on the floor in front of it.  A
    square light hangs above the floor, facing down."""
    b = _Builder()
    mf = b.material(DIFFUSE, rho)
    mm = b.material(MIRROR, 0.0)
    b.quad((-6, 0, -6), (-6, 0, 2), (6, 0, 2), (6, 0, -6), mf)       # floor (+y)
    b.quad((-6, 0.3, 2), (-6, 4, 2), (6, 4, 2), (6, 0.3, 2), mm)     # mirror (-z)
    _ceiling_light(b, 5.0, y=3.0, x=(-0.3, 0.3), z=(0.2, 0.8))
    cam = Camera((0.1, 1.0, 0.0), (0.0, 0.6, 2.0), (0.0, 1.0, 0.0), 0.35, width, height)
    return b.finish(cam, "mirror_floor", params=[mf])


def mirror_corridor_scene(width=32, height=32, length=50.0) -> Scene:
    """A corridor between two parallel mirrors (x = -0.5 facing +x, x = +0.5
    facing -x, 100 high) over a diffuse floor (y = 0), closed by a diffuse end
    wall at z = length; the top is open.  Eye rays bounce between the mirrors
    on their way to the floor or the end wall, up to a few dozen times."""
    b = _Builder()
    mf = b.material(DIFFUSE, 0.5)
    me = b.material(DIFFUSE, 0.7)
    mm = b.material(MIRROR, 0.0)
    L, Hh = length, 100.0
    b.quad((-0.5, 0, -1), (-0.5, 0, L), (0.5, 0, L), (0.5, 0, -1), mf)          # floor (+y)
    b.quad((-0.5, 0, L), (-0.5, Hh, L), (0.5, Hh, L), (0.5, 0, L), me)          # end wall (-z)
    b.quad((-0.5, 0, -1), (-0.5, Hh, -1), (-0.5, Hh, L), (-0.5, 0, L), mm)      # left mirror (+x)
    b.quad((0.5, 0, -1), (0.5, 0, L), (0.5, Hh, L), (0.5, Hh, -1), mm)          # right mirror (-x)
    _ceiling_light(b, 1.0, y=0.99 * Hh, x=(-0.4, 0.4), z=(0.0, 0.8))
    cam = Camera((0.1, 1.0, 0.0), (0.3, 0.75, 5.0), (0.0, 1.0, 0.0), 0.5, width, height)
    return b.finish(cam, "mirror_corridor", params=[mf, me])


def specular_furnace_scene(rho=0.5, Le=1.0, width=16, height=16, glass_level=3) -> Scene:
    """The closed furnace cube (every face diffuse with albedo rho, emitting Le
    inward) holding a floating mirror box and a glass sphere (IOR 1.5).
    Lossless specular surfaces leave the uniform radiance Le / (1 - rho)
    unchanged, so every hit point still sees it."""
    b = _Builder()
    m = b.material(DIFFUSE, rho, Le=Le)
    mm = b.material(MIRROR, 0.0)
    mg = b.material(GLASS, 0.0, ior=1.5)
    tris = _box((0, 0, 0), (1, 1, 1))[:, [0, 2, 1]]   # inward normals
    b.add(tris, m)
    b.add(_box((0.2, 0.3, 0.55), (0.4, 0.5, 0.75)), mm)
    b.add(np.asarray((0.66, 0.5, 0.65)) + 0.16 * _icosphere(glass_level), mg)
    cam = Camera((0.5, 0.5, 0.05), (0.5, 0.5, 1.0), (0.0, 1.0, 0.0), 0.6, width, height)
    return b.finish(cam, "specular_furnace", params=[m])


def polygon_light_mirror_scene(rho=0.5, Le=1.0, half=0.25, height=1.0, mirror_x=0.4, floor_half=40.0,
                               width=32, height_px=24) -> Scene:
    """The polygon-light scene cut by a large vertical mirror at x = mirror_x
    (facing -x): the floor (x < mirror_x) is lit by the square light and by
    its mirror image.  The floor's Russian-roulette survival is 0, so only
    first-bounce photons are stored and the floor radiance is
    (rho/pi) (E(light) + E(image of the light))."""
    b = _Builder()
    mf = b.material(DIFFUSE, rho)
    mm = b.material(MIRROR, 0.0)
    f, xm = floor_half, mirror_x
    b.quad((-f, 0, -f), (-f, 0, f), (xm, 0, f), (xm, 0, -f), mf)        # floor (+y)
    b.quad((xm, 0, -f), (xm, 0, f), (xm, f, f), (xm, f, -f), mm)        # mirror (-x)
    _ceiling_light(b, Le, y=height, x=(-half, half), z=(-half, half))
    cam = Camera((-0.6, 0.9, -0.9), (-0.2, 0.0, 0.0), (0.0, 1.0, 0.0), 0.3, width, height_px)
    s = b.finish(cam, "polygon_light_mirror", params=[mf])
    s.mat_q = s.mat_q.copy()
    s.mat_q[mf] = 0.0
    return s


def soup_scene(n_tri=1 << 20, seed=2) -> Scene:
    """Random triangle soup: centroids uniform in the unit cube, vertex offsets
    of lognormal(-5, 0.5) length along uniform directions."""
    rng = np.random.default_rng(seed)
    c = rng.random((n_tri, 1, 3))
    ell = rng.lognormal(-5.0, 0.5, (n_tri, 1, 1))
    u = rng.standard_normal((n_tri, 3, 3))
    u /= np.linalg.norm(u, axis=2, keepdims=True)
    v = (c + ell * u).astype(np.float32)
    b = _Builder()
    m = b.material(DIFFUSE, 0.5)
    cam = Camera((0.5, 0.5, -1.5), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 0.4, 1920, 1080)
    s = b.finish(cam, "soup")
    s.verts = np.ascontiguousarray(v)
    s.tri_mat = np.zeros(n_tri, np.uint32)
    return s


def pinhole_rays(cam: Camera) -> np.ndarray:
    """Pixel-centre rays of a pinhole camera, row-major, float32 [W*H, 8]."""
    pos = np.asarray(cam.pos, np.float64)
    f = np.asarray(cam.look, np.float64) - pos
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(cam.up, np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    W, H = cam.width, cam.height
    aspect = W / H
    x = (np.arange(W) + 0.5) / W
    y = (np.arange(H) + 0.5) / H
    X, Y = np.meshgrid(x, y)
    sx = (2 * X - 1) * cam.tan_half_fov * aspect
    sy = (1 - 2 * Y) * cam.tan_half_fov
    d = f[None, None] + sx[..., None] * r[None, None] + sy[..., None] * u[None, None]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    out = np.zeros((H * W, 8), np.float32)
    out[:, 0:3] = pos
    out[:, 3] = 0.0
    out[:, 4:7] = d.reshape(-1, 3)
    out[:, 7] = np.inf
    return out


def random_rays(n: int, seed=2, lo=0.0, hi=1.0) -> np.ndarray:
    """Incoherent rays: origins uniform in [lo,hi]^3, directions uniform on the sphere."""
    rng = np.random.default_rng(seed + 1000)
    out = np.zeros((n, 8), np.float32)
    out[:, 0:3] = rng.uniform(lo, hi, (n, 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out[:, 4:7] = d
    out[:, 3] = 0.0
    out[:, 7] = np.inf
    return out


def grazing_rays(verts, n: int, angles, seed=7, dist=(0.05, 1.0), on_edges=False) -> np.ndarray:
    """Rays aimed at points of random triangles of `verts`, each arriving at
    one of `angles` (radians) to the triangle's plane from a distance drawn
    uniformly in dist x the scene's diagonal.  The aim points are uniform over
    the triangle, or (on_edges) on its edges and vertices, where a hit lies on
    a face of the leaf's box."""
    rng = np.random.default_rng(seed)
    v = np.asarray(verts, np.float64)
    diag = float(np.linalg.norm(v.reshape(-1, 3).max(0) - v.reshape(-1, 3).min(0)))
    tri = rng.integers(0, len(v), n)
    a = rng.random(n)
    b = rng.random(n)
    if on_edges:
        k = rng.integers(0, 3, n)               # edge k, or a vertex when the edge parameter is 0
        a = np.where(rng.random(n) < 0.3, 0.0, a)
        bary = np.zeros((n, 3))
        bary[np.arange(n), k] = 1 - a
        bary[np.arange(n), (k + 1) % 3] = a
    else:
        fold = a + b > 1
        a, b = np.where(fold, 1 - a, a), np.where(fold, 1 - b, b)
        bary = np.stack([1 - a - b, a, b], 1)
    P = np.einsum("nk,nkj->nj", bary, v[tri])
    nrm = np.cross(v[tri, 1] - v[tri, 0], v[tri, 2] - v[tri, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    w = rng.standard_normal((n, 3))
    w -= (w * nrm).sum(1, keepdims=True) * nrm
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    th = np.asarray(angles, np.float64)[rng.integers(0, len(angles), n)]
    side = np.where(rng.random(n) < 0.5, -1.0, 1.0)[:, None]
    d = np.cos(th)[:, None] * w + np.sin(th)[:, None] * side * nrm
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    L = rng.uniform(dist[0], dist[1], n) * diag
    out = np.zeros((n, 8), np.float32)
    out[:, 0:3] = P - L[:, None] * d
    out[:, 4:7] = d
    out[:, 7] = np.inf
    return out


def far_origin_rays(verts, n: int, scales=(1e2, 1e3, 1e4, 1e5), seed=8) -> np.ndarray:
    """Rays from far outside the scene (scale x its extent away) aimed at
    random points of random triangles of `verts`."""
    rng = np.random.default_rng(seed)
    v = np.asarray(verts, np.float64)
    pts = v.reshape(-1, 3)
    ext = float((pts.max(0) - pts.min(0)).max())
    tri = rng.integers(0, len(v), n)
    a, b = rng.random(n), rng.random(n)
    fold = a + b > 1
    a, b = np.where(fold, 1 - a, a), np.where(fold, 1 - b, b)
    P = v[tri, 0] + a[:, None] * (v[tri, 1] - v[tri, 0]) + b[:, None] * (v[tri, 2] - v[tri, 0])
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    L = np.asarray(scales, np.float64)[rng.integers(0, len(scales), n)] * ext
    out = np.zeros((n, 8), np.float32)
    out[:, 0:3] = P - L[:, None] * d
    out[:, 4:7] = d
    out[:, 7] = np.inf
    return out


# Build options of the soup's BVH (pm_bvh_opts): spatial splits where the
# children of the best object split overlap by more than 1e-4 of the scene
# box's area, and a node visit costed as two triangle tests in the SAH (fuller
# leaves: 1.53 M nodes for 1.86 M triangle records, 236 MB on the device).
# Against the plain SAH build (0, 1) the incoherent rays visit about a quarter
# fewer nodes.
SOUP_SPLIT_ALPHA = 1e-4
SOUP_TRAV_COST = 2.0


def soup_workload(n_tri=1 << 20, width=1920, height=1080, n_incoherent=1 << 21, seed=2):
    """Traversal-only workload: scene + coherent pinhole rays + incoherent rays."""
    s = soup_scene(n_tri, seed)
    cam = dataclasses.replace(s.camera, width=width, height=height)
    return s, pinhole_rays(cam), random_rays(n_incoherent, seed)


def small_soup(n_tri: int, seed: int, scale=1.0, spread=0.3) -> Scene:
    """Tiny random scenes for property tests (larger triangles, many overlaps)."""
    rng = np.random.default_rng(seed)
    c = rng.random((n_tri, 1, 3))
    u = rng.standard_normal((n_tri, 3, 3))
    v = (c + spread * scale * u).astype(np.float32)
    b = _Builder()
    m = b.material(DIFFUSE, 0.5)
    cam = Camera((0.5, 0.5, -1.5), (0.5, 0.5, 0.5), (0.0, 1.0, 0.0), 0.5, 16, 16)
    s = b.finish(cam, "small_soup")
    s.verts = np.ascontiguousarray(v)
    s.tri_mat = np.zeros(n_tri, np.uint32)
    return s


def batch_workload(n_scenes=32, seed=5, tri_range=(1000, 200000), side_range=(128, 512), photon_log2=(16, 20)):
    """Scenes of uneven size for batched rendering: triangle counts log-uniform
    in tri_range (procedural room + heightfield + spheres), square images with
    sides log-uniform in side_range, photons per iteration 2^U{photon_log2}.

    Returns a list of (scene, n_photons, r0)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_scenes):
        T = float(np.exp(rng.uniform(np.log(tri_range[0]), np.log(tri_range[1]))))
        side = int(round(float(np.exp(rng.uniform(np.log(side_range[0]), np.log(side_range[1]))))))
        Np = 1 << int(rng.integers(photon_log2[0], photon_log2[1] + 1))
        level = 0
        while level < 6 and 80 * 4 ** (level + 1) <= T / 2:
            level += 1
        cells = max(2, int(round(np.sqrt(max(T - 80 * 4 ** level - 12, 8) / 2))))
        sc = procedural_scene(width=side, height=side, hf_cells=cells, sphere_level=level, glass_level=level,
                              seed=seed * 1000 + i)
        v = sc.verts.reshape(-1, 3)
        diag = float(np.linalg.norm(v.max(0) - v.min(0)))
        out.append((sc, Np, 0.05 * diag * 64 / side))
    return out
