"""Seeded synthetic inputs for the ray caster and for its CPU oracle.

This module only *draws* inputs: primitive positions, radii, colours, light
directions, cameras and render parameters.  It holds none of the rendering
arithmetic (no intersection, traversal, sampling or shading), so both the HIP
path and the oracle may import it without sharing any of the method.

The paper renders one molecular scene of 26,318 objects (Sec. 2, Strong
scaling; Fig. 1) with ambient-occlusion lighting at 965x1137 and 3860x4548
pixels (Sec. 2, rendering commands; Tables 2-3).  That scene file is not
available, so the generators below build seeded stand-ins of the same object
count: a random walk of atoms (spheres) joined by bonds (cylinders).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Four-colour palette, components <= 0.8.  Sphere i takes PALETTE[i % 4];
# a cylinder takes the colour of its first atom.
PALETTE = np.array(
    [[0.80, 0.30, 0.30],
     [0.30, 0.75, 0.35],
     [0.30, 0.45, 0.80],
     [0.80, 0.75, 0.30]], dtype=np.float32)

# Directions toward the two white directional lights (not normalised here:
# each consumer normalises).
LIGHT0 = (-0.5, 0.5, 1.0)
LIGHT1 = (1.0, 2.0, 0.5)


@dataclasses.dataclass
class Scene:
    """Host arrays of one scene.  Global primitive ids: spheres [0, n_s),
    cylinders [n_s, n_s + n_c), triangles [n_s + n_c, n_s + n_c + n_t)."""
    sph_center: np.ndarray   # float64 [n_s, 3]
    sph_radius: np.ndarray   # float64 [n_s]
    sph_rgb: np.ndarray      # float32 [n_s, 3]
    cyl_a: np.ndarray        # float64 [n_c, 3]
    cyl_b: np.ndarray        # float64 [n_c, 3]
    cyl_radius: np.ndarray   # float64 [n_c]
    cyl_rgb: np.ndarray      # float32 [n_c, 3]
    light_dir: np.ndarray    # float64 [n_l, 3]  toward the light
    light_rgb: np.ndarray    # float64 [n_l, 3]
    sph_opacity: Optional[np.ndarray] = None  # float32 [n_s] in (0, 1]; None = opaque
    cyl_opacity: Optional[np.ndarray] = None  # float32 [n_c] in (0, 1]; None = opaque
    tri_v: Optional[np.ndarray] = None        # float64 [n_t, 3, 3] triangle vertices
    tri_rgb: Optional[np.ndarray] = None      # float32 [n_t, 3]
    tri_opacity: Optional[np.ndarray] = None  # float32 [n_t] in (0, 1]; None = opaque

    @property
    def n_spheres(self) -> int:
        return int(self.sph_radius.shape[0])

    @property
    def n_cylinders(self) -> int:
        return int(self.cyl_radius.shape[0])

    @property
    def n_triangles(self) -> int:
        return 0 if self.tri_v is None else int(np.asarray(self.tri_v).reshape(-1, 9).shape[0])

    @property
    def n_prims(self) -> int:
        return self.n_spheres + self.n_cylinders + self.n_triangles

    @property
    def n_lights(self) -> int:
        return int(self.light_dir.shape[0])

    def contiguous(self) -> "Scene":
        f = {}
        for k, v in dataclasses.asdict(self).items():
            f[k] = None if v is None else np.ascontiguousarray(v)
        return Scene(**f)


@dataclasses.dataclass
class Camera:
    """Pinhole camera: eye, look-at point, up vector, vertical field of view
    in degrees, and the frame size (width = horizontal pixel count, height =
    vertical), as in the paper's -res W H option (Sec. 2)."""
    eye: tuple
    lookat: tuple
    up: tuple
    fovy_deg: float
    width: int
    height: int


@dataclasses.dataclass
class Params:
    """Render parameters.  light_rescale and skylight are the paper's
    -rescale_lights 0.3 and -add_skylight 1.0 options (Sec. 2)."""
    light_rescale: float = 0.3
    skylight: float = 1.0
    ao_samples: int = 16
    ao_maxdist: float = math.inf
    seed: int = 2
    view_id: int = 0
    background: tuple = (0.0, 0.0, 0.0)
    aa_samples: int = 1    # primary samples per pixel (antialiasing); 1 = pixel centre
    specular: float = 0.0  # Phong highlight strength (0 = none)
    shininess: float = 20.0  # Phong exponent
    max_layers: int = 0    # transparency: surfaces per primary ray (0, 1 = opaque rendering)


def _empty3(dtype=np.float64):
    return np.zeros((0, 3), dtype=dtype)


def _lights(n: int):
    dirs = [LIGHT0, LIGHT1][:n]
    return (np.array(dirs, dtype=np.float64).reshape(-1, 3),
            np.ones((len(dirs), 3), dtype=np.float64))


def _unit_gaussian(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    nrm = np.sqrt((v * v).sum(axis=1))
    # a zero-length draw has probability 0; keep it well defined anyway
    nrm[nrm == 0.0] = 1.0
    return v / nrm[:, None]


def tiny_scene(seed: int = 1, n: int = 64, ball_radius: float = 10.0,
               n_lights: int = 1) -> Scene:
    """n spheres, radii U[0.5, 1.5], centres uniform in a ball of the given
    radius (radius R*u^(1/3), Gaussian-normalised direction)."""
    rng = np.random.default_rng(seed)
    dirs = _unit_gaussian(rng, n)
    u = rng.random(n)
    rad = ball_radius * np.cbrt(u)
    centres = dirs * rad[:, None]
    radii = rng.uniform(0.5, 1.5, n)
    rgb = PALETTE[np.arange(n) % 4]
    ld, lc = _lights(n_lights)
    return Scene(centres, radii, rgb.astype(np.float32),
                 _empty3(), _empty3(), np.zeros(0), _empty3(np.float32), ld, lc)


def random_walk(n_positions: int, ball_radius: float, seed: int,
                step: float = 1.5) -> tuple:
    """Seeded random walk folded into a ball.  Returns (positions, rng)
    with the generator positioned after the step draws."""
    rng = np.random.default_rng(seed)
    dirs = _unit_gaussian(rng, max(n_positions - 1, 0))
    pos = np.zeros((n_positions, 3), dtype=np.float64)
    p = np.zeros(3, dtype=np.float64)
    R = float(ball_radius)
    for i in range(1, n_positions):
        p = p + step * dirs[i - 1]
        nrm = math.sqrt(float(p @ p))
        if nrm > R:
            # fold back inside: reflect the radial coordinate about R
            p = p * ((2.0 * R - nrm) / nrm)
        pos[i] = p
    return pos, rng


def random_walk_scene(n_spheres: int, ball_radius: float, seed: int,
                      n_cylinders: Optional[int] = None, r_lo: float = 1.2,
                      r_hi: float = 1.9, cyl_radius: float = 0.3,
                      n_lights: int = 2) -> Scene:
    """Protein-like scene: atoms on a folded random walk (step 1.5), bonds
    between consecutive walk positions.  With n_cylinders == n_spheres the
    walk has n_spheres + 1 positions: spheres sit on positions 0..n_s-1 and
    each consecutive pair of positions carries one cylinder, so the last
    cylinder dangles from the last atom."""
    if n_cylinders is None:
        n_cylinders = n_spheres
    n_pos = max(n_spheres, n_cylinders + 1)
    pos, rng = random_walk(n_pos, ball_radius, seed)
    radii = rng.uniform(r_lo, r_hi, n_spheres)
    centres = pos[:n_spheres].copy()
    ca = pos[:n_cylinders].copy()
    cb = pos[1:n_cylinders + 1].copy()
    srgb = PALETTE[np.arange(n_spheres) % 4].astype(np.float32)
    crgb = PALETTE[np.arange(n_cylinders) % 4].astype(np.float32)
    ld, lc = _lights(n_lights)
    return Scene(centres, radii, srgb, ca, cb,
                 np.full(n_cylinders, cyl_radius, dtype=np.float64), crgb, ld, lc)


def icosphere(subdiv: int):
    """Unit icosphere: the icosahedron's 20 faces, each split into 4 by edge
    midpoints (pushed to the sphere) `subdiv` times.  Returns (vertices
    [V, 3], faces [F, 3]) with F = 20 * 4^subdiv, faces counter-clockwise
    seen from outside."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0), (0, -1, g), (0, 1, g),
         (0, -1, -g), (0, 1, -g), (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    verts = [np.array(x, dtype=np.float64) / math.sqrt(1.0 + g * g) for x in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        mid = {}

        def midpoint(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, dtype=np.int64)


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly random rotation matrices (QR of Gaussian matrices with the
    signs fixed)."""
    q, r = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    q[np.linalg.det(q) < 0, :, 0] *= -1.0
    return q


def blob_mesh(centres: np.ndarray, radius: float, subdiv: int, seed: int = 0,
              rotate: bool = True) -> np.ndarray:
    """Closed icosphere meshes of the given radius around each centre:
    triangle vertices [n * F, 3, 3].  With rotate, each blob is turned by
    its own random rotation; without, every blob keeps the icosahedron's
    axis-aligned symmetry, whose faces have normals with (rounded) zero
    components and normals perpendicular to a light or nearly so, where a
    whole face's sign decisions rest on rounding."""
    verts, faces = icosphere(subdiv)
    unit = verts[faces]  # [F, 3, 3]
    c = np.asarray(centres, dtype=np.float64).reshape(-1, 1, 1, 3)
    if rotate:
        rot = _random_rotations(np.random.default_rng(seed), c.shape[0])
        turned = np.einsum("nij,fvj->nfvi", rot, unit)
    else:
        turned = np.broadcast_to(unit, (c.shape[0],) + unit.shape)
    return (c + radius * turned).reshape(-1, 3, 3)


def voxel_mesh(centres: np.ndarray, radius: float, cell: float,
               offset=(0.125, 0.375, 0.25)) -> np.ndarray:
    """The boundary of the voxels (cubes of side `cell` on a lattice through
    `offset`) whose centres lie within `radius` of a centre: each face
    between a voxel inside and one outside becomes two triangles, wound
    counter-clockwise seen from outside.  Every normal is an axis direction
    and every vertex a multiple of `cell` (exact for a power of two), like
    the blocky surfaces of a marching-cubes mesh at its lattice directions:
    triangle vertices [n, 3, 3].  The default offset keeps lattice planes
    off the coordinate planes (and so off a camera's axis through the
    origin)."""
    out = []
    off = np.asarray(offset, dtype=np.float64)
    for c in np.asarray(centres, dtype=np.float64).reshape(-1, 3):
        c = c - off
        base = np.floor(c / cell).astype(np.int64)
        m = int(math.ceil(radius / cell)) + 1
        idx = np.arange(-m, m + 1)
        g = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1) + base  # voxel lattice index
        ctr = (g + 0.5) * cell
        inside = ((ctr - c) ** 2).sum(axis=-1) <= radius * radius
        inside = np.pad(inside, 1)
        gp = np.pad(g, ((1, 1), (1, 1), (1, 1), (0, 0)), mode="edge")
        n = inside.shape[0]
        for a in range(3):
            b, e = (a + 1) % 3, (a + 2) % 3
            for sgn in (1, -1):
                sl_in = [slice(1, n - 1)] * 3
                sl_out = list(sl_in)
                sl_out[a] = slice(1 + sgn, n - 1 + sgn)
                face = inside[tuple(sl_in)] & ~inside[tuple(sl_out)]
                vox = gp[tuple(sl_in)][face]  # lattice index of each voxel with that face
                p00 = vox.astype(np.float64)
                p00[:, a] += 1 if sgn > 0 else 0
                p00 = p00 * cell + off
                eb = np.zeros(3)
                eb[b] = cell
                ec = np.zeros(3)
                ec[e] = cell
                p10, p11, p01 = p00 + eb, p00 + eb + ec, p00 + ec
                if sgn > 0:
                    out += [np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)]
                else:
                    out += [np.stack([p00, p11, p10], 1), np.stack([p00, p01, p11], 1)]
    return np.concatenate(out, axis=0)


def with_triangles(scene: Scene, tri_v: np.ndarray, tri_rgb=None, tri_opacity=None) -> Scene:
    tri_v = np.ascontiguousarray(tri_v, dtype=np.float64).reshape(-1, 3, 3)
    if tri_rgb is None:
        tri_rgb = PALETTE[np.arange(tri_v.shape[0]) % 4]
    return Scene(**{**scene.__dict__, "tri_v": tri_v,
                    "tri_rgb": np.ascontiguousarray(tri_rgb, dtype=np.float32).reshape(-1, 3),
                    "tri_opacity": tri_opacity})


def stacked_cylinders(n: int = 14000, half: float = 100.0, radius: float = 1.0) -> Scene:
    """n identical cylinders along the diagonal of a cube of half-size
    `half`, no spheres: every cylinder's box is the whole scene box, so each
    is listed in every grid cell (n x cells references in all; a grid-size
    limit case)."""
    a = np.full((n, 3), -half)
    b = np.full((n, 3), half)
    ld, lc = _lights(1)
    e3 = _empty3()
    return Scene(e3, np.zeros(0), _empty3(np.float32), a, b, np.full(n, radius),
                 PALETTE[np.arange(n) % 4].astype(np.float32), ld, lc)


def mixed_tiny_scene(seed: int = 5) -> Scene:
    """Small scene with all three primitive types: 24 spheres and 12
    cylinders in a ball of radius 10, four icosphere blobs (80 triangles
    each) and a two-triangle floor under them."""
    rng = np.random.default_rng(seed)
    base = tiny_scene(seed=seed, n=24)
    ca = rng.uniform(-8, 8, (12, 3))
    cb = ca + 3.0 * _unit_gaussian(rng, 12)
    blobs = blob_mesh(rng.uniform(-7, 7, (4, 3)), 2.5, 1, seed=seed)
    floor = np.array([[[-14, -11, -14], [14, -11, -14], [14, -11, 14]],
                      [[-14, -11, -14], [14, -11, 14], [-14, -11, 14]]], dtype=np.float64)
    s = Scene(**{**base.__dict__, "cyl_a": ca, "cyl_b": cb,
                 "cyl_radius": rng.uniform(0.3, 0.6, 12),
                 "cyl_rgb": PALETTE[np.arange(12) % 4].astype(np.float32)})
    return with_triangles(s, np.concatenate([blobs, floor]))


def surface_scene(seed: int = 2, every: int = 160, radius: float = 4.0,
                  subdiv: int = 2, rotate: bool = False) -> Scene:
    """Molecular-surface stand-in: closed icosphere blobs (320 triangles at
    subdivision 2) of radius 4 around every 160th position of the protein
    walk -- 83 blobs, 26,560 triangles, about the protein scene's object
    count -- with the protein scene's two lights.  The blobs keep the
    icosahedron's orientation unless rotate."""
    pos, _ = random_walk(PROTEIN_SPHERES + 1, PROTEIN_RADIUS, seed)
    tri = blob_mesh(pos[::every], radius, subdiv, seed=seed, rotate=rotate)
    ld, lc = _lights(2)
    e3 = _empty3()
    s = Scene(e3, np.zeros(0), _empty3(np.float32), e3.copy(), e3.copy(), np.zeros(0),
              _empty3(np.float32), ld, lc)
    per = 20 * 4 ** subdiv
    rgb = PALETTE[(np.arange(tri.shape[0]) // per) % 4]
    return with_triangles(s, tri, rgb)


def voxel_surface_scene(seed: int = 2, every: int = 1100, radius: float = 4.0,
                        cell: float = 0.5, axis_light: bool = True) -> Scene:
    """Axis-aligned surface stand-in: voxel surfaces (voxel_mesh, cubes of
    side 0.5) of radius 4 around every 1100th position of the protein walk
    (12 blobs).  Lights: the protein scene's two, plus (with axis_light) one
    along +z, to which the faces along x and y are exactly perpendicular."""
    pos, _ = random_walk(PROTEIN_SPHERES + 1, PROTEIN_RADIUS, seed)
    tri = voxel_mesh(pos[::every], radius, cell)
    ld, lc = _lights(2)
    if axis_light:
        ld = np.concatenate([ld, [[0.0, 0.0, 1.0]]])
        lc = np.concatenate([lc, [[0.5, 0.5, 0.5]]])
    e3 = _empty3()
    s = Scene(e3, np.zeros(0), _empty3(np.float32), e3.copy(), e3.copy(), np.zeros(0),
              _empty3(np.float32), ld, lc)
    return with_triangles(s, tri)


# ---------------------------------------------------------------------------
# The workloads: one tiny case, the 26,318-object protein-like scene at the
# paper's two resolutions, a serving stream and a 1M-object camera orbit.
# ---------------------------------------------------------------------------

PROTEIN_SPHERES = 13159          # 13,159 + 13,159 = 26,318 objects
PROTEIN_RADIUS = 40.0
RES_1MP = (965, 1137)            # paper: -res 965 1137
RES_4MP = (1930, 2274)           # paper: weak-scaling middle point
RES_17MP = (3860, 4548)          # paper: -res 3860 4548


def tiny_workload():
    scene = tiny_scene(seed=1)
    cam = Camera((0.0, 0.0, 30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 128, 128)
    params = Params(ao_samples=8, seed=1, view_id=0)
    return scene, cam, params


def protein_scene(seed: int = 2) -> Scene:
    return random_walk_scene(PROTEIN_SPHERES, PROTEIN_RADIUS, seed)


def protein_camera(res=RES_1MP) -> Camera:
    return Camera((0.0, 0.0, 120.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0,
                  int(res[0]), int(res[1]))


def protein_workload(res=RES_1MP, seed: int = 2):
    return protein_scene(seed), protein_camera(res), Params(ao_samples=16, seed=2)


def serving_radius(n_total: int) -> float:
    """Ball radius for a serving scene of n_total objects: the protein
    density kept constant, R = 40 (n / 26318)^(1/3)."""
    return PROTEIN_RADIUS * (n_total / (2.0 * PROTEIN_SPHERES)) ** (1.0 / 3.0)


def serving_pool(n_scenes: int = 16, seed0: int = 100, n_min: int = 2000,
                 n_max: int = 200000) -> List[Scene]:
    """Pool of walk scenes with total object counts log-uniform in
    [n_min, n_max], half spheres and half cylinders."""
    out = []
    for k in range(n_scenes):
        rng = np.random.default_rng(seed0 + k)
        n_tot = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        n_s = max(n_tot // 2, 1)
        out.append(random_walk_scene(n_s, serving_radius(2 * n_s), seed0 + k))
    return out


SERVING_RESOLUTIONS = [(256, 256), RES_1MP, (1920, 1080)]


def serving_requests(pool_radii: List[float], n_jobs: int, rate_hz: float = 50.0,
                     seed: int = 3) -> list:
    """Poisson arrival stream of render jobs over a scene pool.  Each job:
    (arrival_s, scene_index, Camera, Params)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for _ in range(n_jobs):
        t += rng.exponential(1.0 / rate_hz)
        si = int(rng.integers(len(pool_radii)))
        W, H = SERVING_RESOLUTIONS[int(rng.integers(len(SERVING_RESOLUTIONS)))]
        az = rng.uniform(0.0, 2.0 * math.pi)
        dist = 3.0 * pool_radii[si]
        eye = (dist * math.sin(az), 0.0, dist * math.cos(az))
        cam = Camera(eye, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, W, H)
        S = int(rng.integers(4, 33))
        params = Params(ao_samples=S, seed=int(rng.integers(1 << 62)), view_id=0)
        jobs.append((t, si, cam, params))
    return jobs


ORBIT_SPHERES = 500000
ORBIT_RADIUS = 250.0
ORBIT_VIEWS = 64
RES_1080P = (1920, 1080)


def orbit_scene(seed: int = 4) -> Scene:
    return random_walk_scene(ORBIT_SPHERES, ORBIT_RADIUS, seed)


def orbit_cameras(n_views: int = ORBIT_VIEWS, dist: float = 625.0,
                  res=RES_1080P) -> List[Camera]:
    cams = []
    for k in range(n_views):
        th = 2.0 * math.pi * k / n_views
        cams.append(Camera((dist * math.sin(th), 0.0, dist * math.cos(th)),
                           (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0,
                           int(res[0]), int(res[1])))
    return cams


def orbit_params(n_views: int = ORBIT_VIEWS) -> List[Params]:
    return [Params(ao_samples=32, seed=4, view_id=k) for k in range(n_views)]


def sample_pixels(width: int, height: int, n: int, seed: int) -> np.ndarray:
    """Distinct seeded pixel indices (j*W + i), sorted, for sampled checks at
    full frame sizes."""
    rng = np.random.default_rng(seed)
    total = width * height
    n = min(n, total)
    return np.sort(rng.choice(total, size=n, replace=False)).astype(np.int64)
