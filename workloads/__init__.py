"""Seeded synthetic inputs for the batched manifold-walk path.

This module is shared by the tests, the benchmark and the oracle harness.  It
holds *data generation only*: triangle meshes, analytic spheres and random
endpoint batches.  It contains none of the method's arithmetic (no
constraints, no walks, no seeds, no guide).  The paper's scenes are
third-party assets that are not available, so the synthetic scenes below stand
in for them; the recipe of each is stated in its docstring.

Every random draw uses numpy's Philox bit generator keyed by ``(seed,
stream)``, so a given (workload, seed) always produces the same arrays.

Array layout conventions (shared by every consumer):

* points / directions in a batch are structure-of-arrays ``float32[3, N]``;
* chain length ``length[N]`` is ``uint8`` in 1..8;
* chain type ``types[N]`` is a ``uint8`` bitmask, bit ``i`` set when vertex
  ``i+1`` is a transmission (T) and clear for a reflection (R);
* ``obj1[N]`` (``int32``) selects how the first specular vertex of a p_0
  seed is drawn: an object id (uniform by area on it), ``-1`` (uniform over
  all specular objects) or ``-2`` (direction mode: w_D uniform in a cone
  about n_D whose half-angle the workload states in ``SEED_CONE_DEG``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MAX_LEN = 8

MAT_MIRROR = 0       # ideal conductor: reflection only
MAT_DIELECTRIC = 1   # smooth dielectric: reflection and transmission

# stream ids for the endpoint generators (key word 1 of the Philox generator)
STREAM_SCENE = 1
STREAM_ENDPOINTS = 2
STREAM_TRAINING = 3
STREAM_LOSS = 4

P0_ANY_OBJECT = -1
P0_DIRECTION = -2


def rng(seed: int, stream: int) -> np.random.Generator:
    """numpy Generator on Philox4x64-10 keyed by (seed, stream)."""
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


@dataclasses.dataclass
class HeightField:
    """Sine-sum height field z(x, y) = z0 + sum_k a_k sin(f_k (cos psi_k x + sin psi_k y) + phi_k).

    The grid has ``res x res`` vertices spanning ``[x0, x1] x [y0, y1]``.
    Cell (i, j) is split along its (i, j)-(i+1, j+1) diagonal; triangle ids
    are ``first_tri + 2 (j (res-1) + i) + {0, 1}``; vertex ids are
    ``first_vert + j res + i``.  The outward (air-side) normal is +z.
    """
    obj: int
    res: int
    x0: float
    x1: float
    y0: float
    y1: float
    z0: float
    amp: np.ndarray     # [S]
    freq: np.ndarray    # [S] angular frequency, rad per unit length
    psi: np.ndarray     # [S] direction angle
    phase: np.ndarray   # [S]
    first_vert: int = 0
    first_tri: int = 0


@dataclasses.dataclass
class Scene:
    verts: np.ndarray          # float32 [V, 3]
    normals: np.ndarray        # float32 [V, 3] unit vertex (shading) normals
    tris: np.ndarray           # int32 [T, 3] vertex indices, counter-clockwise about the outward normal
    tri_obj: np.ndarray        # int32 [T] object id per triangle
    obj_material: np.ndarray   # int32 [O]
    obj_ior: np.ndarray        # float32 [O] index of refraction inside the object (outside is 1)
    spheres: np.ndarray        # float32 [S, 4] centre xyz, radius
    sphere_obj: np.ndarray     # int32 [S]
    scale: float               # longest side of the specular geometry's bounding box
    heightfields: List[HeightField] = dataclasses.field(default_factory=list)
    name: str = ""

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def n_objects(self) -> int:
        return int(self.obj_material.shape[0])


def _empty_mesh():
    return (np.zeros((0, 3), np.float64), np.zeros((0, 3), np.float64),
            np.zeros((0, 3), np.int64), np.zeros((0,), np.int64))


def _finish(name, verts, normals, tris, tri_obj, mats, iors, spheres, sphere_obj, scale, hfs=()):
    return Scene(
        verts=np.ascontiguousarray(verts, np.float32),
        normals=np.ascontiguousarray(normals, np.float32),
        tris=np.ascontiguousarray(tris, np.int32).reshape(-1, 3),
        tri_obj=np.ascontiguousarray(tri_obj, np.int32),
        obj_material=np.asarray(mats, np.int32),
        obj_ior=np.asarray(iors, np.float32),
        spheres=np.asarray(spheres, np.float32).reshape(-1, 4),
        sphere_obj=np.asarray(sphere_obj, np.int32),
        scale=float(scale),
        heightfields=list(hfs),
        name=name,
    )


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------

def sphere_mirror_scene() -> Scene:
    """Analytic unit mirror sphere at the origin (object 0). Scale L = 2."""
    v, n, t, o = _empty_mesh()
    return _finish("sphere_mirror", v, n, t, o, [MAT_MIRROR], [1.0],
                   [[0.0, 0.0, 0.0, 1.0]], [0], 2.0)


def icosphere(subdiv: int):
    """Unit icosphere: the 12-vertex icosahedron with vertices at cyclic
    permutations of (0, +-1, +-phi), each face split 4-to-1 ``subdiv`` times
    with edge midpoints pushed onto the unit sphere.  Returns float64
    vertices and int64 faces (counter-clockwise seen from outside)."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
         (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
         (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, np.float64) / np.linalg.norm(p) for p in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts), np.array(faces, np.int64)


def icosphere_glass_scene(subdiv: int = 4, radius: float = 1.0, ior: float = 1.5) -> Scene:
    """Triangulated glass sphere (object 0): icosphere of ``subdiv`` levels,
    exact vertex normals (position / radius).  subdiv 4 gives 2562 vertices and
    5120 triangles.  Scale L = 2 radius."""
    v, f = icosphere(subdiv)
    return _finish("icosphere_glass", v * radius, v.copy(), f, np.zeros(len(f), np.int64),
                   [MAT_DIELECTRIC], [ior], np.zeros((0, 4)), [], 2.0 * radius)


def _heightfield_mesh(hf: HeightField):
    xs = np.linspace(hf.x0, hf.x1, hf.res)
    ys = np.linspace(hf.y0, hf.y1, hf.res)
    X, Y = np.meshgrid(xs, ys)            # [j, i]
    Z = np.full_like(X, hf.z0)
    HX = np.zeros_like(X)
    HY = np.zeros_like(X)
    for a, fr, ps, ph in zip(hf.amp, hf.freq, hf.psi, hf.phase):
        arg = fr * (math.cos(ps) * X + math.sin(ps) * Y) + ph
        Z += a * np.sin(arg)
        HX += a * fr * math.cos(ps) * np.cos(arg)
        HY += a * fr * math.sin(ps) * np.cos(arg)
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    nrm = np.stack([-HX, -HY, np.ones_like(X)], -1).reshape(-1, 3)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r = hf.res
    i, j = np.meshgrid(np.arange(r - 1), np.arange(r - 1))   # [j, i]
    v00 = (j * r + i).ravel()
    v10 = v00 + 1
    v01 = v00 + r
    v11 = v01 + 1
    tris = np.empty((2 * v00.size, 3), np.int64)
    tris[0::2] = np.stack([v00, v10, v11], 1)
    tris[1::2] = np.stack([v00, v11, v01], 1)
    return verts, nrm, tris


def _random_sines(g: np.random.Generator, count: int, amp: float):
    a = np.full(count, amp)
    f = g.uniform(1.0, 8.0, count)
    psi = g.uniform(0.0, 2.0 * math.pi, count)
    ph = g.uniform(0.0, 2.0 * math.pi, count)
    return a, f, psi, ph


def water_scene(res: int = 256, seed: int = 0, n_sines: int = 8, amp: float = 0.02,
                ior: float = 1.33) -> Scene:
    """Water surface (object 0): ``res x res`` sine height field over [0, 4]^2
    at mean level z = 0, ``n_sines`` sines of amplitude ``amp`` each, angular
    frequency U[1, 8], direction and phase U[0, 2 pi).  Water (IOR 1.33) lies
    below.  res 256 gives 130,050 triangles.  Scale L = 4."""
    g = rng(seed, STREAM_SCENE)
    a, f, psi, ph = _random_sines(g, n_sines, amp)
    hf = HeightField(0, res, 0.0, 4.0, 0.0, 4.0, 0.0, a, f, psi, ph)
    v, n, t = _heightfield_mesh(hf)
    return _finish("water", v, n, t, np.zeros(len(t), np.int64), [MAT_DIELECTRIC], [ior],
                   np.zeros((0, 4)), [], 4.0, [hf])


SLAB_COUNT = 4
SLAB_GAP = 0.5
SLAB_THICK = 0.25
SLAB_SPHERE = (6.0, 2.0, -1.0, 0.5)


def interface_z(k: int) -> float:
    """Mean height of interface k (1-based, counted from the light) of the slab stack."""
    slab, bottom = divmod(k - 1, 2)
    return -SLAB_GAP * slab - (SLAB_THICK if bottom else 0.0)


def slab_stack_scene(res: int = 128, seed: int = 0, n_sines: int = 4, amp: float = 0.01,
                     ior: float = 1.5, theta: Optional[np.ndarray] = None) -> Scene:
    """Four displaced glass slabs over [0, 4]^2 plus an analytic mirror sphere.

    Slab k (0..3): top = ``res x res`` sine height field at mean z = -0.5 k
    (object 2k, outward normal +z), bottom = flat two-triangle quad at
    z = -0.5 k - 0.25 (object 2k+1, outward normal -z); glass IOR 1.5 inside.
    Interfaces 1..8 counted from the light are objects 0..7.  Mirror sphere
    (object 8): centre (6, 2, -1), radius 0.5.  Scale L = 4.

    ``theta`` (float[32]) optionally overrides the differentiable surface
    parameters: for slab k and sine s, ``theta[8k + 2s]`` is the amplitude and
    ``theta[8k + 2s + 1]`` the phase.  Frequencies and directions stay fixed.
    """
    g = rng(seed, STREAM_SCENE + 16)
    V, N, T, O = [], [], [], []
    hfs = []
    nv = 0
    nt = 0
    mats, iors = [], []
    for k in range(SLAB_COUNT):
        a, f, psi, ph = _random_sines(g, n_sines, amp)
        if theta is not None:
            a = np.array([theta[8 * k + 2 * s] for s in range(n_sines)], np.float64)
            ph = np.array([theta[8 * k + 2 * s + 1] for s in range(n_sines)], np.float64)
        hf = HeightField(2 * k, res, 0.0, 4.0, 0.0, 4.0, -SLAB_GAP * k, a, f, psi, ph, nv, nt)
        v, n, t = _heightfield_mesh(hf)
        hfs.append(hf)
        V.append(v); N.append(n); T.append(t + nv); O.append(np.full(len(t), 2 * k))
        nv += len(v); nt += len(t)
        mats.append(MAT_DIELECTRIC); iors.append(ior)
        zb = -SLAB_GAP * k - SLAB_THICK
        qv = np.array([[0, 0, zb], [4, 0, zb], [4, 4, zb], [0, 4, zb]], np.float64)
        qn = np.tile([0.0, 0.0, -1.0], (4, 1))
        qt = np.array([[0, 2, 1], [0, 3, 2]], np.int64)
        V.append(qv); N.append(qn); T.append(qt + nv); O.append(np.full(2, 2 * k + 1))
        nv += 4; nt += 2
        mats.append(MAT_DIELECTRIC); iors.append(ior)
    mats.append(MAT_MIRROR); iors.append(1.0)
    return _finish("slab_stack", np.concatenate(V), np.concatenate(N), np.concatenate(T),
                   np.concatenate(O), mats, iors, [list(SLAB_SPHERE)], [2 * SLAB_COUNT], 4.0, hfs)


def slab_theta(scene: Scene) -> np.ndarray:
    """The 32 differentiable parameters (amplitude, phase per sine) of a slab stack."""
    th = []
    for hf in scene.heightfields:
        for a, ph in zip(hf.amp, hf.phase):
            th += [a, ph]
    return np.asarray(th, np.float64)


# ---------------------------------------------------------------------------
# Endpoint batches
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Endpoints:
    xD: np.ndarray      # float32 [3, N]
    nD: np.ndarray      # float32 [3, N]
    xL: np.ndarray      # float32 [3, N]
    length: np.ndarray  # uint8 [N]
    types: np.ndarray   # uint8 [N]
    obj1: np.ndarray    # int32 [N]

    @property
    def n(self) -> int:
        return int(self.length.shape[0])

    def subset(self, idx) -> "Endpoints":
        return Endpoints(np.ascontiguousarray(self.xD[:, idx]), np.ascontiguousarray(self.nD[:, idx]),
                         np.ascontiguousarray(self.xL[:, idx]), np.ascontiguousarray(self.length[idx]),
                         np.ascontiguousarray(self.types[idx]), np.ascontiguousarray(self.obj1[idx]))


def _pack(xD, nD, xL, length, types, obj1) -> Endpoints:
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64).T.astype(np.float32))
    return Endpoints(f(xD), f(nD), f(xL), np.asarray(length, np.uint8), np.asarray(types, np.uint8),
                     np.asarray(obj1, np.int32))


def _up(n):
    return np.tile([0.0, 0.0, 1.0], (n, 1))


def sphere_mirror_endpoints(n: int = 4096, seed: int = 0) -> Endpoints:
    """Shading points uniform on z = -2 over [-2, 2]^2 facing +z, point light
    uniform in [-1, 1]^2 x [3, 4]; one reflection (type R)."""
    g = rng(seed, STREAM_ENDPOINTS)
    xD = np.stack([g.uniform(-2, 2, n), g.uniform(-2, 2, n), np.full(n, -2.0)], 1)
    xL = np.stack([g.uniform(-1, 1, n), g.uniform(-1, 1, n), g.uniform(3, 4, n)], 1)
    return _pack(xD, _up(n), xL, np.ones(n), np.zeros(n), np.full(n, -1))


def icosphere_endpoints(n: int = 1 << 20, seed: int = 0) -> Endpoints:
    """Shading points uniform on z = -1.5 over [-3, 3]^2 facing +z, point
    light at (0, 0, 3); two transmissions (type TT)."""
    g = rng(seed, STREAM_ENDPOINTS + 16)
    xD = np.stack([g.uniform(-3, 3, n), g.uniform(-3, 3, n), np.full(n, -1.5)], 1)
    xL = np.tile([0.0, 0.0, 3.0], (n, 1))
    return _pack(xD, _up(n), xL, np.full(n, 2), np.full(n, 0b11), np.full(n, -1))


def water_endpoints(n: int = 1 << 22, seed: int = 0, stream: int = STREAM_ENDPOINTS + 32) -> Endpoints:
    """Receiver points uniform in the volume [0, 4]^2 x [-2, -0.5] under the
    water, facing +z, point light at (2, 2, 3); one transmission (type T)."""
    g = rng(seed, stream)
    xD = np.stack([g.uniform(0, 4, n), g.uniform(0, 4, n), g.uniform(-2.0, -0.5, n)], 1)
    xL = np.tile([2.0, 2.0, 3.0], (n, 1))
    return _pack(xD, _up(n), xL, np.ones(n), np.ones(n), np.zeros(n))


WATER_GRID_LO = (0.0, 0.0, -2.0)
WATER_GRID_HI = (4.0, 4.0, -0.5)


def _slab_chains(g: np.random.Generator, lengths: np.ndarray):
    n = lengths.size
    xD = np.empty((n, 3))
    obj1 = np.empty(n, np.int64)
    types = np.empty(n, np.int64)
    refl = lengths == 1
    m = int(refl.sum())
    xD[refl] = np.stack([g.uniform(4, 7, m), g.uniform(0.5, 3.5, m), np.full(m, -2.0)], 1)
    obj1[refl] = 2 * SLAB_COUNT
    types[refl] = 0
    tr = ~refl
    m = int(tr.sum())
    zs = np.array([interface_z(k) - 0.5 * SLAB_THICK for k in range(1, 9)])
    xD[tr] = np.stack([g.uniform(0.5, 3.5, m), g.uniform(0.5, 3.5, m), zs[lengths[tr] - 1]], 1)
    obj1[tr] = P0_DIRECTION
    types[tr] = (1 << lengths[tr]) - 1
    return xD, obj1, types


# Half-angle of the direction-mode p_0 cone used by the slab workloads.  Every
# admissible first segment of a slab chain leaves x_D within ~34 degrees of +z
# (the light is at most 2.1 units aside and >= 3.1 units above), so 40 degrees
# covers all of them with margin.  Seeds drawn by area over a whole 4 x 4
# interface from 0.125 below it are nearly all grazing and leave the stack.
SEED_CONE_DEG = 40.0


def slab_uneven_endpoints(n: int = 1 << 23, seed: int = 0) -> Endpoints:
    """Uneven batch through the slab stack.  Length n = min(G, 8) with G
    geometric(p = 0.4) on {1, 2, ...}.  n = 1: reflection off the mirror
    sphere (seed uniform on its visible cap) from shading points uniform on
    z = -2 over [4, 7] x [0.5, 3.5].  n >= 2: n transmissions through
    interfaces n, ..., 1 from shading points uniform over [0.5, 3.5]^2 at the
    height midway between interfaces n and n + 1 (inside a slab for odd n),
    seeded in direction mode (cone of SEED_CONE_DEG about +z).  Point light at
    (2, 2, 3); all shading points face +z."""
    g = rng(seed, STREAM_ENDPOINTS + 48)
    lengths = np.minimum(g.geometric(0.4, n), MAX_LEN)
    xD, obj1, types = _slab_chains(g, lengths)
    xL = np.tile([2.0, 2.0, 3.0], (n, 1))
    return _pack(xD, _up(n), xL, lengths, types, obj1)


def slab_adjoint_endpoints(n: int = 1 << 20, seed: int = 0) -> Endpoints:
    """As :func:`slab_uneven_endpoints` with lengths uniform on {2, 3, 4}."""
    g = rng(seed, STREAM_ENDPOINTS + 64)
    lengths = g.integers(2, 5, n)
    xD, obj1, types = _slab_chains(g, lengths)
    xL = np.tile([2.0, 2.0, 3.0], (n, 1))
    return _pack(xD, _up(n), xL, lengths, types, obj1)


def loss_weights(n: int, kmax: int = MAX_LEN, seed: int = 0):
    """Fixed random cotangents for a scalar test loss
    l = sum_c (sum_i r_ci . x_ci + g_c G_c): r float32 [3, K, N], g float32 [N]."""
    g = rng(seed, STREAM_LOSS)
    r = g.standard_normal((3, kmax, n)).astype(np.float32)
    gg = g.standard_normal(n).astype(np.float32)
    return r, gg


WORKLOADS = {
    "sphere_mirror": (sphere_mirror_scene, sphere_mirror_endpoints),
    "icosphere_tt": (icosphere_glass_scene, icosphere_endpoints),
    "water_caustic": (water_scene, water_endpoints),
    "slab_uneven": (slab_stack_scene, slab_uneven_endpoints),
    "slab_adjoint": (slab_stack_scene, slab_adjoint_endpoints),
}
