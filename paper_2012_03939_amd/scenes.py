"""Seeded synthetic inputs for every workload of the differentiable path tracer.

This module holds no arithmetic of the rendering method: it only builds meshes,
per-face materials, point lights, an HDR environment map and cameras, all as
plain float32/int32 numpy arrays.  Both the HIP library and the FP64 CPU oracle
receive exactly these arrays, so the two implementations never share anything
but their inputs.

The paper's own data (Stanford meshes inside a Cornell box, real captures;
Sec. 4.1 and 4.2) are not available; these generators stand in for them with
the same kind of content: a closed triangle mesh around the origin, per-face
Torrance-Sparrow parameters (Sec. 3.3, "Representation"), point lights or an
HDR environment map (Sec. 3.1), and calibrated cameras on a ring or a Fibonacci
sphere (Sec. 4.1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# --------------------------------------------------------------------------
# camera record shared by both implementations (host memory, plain numbers)
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple
    fov_y_deg: float
    width: int
    height: int

    def as_row(self) -> List[float]:
        return [*map(float, self.eye), *map(float, self.target), *map(float, self.up),
                float(self.fov_y_deg)]


@dataclasses.dataclass
class Scene:
    V: np.ndarray            # float32 [nv, 3]
    F: np.ndarray            # int32   [nf, 3], counter-clockwise seen from outside
    mat: np.ndarray          # float32 [nf, 7] = kd rgb, ks rgb, roughness
    lights: np.ndarray       # float32 [nl, 6] = position xyz, intensity rgb
    env: Optional[np.ndarray]  # float32 [he, we, 3] or None
    scene_id: int = 0

    @property
    def nv(self):
        return int(self.V.shape[0])

    @property
    def nf(self):
        return int(self.F.shape[0])


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

_T = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array([(-1, _T, 0), (1, _T, 0), (-1, -_T, 0), (1, -_T, 0),
                   (0, -1, _T), (0, 1, _T), (0, -1, -_T), (0, 1, -_T),
                   (_T, 0, -1), (_T, 0, 1), (-_T, 0, -1), (-_T, 0, 1)], dtype=np.float64)
_ICO_F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
          (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
          (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
          (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]


def geodesic_sphere(k: int, radius: float = 1.0):
    """Geodesic icosphere of frequency k: 20k^2 faces, 10k^2+2 vertices.

    Every icosahedron face is cut into a k-by-k triangular grid and the grid
    points are pushed onto the sphere.  Shared grid points are merged by their
    exact integer barycentric key, so the mesh is closed and 2-manifold.
    """
    if k < 1:
        raise ValueError("k must be >= 1")
    keys = {}
    pts = []

    def vid(a, b, c, wa, wb, wc):
        key = tuple(sorted((v, w) for v, w in ((a, wa), (b, wb), (c, wc)) if w > 0))
        idx = keys.get(key)
        if idx is None:
            p = (wa * _ICO_V[a] + wb * _ICO_V[b] + wc * _ICO_V[c]) / k
            idx = len(pts)
            keys[key] = idx
            pts.append(p)
        return idx

    faces = []
    for (a, b, c) in _ICO_F:
        grid = {}
        for i in range(k + 1):
            for j in range(k + 1 - i):
                grid[i, j] = vid(a, b, c, k - i - j, i, j)
        for i in range(k):
            for j in range(k - i):
                faces.append((grid[i, j], grid[i + 1, j], grid[i, j + 1]))
                if i + j < k - 1:
                    faces.append((grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]))
    V = np.asarray(pts, dtype=np.float64)
    V = radius * V / np.linalg.norm(V, axis=1, keepdims=True)
    F = np.asarray(faces, dtype=np.int32)
    # orient every face outward (the icosahedron list above is outward already;
    # this keeps the invariant explicit)
    c = V[F].mean(axis=1)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = (n * c).sum(axis=1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def torus(nu: int = 200, nv: int = 100, R: float = 1.0, r: float = 0.4):
    """Torus around the y axis, nu x nv quads split into 2*nu*nv outward faces.

    Returns (V, F, tube_normals)."""
    th = 2.0 * np.pi * np.arange(nu) / nu
    ph = 2.0 * np.pi * np.arange(nv) / nv
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    ring = R + r * np.cos(PH)
    V = np.stack([ring * np.cos(TH), r * np.sin(PH), ring * np.sin(TH)], axis=-1).reshape(-1, 3)
    N = np.stack([np.cos(PH) * np.cos(TH), np.sin(PH), np.cos(PH) * np.sin(TH)], axis=-1).reshape(-1, 3)
    idx = np.arange(nu * nv).reshape(nu, nv)
    a = idx
    b = np.roll(idx, -1, axis=0)
    c = np.roll(idx, -1, axis=1)
    d = np.roll(np.roll(idx, -1, axis=0), -1, axis=1)
    F = np.concatenate([np.stack([a, c, b], -1).reshape(-1, 3),
                        np.stack([b, c, d], -1).reshape(-1, 3)]).astype(np.int32)
    cen = V[F].mean(axis=1)
    fn = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    out = N[F].mean(axis=1)
    flip = (fn * out).sum(axis=1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    del cen
    return V, F, N


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise(p: np.ndarray, seed: int, octaves: int = 3, base_freq: float = 2.0) -> np.ndarray:
    """3-octave value noise in [-1, 1]: hashed lattice values, quintic-fade trilinear
    interpolation, lacunarity 2, gain 0.5, normalised by the sum of gains."""
    rng = np.random.default_rng(seed)
    total = np.zeros(p.shape[0])
    amp, freq, norm = 1.0, base_freq, 0.0
    for _ in range(octaves):
        perm = rng.permutation(256)
        vals = rng.uniform(-1.0, 1.0, 256)
        q = p * freq
        i0 = np.floor(q).astype(np.int64)
        f = q - i0
        w = _fade(f)
        acc = np.zeros(p.shape[0])
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    h = perm[(perm[(perm[(i0[:, 0] + dx) & 255] + i0[:, 1] + dy) & 255] + i0[:, 2] + dz) & 255]
                    wx = w[:, 0] if dx else 1.0 - w[:, 0]
                    wy = w[:, 1] if dy else 1.0 - w[:, 1]
                    wz = w[:, 2] if dz else 1.0 - w[:, 2]
                    acc += wx * wy * wz * vals[h]
        total += amp * acc
        norm += amp
        amp *= 0.5
        freq *= 2.0
    return total / norm


def noise_sphere(k: int, amplitude: float = 0.1, noise_seed: int = 7):
    V, F = geodesic_sphere(k)
    n = value_noise(V, noise_seed)
    V = V * (1.0 + amplitude * n)[:, None]
    return V, F


def noise_torus(nu=200, nv=100, amplitude=0.1, noise_seed=7):
    V, F, N = torus(nu, nv)
    n = value_noise(V, noise_seed)
    V = V + (amplitude * n)[:, None] * N
    return V, F


# --------------------------------------------------------------------------
# materials, lights, environment map, cameras
# --------------------------------------------------------------------------

def random_materials(nf: int, rng: np.random.Generator) -> np.ndarray:
    """kd ~ U[0.1,0.9]^3, ks ~ U[0,0.3]^3, roughness log-uniform in [0.05, 0.5]."""
    kd = rng.uniform(0.1, 0.9, (nf, 3))
    ks = rng.uniform(0.0, 0.3, (nf, 3))
    al = np.exp(rng.uniform(np.log(0.05), np.log(0.5), (nf, 1)))
    return np.concatenate([kd, ks, al], axis=1).astype(np.float32)


def mesh_color_texels(face_mat: np.ndarray, r: int, rng: np.random.Generator) -> np.ndarray:
    """Mesh-colour texels at resolution r ([nf (r+1)(r+2)/2, 7], triangle blocks in
    face order): each texel is its face's material with kd and ks scaled by
    U[0.6, 1.4] per channel (clipped to [0, 1]) and roughness by U[0.7, 1.3]."""
    T = (r + 1) * (r + 2) // 2
    tex = np.repeat(np.asarray(face_mat, np.float64), T, axis=0)
    tex[:, :6] = np.clip(tex[:, :6] * rng.uniform(0.6, 1.4, (tex.shape[0], 6)), 0.0, 1.0)
    tex[:, 6] = tex[:, 6] * rng.uniform(0.7, 1.3, tex.shape[0])
    return tex.astype(np.float32)


def uniform_materials(nf: int, kd=0.5, ks=0.04, rough=0.3) -> np.ndarray:
    m = np.empty((nf, 7), np.float32)
    m[:, 0:3] = kd
    m[:, 3:6] = ks
    m[:, 6] = rough
    return m


def hemisphere_lights(n: int, rng: np.random.Generator, radius=4.0, imin=5.0, imax=20.0):
    out = np.zeros((n, 6), np.float32)
    for i in range(n):
        while True:
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            if d[1] > 0.05:
                break
        inten = rng.uniform(imin, imax)
        out[i, :3] = radius * d
        out[i, 3:] = inten
    return out


def gaussian_lobe_envmap(rng: np.random.Generator, width=512, height=256, nlobes=6,
                         base=0.05) -> np.ndarray:
    """Equirectangular RGB map [height, width, 3]: base + sum of Gaussian lobes
    (angular sigma U[0.05,0.3] rad, log-normal intensity mu=1 sigma=1.5, tint U[0.5,1]^3).
    Row 0 looks along +y; a texel centre direction is (sin t sin p, cos t, sin t cos p)."""
    th = np.pi * (np.arange(height) + 0.5) / height
    ph = 2.0 * np.pi * (np.arange(width) + 0.5) / width
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(TH) * np.sin(PH), np.cos(TH), np.sin(TH) * np.cos(PH)], -1)
    img = np.full((height, width, 3), base, np.float64)
    for _ in range(nlobes):
        mu = rng.normal(size=3)
        mu /= np.linalg.norm(mu)
        sigma = rng.uniform(0.05, 0.3)
        inten = rng.lognormal(1.0, 1.5)
        tint = rng.uniform(0.5, 1.0, 3)
        ang = np.arccos(np.clip(dirs @ mu, -1.0, 1.0))
        img += inten * tint[None, None, :] * np.exp(-ang ** 2 / (2 * sigma ** 2))[..., None]
    return img.astype(np.float32)


def fibonacci_sphere(n: int) -> np.ndarray:
    ga = np.pi * (3.0 - 5.0 ** 0.5)
    i = np.arange(n)
    y = 1.0 - 2.0 * (i + 0.5) / n
    r = np.sqrt(1.0 - y * y)
    return np.stack([r * np.cos(ga * i), y, r * np.sin(ga * i)], -1)


def look_at_origin(eye, w, h, fov=45.0) -> Camera:
    return Camera(tuple(float(x) for x in eye), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fov, int(w), int(h))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    scenes: List[Scene]
    cams: List[Camera]
    cam_scene: List[int]
    spp: int
    bounces: int
    seed: int = 0
    edges: bool = True

    @property
    def n_paths(self) -> int:
        return sum(c.width * c.height for c in self.cams) * self.spp


def small_sphere(res: int = 64, spp: int = 4) -> Workload:
    """One 64x64 view of a 320-face icosphere (radius 1) lit by one point light of
    intensity 10 at (2,2,2); direct lighting only; 4 spp; seed 0."""
    rng = np.random.default_rng(1000)
    V, F = geodesic_sphere(4)
    sc = Scene(V.astype(np.float32), F, random_materials(F.shape[0], rng),
               np.array([[2, 2, 2, 10, 10, 10]], np.float32), None, 0)
    cams = [look_at_origin((0.0, 0.0, 3.0), res, res)]
    return Workload("sphere320_1x64sq_4spp_b1_point", [sc], cams, [0], spp, 1, 0)


def noise_sphere_ring(res: int = 256, nviews: int = 8, spp: int = 16) -> Workload:
    """8 views on a ring at distance 3; 9,680-face noise-displaced sphere; 3 point
    lights of intensity U[5,20] on a radius-4 upper hemisphere; 2 bounces; 16 spp."""
    rng = np.random.default_rng(1001)
    V, F = noise_sphere(22, 0.1, noise_seed=11)
    sc = Scene(V.astype(np.float32), F, random_materials(F.shape[0], rng),
               hemisphere_lights(3, rng), None, 0)
    cams = []
    for i in range(nviews):
        a = 2.0 * np.pi * i / nviews
        cams.append(look_at_origin((3.0 * np.sin(a), 0.0, 3.0 * np.cos(a)), res, res))
    return Workload("noisesphere9680_8x256sq_16spp_b2_3point", [sc], cams, [0] * nviews, spp, 2, 0)


def torus_envmap(res: int = 512, nviews: int = 16, spp: int = 16, bounces: int = 3) -> Workload:
    """40,000-face noise-displaced torus (R=1, r=0.4) under a 512x256 six-lobe HDR
    environment map; 16 views at 512^2 on a Fibonacci sphere at distance 4;
    3 bounces; silhouette edge sampling on."""
    rng = np.random.default_rng(1002)
    V, F = noise_torus(200, 100, 0.1, noise_seed=13)
    env = gaussian_lobe_envmap(rng)
    sc = Scene(V.astype(np.float32), F, random_materials(F.shape[0], rng),
               np.zeros((0, 6), np.float32), env, 0)
    eyes = 4.0 * fibonacci_sphere(nviews)
    cams = [look_at_origin(e, res, res) for e in eyes]
    return Workload(f"torus40k_env512x256_{nviews}x{res}sq_{spp}spp_b{bounces}", [sc], cams,
                    [0] * nviews, spp, bounces, 0)


def batched_uneven(spp: int = 16, bounces: int = 2) -> Workload:
    """4 noise spheres (2k, 8k, 20,480, 60,500 faces), 24 views (6 per scene) at
    resolutions drawn from {128,256,384,512}^2; scenes 0 and 2 under 3 point
    lights, scenes 1 and 3 under the six-lobe environment map."""
    rng = np.random.default_rng(1003)
    scenes = []
    cams, cam_scene = [], []
    for s, k in enumerate((10, 20, 32, 55)):
        V, F = noise_sphere(k, 0.1, noise_seed=17 + s)
        mat = random_materials(F.shape[0], rng)
        if s % 2 == 0:
            sc = Scene(V.astype(np.float32), F, mat, hemisphere_lights(3, rng), None, s)
        else:
            sc = Scene(V.astype(np.float32), F, mat, np.zeros((0, 6), np.float32),
                       gaussian_lobe_envmap(rng), s)
        scenes.append(sc)
        eyes = 3.0 * fibonacci_sphere(6)
        for e in eyes:
            r = int(rng.choice([128, 256, 384, 512]))
            cams.append(look_at_origin(e, r, r))
            cam_scene.append(s)
    return Workload("batched4scenes_24views_uneven_16spp_b2", scenes, cams, cam_scene, spp, bounces, 0)


def optimisation_problem(nviews: int = 32, res: int = 256):
    """Target: 100,820-face noise sphere with random materials; start: 5,120-face
    sphere (different noise field) with kd 0.5, ks 0.04, roughness 0.3; envmap
    lighting as in the torus workload; views on a Fibonacci sphere at distance 3."""
    rng = np.random.default_rng(1004)
    Vt, Ft = noise_sphere(71, 0.1, noise_seed=23)
    env = gaussian_lobe_envmap(rng)
    target = Scene(Vt.astype(np.float32), Ft, random_materials(Ft.shape[0], rng),
                   np.zeros((0, 6), np.float32), env, 0)
    V0, F0 = noise_sphere(16, 0.05, noise_seed=29)
    start = Scene(V0.astype(np.float32), F0, uniform_materials(F0.shape[0]),
                  np.zeros((0, 6), np.float32), env, 1)
    eyes = 3.0 * fibonacci_sphere(nviews)
    cams = [look_at_origin(e, res, res) for e in eyes]
    return target, start, cams


def perturbed_vertices(V: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (V + rng.normal(0.0, sigma, V.shape)).astype(np.float32)


def camera_rows(cams: List[Camera]) -> np.ndarray:
    return np.array([c.as_row() for c in cams], np.float64)


def camera_res(cams: List[Camera]) -> np.ndarray:
    return np.array([(c.width, c.height) for c in cams], np.int32)
