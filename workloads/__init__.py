"""Seeded synthetic inputs for the MC-BEM / dense-BEM hot path.

This module holds no arithmetic of the method itself: no areas, no
normals, no kernels, no sampling of the estimator.  It only builds the
inputs that both the CPU oracle and the GPU library consume:

* closed triangle meshes (icosphere, noise-displaced ellipsoid,
  cube-sphere ellipsoid), counter-clockwise seen from outside;
* Neumann data (constant, cos(theta), random complex spherical-harmonic
  combinations up to a given degree), given per vertex;
* wavenumbers from frequencies (k = 2 pi f / c, c = 343 m/s);
* query points as (triangle, b1, b2) barycentric records.

The paper's own objects and modal data (Armadillo, Bowl, Bunny, Dragon,
Plate, the phone/cup scenes) are not available, so these stand in for
them at the sizes the paper works with (20k-triangle scenes, 1K-10K
samples, 125 Hz - 8 kHz, objects of 0.1-0.2 m; Sections 5-6).

Random numbers here come from numpy's PCG64 (``numpy.random.default_rng``)
seeded per purpose; none of them are the estimator's own samples, which
both sides draw from the counter generator given by the seed argument.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.special as sps

SOUND_SPEED = 343.0  # m/s
BASE_SEED = 20250606


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int32)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def _orient_outward(v, f):
    """Flip triangles whose winding points towards the origin (star-shaped meshes)."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    f = f.copy()
    bad = s < 0
    f[bad] = f[bad][:, [0, 2, 1]]
    return f


def icosphere_unit(subdiv: int):
    """Unit icosphere: 20*4^s triangles, 10*4^s+2 vertices (unit directions)."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(subdiv):
        cache = {}
        new_f = []

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key in cache:
                return cache[key]
            p = (np.asarray(verts[i]) + np.asarray(verts[j])) * 0.5
            p /= np.linalg.norm(p)
            verts.append(tuple(p))
            cache[key] = len(verts) - 1
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_f += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.asarray(new_f, dtype=np.int32)
    v = np.asarray(verts, dtype=np.float64)
    return v, _orient_outward(v, np.asarray(f, dtype=np.int32))


def icosphere(subdiv: int, radius: float = 1.0):
    u, f = icosphere_unit(subdiv)
    return u * radius, f, u


@functools.lru_cache(maxsize=128)
def _cubesphere_unit_cached(n: int):
    # grid points of the six faces, then merge duplicates on the cube edges
    g = np.linspace(-1.0, 1.0, n + 1)
    A, B = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    pts, faces = [], []
    base = 0
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            p = np.zeros((n + 1, n + 1, 3))
            p[..., axis] = sgn
            p[..., (axis + 1) % 3] = g[A]
            p[..., (axis + 2) % 3] = g[B]
            pts.append(p.reshape(-1, 3))
            idx = base + (A * (n + 1) + B)
            q00, q10 = idx[:-1, :-1], idx[1:, :-1]
            q11, q01 = idx[1:, 1:], idx[:-1, 1:]
            faces.append(np.stack([q00, q10, q11], -1).reshape(-1, 3))
            faces.append(np.stack([q00, q11, q01], -1).reshape(-1, 3))
            base += (n + 1) * (n + 1)
    pts = np.concatenate(pts)
    faces = np.concatenate(faces)
    key = np.round(pts * (2 * n)).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    order = np.argsort(first)                 # keep first-seen vertex order
    remap = np.empty_like(order)
    remap[order] = np.arange(len(order))
    v = pts[first[order]]
    f = remap[inv.reshape(-1)][faces].astype(np.int32)
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    return v, _orient_outward(v, f)


def cubesphere_unit(n: int):
    """Unit cube-sphere: 12 n^2 triangles, 6 n^2 + 2 vertices."""
    v, f = _cubesphere_unit_cached(int(n))
    return v.copy(), f.copy()


def real_sh_basis(u: np.ndarray, lmax: int) -> np.ndarray:
    """Real orthonormal spherical harmonics up to degree lmax at unit directions u.

    Returns an array of shape (len(u), (lmax+1)^2)."""
    theta = np.arccos(np.clip(u[:, 2], -1.0, 1.0))
    phi = np.arctan2(u[:, 1], u[:, 0])
    cols = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            y = sps.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                cols.append(y.real)
            elif m > 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.real)
            else:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.imag)
    return np.stack(cols, axis=1)


def noisy_ellipsoid(seed: int, subdiv: int = 5, axes=(0.10, 0.06, 0.04),
                    amp: float = 0.05, lmax: int = 6):
    """Icosphere mapped to an ellipsoid and displaced radially by a smooth
    seeded field with max |eta| = 1: x = E(u) (1 + amp * eta(u))."""
    u, f = icosphere_unit(subdiv)
    rng = np.random.default_rng([seed, 2])
    basis = real_sh_basis(u, lmax)
    coef = rng.standard_normal(basis.shape[1])
    coef[0] = 0.0
    eta = basis @ coef
    eta /= np.max(np.abs(eta))
    v = u * np.asarray(axes)[None, :] * (1.0 + amp * eta)[:, None]
    return v, f, u


def random_rotation(rng) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def cubesphere_ellipsoid(seed: int, n_tri_target: int, base_radius: float = 0.1):
    """Cube-sphere ellipsoid with random axis ratios in [0.4, 1], uniform
    scale 0.5-2x, random rotation and a translation in [-1, 1]^3 m."""
    rng = np.random.default_rng([seed, 5])
    n = max(2, int(round(math.sqrt(n_tri_target / 12.0))))
    u, f = cubesphere_unit(n)
    ratios = np.concatenate([[1.0], rng.uniform(0.4, 1.0, 2)])
    scale = rng.uniform(0.5, 2.0)
    rot = random_rotation(rng)
    shift = rng.uniform(-1.0, 1.0, 3)
    v = (u * ratios[None, :] * base_radius * scale) @ rot.T + shift[None, :]
    return v, f, u


def torus(major: float, minor: float, nu: int, nv: int):
    """Closed torus about the y axis (tube centre circle of radius `major` in
    the xz plane, tube radius `minor`), nu x nv quads split in two,
    counter-clockwise seen from outside: (V, T)."""
    u = 2.0 * np.pi * np.arange(nu) / nu
    w = 2.0 * np.pi * np.arange(nv) / nv
    U, Wv = np.meshgrid(u, w, indexing="ij")
    rad = major + minor * np.cos(Wv)
    v = np.stack([rad * np.cos(U), minor * np.sin(Wv), rad * np.sin(U)], -1).reshape(-1, 3)
    I, J = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = I * nv + J
    b = ((I + 1) % nu) * nv + J
    c = ((I + 1) % nu) * nv + (J + 1) % nv
    d = I * nv + (J + 1) % nv
    f = np.concatenate([np.stack([a, b, c], -1).reshape(-1, 3),
                        np.stack([a, c, d], -1).reshape(-1, 3)]).astype(np.int32)
    # outward: away from the tube's centre circle
    cen = v[f].mean(axis=1)
    ang = np.arctan2(cen[:, 2], cen[:, 0])
    ring = np.stack([major * np.cos(ang), np.zeros_like(ang), major * np.sin(ang)], -1)
    nrm = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    bad = np.einsum("ij,ij->i", nrm, cen - ring) < 0
    f[bad] = f[bad][:, [0, 2, 1]]
    return v, f


@dataclass
class Scene:
    """Several closed bodies in one mesh (Section 4.1.1's smooth-Neumann
    scenes): vertices and triangles of every body concatenated, the body of
    each triangle, and per-triangle Neumann data g (1 on the speaker's
    vibrating patch, 0 on every other triangle)."""
    vertices: np.ndarray
    tris: np.ndarray
    body: np.ndarray                 # (T,) int32: 0 speaker, 1.. passive bodies
    g_tri: np.ndarray                # (T,) complex128


def scene_speaker_torus(speaker_y: float, speaker_n: int = 12, torus_nu: int = 96,
                        torus_nv: int = 40, major: float = 0.06, minor: float = 0.025,
                        speaker_axes=(0.012, 0.02, 0.012), patch: float = 0.8) -> Scene:
    """A small speaker (cube-sphere ellipsoid, long axis along y) at height
    `speaker_y` on the axis of a passive torus (radius 0.06 m, tube 0.025 m,
    its hole 0.035 m wide): the speaker moves along y through the hole as the
    paper's phone moves along y past the cup (Section 6).  Only the
    speaker's lower end vibrates: g = 1 on its triangles whose unit-sphere
    direction has y < -patch, 0 elsewhere (per triangle)."""
    us, fs = cubesphere_unit(speaker_n)
    vs = us * np.asarray(speaker_axes)[None, :] + np.array([0.0, speaker_y, 0.0])[None, :]
    vt, ft = torus(major, minor, torus_nu, torus_nv)
    v = np.concatenate([vs, vt])
    f = np.concatenate([fs, ft + len(vs)]).astype(np.int32)
    body = np.concatenate([np.zeros(len(fs), np.int32), np.ones(len(ft), np.int32)])
    c = us[fs].mean(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    g = np.zeros(len(f), dtype=np.complex128)
    g[:len(fs)][c[:, 1] < -patch] = 1.0
    return Scene(v, f, body, g)


def config_scenes(n_positions: int = 16, n_modes: int = 8, n_samples: int = 2048,
                  n_queries: int = 4096, seed: int = BASE_SEED + 5, y_range=(-0.15, 0.15)):
    """Speaker-torus scenes at evenly spaced speaker heights (the condition
    variable v of Section 3.4), each with n_modes frequencies log-uniform
    200 Hz - 8 kHz and per-triangle Neumann data (the same patch for every
    frequency), random surface queries on all bodies."""
    out = []
    for i, y in enumerate(np.linspace(y_range[0], y_range[1], n_positions)):
        sc = scene_speaker_torus(float(y))
        k = wavenumber(log_uniform_freqs(n_modes, seed * 100 + i))
        g = np.ascontiguousarray(np.repeat(sc.g_tri[None, :], n_modes, axis=0))
        qt, qb = random_face_queries(len(sc.tris), n_queries, seed * 100 + i)
        out.append(MCWorkload(f"scene{i}_y{y:+.3f}", sc.vertices, sc.tris, g, k, qt, qb, n_samples,
                              seed * 100 + i, {"body": sc.body, "speaker_y": float(y)}))
    return out


# --------------------------------------------------------------------------
# Neumann data, frequencies, queries
# --------------------------------------------------------------------------
def sh_neumann(u: np.ndarray, n_modes: int, seed: int, lmax: int = 4) -> np.ndarray:
    """n_modes complex per-vertex fields sum_{l<=lmax,m} c_lm Y_lm(u), c_lm ~ CN(0,1),
    each normalised to RMS 1.  Shape (n_modes, len(u)), complex128."""
    rng = np.random.default_rng([seed, 3])
    basis = real_sh_basis(u, lmax)
    c = (rng.standard_normal((n_modes, basis.shape[1]))
         + 1j * rng.standard_normal((n_modes, basis.shape[1]))) / math.sqrt(2.0)
    g = c @ basis.T
    g /= np.sqrt(np.mean(np.abs(g) ** 2, axis=1, keepdims=True))
    return np.ascontiguousarray(g.astype(np.complex128))


def log_uniform_freqs(n: int, seed: int, lo: float = 200.0, hi: float = 8000.0) -> np.ndarray:
    rng = np.random.default_rng([seed, 4])
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def wavenumber(freq_hz):
    return 2.0 * math.pi * np.asarray(freq_hz, dtype=np.float64) / SOUND_SPEED


def vertex_queries(tris: np.ndarray, n_vertices: int):
    """One (tri, b1, b2) record per vertex: the first incident triangle and
    the corner the vertex occupies in it."""
    tri = np.full(n_vertices, -1, dtype=np.int32)
    b = np.zeros((n_vertices, 2), dtype=np.float64)
    for t in range(len(tris)):
        for c in range(3):
            vtx = tris[t, c]
            if tri[vtx] < 0:
                tri[vtx] = t
                if c == 1:
                    b[vtx] = (1.0, 0.0)
                elif c == 2:
                    b[vtx] = (0.0, 1.0)
    assert (tri >= 0).all(), "mesh has unreferenced vertices"
    return tri, b


def random_face_queries(n_tris: int, n_queries: int, seed: int):
    """Random interior surface points: triangle uniform by index, barycentrics
    uniform on the open triangle."""
    rng = np.random.default_rng([seed, 1])
    tri = rng.integers(0, n_tris, n_queries).astype(np.int32)
    a = rng.uniform(0.0, 1.0, (n_queries, 2))
    flip = a.sum(axis=1) > 1.0
    a[flip] = 1.0 - a[flip]
    a = np.clip(a, 1e-6, None)
    s = a.sum(axis=1)
    over = s > 1.0 - 1e-6
    a[over] *= (1.0 - 1e-6) / s[over, None]
    return tri, np.ascontiguousarray(a)


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------
@dataclass
class MCWorkload:
    name: str
    vertices: np.ndarray            # (V,3) float64
    tris: np.ndarray                # (T,3) int32, CCW from outside
    g: np.ndarray                   # (n_modes, V) complex128, per-vertex Neumann data
    k: np.ndarray                   # (n_modes,) float64 wavenumbers
    q_tri: np.ndarray               # (Q,) int32
    q_b: np.ndarray                 # (Q,2) float64
    n_samples: int
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def n_modes(self):
        return len(self.k)

    @property
    def n_queries(self):
        return len(self.q_tri)

    def pair_evals(self):
        """Algorithmic pair evaluations per solve: N(N-1) + Q N per mode."""
        n = self.n_samples
        return self.n_modes * (n * (n - 1) + self.n_queries * n)


def config_pulsating_sphere(n_samples: int = 256, seed: int = BASE_SEED + 0):
    """Unit icosphere (1280 tri, 642 vert), v_n = 1, k = 2, vertex queries."""
    v, f, _ = icosphere(3, 1.0)
    g = np.ones((1, len(v)), dtype=np.complex128)
    qt, qb = vertex_queries(f, len(v))
    return MCWorkload("pulsating_sphere_ico3_k2", v, f, g, np.array([2.0]), qt, qb,
                      n_samples, seed, {"radius": 1.0})


def config_oscillating_sphere(n_samples: int = 4096, seed: int = BASE_SEED + 1,
                              ka=(1.0, 5.0, 10.0), subdiv: int = 4, radius: float = 0.1):
    """Icosphere of radius 0.1 m (5120 tri, 2562 vert), v_n = cos(theta), k a in {1,5,10}."""
    v, f, u = icosphere(subdiv, radius)
    k = np.asarray(ka, dtype=np.float64) / radius
    g = np.repeat(u[None, :, 2].astype(np.complex128), len(k), axis=0)
    qt, qb = vertex_queries(f, len(v))
    return MCWorkload(f"oscillating_sphere_ico{subdiv}", v, f, np.ascontiguousarray(g), k,
                      qt, qb, n_samples, seed, {"radius": radius, "u": u})


def config_precision(seed: int = BASE_SEED + 2, n_modes: int = 32, n_queries: int = 4096,
                     n_samples: int = 1024, subdiv: int = 5):
    """Noise-displaced ellipsoid 0.10 x 0.06 x 0.04 m (20480 tri), 32 modes of random
    SH Neumann data up to degree 4, frequencies log-uniform 200 Hz - 8 kHz,
    4096 random surface queries, 1024 samples."""
    v, f, u = noisy_ellipsoid(seed, subdiv)
    g = sh_neumann(u, n_modes, seed)
    k = wavenumber(log_uniform_freqs(n_modes, seed))
    qt, qb = random_face_queries(len(f), n_queries, seed)
    return MCWorkload(f"noisy_ellipsoid_{len(f)}tri_{n_modes}modes_Q{n_queries}_N{n_samples}",
                      v, f, g, k, qt, qb, n_samples, seed)


def log_uniform_int(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size)).round().astype(np.int64)


def config_batched(seed: int = BASE_SEED + 3, n_instances: int = 256, scale: float = 1.0):
    """256 cube-sphere ellipsoid instances of 2k-40k triangles (log-uniform),
    8-64 modes, 2k-16k queries, 512-2048 samples.  ``scale`` shrinks the
    per-instance sizes for tests."""
    rng = np.random.default_rng([seed, 6])
    out = []
    for i in range(n_instances):
        t_target = int(log_uniform_int(rng, 2000, 40000) * scale)
        n_modes = int(rng.integers(8, 65))
        q = int(log_uniform_int(rng, 2000, 16000) * scale)
        n = int(log_uniform_int(rng, 512, 2048) * scale)
        v, f, u = cubesphere_ellipsoid(seed * 1000 + i, max(t_target, 48))
        g = sh_neumann(u, n_modes, seed * 1000 + i)
        k = wavenumber(log_uniform_freqs(n_modes, seed * 1000 + i))
        qt, qb = random_face_queries(len(f), max(q, 1), seed * 1000 + i)
        out.append(MCWorkload(f"batch{i}", v, f, g, k, qt, qb, max(n, 2), seed * 1000 + i))
    return out


@dataclass
class ServedMesh:
    vertices: np.ndarray
    tris: np.ndarray
    g_vertex: np.ndarray            # (pool_modes, V) complex128, per-vertex Neumann pool
    g_tri: np.ndarray               # (dense_modes, T) complex128, per-triangle Neumann pool
    q_tri: np.ndarray               # (pool_queries,) int32
    q_b: np.ndarray                 # (pool_queries, 2) float64


@dataclass
class ServedRequest:
    kind: str                       # "mc" or "dense"
    mesh: int                       # index into the resident meshes
    m0: int                         # first mode of the mesh's pool
    k: np.ndarray                   # (n_modes,) wavenumbers
    n_queries: int                  # Monte-Carlo: first Q queries of the pool
    n_samples: int
    seed: int
    gap: float                      # unit-rate exponential inter-arrival gap

    @property
    def n_modes(self):
        return len(self.k)

    def pair_evals(self):
        if self.kind != "mc":
            return 0
        n = self.n_samples
        return self.n_modes * (n * (n - 1) + self.n_queries * n)


def config_served(seed: int = BASE_SEED + 4, n_meshes: int = 64, n_requests: int = 2000,
                  t_range=(1000, 50000), q_range=(1, 16384), n_range=(512, 2048),
                  pool_modes: int = 64, dense_fraction: float = 0.1, dense_max_tris: int = 8000,
                  dense_modes: int = 4):
    """Resident cube-sphere meshes of T log-uniform in t_range and a request
    stream over them.  Monte-Carlo requests: modes uniform {1..pool_modes}
    (a contiguous slice of the mesh's Neumann pool, wavenumbers of their own,
    log-uniform 200 Hz - 8 kHz), Q log-uniform in q_range (the first Q of the
    mesh's query pool), N log-uniform in n_range.  Dense requests (a
    dense_fraction share) go to meshes of at most dense_max_tris triangles
    with 1..dense_modes modes.  Arrivals are Poisson: `gap` is a unit-rate
    exponential, scaled by 1/rate by the caller."""
    rng = np.random.default_rng([seed, 7])
    meshes = []
    for i in range(n_meshes):
        t_target = int(log_uniform_int(rng, *t_range))
        v, f, u = cubesphere_ellipsoid(seed * 1000 + i, max(t_target, 48))
        g_v = sh_neumann(u, pool_modes, seed * 1000 + i)
        c = u[f].mean(axis=1)
        c /= np.linalg.norm(c, axis=1, keepdims=True)
        g_t = sh_neumann(c, dense_modes, seed * 1000 + i + 500)
        qt, qb = random_face_queries(len(f), q_range[1], seed * 1000 + i)
        meshes.append(ServedMesh(v, f, g_v, g_t, qt, qb))
    small = [i for i, m in enumerate(meshes) if len(m.tris) <= dense_max_tris]
    reqs = []
    for r in range(n_requests):
        dense = bool(small) and rng.random() < dense_fraction
        if dense:
            mi = int(rng.choice(small))
            M = int(rng.integers(1, dense_modes + 1))
            m0 = int(rng.integers(0, dense_modes - M + 1))
            q, n = 0, 0
        else:
            mi = int(rng.integers(0, n_meshes))
            M = int(rng.integers(1, pool_modes + 1))
            m0 = int(rng.integers(0, pool_modes - M + 1))
            q = int(log_uniform_int(rng, *q_range))
            n = int(log_uniform_int(rng, *n_range))
        k = wavenumber(log_uniform_freqs(M, seed * 100000 + r))
        reqs.append(ServedRequest("dense" if dense else "mc", mi, m0, k, q, max(n, 2),
                                  seed * 100000 + r, float(rng.exponential(1.0))))
    return meshes, reqs


# ------------------------------------------------- neural-field training rows
def nf_rows(B: int, n_v: int, seed: int, r_lo: float = 1.5, r_hi: float = 3.0):
    """Seeded listener rows of the neural field's training shell (Section
    3.4): directions uniform on the sphere (theta = arccos(1 - 2 u)), radius
    uniform in [r_lo, r_hi], condition variables and normalised frequency
    uniform in [0, 1].  Returns float64 arrays theta, phi, r, v [B, n_v], f."""
    rng = np.random.default_rng([seed, 31])
    th = np.arccos(1.0 - 2.0 * rng.uniform(0.0, 1.0, B))
    ph = rng.uniform(0.0, 2.0 * np.pi, B)
    r = rng.uniform(r_lo, r_hi, B)
    v = rng.uniform(0.0, 1.0, (B, n_v))
    f = rng.uniform(0.0, 1.0, B)
    return th, ph, r, v, f


def nf_smooth_target(th, ph, r, v, f, n_out: int = 1):
    """A smooth positive stand-in for |p| over the shell (synthetic training
    values; output o adds a phase o to the azimuthal term)."""
    vs = v.sum(axis=1) if v.shape[1] else np.zeros_like(th)
    cols = [(1.0 + 0.5 * np.cos(th) * np.sin(ph + 2.0 * vs + o) + 0.3 * f) / r for o in range(n_out)]
    return np.stack(cols, 1)
