"""Python driver for the FP64 CPU oracle (``nat_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The GPU library never
imports this module and this module never imports the GPU library.

Every function takes and returns numpy arrays (complex128 for complex
data) and forwards to the plain C implementation, which follows the
paper's Section 4 step by step in double precision.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "nat_oracle.c"
LIB = HERE / "liboracle.so"

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        tmp = LIB.with_suffix(".so.tmp")
        subprocess.run(["gcc", *CFLAGS, "-o", str(tmp), str(SRC), "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None

_d = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(str(LIB))
        L.orc_num_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_geometry.argtypes = [_d, _i, C.c_int32, _d, _d, _d]
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_rng_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.orc_rng_word.restype = C.c_uint64
        L.orc_cdf_search.argtypes = [_d, C.c_int32, C.c_double]
        L.orc_cdf_search.restype = C.c_int32
        L.orc_samples.argtypes = [_d, C.c_int32, C.c_int32, C.c_uint64, _i, _d]
        L.orc_surface_points.argtypes = [_d, _i, C.c_int32, _i, _d, _d]
        L.orc_poisson_candidates.argtypes = [_d, _i, _d, C.c_int32, C.c_int32, C.c_uint64, _i, _d, _d]
        L.orc_poisson_samples.argtypes = [_d, C.c_int32, _i, C.c_int32, C.c_int32, C.c_uint64,
                                          C.c_double, C.c_int32, C.c_int32, _i, _d]
        L.orc_poisson_samples.restype = C.c_int32
        L.orc_neumann_at.argtypes = [_i, C.c_int32, _d, C.c_int32, _i, _d, _d]
        L.orc_kernels.argtypes = [C.c_double, _d, _d, _d, _d, _d]
        L.orc_mc_matrix.argtypes = [C.c_int32, _d, _d, C.c_double, C.c_double, C.c_double, _d]
        L.orc_mc_rhs.argtypes = [C.c_int32, _d, C.c_double, C.c_double, C.c_double, _d, C.c_int32, _d]
        L.orc_mc_eval.argtypes = [C.c_int32, _d, C.c_void_p, C.c_double, C.c_void_p, C.c_int32,
                                  _d, _d, _d, _d, C.c_double, C.c_double, C.c_double, C.c_int32, _d]
        L.orc_free_terms.argtypes = [_d, _i, C.c_int32, _i, _d, C.c_int32, C.c_int32, _d]
        L.orc_field_points.argtypes = [_d, C.c_double, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                       C.c_double, C.c_uint64, _d, _d]
        L.orc_gmres.argtypes = [C.c_int32, _d, _d, _d, C.c_double, C.c_int32,
                                C.POINTER(C.c_double)]
        L.orc_gmres.restype = C.c_int32
        L.orc_mcbem.argtypes = [_d, C.c_int32, _i, C.c_int32, _d, C.c_int32, C.c_int32, _d,
                                _i, _d, C.c_int32, C.c_int32, C.c_uint64, C.c_double,
                                C.c_double, C.c_int32, _d, C.c_void_p, _i, _d, _i, _d, C.c_int32,
                                C.c_int32, C.c_int32]
        L.orc_mcbem.restype = C.c_int32
        L.orc_gauss_legendre01.argtypes = [C.c_int32, _d, _d]
        L.orc_self_panel.argtypes = [C.c_double, _d, _d, _d, _d]
        L.orc_panel_integrals.argtypes = [C.c_double, _d, _d, _d, _d, _d, _d]
        L.orc_bem_assemble.argtypes = [_d, _i, C.c_int32, C.c_double, C.c_int32, _d, _d]
        L.orc_panel_data.argtypes = [_i, C.c_int32, _d, _d]
        L.orc_bem_solve.argtypes = [C.c_int32, _d, _d, _d, C.c_double, C.c_int32, _d,
                                    C.POINTER(C.c_double)]
        L.orc_bem_solve.restype = C.c_int32
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _c2d(a):
    """complex128 array -> contiguous float64 view of interleaved (re, im)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64).reshape(-1)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Thread count of the OpenMP loops that follow (the timing leg's single-thread run)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------- geometry
def geometry(V, T):
    V, T = _f64(V), _i32(T)
    nT = len(T)
    area = np.empty(nT)
    nrm = np.empty((nT, 3))
    cdf = np.empty(nT)
    lib().orc_geometry(V.reshape(-1), T.reshape(-1), nT, area, nrm.reshape(-1), cdf)
    return area, nrm, cdf


def rng_word(seed, stream, counter):
    return int(lib().orc_rng_word(seed, stream, counter))


def splitmix64(state):
    return int(lib().orc_splitmix64(state))


def cdf_search(cdf, tau):
    cdf = _f64(cdf)
    return int(lib().orc_cdf_search(cdf, len(cdf), float(tau)))


def samples(V, T, N, seed):
    """Sample triangle indices and barycentrics (b1, b2)."""
    _, _, cdf = geometry(V, T)
    tri = np.empty(N, dtype=np.int32)
    bary = np.empty((N, 2))
    lib().orc_samples(cdf, len(cdf), N, seed, tri, bary.reshape(-1))
    return tri, bary


POISSON_RSCALE = 0.72      # r = POISSON_RSCALE sqrt(|Gamma| / N)
POISSON_CANDIDATES = 16    # candidates per requested sample


def poisson_candidates(V, T, M, seed):
    """The candidate pool of the Poisson-disk sampler: (tri, bary, xyz)."""
    V, T = _f64(V), _i32(T)
    _, _, cdf = geometry(V, T)
    tri = np.empty(M, dtype=np.int32)
    bary = np.empty((M, 2))
    xyz = np.empty((M, 3))
    lib().orc_poisson_candidates(V.reshape(-1), T.reshape(-1), cdf, len(T), int(M), seed, tri,
                                 bary.reshape(-1), xyz.reshape(-1))
    return tri, bary, xyz


def poisson_samples(V, T, N, seed, rscale=POISSON_RSCALE, cand_factor=POISSON_CANDIDATES,
                    all_accepted=False):
    """Poisson-disk samples (Section 4.2): the first N accepted points (every
    accepted point with all_accepted).  Returns (tri, bary, n_accepted)."""
    V, T = _f64(V), _i32(T)
    cap = cand_factor * N if all_accepted else N
    tri = np.empty(cap, dtype=np.int32)
    bary = np.empty((cap, 2))
    n = int(lib().orc_poisson_samples(V.reshape(-1), len(V), T.reshape(-1), len(T), int(N), seed,
                                      float(rscale), int(cand_factor), int(cap), tri, bary.reshape(-1)))
    m = min(cap, n)
    return tri[:m], bary[:m], n


def surface_points(V, T, tri, bary):
    tri, bary = _i32(tri), _f64(bary)
    out = np.empty((len(tri), 3))
    lib().orc_surface_points(_f64(V).reshape(-1), _i32(T).reshape(-1), len(tri), tri,
                             bary.reshape(-1), out.reshape(-1))
    return out


def neumann_at(T, g, tri, bary, layout=0):
    tri, bary = _i32(tri), _f64(bary)
    out = np.empty(len(tri), dtype=np.complex128)
    lib().orc_neumann_at(_i32(T).reshape(-1), layout, _c2d(g), len(tri), tri,
                         bary.reshape(-1), out.view(np.float64))
    return out


def kernels(k, x, nx, y, ny):
    """(G, dG/dn_y, dG/dn_x, d2G/dn_x dn_y) at one point pair."""
    out = np.empty(4, dtype=np.complex128)
    lib().orc_kernels(float(k), _f64(x), _f64(nx), _f64(y), _f64(ny), out.view(np.float64))
    return out


# --------------------------------------------------------------- MC pieces
def mc_constants(area_total, N, eps_scale=1.0):
    """w = |Gamma|/N and eps = eps_scale sqrt(|Gamma| / (pi N))."""
    return area_total / N, eps_scale * np.sqrt(area_total / (np.pi * N))


def mc_matrix(y, ny, k, w, eps):
    y, ny = _f64(y), _f64(ny)
    N = len(y)
    M = np.empty((N, N), dtype=np.complex128)
    lib().orc_mc_matrix(N, y.reshape(-1), ny.reshape(-1), float(k), float(w), float(eps),
                        M.view(np.float64).reshape(-1))
    return M


def mc_rhs(y, k, w, eps, g, exact_disk=False):
    y = _f64(y)
    N = len(y)
    b = np.empty(N, dtype=np.complex128)
    lib().orc_mc_rhs(N, y.reshape(-1), float(k), float(w), float(eps), _c2d(g), int(exact_disk),
                     b.view(np.float64))
    return b


def mc_eval(x, gx, c_q, y, ny, g, p, k, w, eps, exact_disk=False):
    """Stage-B sum at targets x; gx=None drops the disk term (exterior use).
    c_q: one free term for every target, or an array of one per target."""
    x, y, ny = _f64(x), _f64(y), _f64(ny)
    out = np.empty(len(x), dtype=np.complex128)
    gxa = None
    if gx is not None:
        gxa = _c2d(gx)
    carr = None
    if np.ndim(c_q) > 0:
        carr = _f64(c_q)
        assert carr.shape == (len(x),)
    lib().orc_mc_eval(len(x), x.reshape(-1),
                      gxa.ctypes.data_as(C.c_void_p) if gxa is not None else None,
                      0.5 if carr is not None else float(c_q),
                      carr.ctypes.data_as(C.c_void_p) if carr is not None else None,
                      len(y), y.reshape(-1), ny.reshape(-1), _c2d(g), _c2d(p),
                      float(k), float(w), float(eps), int(exact_disk), out.view(np.float64))
    return out


def bounding_sphere(V):
    """(centre, radius) of the axis-aligned bounding box: its centre and half its diagonal."""
    V = _f64(V)
    lo, hi = V.min(axis=0), V.max(axis=0)
    return 0.5 * (lo + hi), 0.5 * float(np.linalg.norm(hi - lo))


def field_points(V, kind, n_a, n_b=1, r_lo=1.5, r_hi=3.0, seed=0):
    """Field points around the mesh (Section 3.4 shell, kind 0; FFAT grid of
    n_a x n_b directions at radius r_lo R, kind 1).  Returns (xyz, coords)
    with coords = (r, theta, phi) per point."""
    c, R = bounding_sphere(V)
    n = n_a if kind == 0 else n_a * n_b
    xyz = np.empty((n, 3))
    coords = np.empty((n, 3))
    lib().orc_field_points(_f64(c), float(R), int(kind), int(n_a), int(n_b), float(r_lo),
                           float(r_hi), seed, xyz.reshape(-1), coords.reshape(-1))
    return xyz, coords


def mcbem_field(V, T, g, k, N, seed, points, p_samples, eps_scale=1.0, layout=0, poisson=False):
    """Pressure at exterior points from the sample values of an estimate
    (Section 3.4: the field from the Neumann and Dirichlet data): the
    representation formula p(x) = sum_j w (dG/dn_j p_j - G g_j) over the same
    samples, with c = 1 and no disk term.  p_samples: (n_modes, N), e.g. the
    p_samples of mcbem() with the same N and seed."""
    V, T = _f64(V), _i32(T)
    g = np.ascontiguousarray(np.atleast_2d(g), dtype=np.complex128)
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    p_samples = np.ascontiguousarray(np.atleast_2d(p_samples), dtype=np.complex128)
    area, nrm, cdf = geometry(V, T)
    if poisson:
        tri, bary, _ = poisson_samples(V, T, N, seed)
    else:
        tri, bary = samples(V, T, N, seed)
    y = surface_points(V, T, tri, bary)
    ny = np.ascontiguousarray(nrm[tri])
    w, eps = mc_constants(cdf[-1], N, eps_scale)
    out = np.empty((len(k), len(points)), dtype=np.complex128)
    for m in range(len(k)):
        gj = neumann_at(T, g[m], tri, bary, layout)
        out[m] = mc_eval(points, None, 1.0, y, ny, gj, p_samples[m], k[m], w, eps)
    return out


def free_terms(V, T, q_tri, q_bary, jump=1):
    """Free term c of the surface identity at each query (1/2 on smooth parts;
    one minus the body's solid angle over 4 pi at vertices and edges)."""
    V, T, q_tri, q_bary = _f64(V), _i32(T), _i32(q_tri), _f64(q_bary)
    out = np.empty(len(q_tri))
    lib().orc_free_terms(V.reshape(-1), T.reshape(-1), len(T), q_tri, q_bary.reshape(-1),
                         len(q_tri), int(jump), out)
    return out


def gmres(A, b, tol=1e-12, max_iter=200):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    x = np.empty(n, dtype=np.complex128)
    res = C.c_double()
    it = lib().orc_gmres(n, A.view(np.float64).reshape(-1), _c2d(b), x.view(np.float64),
                         float(tol), int(max_iter), C.byref(res))
    return x, int(it), float(res.value)


def mcbem(V, T, g, k, q_tri, q_bary, N, seed, eps_scale=1.0, tol=1e-12, max_iter=200,
          layout=0, want_samples=False, jump=0, exact_disk=False, poisson=False):
    """The whole MC-BEM estimate for n_modes (k_m, g_m) pairs.

    g: complex (n_modes, V) per-vertex (layout 0) or (n_modes, T) per triangle.
    Returns dict with p (n_modes, Q), iters, resid, tri, bary and optionally
    p_samples (n_modes, N)."""
    V, T = _f64(V), _i32(T)
    g = np.ascontiguousarray(np.atleast_2d(g), dtype=np.complex128)
    k = _f64(np.atleast_1d(k))
    n_modes = len(k)
    assert g.shape[0] == n_modes
    q_tri, q_bary = _i32(q_tri), _f64(q_bary)
    Q = len(q_tri)
    p = np.empty((n_modes, Q), dtype=np.complex128)
    ps = np.empty((n_modes, N), dtype=np.complex128) if want_samples else None
    iters = np.empty(n_modes, dtype=np.int32)
    resid = np.empty(n_modes)
    tri = np.empty(N, dtype=np.int32)
    bary = np.empty((N, 2))
    st = lib().orc_mcbem(V.reshape(-1), len(V), T.reshape(-1), len(T), g.view(np.float64).reshape(-1),
                         layout, n_modes, k, q_tri, q_bary.reshape(-1), Q, N, seed,
                         float(eps_scale), float(tol), int(max_iter),
                         p.view(np.float64).reshape(-1),
                         ps.ctypes.data_as(C.c_void_p) if ps is not None else None,
                         iters, resid, tri, bary.reshape(-1), int(jump), int(exact_disk),
                         int(bool(poisson)))
    if st == 5:
        raise ValueError(f"Poisson-disk sampling accepted fewer than N = {N} points")
    out = dict(p=p, iters=iters, resid=resid, tri=tri, bary=bary, status=int(st))
    if want_samples:
        out["p_samples"] = ps
    return out


# ------------------------------------------------------------- dense BEM
def gauss_legendre01(n):
    x = np.empty(n)
    w = np.empty(n)
    lib().orc_gauss_legendre01(n, x, w)
    return x, w


def self_panel(k, v0, v1, v2):
    out = np.empty(2, dtype=np.complex128)
    lib().orc_self_panel(float(k), _f64(v0), _f64(v1), _f64(v2), out.view(np.float64))
    return out


def panel_integrals(k, x, nx, a, b, c):
    out = np.empty(4, dtype=np.complex128)
    lib().orc_panel_integrals(float(k), _f64(x), _f64(nx), _f64(a), _f64(b), _f64(c),
                              out.view(np.float64))
    return out


def bem_assemble(V, T, k, burton_miller=True):
    """Matrices (A, B) of A p = B g, P0 collocation at centroids."""
    V, T = _f64(V), _i32(T)
    n = len(T)
    A = np.empty((n, n), dtype=np.complex128)
    B = np.empty((n, n), dtype=np.complex128)
    lib().orc_bem_assemble(V.reshape(-1), T.reshape(-1), n, float(k), int(bool(burton_miller)),
                           A.view(np.float64).reshape(-1), B.view(np.float64).reshape(-1))
    return A, B


def panel_data(T, gv):
    T = _i32(T)
    out = np.empty(len(T), dtype=np.complex128)
    lib().orc_panel_data(T.reshape(-1), len(T), _c2d(gv), out.view(np.float64))
    return out


def bem_solve(A, B, g_panel, tol=1e-10, max_iter=500):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    n = A.shape[0]
    p = np.empty(n, dtype=np.complex128)
    res = C.c_double()
    it = lib().orc_bem_solve(n, A.view(np.float64).reshape(-1), B.view(np.float64).reshape(-1),
                             _c2d(g_panel), float(tol), int(max_iter), p.view(np.float64),
                             C.byref(res))
    return p, int(it), float(res.value)


def centroids(V, T):
    V, T = _f64(V), _i32(T)
    return (V[T[:, 0]] + V[T[:, 1]] + V[T[:, 2]]) / 3.0
