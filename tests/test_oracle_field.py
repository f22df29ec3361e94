"""Pins for the oracle's exterior field (Section 3.4: the field at points
around the scene from the surface Neumann and Dirichlet data; Section 3.1:
FFAT maps on a sphere of directions): the shell and grid point sets by
their distributions and symmetries, and the representation formula over
the Monte-Carlo samples by the pulsating sphere's exterior closed form and
an interior point source."""
import math

import numpy as np
import pytest
import scipy.stats as st

import workloads as W
from oracle import closed_forms as CF
from oracle import oracle as O


def test_shell_points_distribution():
    """Radius uniform in [1.5 R, 3 R), direction uniform on the sphere."""
    v, f, _ = W.noisy_ellipsoid(3, subdiv=3)
    c, R = O.bounding_sphere(v)
    n = 20000
    x, co = O.field_points(v, 0, n, r_lo=1.5, r_hi=3.0, seed=5)
    r, th, ph = co[:, 0], co[:, 1], co[:, 2]
    d = x - c[None, :]
    assert np.allclose(np.linalg.norm(d, axis=1), r, rtol=1e-14, atol=0)
    assert r.min() >= 1.5 * R and r.max() < 3.0 * R
    assert st.kstest((r / R - 1.5) / 1.5, "uniform").pvalue > 1e-3
    assert st.kstest((1.0 - np.cos(th)) / 2.0, "uniform").pvalue > 1e-3
    assert st.kstest(ph / (2 * np.pi), "uniform").pvalue > 1e-3
    u = d / r[:, None]
    assert np.allclose(u[:, 2], np.cos(th), atol=1e-15)
    # mean direction of n uniform unit vectors: each component has sd 1/sqrt(3n)
    assert np.all(np.abs(u.mean(axis=0)) < 4.0 / math.sqrt(3 * n))
    # every point lies outside the mesh's bounding box
    lo, hi = v.min(axis=0), v.max(axis=0)
    assert not np.any(np.all((x >= lo) & (x <= hi), axis=1))
    # a different seed gives different points
    x2, _ = O.field_points(v, 0, 10, seed=6)
    assert not np.allclose(x2, x[:10])


def test_ffat_grid_geometry():
    """The 32 x 64 FFAT grid: all points at r_lo R, theta constant along a row
    and increasing down the rows, phi increasing along a row, every point's
    antipode in the grid, directions summing to zero."""
    v, f, _ = W.cubesphere_ellipsoid(4, 3000)
    c, R = O.bounding_sphere(v)
    na, nb = 32, 64
    x, co = O.field_points(v, 1, na, nb, r_lo=2.0)
    assert x.shape == (na * nb, 3)
    d = (x - c[None, :]).reshape(na, nb, 3)
    assert np.allclose(np.linalg.norm(d, axis=2), 2.0 * R, rtol=1e-14, atol=0)
    th = co[:, 1].reshape(na, nb)
    ph = co[:, 2].reshape(na, nb)
    assert np.all(th == th[:, :1]) and np.all(np.diff(th[:, 0]) > 0)
    assert np.all(np.diff(ph, axis=1) > 0) and 0 < th.min() and th.max() < np.pi
    anti = d[::-1][:, (np.arange(nb) + nb // 2) % nb]
    assert np.allclose(anti, -d, atol=1e-14 * R)
    assert np.allclose(d.reshape(-1, 3).sum(axis=0), 0.0, atol=1e-11 * R)


def test_field_pulsating_sphere_closed_form():
    """P1 outside the body: dp/dr = 1 on the unit sphere, k = 2; the field at
    shell points from the estimate's own sample values against the monopole
    g a^2 e^{ik(r-a)} / ((ika - 1) r), error falling with N."""
    wl = W.config_pulsating_sphere()
    x, co = O.field_points(wl.vertices, 0, 300, seed=1)
    ex = CF.pulsating_sphere_field(2.0, 1.0, co[:, 0])
    assert ex[0] == pytest.approx(CF.pulsating_sphere(2.0, 1.0) * np.exp(2j * (co[0, 0] - 1)) / co[0, 0])
    errs = {}
    for N in (256, 1024, 4096):
        e = []
        for s in range(3 if N < 4096 else 1):
            r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, N, wl.seed + s,
                        want_samples=True)
            p = O.mcbem_field(wl.vertices, wl.tris, wl.g, wl.k, N, wl.seed + s, x, r["p_samples"])
            e.append(np.linalg.norm(p[0] - ex) / np.linalg.norm(ex))
        errs[N] = float(np.mean(e))
    assert errs[4096] < errs[1024] < errs[256]
    assert errs[4096] < 0.1


def test_field_interior_point_source():
    """Interior point source x0 on a noise-displaced ellipsoid: with the exact
    surface values p = G(., x0) at the samples and per-vertex g = dG/dn, the
    representation formula reproduces G(x, x0) outside; averaged over seeds
    the estimate is unbiased up to the interpolation error of g."""
    v, f, u = W.noisy_ellipsoid(11, subdiv=4)
    k = 40.0
    x0 = np.array([0.02, 0.01, -0.005])
    _, nrm, _ = O.geometry(v, f)
    vn = np.zeros_like(v)
    for c in range(3):
        np.add.at(vn, f[:, c], nrm)
    vn /= np.linalg.norm(vn, axis=1, keepdims=True)
    gv = CF.point_source_normal_derivative(k, v, vn, x0)
    x, co = O.field_points(v, 0, 200, seed=2)
    ex = CF.point_source_field(k, x, x0)
    ests, errs = [], []
    N = 2048
    for s in range(16):
        tri, bary = O.samples(v, f, N, 100 + s)
        y = O.surface_points(v, f, tri, bary)
        ps = CF.point_source_field(k, y, x0)
        p = O.mcbem_field(v, f, gv[None, :], [k], N, 100 + s, x, ps[None, :])[0]
        ests.append(p)
        errs.append(np.linalg.norm(p - ex) / np.linalg.norm(ex))
    mean = np.mean(ests, axis=0)
    assert np.linalg.norm(mean - ex) / np.linalg.norm(ex) < 0.25 * float(np.mean(errs))
    assert float(np.mean(errs)) < 0.2
