"""Pins for the oracle's geometry, counter RNG and area-uniform sampling
(Section 4.1.1: uniform sampling, density 1/|Gamma|)."""
import math
from pathlib import Path

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import oracle as O

GOLD = Path(__file__).parent / "golden"


def _golden_ints(name):
    return [int(l) for l in (GOLD / name).read_text().splitlines() if l and not l.startswith("#")]


def test_splitmix64_reference_vector():
    expect = _golden_ints("splitmix64_seed1234567.txt")
    got = [O.rng_word(1234567, 0, i) for i in range(len(expect))]
    assert got == expect


def test_rng_streams_and_counters_differ():
    a = [O.rng_word(7, 0, i) for i in range(1000)]
    b = [O.rng_word(7, 1, i) for i in range(1000)]
    assert len(set(a)) == 1000 and not set(a) & set(b)


def test_geometry_areas_normals_cdf():
    v, f, u = W.icosphere(2, 1.0)
    area, nrm, cdf = O.geometry(v, f)
    # areas from the determinant formula computed independently (Heron's formula)
    a = np.linalg.norm(v[f[:, 1]] - v[f[:, 0]], axis=1)
    b = np.linalg.norm(v[f[:, 2]] - v[f[:, 1]], axis=1)
    c = np.linalg.norm(v[f[:, 0]] - v[f[:, 2]], axis=1)
    s = 0.5 * (a + b + c)
    heron = np.sqrt(s * (s - a) * (s - b) * (s - c))
    np.testing.assert_allclose(area, heron, rtol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=1), 1.0, rtol=1e-14)
    cen = O.centroids(v, f)
    assert (np.einsum("ij,ij->i", nrm, cen) > 0).all()          # outward
    for t in range(0, len(f), 37):                                # normal is perpendicular to edges
        assert abs(np.dot(nrm[t], v[f[t, 1]] - v[f[t, 0]])) < 1e-14
    assert np.all(np.diff(cdf) > 0) and cdf[0] == area[0]
    assert cdf[-1] == pytest.approx(area.sum(), rel=1e-14)
    # inscribed polyhedron: area below the sphere's and converging to it
    assert 0.98 * 4 * math.pi < cdf[-1] < 4 * math.pi


def test_cdf_search_is_smallest_index_with_cdf_above_tau():
    rng = np.random.default_rng(0)
    cdf = np.cumsum(rng.uniform(0.0, 1.0, 200))
    cdf[50] = cdf[49]  # a zero-area triangle is never chosen
    cdf[120:123] = cdf[119]
    taus = np.concatenate([rng.uniform(0, cdf[-1], 5000), cdf[:-1], [0.0, np.nextafter(cdf[-1], 0)]])
    for tau in taus:
        lin = int(np.argmax(cdf > tau)) if (cdf > tau).any() else len(cdf) - 1
        assert O.cdf_search(cdf, tau) == lin
    chosen = {O.cdf_search(cdf, t) for t in taus}
    assert 50 not in chosen and not chosen & {120, 121, 122}


def test_triangle_hits_follow_area_chi2():
    v, f, _ = W.cubesphere_ellipsoid(11, 600)
    area, _, _ = O.geometry(v, f)
    N = 200_000
    tri, bary = O.samples(v, f, N, 99)
    counts = np.bincount(tri, minlength=len(f))
    expected = N * area / area.sum()
    chi2, p = stats.chisquare(counts, expected)
    assert p > 1e-3


def test_barycentrics_uniform_on_triangle():
    v, f, _ = W.icosphere(1, 1.0)
    tri, bary = O.samples(v, f, 50_000, 5)
    b1, b2 = bary[:, 0], bary[:, 1]
    b0 = 1.0 - b1 - b2
    assert (b1 >= 0).all() and (b2 >= 0).all() and (b0 >= -1e-15).all()
    # each barycentric of a uniform point has CDF 1 - (1 - t)^2
    for b in (b0, b1, b2):
        ks = stats.kstest(b, lambda t: 1.0 - (1.0 - np.clip(t, 0, 1)) ** 2)
        assert ks.pvalue > 1e-3


def test_sample_points_on_their_triangle():
    v, f, _ = W.noisy_ellipsoid(3, subdiv=2)
    tri, bary = O.samples(v, f, 2000, 3)
    y = O.surface_points(v, f, tri, bary)
    _, nrm, _ = O.geometry(v, f)
    off = np.einsum("ij,ij->i", y - v[f[tri, 0]], nrm[tri])
    assert np.abs(off).max() < 1e-15


def test_neumann_interpolation_reproduces_linear_fields():
    v, f, _ = W.icosphere(2, 1.0)
    coef = np.array([0.3 - 0.1j, -1.2 + 0.5j, 0.7j])
    gv = v @ coef + (0.25 + 0.5j)                      # linear in space
    tri, bary = O.samples(v, f, 500, 17)
    y = O.surface_points(v, f, tri, bary)
    got = O.neumann_at(f, gv, tri, bary, layout=0)
    np.testing.assert_allclose(got, y @ coef + (0.25 + 0.5j), rtol=1e-13, atol=1e-14)
    gt = np.arange(len(f)) * (1 + 2j)
    np.testing.assert_array_equal(O.neumann_at(f, gt, tri, bary, layout=1), gt[tri])
