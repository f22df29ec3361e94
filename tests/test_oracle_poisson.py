"""Pins for the oracle's Poisson-disk sample set (Section 4.2: parallel
Poisson-disk sampling; Section 6.1: Poisson samples beat random ones at the
same count): minimum spacing, maximality over the candidate pool, the grid
and phase schedule against a brute-force sequential definition on a tiny
mesh, even spread by area, enough accepted points for the estimate, and a
lower estimator error than independent samples on the closed-form spheres."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import oracle as O


def _radius(v, f, N):
    _, _, cdf = O.geometry(v, f)
    return O.POISSON_RSCALE * math.sqrt(cdf[-1] / N)


@pytest.mark.parametrize("kind", ["ico3", "ellipsoid", "scene"])
def test_spacing_maximality_and_count(kind):
    if kind == "ico3":
        v, f, _ = W.icosphere(3, 1.0)
    elif kind == "ellipsoid":
        v, f, _ = W.noisy_ellipsoid(3, subdiv=4)
    else:
        sc = W.scene_speaker_torus(0.0)
        v, f = sc.vertices, sc.tris
    N = 1024
    r = _radius(v, f, N)
    tri, bary, n = O.poisson_samples(v, f, N, 5, all_accepted=True)
    assert len(tri) == n and n >= 1.05 * N
    x = O.surface_points(v, f, tri, bary)
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    assert d2.min() >= r * r                       # no two accepted points closer than r
    # every candidate lies within r of an accepted point (nothing more fits)
    _, _, cx = O.poisson_candidates(v, f, O.POISSON_CANDIDATES * N, 5)
    dmin = np.sqrt(((cx[:, None, :] - x[None, :, :]) ** 2).sum(-1).min(axis=1))
    assert dmin.max() <= r * (1 + 1e-12)
    # the estimator's set is the first N in acceptance order
    t1, b1, n1 = O.poisson_samples(v, f, N, 5)
    assert n1 == n and np.array_equal(t1, tri[:N]) and np.array_equal(b1, bary[:N])


def _brute_force(v, f, N, seed):
    """The same candidates, cells, phases and passes, but every candidate is
    checked against all points accepted so far (no neighbour-cell search)."""
    _, _, cdf = O.geometry(v, f)
    r = O.POISSON_RSCALE * math.sqrt(cdf[-1] / N)
    r2 = r * r
    inv_h = math.sqrt(3.0) / r
    lo, hi = v.min(axis=0), v.max(axis=0)
    dim = np.floor((hi - lo) * inv_h).astype(np.int64) + 1
    M = O.POISSON_CANDIDATES * N
    _, _, x = O.poisson_candidates(v, f, M, seed)
    cc = np.clip(np.floor((x - lo) * inv_h).astype(np.int64), 0, dim - 1)
    key = (cc[:, 0] * dim[1] + cc[:, 1]) * dim[2] + cc[:, 2]
    cells = {}
    for i in np.lexsort((np.arange(M), key)):
        cells.setdefault(int(key[i]), []).append(int(i))
    order = sorted(cells)
    phase = {k: int((k // (dim[1] * dim[2])) % 3 * 9 + (k // dim[2]) % dim[1] % 3 * 3 + k % dim[2] % 3)
             for k in order}
    done, acc = set(), []
    for p in range(max(len(c) for c in cells.values())):
        for ph in range(27):
            for k in order:
                if phase[k] != ph or k in done or len(cells[k]) <= p:
                    continue
                i = cells[k][p]
                if all(((x[i] - x[a]) ** 2).sum() >= r2 for a in acc):
                    done.add(k)
                    acc.append(i)
    return acc


def test_schedule_matches_brute_force_on_a_tiny_mesh():
    v, f, _ = W.icosphere(1, 1.0)
    for N, seed in ((40, 3), (64, 2**40 + 1)):
        acc = _brute_force(v, f, N, seed)
        tri, bary, n = O.poisson_samples(v, f, N, seed, all_accepted=True)
        ctri, cbary, _ = O.poisson_candidates(v, f, O.POISSON_CANDIDATES * N, seed)
        assert n == len(acc)
        assert np.array_equal(tri, ctri[acc]) and np.array_equal(bary, cbary[acc])


def test_even_spread_by_area():
    """Counts in the 8 octants of the unit sphere: proportional to area and far
    less dispersed than independent samples (binomial variance)."""
    v, f, _ = W.icosphere(4, 1.0)
    N = 2048
    tri, bary, _ = O.poisson_samples(v, f, N, 9)
    x = O.surface_points(v, f, tri, bary)
    octant = (x[:, 0] > 0) * 4 + (x[:, 1] > 0) * 2 + (x[:, 2] > 0)
    counts = np.bincount(octant, minlength=8)
    expect = N / 8
    assert np.all(np.abs(counts - expect) < 0.1 * expect)
    binom_var = N * (1 / 8) * (7 / 8)
    assert counts.var() < 0.25 * binom_var


def test_poisson_samples_lower_the_error():
    """Section 6.1: at the same N the Poisson-disk estimate is closer to the
    closed form than the independent-sample one (pulsating sphere at
    N = 256, 1024; oscillating sphere at ka = 5, N = 1024; seed averages)."""
    wl = W.config_pulsating_sphere()
    ex = CF.pulsating_sphere(2.0, 1.0)
    for N in (256, 1024):
        err = {}
        for pois in (False, True):
            e = [np.linalg.norm(O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, N, 100 + s,
                                        poisson=pois)["p"][0] - ex) / (abs(ex) * math.sqrt(wl.n_queries))
                 for s in range(3)]
            err[pois] = float(np.mean(e))
        assert err[True] < 0.75 * err[False], (N, err)
    wl = W.config_oscillating_sphere(ka=(5.0,))
    exo = CF.oscillating_sphere_factor(wl.k[0], 0.1) * wl.extra["u"][:, 2]
    err = {}
    for pois in (False, True):
        e = [np.linalg.norm(O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, 1024, 200 + s,
                                    poisson=pois)["p"][0] - exo) / np.linalg.norm(exo) for s in range(2)]
        err[pois] = float(np.mean(e))
    assert err[True] < 0.6 * err[False], err
