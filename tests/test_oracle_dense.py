"""Pins for the oracle's dense collocation Burton-Miller BEM (Section 4,
eq. BurtonMiller; Section 4.1 direct assembly of A p = B g): quadrature
rules, self-panel finite parts, operator identities on the sphere, closed
forms and the resonance the Burton-Miller term removes."""
import math
from pathlib import Path

import numpy as np
import pytest

import workloads as W
from oracle import closed_forms as CF
from oracle import oracle as O

GOLD = Path(__file__).parent / "golden"


def test_gauss_legendre_against_tables():
    rows = [l.split() for l in (GOLD / "gauss_legendre_n3.txt").read_text().splitlines()
            if l and not l.startswith("#")]
    ref = np.array([[float(a), float(b)] for a, b in rows])
    x, w = O.gauss_legendre01(3)
    np.testing.assert_allclose(2 * x - 1, ref[:, 0], atol=1e-15)
    np.testing.assert_allclose(2 * w, ref[:, 1], atol=1e-15)
    for n in (5, 16):
        x, w = O.gauss_legendre01(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        np.testing.assert_allclose(2 * x - 1, xr, atol=1e-14)
        np.testing.assert_allclose(2 * w, wr, atol=1e-14)


def _duffy_points(x, a, b, n):
    """Gauss points of a collapsed rule with the singular corner at x on the
    triangle (x, a, b): y = x + s (a - x) + s t (b - a), dS = 2A s ds dt."""
    g, gw = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1)
    gw = 0.5 * gw
    two_a = np.linalg.norm(np.cross(a - x, b - x))
    S, T = np.meshgrid(g, g, indexing="ij")
    WS, WT = np.meshgrid(gw, gw, indexing="ij")
    pts = x + S[..., None] * (a - x) + (S * T)[..., None] * (b - a)
    wts = WS * WT * S * two_a
    return pts.reshape(-1, 3), wts.reshape(-1)


@pytest.mark.parametrize("k", [0.0, 7.0, 60.0])
def test_self_panel_against_duffy_brute_force(k):
    """P14: S_ii by Duffy-regularised quadrature; W_ii as its k = 0 finite part
    in closed form plus the (weakly singular) difference by Duffy."""
    v0 = np.array([0.0, 0.0, 0.0])
    v1 = np.array([0.11, 0.01, 0.0])
    v2 = np.array([0.03, 0.07, 0.0])
    x = (v0 + v1 + v2) / 3
    S_ref = 0.0
    dW = 0.0
    W0 = 0.0
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        pts, wts = _duffy_points(x, a, b, 60)
        r = np.linalg.norm(pts - x, axis=1)
        S_ref += np.sum(wts * np.exp(1j * k * r) / (4 * np.pi * r))
        dW += np.sum(wts * (np.exp(1j * k * r) * (1 - 1j * k * r) - 1.0) / (4 * np.pi * r ** 3))
        # k = 0 finite part: -(1/4pi) int dtheta / rho = -(sin tb - sin ta)/(4 pi d)
        e = b - a
        L = np.linalg.norm(e)
        uu = e / L
        along = np.dot(x - a, uu)
        d = np.linalg.norm((x - a) - along * uu)
        ta, tb = math.atan(-along / d), math.atan((L - along) / d)
        W0 += -(math.sin(tb) - math.sin(ta)) / (4 * np.pi * d)
    S, Wii = O.self_panel(k, v0, v1, v2)
    assert abs(S - S_ref) < 1e-7 * abs(S_ref)   # 16-point theta rule
    assert abs(Wii - (W0 + dW)) < 1e-7 * abs(W0)


def test_self_panel_k0_closed_form():
    v0, v1, v2 = np.array([0, 0, 0.0]), np.array([1.0, 0, 0]), np.array([0.2, 0.9, 0])
    x = (v0 + v1 + v2) / 3
    S_ref = 0.0
    for a, b in ((v0, v1), (v1, v2), (v2, v0)):
        e = b - a
        L = np.linalg.norm(e)
        uu = e / L
        along = np.dot(x - a, uu)
        d = np.linalg.norm((x - a) - along * uu)
        ta, tb = math.atan(-along / d), math.atan((L - along) / d)
        S_ref += d * (math.asinh(math.tan(tb)) - math.asinh(math.tan(ta))) / (4 * np.pi)
    S, _ = O.self_panel(0.0, v0, v1, v2)
    assert S.real == pytest.approx(S_ref, rel=1e-10) and S.imag == 0.0  # 16-point theta rule


def test_near_panel_rule_against_fine_quadrature():
    """Subdivision rule for a target close to an edge-adjacent panel."""
    a, b, c = np.array([0, 0, 0.0]), np.array([1.0, 0, 0]), np.array([0.4, 0.8, 0.05])
    x = np.array([0.5, -0.29, 0.02])
    nx = np.array([0.0, 0.1, 1.0])
    nx /= np.linalg.norm(nx)
    k = 4.0
    got = O.panel_integrals(k, x, nx, a, b, c)
    # reference: uniform 64 x 64 split of the triangle, 7-point-equivalent
    # collapsed Gauss 6x6 on each sub-triangle
    n = 64
    e1, e2 = (b - a) / n, (c - a) / n
    nrm = np.cross(b - a, c - a)
    ny = nrm / np.linalg.norm(nrm)
    subs = []
    for i in range(n):
        for j in range(n - i):
            p0 = a + i * e1 + j * e2
            subs.append((p0, p0 + e1, p0 + e2))
            if i + j < n - 1:
                subs.append((p0 + e1, p0 + e1 + e2, p0 + e2))
    g, gw = np.polynomial.legendre.leggauss(6)
    g, gw = 0.5 * (g + 1), 0.5 * gw
    ref = np.zeros(4, dtype=complex)
    for (p, q, r) in subs:
        two_a = np.linalg.norm(np.cross(q - p, r - p))
        for s, ws in zip(g, gw):
            for t, wt in zip(g, gw):
                y = p + s * (q - p) + t * (1 - s) * (r - p)
                ref += ws * wt * (1 - s) * two_a * O.kernels(k, x, nx, y, ny)
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() < 2e-3


def _sphere_operators(subdiv, k):
    v, f, u = W.icosphere(subdiv, 1.0)
    _, nrm, _ = O.geometry(v, f)
    cen = O.centroids(v, f)
    n = len(f)
    rows = np.zeros(4, dtype=complex)
    sums = np.zeros((n, 4), dtype=complex)
    idx = np.arange(0, n, max(1, n // 40))
    for i in idx:
        acc = np.zeros(4, dtype=complex)
        for j in range(n):
            if i == j:
                S, Wd = O.self_panel(k, v[f[j, 0]], v[f[j, 1]], v[f[j, 2]])
                acc += np.array([S, 0, 0, Wd])
            else:
                acc += O.panel_integrals(k, cen[i], nrm[i], v[f[j, 0]], v[f[j, 1]], v[f[j, 2]])
        sums[i] = acc
    return sums[idx], idx, v, f


def test_operator_identities_on_sphere():
    """Operators applied to the constant 1 on the unit sphere (k = 0):
    S 1 = 1, K 1 = -1/2, K' 1 = -1/2, W 1 = 0; at k > 0 S 1 = e^{ika} sin(ka)/k (k = 1.5)."""
    sums, idx, v, f = _sphere_operators(2, 0.0)
    S, K, Kp, Wd = sums.T
    assert np.abs(S - 1.0).max() < 0.01          # O(h^2) geometric error
    assert np.abs(K + 0.5).max() < 1e-5          # Gauss: exact on any closed polyhedron
    assert np.abs(Kp + 0.5).max() < 0.05         # O(h): centroids lie inside the sphere
    # W 1 = 0 (the double layer of 1 is piecewise constant), relative to the
    # self term ~ 1/h: a wrong sign of the finite part would leave ~2 |W_ii|
    Wself = np.array([O.self_panel(0.0, *[v[f[i, c]] for c in range(3)])[1] for i in idx])
    assert np.abs(Wd).max() < 1e-4 * np.abs(Wself).min()
    sums3, _, _, _ = _sphere_operators(2, 1.5)
    ref = CF.sphere_single_layer_of_one(1.5, 1.0)
    assert np.abs(sums3[:, 0] - ref).max() < 0.03 * abs(ref)


def _dense(v, f, k, g_vertex, bm=True):
    A, B = O.bem_assemble(v, f, k, bm)
    gp = O.panel_data(f, g_vertex)
    p, it, res = O.bem_solve(A, B, gp, tol=1e-10)
    assert res <= 1e-10
    return p, A, B, gp


def test_pulsating_sphere_dense_first_order():
    """P1 for the dense solver: error halves with each refinement."""
    ex = CF.pulsating_sphere(2.0, 1.0)
    errs = []
    for s in (2, 3):
        v, f, u = W.icosphere(s, 1.0)
        p, *_ = _dense(v, f, 2.0, np.ones(len(v), dtype=complex))
        errs.append(np.abs(p - ex).max() / abs(ex))
    assert errs[1] < 0.025 and errs[1] < 0.6 * errs[0]


@pytest.mark.parametrize("ka,tol", [(1.0, 0.05), (5.0, 0.04), (10.0, 0.04)])
def test_oscillating_sphere_dense(ka, tol):
    """P2: dp/dr = cos(theta), a = 0.1 m."""
    a = 0.1
    v, f, u = W.icosphere(3, a)
    p, *_ = _dense(v, f, ka / a, u[:, 2].astype(complex))
    cen = O.centroids(v, f)
    cosq = cen[:, 2] / np.linalg.norm(cen, axis=1)
    ex = CF.oscillating_sphere_factor(ka / a, a) * cosq
    assert np.linalg.norm(p - ex) / np.linalg.norm(ex) < tol


def test_burton_miller_removes_interior_resonance():
    """At ka = pi (j_0(ka) = 0, an interior Dirichlet eigenvalue) the
    conventional equation fails and the Burton-Miller one does not; away
    from it both agree with the closed form."""
    v, f, u = W.icosphere(3, 1.0)
    one = np.ones(len(v), dtype=complex)
    ex = CF.pulsating_sphere(math.pi, 1.0)
    p_bm, *_ = _dense(v, f, math.pi, one, True)
    p_cb, *_ = _dense(v, f, math.pi, one, False)
    e_bm = np.abs(p_bm - ex).max() / abs(ex)
    e_cb = np.abs(p_cb - ex).max() / abs(ex)
    assert e_bm < 0.03 and e_cb > 0.08


def test_interior_point_source_dense_and_reciprocity():
    """P3 on a noise-displaced ellipsoid, P10 against LU, P11/P12."""
    v, f, u = W.noisy_ellipsoid(3, subdiv=2)
    k = 40.0
    x0 = np.array([0.01, 0.005, -0.003])
    _, nrm, _ = O.geometry(v, f)
    cen = O.centroids(v, f)
    A, B = O.bem_assemble(v, f, k, True)
    g = CF.point_source_normal_derivative(k, cen, nrm, x0)
    p, it, res = O.bem_solve(A, B, g, tol=1e-12)
    ex = CF.point_source_field(k, cen, x0)
    assert np.linalg.norm(p - ex) / np.linalg.norm(ex) < 0.08
    ref = np.linalg.solve(A, B @ g)
    assert np.linalg.norm(p - ref) / np.linalg.norm(ref) < 1e-10 * np.linalg.cond(A)
    area, _, _ = O.geometry(v, f)
    gs = W.sh_neumann(u, 2, 4, lmax=2)
    p1, _, _ = O.bem_solve(A, B, O.panel_data(f, gs[0]))
    p2, _, _ = O.bem_solve(A, B, O.panel_data(f, gs[1]))
    g1, g2 = O.panel_data(f, gs[0]), O.panel_data(f, gs[1])
    rec = np.sum(area * (p1 * g2 - p2 * g1))
    assert abs(rec) < 0.05 * np.sum(area * np.abs(p1 * g2))
    assert np.sum(area * p1 * np.conj(g1)).imag < 0
