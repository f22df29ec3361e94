"""Pins for the oracle's free term of the surface identity (the jump factor
c_q of the Stage-B evaluation, Section 4.2): 1/2 on smooth parts, and at
mesh vertices and edges one minus the solid angle the body subtends there
over 4 pi.  Closed forms: the cube (corner 7/8, edge 3/4, face diagonal
1/2), the regular icosahedron (vertex solid angle from the spherical excess
of its vertex figure, edge from its dihedral angle) and a non-convex
L-shaped prism (a reflex edge, c = 1/4, and a reflex corner, c = 5/8)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O


def prism(poly, h=1.0):
    """Closed, outward-oriented extrusion of a CCW polygon star-shaped from
    its first vertex."""
    P = np.asarray(poly, dtype=np.float64)
    n = len(P)
    V = np.vstack([np.c_[P, np.zeros(n)], np.c_[P, np.full(n, h)]])
    F = []
    for i in range(1, n - 1):
        F.append((0, i + 1, i))              # bottom, normal -z
        F.append((n, n + i, n + i + 1))      # top, normal +z
    for i in range(n):
        a, b = i, (i + 1) % n
        F.append((a, b, n + b))
        F.append((a, n + b, n + a))
    return V, np.asarray(F, dtype=np.int32)


def cube():
    return prism([(0, 0), (1, 0), (1, 1), (0, 1)])


def l_prism():
    return prism([(0, 0), (2, 0), (2, 1), (1, 1), (1, 2), (0, 2)])


def vertex_query(T, v):
    """(triangle, b1, b2) placing the query exactly on vertex v."""
    t = int(np.nonzero((T == v).any(axis=1))[0][0])
    c = int(np.nonzero(T[t] == v)[0][0])
    return t, [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)][c]


def edge_query(T, a, b, s=0.3):
    """(triangle, b1, b2) placing the query on edge (a, b), a fraction s from
    one end: the barycentric weight of the third corner is exactly 0."""
    for t, tv in enumerate(T):
        if a in tv and b in tv:
            c = [i for i in range(3) if tv[i] not in (a, b)][0]
            wt = [0.0, 0.0, 0.0]
            others = [i for i in range(3) if i != c]
            wt[others[0]], wt[others[1]] = s, 1.0 - s
            b1, b2 = wt[1], wt[2]
            if c == 0:          # the weight 1 - b1 - b2 must round to exactly 0
                b2 = 1.0 - b1
            return t, (b1, b2)
    raise AssertionError("edge not in mesh")


def free_at(V, T, queries, jump=1):
    qt = np.array([q[0] for q in queries], dtype=np.int32)
    qb = np.array([q[1] for q in queries], dtype=np.float64)
    return O.free_terms(V, T, qt, qb, jump)


def test_cube_corners_edges_faces():
    V, T = cube()
    corners = [vertex_query(T, v) for v in range(8)]
    assert np.allclose(free_at(V, T, corners), 7 / 8, atol=1e-14)
    # the 12 cube edges and the 6 face diagonals
    E = {}
    for tv in T:
        for i in range(3):
            a, b = sorted((tv[i], tv[(i + 1) % 3]))
            E[(a, b)] = np.linalg.norm(V[a] - V[b])
    real = [e for e, L in E.items() if abs(L - 1.0) < 1e-12]
    diag = [e for e, L in E.items() if abs(L - math.sqrt(2)) < 1e-12]
    assert len(real) == 12 and len(diag) == 6
    assert np.allclose(free_at(V, T, [edge_query(T, *e) for e in real]), 3 / 4, atol=1e-14)
    assert np.allclose(free_at(V, T, [edge_query(T, *e) for e in diag]), 1 / 2, atol=1e-14)
    # face interiors and the paper's constant
    inner = [(t, (0.2, 0.3)) for t in range(len(T))]
    assert np.all(free_at(V, T, inner) == 0.5)
    assert np.all(free_at(V, T, corners, jump=0) == 0.5)


def test_regular_icosahedron():
    u, f = W.icosphere_unit(0)
    assert len(f) == 20
    dihedral = math.acos(-math.sqrt(5.0) / 3.0)
    omega_v = 5 * dihedral - 3 * math.pi           # spherical excess of the vertex figure
    c_v = free_at(u, f, [vertex_query(f, v) for v in range(12)])
    assert np.allclose(c_v, 1 - omega_v / (4 * math.pi), atol=1e-13)
    edges = {tuple(sorted((tv[i], tv[(i + 1) % 3]))) for tv in f for i in range(3)}
    assert len(edges) == 30
    c_e = free_at(u, f, [edge_query(f, *e, s=0.61) for e in edges])
    assert np.allclose(c_e, 1 - dihedral / (2 * math.pi), atol=1e-13)


def test_non_convex_l_prism():
    V, T = l_prism()
    # the reflex vertical edge at (1, 1): interior dihedral 3 pi / 2
    a = int(np.nonzero(np.all(V == (1, 1, 0), axis=1))[0][0])
    b = int(np.nonzero(np.all(V == (1, 1, 1), axis=1))[0][0])
    assert free_at(V, T, [edge_query(T, a, b)])[0] == pytest.approx(0.25, abs=1e-14)
    # its end points: three octants of the body meet there
    assert np.allclose(free_at(V, T, [vertex_query(T, a), vertex_query(T, b)]), 5 / 8, atol=1e-14)
    # a convex corner and a convex vertical edge
    c = int(np.nonzero(np.all(V == (2, 0, 0), axis=1))[0][0])
    d = int(np.nonzero(np.all(V == (2, 0, 1), axis=1))[0][0])
    assert free_at(V, T, [vertex_query(T, c)])[0] == pytest.approx(7 / 8, abs=1e-14)
    assert free_at(V, T, [edge_query(T, c, d)])[0] == pytest.approx(3 / 4, abs=1e-14)


def test_smooth_limit_and_rigid_motion():
    """On refined spheres the vertex values approach 1/2 from above: a vertex
    with angle defect d is close to a circular cone whose solid-angle
    deficit is 2 pi sqrt(d / pi), so c - 1/2 ~ sqrt(d / (4 pi)) halves with
    each subdivision (d falls 4x).  A rigid motion changes nothing."""
    excess = []
    for sub in (1, 2, 3):
        u, f = W.icosphere_unit(sub)
        q = [vertex_query(f, v) for v in range(0, len(u), 7)]
        c = free_at(u, f, q)
        assert np.all(c > 0.5)
        d = 4 * math.pi / len(u)                     # mean angle defect (Descartes)
        assert np.mean(c) - 0.5 == pytest.approx(math.sqrt(d / (4 * math.pi)), rel=0.15)
        excess.append(np.mean(c) - 0.5)
    assert 1.6 < excess[0] / excess[1] < 2.4 and 1.6 < excess[1] / excess[2] < 2.4
    rng = np.random.default_rng(5)
    R = W.random_rotation(rng)
    c2 = free_at(u @ R.T + np.array([0.3, -2.0, 1.1]), f, q)
    assert np.allclose(c, c2, atol=1e-12)


def test_estimate_uses_the_free_term():
    """With jump = 1 the oracle's estimate at a vertex query equals the
    jump = 0 estimate rescaled by 1/2 over that query's free term."""
    V, T = cube()
    k = np.array([3.0])
    g = np.ones((1, len(V)), dtype=np.complex128)
    qs = [vertex_query(T, 0), edge_query(T, 0, 1), (5, (0.25, 0.25))]
    qt = np.array([q[0] for q in qs], dtype=np.int32)
    qb = np.array([q[1] for q in qs])
    r0 = O.mcbem(V, T, g, k, qt, qb, 256, 7, jump=0)
    r1 = O.mcbem(V, T, g, k, qt, qb, 256, 7, jump=1)
    c = O.free_terms(V, T, qt, qb, 1)
    assert np.allclose(c, [7 / 8, 3 / 4, 1 / 2], atol=1e-14)
    assert np.allclose(r1["p"][0], r0["p"][0] * 0.5 / c, rtol=1e-14, atol=0)
