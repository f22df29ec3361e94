"""The library's free terms for NAT_JUMP_POLYHEDRAL (host code, no GPU):
vertex values from a cap closing the vertex's cone, edge values from the
dihedral angle.  Checked against the closed forms the oracle is pinned to and
against the oracle's own definition (the body's solid angle summed over every
other triangle) on curved and irregular meshes."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from paper_2506_06190_amd import nat
from test_oracle_free_terms import cube, edge_query, l_prism, vertex_query


def test_closed_forms():
    V, T = cube()
    cv, ce = nat.nat_mesh_free_terms(V, T)
    assert np.allclose(cv, 7 / 8, atol=1e-14)
    for t, tv in enumerate(T):
        for i in range(3):
            a, b = tv[(i + 1) % 3], tv[(i + 2) % 3]
            L = np.linalg.norm(V[a] - V[b])
            assert ce[t, i] == pytest.approx(3 / 4 if abs(L - 1) < 1e-12 else 1 / 2, abs=1e-14)
    V, T = l_prism()
    cv, ce = nat.nat_mesh_free_terms(V, T)
    a = int(np.nonzero(np.all(V == (1, 1, 0), axis=1))[0][0])
    b = int(np.nonzero(np.all(V == (1, 1, 1), axis=1))[0][0])
    assert cv[a] == pytest.approx(5 / 8, abs=1e-14) and cv[b] == pytest.approx(5 / 8, abs=1e-14)
    t, (b1, b2) = edge_query(T, a, b)
    corner = [i for i in range(3) if T[t][i] not in (a, b)][0]
    assert ce[t, corner] == pytest.approx(1 / 4, abs=1e-14)
    u, f = W.icosphere_unit(0)
    cv, ce = nat.nat_mesh_free_terms(u, f)
    dihedral = math.acos(-math.sqrt(5.0) / 3.0)
    assert np.allclose(cv, 1 - (5 * dihedral - 3 * math.pi) / (4 * math.pi), atol=1e-13)
    assert np.allclose(ce, 1 - dihedral / (2 * math.pi), atol=1e-13)


@pytest.mark.parametrize("kind", ["icosphere", "ellipsoid", "cubesphere"])
def test_against_oracle(kind):
    if kind == "icosphere":
        V, T = W.icosphere_unit(3)
    elif kind == "ellipsoid":
        V, T, _ = W.noisy_ellipsoid(11, subdiv=3)
    else:
        V, T = W.cubesphere_unit(6)
    cv, ce = nat.nat_mesh_free_terms(V, T)
    vs = list(range(0, len(V), 5))
    q = [vertex_query(T, v) for v in vs]
    ref = O.free_terms(V, T, np.array([x[0] for x in q], np.int32), np.array([x[1] for x in q]), 1)
    assert np.allclose(cv[vs], ref, rtol=0, atol=1e-12)
    edges = []
    for t in range(0, len(T), 9):
        i = t % 3
        edges.append((t, i, T[t][(i + 1) % 3], T[t][(i + 2) % 3]))
    q = [edge_query(T, a, b, s=0.37) for (_, _, a, b) in edges]
    ref = O.free_terms(V, T, np.array([x[0] for x in q], np.int32), np.array([x[1] for x in q]), 1)
    got = np.array([ce[t, i] for (t, i, _, _) in edges])
    assert np.allclose(got, ref, rtol=0, atol=1e-12)
