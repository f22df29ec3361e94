"""Pins for the oracle on scenes of several closed bodies (Section 4.1.1: a
speaker surface with Neumann data 1 and passive objects with 0; Section
3.4: data constant per triangle): samples spread over the bodies by area,
an interior point source inside either body of a speaker-torus scene
(exact on the polyhedra themselves), and two spheres far apart, where the
pulsating one keeps its closed form and the passive one sees the incident
monopole."""
import numpy as np
import scipy.stats as st

import workloads as W
from oracle import closed_forms as CF
from oracle import oracle as O


def _vertex_normals(v, f):
    _, nrm, _ = O.geometry(v, f)
    vn = np.zeros_like(v)
    for c in range(3):
        np.add.at(vn, f[:, c], nrm)
    return vn / np.linalg.norm(vn, axis=1, keepdims=True)


def test_scene_mesh_and_samples_by_body_area():
    sc = W.scene_speaker_torus(0.05)
    area, nrm, cdf = O.geometry(sc.vertices, sc.tris)
    a_body = np.array([area[sc.body == b].sum() for b in (0, 1)])
    # the speaker's vibrating patch is its lower end only
    assert 0 < np.count_nonzero(sc.g_tri) < np.count_nonzero(sc.body == 0)
    assert np.all(sc.g_tri[sc.body == 1] == 0)
    tri, _ = O.samples(sc.vertices, sc.tris, 20000, 3)
    hits = np.bincount(sc.body[tri], minlength=2)
    assert st.chisquare(hits, 20000 * a_body / a_body.sum()).pvalue > 1e-3


def test_scene_interior_point_source():
    """x0 inside the speaker, then inside the torus's tube: g = dG(., x0)/dn on
    both bodies gives p = G(., x0) on both surfaces."""
    sc = W.scene_speaker_torus(0.1)
    v, f = sc.vertices, sc.tris
    vn = _vertex_normals(v, f)
    k = 30.0
    qt, qb = W.random_face_queries(len(f), 400, 3)
    xq = O.surface_points(v, f, qt, qb)
    on = sc.body[qt]
    bars = {0: (0.2, 0.4), 1: (0.2, 0.15)}   # (speaker, torus) error bars per source body
    for src_body, x0 in ((0, np.array([0.0, 0.1, 0.0])), (1, np.array([0.06, 0.0, 0.0]))):
        gv = CF.point_source_normal_derivative(k, v, vn, x0)
        r = O.mcbem(v, f, gv[None, :], [k], qt, qb, 4096, 5)
        ex = CF.point_source_field(k, xq, x0)
        for b in (0, 1):
            m = on == b
            e = np.linalg.norm(r["p"][0][m] - ex[m]) / np.linalg.norm(ex[m])
            assert e < bars[src_body][b], (src_body, b, e)


def test_two_spheres_far_apart():
    """Sphere A (radius 0.05, g = 1) and sphere B (g = 0) 0.5 m apart, k = 2:
    on A the single pulsating sphere's closed form, on B the incident monopole
    g a^2 e^{ik(d - a)} / ((ika - 1) d) on average (ka = 0.1: the passive
    sphere barely scatters)."""
    va, fa, _ = W.icosphere(3, 0.05)
    vb = va + np.array([0.5, 0.0, 0.0])
    v = np.concatenate([va, vb])
    f = np.concatenate([fa, fa + len(va)]).astype(np.int32)
    g = np.concatenate([np.ones(len(va)), np.zeros(len(vb))]).astype(complex)
    k = 2.0
    qt, qb = W.random_face_queries(len(f), 600, 4)
    onA = qt < len(fa)
    pa = CF.pulsating_sphere(k, 0.05)
    pinc = CF.pulsating_sphere_field(k, 0.05, 0.5)
    for s in range(2):
        p = O.mcbem(v, f, g[None], [k], qt, qb, 4096, 10 + s)["p"][0]
        assert np.linalg.norm(p[onA] - pa) / (abs(pa) * np.sqrt(onA.sum())) < 0.08
        assert abs(np.mean(p[~onA]) / pinc - 1.0) < 0.06
