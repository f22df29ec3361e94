"""GPU tests of scenes of several closed bodies (Section 4.1.1's
smooth-Neumann scenes: a speaker patch with g = 1, passive bodies with
g = 0; Section 3.4: data constant per triangle) through the C ABI: the
speaker-torus scene in the plain FP64 form (within 1e-10 of the oracle) and
the FP32 form (1e-3), per mode and element by element, a batch of speaker
positions equal to the single estimates bit for bit, the exterior field of
a scene, the dense Burton-Miller path on a scene, and the per-body
orientation check of mesh registration."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_06190_amd import nat  # noqa: E402
from _parity import check_modes, say as _say  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nat.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _scene_workload(y, n_modes=4, N=1500, Q=700, seed=31):
    sc = W.scene_speaker_torus(y)
    k = W.wavenumber(W.log_uniform_freqs(n_modes, seed))
    g = np.ascontiguousarray(np.repeat(sc.g_tri[None, :], n_modes, axis=0))
    qt, qb = W.random_face_queries(len(sc.tris), Q, seed)
    return W.MCWorkload(f"scene_y{y:+.2f}", sc.vertices, sc.tris, g, k, qt, qb, N, seed,
                        {"body": sc.body})


def _estimate(ctx, wl, prec, tol, flags=0):
    mesh = nat.Mesh(ctx, wl.vertices, wl.tris)
    opts = nat.nat_mc_opts_default()
    opts.precision = prec
    opts.gmres_tol = tol
    opts.layout = nat.NAT_NEUMANN_PER_TRIANGLE
    opts.flags = flags
    ps = torch.empty((wl.n_modes, wl.n_samples), dtype=torch.complex128, device=DEV)
    p, rep = nat.nat_mcbem_estimate(mesh, _dev(wl.g), wl.k, _dev(wl.q_tri), _dev(wl.q_b), wl.n_samples,
                                    wl.seed, opts, p_samples=ps)
    torch.cuda.synchronize()
    return mesh, p.cpu().numpy(), ps, rep


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_scene_matches_oracle(ctx, prec):
    wl = _scene_workload(0.02)
    _say(f"scene {prec}: T={len(wl.tris)} M={wl.n_modes} N={wl.n_samples} Q={wl.n_queries}")
    P = nat.NAT_PREC_FP64 if prec == "fp64" else nat.NAT_PREC_FP32
    mesh, p, ps, rep = _estimate(ctx, wl, P, 1e-12 if prec == "fp64" else 1e-6)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed, tol=1e-12,
                layout=1, want_samples=True)
    bar = 1e-10 if prec == "fp64" else 1e-3
    check_modes(p, r["p"], bar, f"scene {prec} queries")
    check_modes(ps.cpu().numpy(), r["p_samples"], bar, f"scene {prec} samples")
    # the passive body's pressure is not zero: it comes from the speaker
    on_torus = wl.extra["body"][wl.q_tri] == 1
    assert np.all(np.abs(p[:, on_torus]).mean(axis=1) > 1e-3 * np.abs(p).max(axis=1))
    _say(f"  iterations {[x['iters'] for x in rep]}")
    mesh.close()


def test_scene_batch_of_positions(ctx):
    """Four speaker heights (the scene's condition variable) in one batch:
    each equals its single estimate bit for bit and the oracle within the
    FP32 bar."""
    wls = [_scene_workload(y, n_modes=3, N=800, Q=300, seed=40 + i)
           for i, y in enumerate((-0.12, -0.03, 0.0, 0.09))]
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    opts = nat.nat_mc_opts_default()
    opts.layout = nat.NAT_NEUMANN_PER_TRIANGLE
    jobs = [nat.McJob(m, _dev(wl.g), wl.k, _dev(wl.q_tri), _dev(wl.q_b), wl.n_samples, wl.seed,
                      layout=nat.NAT_NEUMANN_PER_TRIANGLE) for wl, m in zip(wls, meshes)]
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    torch.cuda.synchronize()
    for wl, mesh, job in zip(wls, meshes, jobs):
        p1, _ = nat.nat_mcbem_estimate(mesh, job.v_n, wl.k, job.q_tri, job.q_bary, wl.n_samples,
                                       wl.seed, opts)
        torch.cuda.synchronize()
        assert torch.equal(job.p_out, p1)
        r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                    tol=1e-12, layout=1)
        check_modes(p1.cpu().numpy(), r["p"], 1e-3, wl.name)
    for m in meshes:
        m.close()


def test_scene_exterior_field(ctx):
    """Training tuples of a scene: the field at 2000 shell points around the
    whole scene from the GPU estimate, against the oracle end to end."""
    wl = _scene_workload(0.05, n_modes=3, N=1200, Q=10)
    mesh, _, ps, _ = _estimate(ctx, wl, nat.NAT_PREC_FP32, 1e-6)
    xs, _ = O.field_points(wl.vertices, 0, 2000, seed=9)
    opts = nat.nat_mc_opts_default()
    opts.layout = nat.NAT_NEUMANN_PER_TRIANGLE
    p, _ = nat.nat_mcbem_field(mesh, _dev(wl.g), wl.k, ps, wl.n_samples, wl.seed, _dev(xs), opts)
    torch.cuda.synchronize()
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed, tol=1e-12,
                layout=1, want_samples=True)
    po = O.mcbem_field(wl.vertices, wl.tris, wl.g, wl.k, wl.n_samples, wl.seed, xs, r["p_samples"],
                       layout=1)
    check_modes(p.cpu().numpy(), po, 1e-3, "scene field")
    mesh.close()


def test_scene_dense_burton_miller(ctx):
    """Dense collocation BEM on a coarse speaker-torus scene (per-triangle
    data): matrices and solution against the oracle."""
    sc = W.scene_speaker_torus(0.07, speaker_n=6, torus_nu=40, torus_nv=16)
    k = 40.0
    mesh = nat.Mesh(ctx, sc.vertices, sc.tris)
    op = nat.nat_bem_assemble(mesh, k, True)
    A, B = nat.nat_bem_op_matrices(op)
    p, rep = nat.nat_bem_solve(op, _dev(sc.g_tri[None, :]), layout=nat.NAT_NEUMANN_PER_TRIANGLE,
                               tol=1e-12)
    torch.cuda.synchronize()
    Ao, Bo = O.bem_assemble(sc.vertices, sc.tris, k, True)
    assert np.abs(A.cpu().numpy() - Ao).max() <= 1e-12 * np.abs(Ao).max()
    assert np.abs(B.cpu().numpy() - Bo).max() <= 1e-12 * np.abs(Bo).max()
    po, _, _ = O.bem_solve(Ao, Bo, sc.g_tri, tol=1e-12)
    check_modes(p.cpu().numpy()[0], po, 1e-9, f"scene dense n={len(sc.tris)}")
    op.close()
    mesh.close()


def test_scene_body_orientation_checked(ctx):
    sc = W.scene_speaker_torus(0.0)
    f = sc.tris.copy()
    f[sc.body == 1] = f[sc.body == 1][:, [0, 2, 1]]      # the torus turned inside out
    with pytest.raises(nat.NatError, match="body 1 of 2"):
        nat.Mesh(ctx, sc.vertices, f)
