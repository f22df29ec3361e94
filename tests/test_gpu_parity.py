"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.

Bars: sample triangle indices bit-exact and barycentrics within 4 ulp; the
plain FP64 form within 1e-10 per mode, the FP32 form within 1e-3 per mode,
each both as relative L2 and element by element (largest deviation at any
query over the largest reference value; the per-mode errors are printed);
the dense Burton-Miller matrices within 1e-12 of the largest entry and its
solutions within 1e-9, also element by element."""

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_06190_amd import nat  # noqa: E402
from _parity import check_modes, rel_l2 as _rel, say as _say  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nat.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _run_gpu(ctx, wl, prec, tol, layout=0, want_samples=False, max_iter=200, jump=0, flags=0):
    mesh = nat.Mesh(ctx, wl.vertices, wl.tris)
    g = torch.from_numpy(np.ascontiguousarray(wl.g)).to(DEV)
    qt = torch.from_numpy(np.ascontiguousarray(wl.q_tri)).to(DEV)
    qb = torch.from_numpy(np.ascontiguousarray(wl.q_b)).to(DEV)
    opts = nat.nat_mc_opts_default()
    opts.precision = prec
    opts.gmres_tol = tol
    opts.layout = layout
    opts.gmres_max_iter = max_iter
    opts.jump = jump
    opts.flags = flags
    ps = None
    if want_samples:
        ps = torch.empty((wl.n_modes, wl.n_samples), dtype=torch.complex128, device=DEV)
    p, rep = nat.nat_mcbem_estimate(mesh, g, wl.k, qt, qb, wl.n_samples, wl.seed, opts, p_samples=ps)
    torch.cuda.synchronize()
    out = p.cpu().numpy(), rep, (ps.cpu().numpy() if ps is not None else None)
    mesh.close()
    return out


def _small_ellipsoid(n_modes=11, Q=700, N=600, seed=77):
    v, f, u = W.noisy_ellipsoid(seed, subdiv=3)
    g = W.sh_neumann(u, n_modes, seed)
    k = W.wavenumber(W.log_uniform_freqs(n_modes, seed))
    qt, qb = W.random_face_queries(len(f), Q, seed)
    return W.MCWorkload("small_ellipsoid", v, f, g, k, qt, qb, N, seed)


def _edge_and_vertex_workload(seed, subdiv=3, n_modes=4, N=700):
    """Noise-displaced ellipsoid with queries on every vertex, on a spread of
    edges (one barycentric weight exactly 0) and at random face points."""
    v, f, u = W.noisy_ellipsoid(seed, subdiv=subdiv)
    vt, vb = W.vertex_queries(f, len(v))
    et, eb = [], []
    for t in range(0, len(f), 7):
        i = t % 3
        et.append(t)
        eb.append([(0.37, 1.0 - 0.37), (0.0, 0.37), (0.37, 0.0)][i])
    ft, fb = W.random_face_queries(len(f), 200, seed)
    qt = np.concatenate([vt, np.array(et, np.int32), ft]).astype(np.int32)
    qb = np.concatenate([vb, np.array(eb), fb])
    g = W.sh_neumann(u, n_modes, seed)
    k = W.wavenumber(W.log_uniform_freqs(n_modes, seed))
    return W.MCWorkload("edge_vertex_ellipsoid", v, f, g, k, qt, qb, N, seed)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_polyhedral_free_term(ctx, prec):
    """NAT_JUMP_POLYHEDRAL: queries on mesh vertices and edges use the free
    term of the body's solid angle there; GPU against the oracle (its own
    all-triangle solid-angle sum) element by element, and the default c = 1/2
    estimate is unchanged."""
    wl = _edge_and_vertex_workload(5)
    _say(f"polyhedral jump {prec}: T={len(wl.tris)} Q={wl.n_queries} N={wl.n_samples}")
    P = nat.NAT_PREC_FP64 if prec == "fp64" else nat.NAT_PREC_FP32
    tol = 1e-12 if prec == "fp64" else 1e-6
    p1, rep, _ = _run_gpu(ctx, wl, P, tol, jump=nat.NAT_JUMP_POLYHEDRAL)
    p0, _, _ = _run_gpu(ctx, wl, P, tol, jump=nat.NAT_JUMP_HALF)
    r1 = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                 tol=1e-12, jump=1)
    r0 = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                 tol=1e-12, jump=0)
    bar = 1e-10 if prec == "fp64" else 1e-3
    check_modes(p1, r1["p"], bar, f"polyhedral {prec}")
    check_modes(p0, r0["p"], bar, f"half {prec}")
    # the two forms differ exactly by the free-term ratio at every query
    c = O.free_terms(wl.vertices, wl.tris, wl.q_tri, wl.q_b, 1)
    assert np.any(c != 0.5)
    assert np.allclose(p1, p0 * (0.5 / c)[None, :], rtol=1e-13, atol=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_exact_disk_term(ctx, prec):
    """NAT_MC_EXACT_DISK: the disk term in closed form in both stages, against
    the oracle's same option; it moves the estimate by O(k eps^2)."""
    wl = _small_ellipsoid(n_modes=5, Q=400, N=500, seed=91)
    _say(f"exact disk {prec}: modes={wl.n_modes} N={wl.n_samples} Q={wl.n_queries}")
    P = nat.NAT_PREC_FP64 if prec == "fp64" else nat.NAT_PREC_FP32
    tol = 1e-12 if prec == "fp64" else 1e-6
    p1, _, _ = _run_gpu(ctx, wl, P, tol, flags=nat.NAT_MC_EXACT_DISK)
    r1 = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                 tol=1e-12, exact_disk=True)
    r0 = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                 tol=1e-12)
    bar = 1e-10 if prec == "fp64" else 1e-3
    check_modes(p1, r1["p"], bar, f"exact disk {prec}")
    assert max(_rel(r1["p"][m], r0["p"][m]) for m in range(wl.n_modes)) > 10 * bar or prec == "fp32"


def test_polyhedral_free_term_batch(ctx):
    """Two instances of different sizes in one batch with per-query free
    terms: each equals its single estimate bit for bit."""
    wls = [_edge_and_vertex_workload(8, subdiv=2, n_modes=3, N=300),
           _edge_and_vertex_workload(9, subdiv=3, n_modes=2, N=500)]
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    opts = nat.nat_mc_opts_default()
    opts.jump = nat.NAT_JUMP_POLYHEDRAL
    jobs = [nat.McJob(m, torch.from_numpy(wl.g).to(DEV), wl.k, torch.from_numpy(wl.q_tri).to(DEV),
                      torch.from_numpy(wl.q_b).to(DEV), wl.n_samples, wl.seed)
            for wl, m in zip(wls, meshes)]
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    torch.cuda.synchronize()
    for wl, mesh, job in zip(wls, meshes, jobs):
        p1, _ = nat.nat_mcbem_estimate(mesh, job.v_n, wl.k, job.q_tri, job.q_bary, wl.n_samples,
                                       wl.seed, opts)
        torch.cuda.synchronize()
        assert torch.equal(job.p_out, p1)
    for m in meshes:
        m.close()


def test_samples_bit_exact(ctx):
    for (v, f), N, seed in [(W.icosphere(3, 1.0)[:2], 256, 20250606),
                            (W.noisy_ellipsoid(3, subdiv=5)[:2], 4099, 12345),
                            (W.cubesphere_ellipsoid(9, 40000)[:2], 2048, 2**63 + 17)]:
        _say(f"samples T={len(f)} N={N} seed={seed}")
        mesh = nat.Mesh(ctx, v, f)
        tri = torch.empty(N, dtype=torch.int32, device=DEV)
        bary = torch.empty((N, 2), dtype=torch.float64, device=DEV)
        nat.nat_mcbem_samples(mesh, N, seed, tri, bary)
        torch.cuda.synchronize()
        t_o, b_o = O.samples(v, f, N, seed)
        assert np.array_equal(tri.cpu().numpy(), t_o)
        ulp = np.spacing(np.abs(b_o)) + 1e-300
        assert (np.abs(bary.cpu().numpy() - b_o) <= 4 * ulp).all()
        mesh.close()


def test_plain_fp64_matches_oracle_pulsating_sphere(ctx):
    wl = W.config_pulsating_sphere()
    _say(f"fp64 {wl.name} N={wl.n_samples} Q={wl.n_queries}")
    p, rep, ps = _run_gpu(ctx, wl, nat.NAT_PREC_FP64, 1e-12, want_samples=True)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                tol=1e-12, want_samples=True)
    _say(f"  iters gpu {rep[0]['iters']} oracle {r['iters'][0]}")
    check_modes(p, r["p"], 1e-10, "queries")
    check_modes(ps, r["p_samples"], 1e-10, "samples")
    assert rep[0]["converged"] == 1 and rep[0]["eps"] > 0
    assert rep[0]["area"] == pytest.approx(O.geometry(wl.vertices, wl.tris)[2][-1], rel=1e-15)


def test_plain_fp64_ragged_multimode(ctx):
    wl = _small_ellipsoid()
    _say(f"fp64 ragged modes={wl.n_modes} N={wl.n_samples} Q={wl.n_queries}")
    p, rep, ps = _run_gpu(ctx, wl, nat.NAT_PREC_FP64, 1e-12, want_samples=True)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                tol=1e-12, want_samples=True)
    check_modes(p, r["p"], 1e-10, "queries")
    check_modes(ps, r["p_samples"], 1e-10, "samples")


def test_fp32_ragged_multimode(ctx):
    wl = _small_ellipsoid()
    _say(f"fp32 ragged modes={wl.n_modes} N={wl.n_samples} Q={wl.n_queries}")
    p, rep, ps = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-6, want_samples=True)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                tol=1e-12, want_samples=True)
    check_modes(p, r["p"], 1e-3, "fp32 queries")
    check_modes(ps, r["p_samples"], 1e-3, "fp32 samples")
    assert all(rr["converged"] for rr in rep)
    # stage times of the call (device events), the same for every mode
    for key in ("t_sample_ms", "t_rhs_ms", "t_solve_ms", "t_eval_ms"):
        assert rep[0][key] > 0.0 and all(rr[key] == rep[0][key] for rr in rep), key
    assert rep[0]["t_solve_ms"] > rep[0]["t_rhs_ms"]


def test_fp32_long_phases(ctx):
    """Wavenumbers high enough that k r / (2 pi) exceeds 64 revolutions on the
    mesh (about 100), so the FP32 sums reduce the phase before the hardware
    sine and cosine; N = 150 samples, so unrestarted GMRES with 200
    iterations converges; within the FP32 bar of the oracle."""
    v, f, u = W.noisy_ellipsoid(13, subdiv=3)
    k = np.array([2200.0, 2500.0])
    g = W.sh_neumann(u, 2, 13)
    qt, qb = W.random_face_queries(len(f), 200, 13)
    wl = W.MCWorkload("long_phases", v, f, g, k, qt, qb, 150, 13)
    diam = np.linalg.norm(v.max(axis=0) - v.min(axis=0))
    assert k.max() / (2 * np.pi) * diam > 64
    _say(f"fp32 long phases: k={k.tolist()} diam={diam:.3f} N={wl.n_samples}")
    p, rep, _ = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-9)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed, tol=1e-12)
    check_modes(p, r["p"], 1e-3, "long phases")


def test_fp64_phase_long_phases(ctx):
    """NAT_MC_FP64_PHASE at phases of about 100 revolutions: the phase formed
    from FP64 positions and reduced in FP64, in both matvec forms, against
    the oracle; the FP64 phase is at least as close to the oracle as the
    FP32 phase."""
    v, f, u = W.noisy_ellipsoid(13, subdiv=3)
    k = np.array([2200.0, 2500.0])
    g = W.sh_neumann(u, 2, 13)
    qt, qb = W.random_face_queries(len(f), 200, 13)
    wl = W.MCWorkload("long_phases", v, f, g, k, qt, qb, 150, 13)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed, tol=1e-12)
    worst = {}
    for name, flags in (("fp32 phase", 0), ("fp64 phase", nat.NAT_MC_FP64_PHASE),
                        ("fp64 phase, ordered", nat.NAT_MC_FP64_PHASE | nat.NAT_MC_ORDERED_SUM)):
        p, rep, ps = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-9, flags=flags, want_samples=True)
        errs = check_modes(p, r["p"], 1e-3, name)
        worst[name] = max(max(e) for e in errs)
    _say(f"  worst error: {worst}")
    assert worst["fp64 phase"] <= worst["fp32 phase"]
    assert worst["fp64 phase, ordered"] <= worst["fp32 phase"]


def test_fp64_phase_batch_equals_alone(ctx):
    """The FP64-phase form in a batch of uneven instances: each equals its
    single estimate bit for bit and the oracle within the FP32 bar."""
    wls = [_small_ellipsoid(n_modes=3, Q=300, N=400, seed=61), _small_ellipsoid(n_modes=9, Q=200, N=257,
                                                                              seed=62)]
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    opts = nat.nat_mc_opts_default()
    opts.flags = nat.NAT_MC_FP64_PHASE
    jobs = [nat.McJob(m, torch.from_numpy(wl.g).to(DEV), wl.k, torch.from_numpy(wl.q_tri).to(DEV),
                      torch.from_numpy(wl.q_b).to(DEV), wl.n_samples, wl.seed)
            for wl, m in zip(wls, meshes)]
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    torch.cuda.synchronize()
    for wl, mesh, job in zip(wls, meshes, jobs):
        p1, _ = nat.nat_mcbem_estimate(mesh, job.v_n, wl.k, job.q_tri, job.q_bary, wl.n_samples,
                                       wl.seed, opts)
        torch.cuda.synchronize()
        assert torch.equal(job.p_out, p1)
        r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                    tol=1e-12)
        check_modes(p1.cpu().numpy(), r["p"], 1e-3, "fp64 phase in a batch")
    for m in meshes:
        m.close()


def test_fp32_full_precision_workload(ctx):
    """Noise-displaced ellipsoid, 20480 triangles, 32 modes, 4096 queries x 1024
    samples, the launch configuration the benchmark times."""
    wl = W.config_precision()
    _say(f"fp32 {wl.name}")
    p, rep, _ = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-6)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed, tol=1e-12)
    _say(f"  iterations: {[rr['iters'] for rr in rep]}")
    check_modes(p, r["p"], 1e-3, "precision workload")


def test_oscillating_sphere_mc_full_size(ctx):
    """The Monte-Carlo half of the dense-path workload at full size: 5120
    triangles, N = 4096 samples, all 2562 vertex queries, ka = 1, 5, 10; plain
    FP64 within 1e-10 and FP32 within 1e-3 of the oracle.  Against the
    closed-form dipole pressure the estimate carries the method's own
    Monte-Carlo error at N = 4096 (the oracle's: 5 %, 15 % and 32 % at ka = 1,
    5, 10), which the test prints and bounds loosely."""
    from oracle import closed_forms as CF
    wl = W.config_oscillating_sphere()
    _say(f"oscillating sphere MC: T={len(wl.tris)} N={wl.n_samples} Q={wl.n_queries} ka=1,5,10")
    ref = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                  tol=1e-12)
    p64, _, _ = _run_gpu(ctx, wl, nat.NAT_PREC_FP64, 1e-12)
    p32, rep, _ = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-6)
    a = wl.extra["radius"]
    cos_t = wl.extra["u"][:, 2]
    check_modes(p64, ref["p"], 1e-10, "FP64")
    check_modes(p32, ref["p"], 1e-3, "FP32")
    for m in range(wl.n_modes):
        exact = CF.oscillating_sphere_factor(wl.k[m], a) * cos_t
        e_cf = _rel(p32[m], exact)
        _say(f"  ka={wl.k[m] * a:g}: {e_cf:.3f} vs closed form; iters {rep[m]['iters']}")
        assert e_cf <= 0.5


def test_per_triangle_layout_and_no_queries(ctx):
    v, f, u = W.icosphere(3, 1.0)
    rng = np.random.default_rng(5)
    gt = (rng.standard_normal((2, len(f))) + 1j * rng.standard_normal((2, len(f))))
    qt, qb = W.random_face_queries(len(f), 130, 9)
    wl = W.MCWorkload("per_tri", v, f, gt, np.array([2.0, 7.5]), qt, qb, 300, 3)
    p, rep, ps = _run_gpu(ctx, wl, nat.NAT_PREC_FP64, 1e-12, layout=1, want_samples=True)
    r = O.mcbem(v, f, gt, wl.k, qt, qb, 300, 3, tol=1e-12, layout=1, want_samples=True)
    check_modes(p, r["p"], 1e-10, "per triangle")
    check_modes(ps, r["p_samples"], 1e-10, "per triangle samples")
    # Q = 0: only the sample values are produced
    wl0 = W.MCWorkload("noq", v, f, gt, wl.k, qt[:0], qb[:0], 300, 3)
    p0, rep0, ps0 = _run_gpu(ctx, wl0, nat.NAT_PREC_FP64, 1e-12, layout=1, want_samples=True)
    assert p0.shape == (2, 0)
    check_modes(ps0, r["p_samples"], 1e-10, "no queries, samples")


def test_minimum_sample_count(ctx):
    wl = W.config_pulsating_sphere(n_samples=2)
    p, rep, ps = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-6, want_samples=True)
    r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, 2, wl.seed, tol=1e-12,
                want_samples=True)
    check_modes(p, r["p"], 1e-3, "N = 2")
    check_modes(ps, r["p_samples"], 1e-3, "N = 2 samples")


def test_deterministic_and_rigid_motion(ctx):
    wl = _small_ellipsoid(n_modes=3, Q=257, N=513, seed=8)
    a, _, _ = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-6)
    b, _, _ = _run_gpu(ctx, wl, nat.NAT_PREC_FP32, 1e-6)
    assert np.array_equal(a, b)
    rot = W.random_rotation(np.random.default_rng(1))
    moved = W.MCWorkload("moved", wl.vertices @ rot.T + np.array([0.4, -0.3, 0.2]), wl.tris, wl.g,
                         wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed)
    c, _, _ = _run_gpu(ctx, moved, nat.NAT_PREC_FP32, 1e-6)
    for m in range(3):
        assert _rel(c[m], a[m]) <= 1e-4


def test_context_closes_what_it_made():
    """Closing a context first closes the meshes, servers and fields made
    from it, so a later close (or garbage collection) of those is a no-op."""
    c = nat.Context(0)
    v, f = W.icosphere(2, 1.0)[:2]
    m = nat.Mesh(c, v, f)
    so = nat.nat_server_opts_default()
    so.hbm_budget = 1 << 28
    srv = nat.Server(c, so)
    nf = nat.NeuralField(c, 0, 1, 1.5, 3.0)
    c.close()
    assert m.handle is None and srv.handle is None and nf.handle is None and c.handle is None
    m.close()
    nf.close()


def test_error_paths(ctx):
    v, f, u = W.icosphere(2, 1.0)
    mesh = nat.Mesh(ctx, v, f)
    g = torch.ones((1, len(v)), dtype=torch.complex128, device=DEV)
    qt = torch.zeros(4, dtype=torch.int32, device=DEV)
    qb = torch.zeros((4, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(nat.NatError) as ei:            # k <= 0
        nat.nat_mcbem_estimate(mesh, g, [0.0], qt, qb, 64, 1)
    assert ei.value.status == nat.NAT_E_INVALID
    bad = qt.clone()
    bad[2] = len(f)
    with pytest.raises(nat.NatError) as ei:            # triangle out of range
        nat.nat_mcbem_estimate(mesh, g, [1.0], bad, qb, 64, 1)
    assert ei.value.status == nat.NAT_E_INVALID
    gn = g.clone()
    gn[0, 3] = float("nan")
    with pytest.raises(nat.NatError) as ei:            # NaN Neumann data
        nat.nat_mcbem_estimate(mesh, gn, [1.0], qt, qb, 64, 1)
    assert ei.value.status == nat.NAT_E_INVALID
    opts = nat.nat_mc_opts_default()
    opts.gmres_max_iter = 1
    opts.precision = nat.NAT_PREC_FP64
    p, rep = nat.nat_mcbem_estimate(mesh, g, [1.0], qt, qb, 64, 1, opts, allow_noconv=True)
    assert rep[0]["iters"] == 1 and rep[0]["converged"] == 0 and torch.isfinite(p).all()
    with pytest.raises(nat.NatError) as ei:
        nat.nat_mcbem_estimate(mesh, g, [1.0], qt, qb, 64, 1, opts)
    assert ei.value.status == nat.NAT_E_NOCONV
    for field, value in (("jump", 2), ("flags", nat.NAT_MC_ASSEMBLED | nat.NAT_MC_MATRIX_FREE),
                         ("flags", nat.NAT_MC_ASSEMBLED | nat.NAT_MC_FP64_PHASE),
                         ("flags", 128), ("eps_scale", 0.0)):
        o = nat.nat_mc_opts_default()
        setattr(o, field, value)
        with pytest.raises(nat.NatError) as ei:        # invalid options
            nat.nat_mcbem_estimate(mesh, g, [1.0], qt, qb, 64, 1, o)
        assert ei.value.status == nat.NAT_E_INVALID, (field, value)
    mesh.close()
    small = nat.Context(0, hbm_budget_bytes=1 << 16)
    m2 = nat.Mesh(small, v, f)
    with pytest.raises(nat.NatError) as ei:
        nat.nat_mcbem_estimate(m2, g, [1.0], qt, qb, 4096, 1)
    assert ei.value.status == nat.NAT_E_BUDGET
    m2.close()
    small.close()


# ------------------------------------------------------------- dense BEM
def _dense_gpu(ctx, v, f, k, gv, bm=True, tol=1e-12):
    mesh = nat.Mesh(ctx, v, f)
    op = nat.nat_bem_assemble(mesh, k, bm)
    A, B = nat.nat_bem_op_matrices(op)
    g = torch.from_numpy(np.ascontiguousarray(np.atleast_2d(gv))).to(DEV)
    p, rep = nat.nat_bem_solve(op, g, tol=tol)
    torch.cuda.synchronize()
    out = A.cpu().numpy(), B.cpu().numpy(), p.cpu().numpy(), rep
    op.close()
    mesh.close()
    return out


@pytest.mark.parametrize("bm", [True, False])
def test_dense_matrices_match_oracle(ctx, bm):
    v, f, u = W.noisy_ellipsoid(3, subdiv=2)
    k = 40.0
    _say(f"dense assemble n={len(f)} bm={bm}")
    A, B, p, rep = _dense_gpu(ctx, v, f, k, u[:, 2].astype(complex), bm)
    Ao, Bo = O.bem_assemble(v, f, k, bm)
    assert np.abs(A - Ao).max() <= 1e-12 * np.abs(Ao).max()
    assert np.abs(B - Bo).max() <= 1e-12 * np.abs(Bo).max()
    po, _, _ = O.bem_solve(Ao, Bo, O.panel_data(f, u[:, 2].astype(complex)), tol=1e-12)
    check_modes(p[0], po, 1e-9, "dense")


def test_dense_oscillating_sphere_full_size(ctx):
    """Icosphere of radius 0.1 m, 5120 panels, v_n = cos(theta), k a in {1, 5, 10}."""
    wl = W.config_oscillating_sphere()
    a = wl.extra["radius"]
    u = wl.extra["u"]
    for k in wl.k:
        _say(f"dense n={len(wl.tris)} ka={k * a}")
        A, B, p, rep = _dense_gpu(ctx, wl.vertices, wl.tris, k, u[:, 2].astype(complex))
        Ao, Bo = O.bem_assemble(wl.vertices, wl.tris, k, True)
        assert np.abs(A - Ao).max() <= 1e-12 * np.abs(Ao).max()
        po, it, res = O.bem_solve(Ao, Bo, O.panel_data(wl.tris, u[:, 2].astype(complex)), tol=1e-12)
        _say(f"  iters {rep[0]['iters']}")
        check_modes(p[0], po, 1e-9, f"dense ka={k * a:g}")
        del A, B, Ao, Bo


@pytest.mark.parametrize("mesh_kind,n_rhs", [("ico3", 9), ("ico3", 20), ("cube13", 16)])
def test_dense_multi_rhs_matrix_cores(ctx, mesh_kind, n_rhs):
    """From 8 right-hand sides on, the dense products run on the FP64 matrix
    cores (16 per pass over the matrix, split over K segments); every solution
    matches the FP64 oracle's collocation solve of the same right-hand side
    (oracle assembly and GMRES) within 1e-9, element by element, and agrees
    with the same right-hand side solved alone (GEMV path).  The
    2028-triangle cube-sphere leaves a ragged last row tile and a last K
    segment with one whole step and a partial one."""
    if mesh_kind == "ico3":
        v, f, u = W.icosphere(3, 0.1)
    else:
        u, f = W.cubesphere_unit(13)
        v = 0.1 * u
    c = u[f].mean(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    g = torch.from_numpy(W.sh_neumann(c, n_rhs, 77)).to(DEV)
    mesh = nat.Mesh(ctx, v, f)
    op = nat.nat_bem_assemble(mesh, 30.0, True)
    _say(f"dense multi-rhs: n={len(f)} n_rhs={n_rhs}")
    p_all, rep_all = nat.nat_bem_solve(op, g, layout=nat.NAT_NEUMANN_PER_TRIANGLE, tol=1e-12)
    torch.cuda.synchronize()
    Ao, Bo = O.bem_assemble(v, f, 30.0, True)
    gh = g.cpu().numpy()
    ref = np.stack([O.bem_solve(Ao, Bo, gh[r], tol=1e-12)[0] for r in range(n_rhs)])
    del Ao, Bo
    check_modes(p_all.cpu().numpy(), ref, 1e-9, f"matrix cores, {n_rhs} rhs vs oracle")
    for r in range(n_rhs):
        p1, rep1 = nat.nat_bem_solve(op, g[r:r + 1].contiguous(), layout=nat.NAT_NEUMANN_PER_TRIANGLE,
                                     tol=1e-12)
        torch.cuda.synchronize()
        a, b = p_all[r].cpu().numpy(), p1[0].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b), r
        assert abs(rep_all[r]["iters"] - rep1[0]["iters"]) <= 1
        assert rep_all[r]["t_solve_ms"] > 0.0 and rep_all[r]["t_rhs_ms"] == 0.0
    op.close()
    mesh.close()


@pytest.mark.parametrize("sub,n_rhs", [(19, 7), (13, 6)])
def test_dense_few_rhs_vector_products(ctx, sub, n_rhs):
    """Below 8 right-hand sides the dense products run on the vector units,
    up to 4 right-hand sides per pass over the matrix: 4332 triangles take
    the four-rows-per-workgroup form (passes of 4 and 3), 2028 triangles the
    one-row form (passes of 4 and 2); every solution matches the FP64
    oracle's collocation solve of the same right-hand side within 1e-9,
    element by element."""
    u, f = W.cubesphere_unit(sub)
    v = 0.1 * u
    c = u[f].mean(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    g = torch.from_numpy(W.sh_neumann(c, n_rhs, 78)).to(DEV)
    mesh = nat.Mesh(ctx, v, f)
    op = nat.nat_bem_assemble(mesh, 30.0, True)
    _say(f"dense few-rhs: n={len(f)} n_rhs={n_rhs}")
    p_all, rep_all = nat.nat_bem_solve(op, g, layout=nat.NAT_NEUMANN_PER_TRIANGLE, tol=1e-12)
    torch.cuda.synchronize()
    op.close()
    mesh.close()
    Ao, Bo = O.bem_assemble(v, f, 30.0, True)
    gh = g.cpu().numpy()
    ref = np.stack([O.bem_solve(Ao, Bo, gh[r], tol=1e-12)[0] for r in range(n_rhs)])
    check_modes(p_all.cpu().numpy(), ref, 1e-9, f"vector products, {n_rhs} rhs vs oracle")


def test_options_together_in_a_batch(ctx):
    """The polyhedral free term, the exact disk term and the assembled-operator
    matvec at once, in a two-instance batch: each instance equals its single
    estimate bit for bit and the oracle with the same options within the
    FP32 bar."""
    wls = [_edge_and_vertex_workload(41, subdiv=2, n_modes=3, N=300),
           _edge_and_vertex_workload(42, subdiv=3, n_modes=2, N=450)]
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    opts = nat.nat_mc_opts_default()
    opts.jump = nat.NAT_JUMP_POLYHEDRAL
    opts.flags = nat.NAT_MC_EXACT_DISK | nat.NAT_MC_ASSEMBLED
    jobs = [nat.McJob(m, torch.from_numpy(wl.g).to(DEV), wl.k, torch.from_numpy(wl.q_tri).to(DEV),
                      torch.from_numpy(wl.q_b).to(DEV), wl.n_samples, wl.seed)
            for wl, m in zip(wls, meshes)]
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    torch.cuda.synchronize()
    for wl, mesh, job in zip(wls, meshes, jobs):
        p1, _ = nat.nat_mcbem_estimate(mesh, job.v_n, wl.k, job.q_tri, job.q_bary, wl.n_samples,
                                       wl.seed, opts)
        torch.cuda.synchronize()
        assert torch.equal(job.p_out, p1)
        r = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                    tol=1e-12, jump=1, exact_disk=True)
        check_modes(p1.cpu().numpy(), r["p"], 1e-3, "options together")
    for m in meshes:
        m.close()
