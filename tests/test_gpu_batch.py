"""GPU tests of the batched form: many instances of uneven size in one set
of launches.  Each job's results must be bit-for-bit those of the same job
run alone, graph replay must equal direct launches bit for bit, and a mixed
batch must match the FP64 oracle within 1e-3 relative L2 per mode."""
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_06190_amd import nat  # noqa: E402
from _parity import check_modes, mode_errors, say as _say  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nat.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _mixed_workloads(n=5, seed=31):
    """Small cube-sphere instances of uneven size: N, Q, modes all differ."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        T = int(rng.integers(300, 2500))
        v, f, u = W.cubesphere_ellipsoid(seed * 100 + i, T)
        M = int(rng.integers(1, 12))
        g = W.sh_neumann(u, M, seed * 100 + i)
        k = W.wavenumber(W.log_uniform_freqs(M, seed * 100 + i))
        Q = int(rng.integers(1, 900))
        N = int(rng.integers(70, 700))
        qt, qb = W.random_face_queries(len(f), Q, seed * 100 + i)
        out.append(W.MCWorkload(f"mix{i}", v, f, g, k, qt, qb, N, seed * 100 + i))
    return out


def _jobs(ctx, wls, meshes):
    jobs = []
    for wl, mesh in zip(wls, meshes):
        jobs.append(nat.McJob(mesh, torch.from_numpy(wl.g).to(DEV), wl.k,
                              torch.from_numpy(wl.q_tri).to(DEV), torch.from_numpy(wl.q_b).to(DEV),
                              wl.n_samples, wl.seed,
                              p_samples=torch.empty((wl.n_modes, wl.n_samples),
                                                    dtype=torch.complex128, device=DEV)))
    return jobs


def test_batch_equals_single_and_oracle(ctx):
    wls = _mixed_workloads()
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    _say("batch sizes: " + ", ".join(f"(T={len(w.tris)}, M={w.n_modes}, N={w.n_samples}, Q={w.n_queries})"
                                     for w in wls))
    opts = nat.nat_mc_opts_default()
    jobs = _jobs(ctx, wls, meshes)
    reps = nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    torch.cuda.synchronize()
    for wl, mesh, job, rep in zip(wls, meshes, jobs, reps):
        p_single, rep1 = nat.nat_mcbem_estimate(
            mesh, job.v_n, wl.k, job.q_tri, job.q_bary, wl.n_samples, wl.seed, opts)
        torch.cuda.synchronize()
        assert torch.equal(p_single, job.p_out), wl.name
        assert [r["iters"] for r in rep1] == [r["iters"] for r in rep]
        ref = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed)
        check_modes(job.p_out.cpu().numpy(), ref["p"], 1e-3, f"{wl.name} vs oracle")
    for m in meshes:
        m.close()


def test_system_alone_equals_forty_copies_in_one_batch(ctx):
    """One system alone (8 chunks of 256 rows) and 40 copies of it in one
    batch (320 chunks, 40 instances sharing every launch) agree bit for bit in
    results and iteration counts, with and without graph replay."""
    v, f, u = W.cubesphere_ellipsoid(77, 3000)
    g = torch.from_numpy(W.sh_neumann(u, 1, 77)).to(DEV)
    k = [float(W.wavenumber(np.array([2500.0]))[0])]
    N = 2048
    qt, qb = W.random_face_queries(len(f), 300, 77)
    qt, qb = torch.from_numpy(qt).to(DEV), torch.from_numpy(qb).to(DEV)
    mesh = nat.Mesh(ctx, v, f)
    for flags in (0, nat.NAT_MC_NO_GRAPH):
        opts = nat.nat_mc_opts_default()
        opts.flags = flags
        p_alone, rep_alone = nat.nat_mcbem_estimate(mesh, g, k, qt, qb, N, 5, opts)
        jobs = [nat.McJob(mesh, g, k, qt, qb, N, 5) for _ in range(40)]
        reps = nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
        torch.cuda.synchronize()
        _say(f"  flags {flags}: {rep_alone[0]['iters']} iterations")
        assert rep_alone[0]["iters"] >= 5
        for job, rep in zip(jobs, reps):
            assert rep[0]["iters"] == rep_alone[0]["iters"]
            assert torch.equal(job.p_out, p_alone)
    mesh.close()


def test_graph_replay_equals_direct_launches(ctx):
    # one mode of this batch is close to an interior resonance of the
    # conventional equation and stops at 200 iterations above 1e-6 (the FP64
    # oracle does too), so the runs also cover the max-iteration exit
    wls = _mixed_workloads(4, seed=7)
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    results = []
    for flags in (0, nat.NAT_MC_NO_GRAPH, 0, 0):
        opts = nat.nat_mc_opts_default()
        opts.flags = flags
        jobs = _jobs(ctx, wls, meshes)
        reps = nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
        torch.cuda.synchronize()
        assert max(r["iters"] for r in reps[3]) == 200 and not all(r["converged"] for r in reps[3])
        results.append([(j.p_out.cpu(), j.p_samples.cpu()) for j in jobs])
    for r in results[1:]:
        for (a, b), (c, d) in zip(results[0], r):
            assert torch.equal(a, c) and torch.equal(b, d)
    for m in meshes:
        m.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_concurrent_parts_equal_one_stream(ctx, prec):
    """nat_mc_opts.n_streams: the batch split into 2, 3 or 5 parts on streams
    of their own gives the same bits (outputs, samples, iteration counts) as
    the whole batch on the caller's stream."""
    wls = _mixed_workloads(5, seed=11)
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    results = []
    for n_streams in (1, 2, 3, 5, 0):
        opts = nat.nat_mc_opts_default()
        opts.precision = nat.NAT_PREC_FP32 if prec == "fp32" else nat.NAT_PREC_FP64
        opts.n_streams = n_streams
        jobs = _jobs(ctx, wls, meshes)
        _say(f"{prec} n_streams={n_streams}")
        reps = nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
        torch.cuda.synchronize()
        results.append(([(j.p_out.cpu(), j.p_samples.cpu()) for j in jobs],
                        [[r["iters"] for r in rr] for rr in reps]))
    for outs, iters in results[1:]:
        assert iters == results[0][1]
        for (a, b), (c, d) in zip(results[0][0], outs):
            assert torch.equal(a, c) and torch.equal(b, d)
    for m in meshes:
        m.close()


def test_concurrent_parts_grow_scratch():
    """Parts whose scratch has to grow while other parts capture their GMRES
    graphs (a fresh context: small batch first, then a larger one), against
    the one-stream run of the larger batch."""
    c = nat.Context(0)
    small = _mixed_workloads(4, seed=17)
    large = _mixed_workloads(8, seed=19)
    for wls in (small, large):
        meshes = [nat.Mesh(c, wl.vertices, wl.tris) for wl in wls]
        outs = []
        for n_streams in (4, 1):
            opts = nat.nat_mc_opts_default()
            opts.n_streams = n_streams
            jobs = _jobs(c, wls, meshes)
            _say(f"grow: {len(wls)} jobs, n_streams={n_streams}")
            nat.nat_mcbem_estimate_batch(c, jobs, opts, allow_noconv=True)
            torch.cuda.synchronize()
            outs.append([j.p_out.cpu() for j in jobs])
        for a, b in zip(*outs):
            assert torch.equal(a, b)
        for m in meshes:
            m.close()
    c.close()


def test_concurrent_parts_errors(ctx):
    """A bad job anywhere in a split batch is refused before any part runs,
    and n_streams outside 0..8 is refused."""
    wls = _mixed_workloads(4, seed=13)
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    jobs = _jobs(ctx, wls, meshes)
    opts = nat.nat_mc_opts_default()
    opts.n_streams = 9
    with pytest.raises(nat.NatError):
        nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    opts.n_streams = 4
    jobs[2].k = np.array([-1.0] * wls[2].n_modes)
    with pytest.raises(nat.NatError, match="k\\[0\\]"):
        nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    for m in meshes:
        m.close()


def test_batch_fp64_plain_matches_oracle(ctx):
    wls = _mixed_workloads(3, seed=3)
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    opts = nat.nat_mc_opts_default()
    opts.precision = nat.NAT_PREC_FP64
    opts.gmres_tol = 1e-12
    jobs = _jobs(ctx, wls, meshes)
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts)
    torch.cuda.synchronize()
    for wl, job in zip(wls, jobs):
        ref = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                      want_samples=True)
        check_modes(job.p_out.cpu().numpy(), ref["p"], 1e-10, f"{wl.name} FP64 vs oracle")
        check_modes(job.p_samples.cpu().numpy(), ref["p_samples"], 1e-10,
                    f"{wl.name} FP64 samples vs oracle")
    for m in meshes:
        m.close()


@pytest.fixture(scope="module")
def full_batch(ctx):
    """The headline workload at full size, in the form the benchmark times
    (one batch of 256 instances, graph-replayed GMRES, concurrent parts)."""
    wls = W.config_batched()
    meshes = [nat.Mesh(ctx, wl.vertices, wl.tris) for wl in wls]
    jobs = [nat.McJob(m, torch.from_numpy(wl.g).to(DEV), wl.k, torch.from_numpy(wl.q_tri).to(DEV),
                      torch.from_numpy(wl.q_b).to(DEV), wl.n_samples, wl.seed)
            for wl, m in zip(wls, meshes)]
    _say(f"full batch: {len(jobs)} instances, {sum(j.n_modes for j in jobs)} systems")
    reps = nat.nat_mcbem_estimate_batch(ctx, jobs, nat.nat_mc_opts_default(), allow_noconv=True)
    torch.cuda.synchronize()
    yield wls, jobs, reps
    del jobs
    for m in meshes:
        m.close()


_ORACLE_CACHE = {}


def _oracle_systems(wl, i, modes):
    key = (i, tuple(modes))
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = O.mcbem(wl.vertices, wl.tris, wl.g[modes], wl.k[modes], wl.q_tri, wl.q_b,
                                     wl.n_samples, wl.seed, tol=1e-6, max_iter=200)
    return _ORACLE_CACHE[key]


def _check_systems(full_batch, picks, label, outs=None):
    """picks: {instance: [modes]}; each system against the FP64 oracle at the
    same GMRES settings (tol 1e-6, at most 200 iterations), per system both
    bars at 1e-3; every system's error is printed.  outs: per-instance
    outputs to check instead of the batch's own."""
    wls, jobs, reps = full_batch
    worst = 0.0
    for i in sorted(picks):
        wl = wls[i]
        modes = sorted(set(picks[i]))
        ref = _oracle_systems(wl, i, modes)
        got = (outs[i] if outs is not None else jobs[i].p_out)[modes].cpu().numpy()
        diam = float(np.linalg.norm(wl.vertices.max(axis=0) - wl.vertices.min(axis=0)))
        for a, (m, (e2, ei)) in enumerate(zip(modes, mode_errors(got, ref["p"]))):
            r = reps[i][m]
            _say(f"  {label} instance {i} (N={wl.n_samples}, Q={wl.n_queries}) mode {m} "
                 f"k*diam={wl.k[m] * diam:.1f}: rel L2 {e2:.2e}, element-wise {ei:.2e}, "
                 f"iters gpu {r['iters']}{'' if r['converged'] else ' (cap)'} "
                 f"oracle {ref['iters'][a]}")
            worst = max(worst, e2, ei)
            assert e2 <= 1e-3 and ei <= 1e-3, (i, m, e2, ei)
    _say(f"  {label}: worst {worst:.2e} over {sum(len(set(v)) for v in picks.values())} systems")
    return worst


def test_full_batched_workload_finite(full_batch):
    wls, jobs, reps = full_batch
    assert all(bool(torch.isfinite(torch.view_as_real(j.p_out)).all()) for j in jobs)
    capped = sum(1 for rr in reps for r in rr if not r["converged"])
    _say(f"  systems stopped at the iteration cap: {capped}")
    assert all(r["iters"] == 200 for rr in reps for r in rr if not r["converged"])


@pytest.mark.parametrize("half", [0, 1])
def test_full_batched_first_and_last_modes(full_batch, half):
    """The first and the last mode of every instance of the headline batch
    against the oracle (instances split in two halves to keep each test
    short)."""
    wls = full_batch[0]
    n = len(wls)
    picks = {i: [0, wls[i].n_modes - 1] for i in range(half * n // 2, (half + 1) * n // 2)}
    _check_systems(full_batch, picks, f"first/last half {half}:")


def test_full_batched_capped_systems(full_batch):
    """Every system of the headline batch that stops at the 200-iteration cap
    (the highest k times object size, near interior resonances of the
    conventional equation) against the oracle run with the same cap."""
    wls, jobs, reps = full_batch
    picks = {}
    for i, rr in enumerate(reps):
        for m, r in enumerate(rr):
            if not r["converged"]:
                picks.setdefault(i, []).append(m)
    assert picks
    _check_systems(full_batch, picks, "capped:")


def test_full_batched_capped_systems_fp64_phase(full_batch, ctx):
    """The headline batch again with NAT_MC_FP64_PHASE (phase from FP64
    positions, reduced in FP64): the systems that stop at the iteration cap
    against the same oracle references; both forms' errors are printed."""
    wls, jobs, reps = full_batch
    picks = {}
    for i, rr in enumerate(reps):
        for m, r in enumerate(rr):
            if not r["converged"]:
                picks.setdefault(i, []).append(m)
    opts = nat.nat_mc_opts_default()
    opts.flags = nat.NAT_MC_FP64_PHASE
    outs = [torch.empty_like(j.p_out) for j in jobs]
    jobs2 = [nat.McJob(j.mesh, j.v_n, j.k, j.q_tri, j.q_bary, j.n_samples, j.seed, p_out=o)
             for j, o in zip(jobs, outs)]
    nat.nat_mcbem_estimate_batch(ctx, jobs2, opts, allow_noconv=True)
    torch.cuda.synchronize()
    w32 = _check_systems(full_batch, picks, "capped, fp32 phase:")
    w64 = _check_systems(full_batch, picks, "capped, fp64 phase:", outs=outs)
    _say(f"  capped systems worst error: fp32 phase {w32:.2e}, fp64 phase {w64:.2e}")
