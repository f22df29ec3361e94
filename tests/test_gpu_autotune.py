"""GPU tests of the tiling autotuner: the sweep fills every bucket with one
of the candidates and round-trips through its JSON cache, and the FP32
results stay within the oracle tolerance, and bit-for-bit batch invariant,
under tables far from the defaults."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_06190_amd import nat  # noqa: E402

DEV = "cuda:0"
CANDIDATES = {16, 32, 64, 128, 256, 512}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_sweep_and_cache(gpu, tmp_path):
    path = tmp_path / "tune.json"
    c1 = nat.Context(0)
    assert nat.nat_tune_get(c1) == {"items_a": [64] * 10, "items_b": [64] * 10, "tuned": False}
    t = nat.nat_autotune(c1, path, force=True)
    torch.cuda.synchronize()
    _say(f"tuned table: {t}")
    assert t["tuned"] and set(t["items_a"]) <= CANDIDATES and set(t["items_b"]) <= CANDIDATES
    form = nat.nat_tune_get_form(c1)
    _say(f"matvec form per bucket (1 = assembled): {form}")
    assert set(form) <= {0, 1}
    assert path.exists()
    c2 = nat.Context(0)
    assert nat.nat_autotune(c2, path) == t          # loaded, not swept
    assert nat.nat_tune_get_form(c2) == form
    c1.close()
    c2.close()


def _job(ctx, seed, n_tri, M, Q, N):
    v, f, u = W.cubesphere_ellipsoid(seed, n_tri)
    g = W.sh_neumann(u, M, seed)
    k = W.wavenumber(W.log_uniform_freqs(M, seed))
    qt, qb = W.random_face_queries(len(f), Q, seed)
    mesh = nat.Mesh(ctx, v, f)
    job = nat.McJob(mesh, torch.from_numpy(g).to(DEV), k, torch.from_numpy(qt).to(DEV),
                    torch.from_numpy(qb).to(DEV), N, seed)
    return (v, f, g, k, qt, qb, N, seed), mesh, job


def _estimate(mesh, job, flags):
    opts = nat.nat_mc_opts_default()
    opts.flags = flags
    p, rep = nat.nat_mcbem_estimate(mesh, job.v_n, job.k, job.q_tri, job.q_bary, job.n_samples,
                                    job.seed, opts)
    torch.cuda.synchronize()
    return p


def test_assembled_operator_form(gpu):
    """The GMRES matvec from the assembled operator: within the FP32 bar of
    the oracle and close to the matrix-free form; graph replay equals direct
    launches bit for bit."""
    ctx = nat.Context(0)
    args, mesh, job = _job(ctx, 21, 1500, 5, 600, 700)
    p_asm = _estimate(mesh, job, nat.NAT_MC_ASSEMBLED)
    p_asm2 = _estimate(mesh, job, nat.NAT_MC_ASSEMBLED | nat.NAT_MC_NO_GRAPH)
    p_free = _estimate(mesh, job, nat.NAT_MC_MATRIX_FREE)
    assert torch.equal(p_asm, p_asm2)
    ref = O.mcbem(*args[:8])["p"]
    a, b = p_asm.cpu().numpy(), p_free.cpu().numpy()
    e_or = max(np.linalg.norm(a[m] - ref[m]) / np.linalg.norm(ref[m]) for m in range(len(a)))
    e_mf = max(np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m]) for m in range(len(a)))
    _say(f"assembled: max rel L2 vs oracle {e_or:.2e}, vs matrix-free {e_mf:.2e}")
    assert e_or <= 1e-3 and e_mf <= 1e-4
    mesh.close()
    ctx.close()


def test_mixed_forms_in_one_batch(gpu):
    """A batch whose instances take different matvec forms by the table (one
    bucket assembled, the other matrix-free) equals each instance alone bit
    for bit and stays within the oracle bar."""
    ctx = nat.Context(0)
    a1, m1, j1 = _job(ctx, 31, 900, 3, 300, 200)     # N = 200: bucket 1
    a2, m2, j2 = _job(ctx, 32, 1500, 4, 500, 700)    # N = 700: bucket 3
    form = [0] * 10
    form[1] = 1
    nat.nat_tune_set_form(ctx, form)
    nat.nat_mcbem_estimate_batch(ctx, [j1, j2])
    torch.cuda.synchronize()
    for args, mesh, job in ((a1, m1, j1), (a2, m2, j2)):
        p1 = _estimate(mesh, job, 0)
        assert torch.equal(job.p_out, p1)
        ref = O.mcbem(*args[:8])["p"]
        got = p1.cpu().numpy()
        e = max(np.linalg.norm(got[m] - ref[m]) / np.linalg.norm(ref[m]) for m in range(len(got)))
        assert e <= 1e-3
    # the assembled instance differs from its matrix-free form only by rounding
    p_free = _estimate(m1, j1, nat.NAT_MC_MATRIX_FREE)
    assert not torch.equal(p_free, j1.p_out)
    m1.close()
    m2.close()
    ctx.close()


@pytest.mark.parametrize("items", [16, 512])
def test_results_under_other_tables(gpu, items):
    ctx = nat.Context(0)
    nat.nat_tune_set(ctx, [items] * 10, [items] * 10)
    v, f, u = W.cubesphere_ellipsoid(11, 1500)
    M, Q, N, seed = 5, 700, 600, 4242
    g = W.sh_neumann(u, M, seed)
    k = W.wavenumber(W.log_uniform_freqs(M, seed))
    qt, qb = W.random_face_queries(len(f), Q, seed)
    mesh = nat.Mesh(ctx, v, f)
    gd, qtd, qbd = (torch.from_numpy(x).to(DEV) for x in (g, qt, qb))
    p, _ = nat.nat_mcbem_estimate(mesh, gd, k, qtd, qbd, N, seed)
    # the same job inside a batch with another instance
    v2, f2, u2 = W.cubesphere_ellipsoid(12, 900)
    mesh2 = nat.Mesh(ctx, v2, f2)
    g2 = torch.from_numpy(W.sh_neumann(u2, 3, 7)).to(DEV)
    qt2, qb2 = W.random_face_queries(len(f2), 300, 7)
    jobs = [nat.McJob(mesh2, g2, W.wavenumber(W.log_uniform_freqs(3, 7)), torch.from_numpy(qt2).to(DEV),
                      torch.from_numpy(qb2).to(DEV), 250, 7),
            nat.McJob(mesh, gd, k, qtd, qbd, N, seed)]
    nat.nat_mcbem_estimate_batch(ctx, jobs)
    torch.cuda.synchronize()
    assert torch.equal(jobs[1].p_out, p)
    ref = O.mcbem(v, f, g, k, qt, qb, N, seed)
    got = p.cpu().numpy()
    errs = [float(np.linalg.norm(got[m] - ref["p"][m]) / np.linalg.norm(ref["p"][m])) for m in range(M)]
    _say(f"items {items}: max rel L2 vs oracle {max(errs):.2e}")
    assert max(errs) <= 1e-3
    mesh.close()
    mesh2.close()
    ctx.close()
