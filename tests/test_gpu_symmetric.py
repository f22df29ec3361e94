"""GPU tests of the symmetric form of the FP32 GMRES matvec (each unordered
sample pair evaluated once for both of its targets) against the ordered
form and the FP64 oracle: within the FP32 bar of the oracle, within 1e-4 of
the ordered form, the same bits with and without graph replay, and the same
bits alone and inside a batch, for groups of 1 to 8 modes and sample
counts that fill a 64-sample sub-tile exactly, leave a ragged one, or stay
below one."""
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
    return p, rep


def test_symmetric_against_ordered_and_oracle(ctx):
    # N = 600: nine full sub-tiles and a ragged one; 11 modes: groups of 8 and 3
    args, mesh, job = _job(ctx, 41, 1500, 11, 600, 600)
    _say("symmetric vs ordered: M=11 Q=600 N=600")
    p_sym, rep = _estimate(mesh, job, nat.NAT_MC_MATRIX_FREE)
    p_sym2, _ = _estimate(mesh, job, nat.NAT_MC_MATRIX_FREE | nat.NAT_MC_NO_GRAPH)
    p_ord, _ = _estimate(mesh, job, nat.NAT_MC_MATRIX_FREE | nat.NAT_MC_ORDERED_SUM)
    assert torch.equal(p_sym, p_sym2)
    assert not torch.equal(p_sym, p_ord)
    ref = O.mcbem(*args[:8])["p"]
    a, b = p_sym.cpu().numpy(), p_ord.cpu().numpy()
    check_modes(a, ref, 1e-3, "symmetric vs oracle")
    check_modes(b, ref, 1e-3, "ordered vs oracle")
    check_modes(a, b, 1e-4, "symmetric vs ordered")
    assert all(r["converged"] for r in rep)
    mesh.close()


@pytest.mark.parametrize("case", ["small_groups", "tiny", "widths_4_to_7"])
def test_symmetric_batch_equals_alone(ctx, case):
    if case == "small_groups":
        # groups of 1, 2 and 3 modes; N = 64, 65, 130
        specs = [(51, 600, 1, 200, 64), (52, 700, 2, 250, 65), (53, 900, 3, 300, 130)]
    elif case == "tiny":
        # fewer samples than one sub-tile, and exactly two
        specs = [(54, 500, 2, 100, 2), (55, 500, 9, 150, 40), (56, 600, 1, 120, 128)]
    else:
        # groups of 4, 5, 6 and 7 modes; N = 191, 256, 300
        specs = [(57, 600, 4, 120, 191), (58, 700, 5, 150, 256), (59, 800, 6, 100, 300),
                 (60, 600, 7, 90, 191)]
    made = [_job(ctx, *s) for s in specs]
    _say(f"symmetric batch {case}: " + ", ".join(f"M={s[2]} N={s[4]}" for s in specs))
    nat.nat_mcbem_estimate_batch(ctx, [j for _, _, j in made])
    torch.cuda.synchronize()
    for args, mesh, job in made:
        p1, _ = _estimate(mesh, job, 0)
        assert torch.equal(job.p_out, p1)
        ref = O.mcbem(*args[:8])["p"]
        check_modes(p1.cpu().numpy(), ref, 1e-3, f"M={args[3].shape[0]} N={args[6]} vs oracle")
    for _, mesh, _ in made:
        mesh.close()
