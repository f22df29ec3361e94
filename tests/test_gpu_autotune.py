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
    assert path.exists()
    c2 = nat.Context(0)
    assert nat.nat_autotune(c2, path) == t          # loaded, not swept
    c1.close()
    c2.close()


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
