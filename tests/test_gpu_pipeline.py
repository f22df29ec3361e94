"""The NAT pipeline end to end on the GPU (Section 3.4): Monte-Carlo BEM
solves of speaker-torus scenes, the field at shell points from each solve's
sample values, and the neural field trained on the resulting (theta, phi, r,
v, f, |p|) tuples.  The training is checked by its own properties (the loss
falls more than three-fold, the held-out relative error of |p| stays below
one half); the pieces are checked against the oracle elsewhere."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2506_06190_amd import nat  # noqa: E402
from _parity import say  # noqa: E402

DEV = "cuda:0"


def test_neural_field_learns_the_generated_field():
    import bench
    ctx = nat.Context(0)
    wls = W.config_scenes(n_positions=3, n_modes=2, n_samples=1024, n_queries=64)
    opts = nat.nat_mc_opts_default()
    opts.layout = nat.NAT_NEUMANN_PER_TRIANGLE
    meshes, jobs, ps = [], [], []
    for wl in wls:
        m = nat.Mesh(ctx, wl.vertices, wl.tris)
        meshes.append(m)
        p_s = torch.empty((wl.n_modes, wl.n_samples), dtype=torch.complex128, device=DEV)
        ps.append(p_s)
        jobs.append(nat.McJob(m, torch.from_numpy(wl.g).to(DEV), wl.k, torch.from_numpy(wl.q_tri).to(DEV),
                              torch.from_numpy(wl.q_b).to(DEV), wl.n_samples, wl.seed, p_samples=p_s,
                              layout=nat.NAT_NEUMANN_PER_TRIANGLE))
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
    P = 4000
    coords, fabs = [], []
    for i, (wl, m) in enumerate(zip(wls, meshes)):
        pts, co = nat.nat_field_points(m, nat.NAT_FIELD_SHELL, P, 1, 1.5, 3.0, 100 + i)
        _, a = nat.nat_mcbem_field(m, jobs[i].v_n, wl.k, ps[i], wl.n_samples, wl.seed, pts, opts, want_abs=True)
        coords.append(co)
        fabs.append(a)
    torch.cuda.synchronize()
    X, Y = bench.scene_training_rows(torch, wls, coords, fabs)
    assert X.shape == (3 * 2 * P, 5) and torch.isfinite(X).all() and (Y >= 0).all()
    assert float(X[:, 2].min()) >= 1.5 - 1e-6 and float(X[:, 2].max()) <= 3.0 + 1e-6
    res = bench.train_on_scene_tuples(nat, torch, ctx, DEV, wls, coords, fabs, steps=600, batch=4096)
    say(f"  {res}")
    assert res["loss_last"] < 0.3 * res["loss_first"]
    assert res["held_out_rel_rms_error_abs_p"] < 0.5
    for m in meshes:
        m.close()
    ctx.close()
