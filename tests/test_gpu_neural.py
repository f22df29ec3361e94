"""GPU parity of the neural acoustic transfer field (include/nat_neural.h)
against the numpy oracle (oracle/neural.py, Sections 3.2-3.4) with its
bfloat16 storage emulation, on the same float32 parameters and inputs.

Tolerances: the GPU forms every sum in FP32 where the oracle uses float64,
so a value that lies within that difference of a bfloat16 rounding midpoint
can round the other way (one bfloat16 ulp, 2^-8 relative, on a few values
per thousand rows); outputs then differ by about 1e-4 of their scale.  The
bars are 5e-3 of the largest value (max-norm) and 1e-3 relative L2 for
outputs and loss, 2e-2 and 5e-3 for gradient blocks.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import neural as NF
from tests._parity import rel_l2, rel_max, say
from workloads import nf_rows, nf_smooth_target

pytestmark = pytest.mark.gpu

R_LO, R_HI = 1.5, 3.0


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2506_06190_amd import nat
    ctx = nat.Context(0)
    yield nat, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def oracle_params(n_v, n_out, seed, grid_scale=0.5):
    """Oracle initialisation with a grid large enough to matter, rounded to
    float32 (the GPU's parameter precision)."""
    p = NF.init_params(n_v, n_out, seed)
    rng = np.random.default_rng([seed, 5])
    p["grid"] = [rng.uniform(-grid_scale, grid_scale, g.shape) for g in p["grid"]]
    p["b"] = [rng.uniform(-0.1, 0.1, b.shape) for b in p["b"]]
    return {k: [f32(a) for a in v] for k, v in p.items()}


def flatten(p):
    parts = []
    for W, b in zip(p["W"], p["b"]):
        parts += [W.ravel(), b.ravel()]
    parts += [g.ravel() for g in p["grid"]]
    return np.concatenate(parts)


def blocks(flat, like):
    """Split a flat array in the C layout into the oracle's named blocks."""
    out, o = [], 0
    for i, (W, b) in enumerate(zip(like["W"], like["b"])):
        out.append((f"W{i}", flat[o:o + W.size].reshape(W.shape)))
        o += W.size
        out.append((f"b{i}", flat[o:o + b.size]))
        o += b.size
    for l, g in enumerate(like["grid"]):
        out.append((f"grid{l}", flat[o:o + g.size].reshape(g.shape)))
        o += g.size
    assert o == flat.size
    return out


def make_rows(B, n_v, n_out, seed):
    th, ph, r, v, f = nf_rows(B, n_v, seed, R_LO, R_HI)
    th, ph, r, v, f = f32(th), f32(ph), f32(r), f32(v), f32(f)
    tgt = f32(nf_smooth_target(th, ph, r, v, f, n_out))
    rows = np.concatenate([th[:, None], ph[:, None], r[:, None], v, f[:, None]], axis=1)
    return (th, ph, r, v, f), tgt, rows


def field(env, n_v, n_out, params):
    nat, ctx, torch = env
    nf = nat.NeuralField(ctx, n_v, n_out, R_LO, R_HI, seed=1)
    assert nf.n_params == flatten(params).size
    nf.set_params(flatten(params))
    return nf


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n_v,n_out,B", [(0, 1, 1), (0, 1, 300), (2, 3, 1000), (1, 1, 4096), (9, 2, 700),
                                         (16, 1, 513)])
def test_infer_matches_oracle(env, n_v, n_out, B):
    nat, ctx, torch = env
    p = oracle_params(n_v, n_out, 10 + B)
    (th, ph, r, v, f), _, rows = make_rows(B, n_v, n_out, 20 + B)
    nf = field(env, n_v, n_out, p)
    got = nf.infer(dev(torch, rows)).cpu().numpy().astype(np.float64)
    x = NF.encode(th, ph, r, v, f, p["grid"], R_LO, R_HI)
    ref, _ = NF.forward(x, p, bf=True)
    say(f"  infer n_v={n_v} n_out={n_out} B={B}: rel_max {rel_max(got, ref):.2e} rel_l2 {rel_l2(got, ref):.2e}")
    assert rel_max(got, ref) <= 5e-3 and rel_l2(got, ref) <= 1e-3
    nf.close()


@pytest.mark.parametrize("n_v,n_out,B", [(0, 1, 300), (2, 3, 1000), (1, 1, 2048), (9, 2, 700), (16, 1, 513)])
def test_loss_and_gradients_match_oracle(env, n_v, n_out, B):
    # input widths 32, 64, 48, 144 and 224: every block count of the products
    nat, ctx, torch = env
    p = oracle_params(n_v, n_out, 30 + B)
    (th, ph, r, v, f), tgt, rows = make_rows(B, n_v, n_out, 40 + B)
    nf = field(env, n_v, n_out, p)
    loss = nf.loss_grad(dev(torch, rows), dev(torch, tgt))
    grads = nf.get_grads().astype(np.float64)
    ref_loss, g = NF.loss_and_grad(th, ph, r, v, f, tgt, p, R_LO, R_HI, bf=True)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss, (loss, ref_loss)
    ref = flatten(g)
    worst = []
    for (name, a), (_, b) in zip(blocks(grads, p), blocks(ref, p)):
        if not np.any(b):
            assert not np.any(a), name
            continue
        worst.append((name, rel_max(a, b), rel_l2(a, b)))
    say("  " + ", ".join(f"{n} {m:.1e}/{l:.1e}" for n, m, l in worst))
    for name, m, l in worst:
        assert m <= 2e-2 and l <= 5e-3, (name, m, l)
    nf.close()


def test_gradient_is_reproducible(env):
    """Every sum of the gradient runs in a fixed order or in integers: two
    evaluations at the same parameters agree bit for bit."""
    nat, ctx, torch = env
    n_v, n_out, B = 1, 2, 5000
    p = oracle_params(n_v, n_out, 21)
    _, tgt, rows = make_rows(B, n_v, n_out, 22)
    nf = field(env, n_v, n_out, p)
    x, t = dev(torch, rows), dev(torch, tgt)
    l1 = nf.loss_grad(x, t)
    g1 = nf.get_grads()
    l2 = nf.loss_grad(x, t)
    g2 = nf.get_grads()
    assert l1 == l2 and np.array_equal(g1, g2)
    nf.close()


def test_train_step_matches_oracle(env):
    """One Adam step from the same parameters: where the gradient is clearly
    nonzero the move is lr g / (|g| + eps) on both sides and must agree to
    1e-3 of lr; elsewhere it is at most 2 lr apart (a sign decided by
    rounding)."""
    nat, ctx, torch = env
    n_v, n_out, B = 1, 1, 1024
    p = oracle_params(n_v, n_out, 7)
    (th, ph, r, v, f), tgt, rows = make_rows(B, n_v, n_out, 8)
    nf = field(env, n_v, n_out, p)
    p0 = flatten(p)
    loss = nf.train_step(dev(torch, rows), dev(torch, tgt), 0, 30)
    moved = nf.get_params().astype(np.float64) - p0
    ref_loss, g = NF.loss_and_grad(th, ph, r, v, f, tgt, p, R_LO, R_HI, bf=True)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    q = {k: [a.copy() for a in vv] for k, vv in p.items()}
    NF.adam_step(q, g, {}, 0, 30)
    ref_moved = flatten(q) - p0
    gf = np.abs(flatten(g))
    firm = gf > 1e-5
    lr = 1e-3
    d = np.abs(moved - ref_moved)
    say(f"  firm {firm.sum()} of {firm.size}: worst {d[firm].max() / lr:.2e} lr; others {d[~firm].max() / lr:.2e} lr")
    assert d[firm].max() <= 1e-3 * lr
    assert d.max() <= 2.0 * lr * (1 + 1e-3)
    nf.close()


def test_training_tracks_oracle(env):
    """Twenty steps on one batch: the GPU's loss follows the oracle's."""
    nat, ctx, torch = env
    n_v, n_out, B, steps = 1, 1, 1024, 20
    p = oracle_params(n_v, n_out, 9, grid_scale=1e-2)
    (th, ph, r, v, f), tgt, rows = make_rows(B, n_v, n_out, 10)
    nf = field(env, n_v, n_out, p)
    x, t = dev(torch, rows), dev(torch, tgt)
    q = {k: [a.copy() for a in vv] for k, vv in p.items()}
    st = {}
    gl, ol = [], []
    for s in range(steps):
        gl.append(nf.train_step(x, t, s, steps))
        lo, g = NF.loss_and_grad(th, ph, r, v, f, tgt, q, R_LO, R_HI, bf=True)
        ol.append(lo)
        NF.adam_step(q, g, st, s, steps)
    rel = np.abs(np.array(gl) - np.array(ol)) / np.array(ol)
    say(f"  losses gpu {gl[0]:.4e} -> {gl[-1]:.4e}, oracle {ol[0]:.4e} -> {ol[-1]:.4e}, worst rel {rel.max():.2e}")
    assert rel.max() <= 2e-2
    assert gl[-1] < gl[0]
    nf.close()


def test_training_fits_a_smooth_field(env):
    """300 steps over a 16384-row set of a smooth field bring the loss below a
    tenth of its start (the oracle's own fit shows the same)."""
    nat, ctx, torch = env
    n_v, n_out, B, steps = 1, 1, 16384, 300
    _, tgt, rows = make_rows(B, n_v, n_out, 12)
    nf = nat.NeuralField(ctx, n_v, n_out, R_LO, R_HI, seed=3)
    x, t = dev(torch, rows), dev(torch, tgt)
    first = nf.train_step(x, t, 0, steps)
    for s in range(1, steps - 1):
        nf.train_step(x, t, s, steps, want_loss=False)
    last = nf.train_step(x, t, steps - 1, steps)
    say(f"  loss {first:.4e} -> {last:.4e}")
    assert last < 0.1 * first
    nf.close()


def test_full_batch_sampled_rows(env):
    """The bench's batch of 262144 rows: the loss over all rows and 512
    sampled outputs against the oracle (whose forward pass runs on the full
    batch in a few seconds)."""
    nat, ctx, torch = env
    n_v, n_out, B = 1, 1, 1 << 18
    p = oracle_params(n_v, n_out, 13)
    (th, ph, r, v, f), tgt, rows = make_rows(B, n_v, n_out, 14)
    nf = field(env, n_v, n_out, p)
    x, t = dev(torch, rows), dev(torch, tgt)
    got = nf.infer(x).cpu().numpy().astype(np.float64)
    loss = nf.loss_grad(x, t)
    idx = np.random.default_rng(15).choice(B, 512, replace=False)
    xo = NF.encode(th[idx], ph[idx], r[idx], v[idx], f[idx], p["grid"], R_LO, R_HI)
    ref, _ = NF.forward(xo, p, bf=True)
    assert rel_max(got[idx], ref) <= 5e-3 and rel_l2(got[idx], ref) <= 1e-3
    xa = NF.encode(th, ph, r, v, f, p["grid"], R_LO, R_HI)
    ya, _ = NF.forward(xa, p, bf=True)
    ref_loss = float(np.mean((ya - tgt) ** 2))
    say(f"  sampled rel_max {rel_max(got[idx], ref):.2e}; loss {loss:.6e} vs {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    nf.close()


def test_save_and_load_round_trip(env, tmp_path):
    """A trained field written with save() and read back with load() gives
    the same inference bit for bit, on a field with two condition variables
    and three outputs over a shell other than the default."""
    nat, ctx, torch = env
    _, tgt, rows = make_rows(2048, 2, 3, 21)
    nf = nat.NeuralField(ctx, 2, 3, 1.2, 2.5, seed=4)
    x, t = dev(torch, rows), dev(torch, tgt)
    for s_ in range(5):
        nf.train_step(x, t, s_, 5, want_loss=False)
    path = tmp_path / "field.npz"
    nf.save(path)
    nf2 = nat.NeuralField.load(ctx, path)
    assert (nf2.n_v, nf2.n_out, nf2.r_lo, nf2.r_hi) == (2, 3, 1.2, 2.5)
    assert np.array_equal(nf2.get_params(), nf.get_params())
    assert torch.equal(nf2.infer(x), nf.infer(x))
    nf.close()
    nf2.close()


def test_inference_allocates_nothing(env):
    """Inference runs entirely in on-chip memory: the context's charged
    bytes do not move, however large the batch."""
    nat, ctx, torch = env
    nf = nat.NeuralField(ctx, 1, 1, R_LO, R_HI, seed=2)
    _, _, rows = make_rows(100000, 1, 1, 3)
    x = dev(torch, rows)
    out = torch.empty((100000, 1), dtype=torch.float32, device="cuda")
    before = ctx.bytes_in_use()
    nf.infer(x, out=out)
    torch.cuda.synchronize()
    assert ctx.bytes_in_use() == before and torch.isfinite(out).all()
    nf.close()


def test_neural_field_errors(env):
    nat, ctx, torch = env
    with pytest.raises(nat.NatError):
        nat.NeuralField(ctx, -1, 1, R_LO, R_HI)
    with pytest.raises(nat.NatError):
        nat.NeuralField(ctx, 0, 0, R_LO, R_HI)
    with pytest.raises(nat.NatError):
        nat.NeuralField(ctx, 0, 1, 3.0, 1.5)
    nf = nat.NeuralField(ctx, 0, 1, R_LO, R_HI)
    with pytest.raises(nat.NatError):
        nf.set_params(np.zeros(nf.n_params + 1, np.float32))
    x = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(nat.NatError):
        nf.infer(x)
    nf.close()
