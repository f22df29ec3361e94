"""GPU tests of the served form through the C ABI: every result served from
a mixed stream equals the same request run alone (bit for bit: the batch
tiling of a request depends only on its own sizes, and a dense request runs
the same assembly and solve), the arena budget bounds the device memory,
a request larger than the arena is refused at submission, and a request
whose data fails the device checks fails alone inside its batch; every
served result of a mixed stream matches the FP64 oracle (Monte-Carlo
requests within 1e-3, dense requests within 1e-9, per mode and element by
element)."""
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


@pytest.fixture(scope="module")
def stream_setup(ctx):
    meshes, reqs = W.config_served(seed=99, n_meshes=5, n_requests=40, t_range=(300, 2500),
                                   q_range=(1, 600), n_range=(70, 500), pool_modes=6,
                                   dense_fraction=0.15, dense_max_tris=900, dense_modes=3)
    res = []
    for m in meshes:
        res.append({"mesh": nat.Mesh(ctx, m.vertices, m.tris),
                    "gv": torch.from_numpy(m.g_vertex).to(DEV),
                    "gt": torch.from_numpy(m.g_tri).to(DEV),
                    "qt": torch.from_numpy(m.q_tri).to(DEV),
                    "qb": torch.from_numpy(m.q_b).to(DEV)})
    torch.cuda.synchronize()
    yield meshes, reqs, res
    for r in res:
        r["mesh"].close()


def _request(rq, R):
    M = rq.n_modes
    if rq.kind == "mc":
        return nat.Request(nat.NAT_REQ_MCBEM, R["mesh"], R["gv"][rq.m0:rq.m0 + M], rq.k,
                           R["qt"][:rq.n_queries], R["qb"][:rq.n_queries], rq.n_samples, rq.seed)
    return nat.Request(nat.NAT_REQ_DENSE, R["mesh"], R["gt"][rq.m0:rq.m0 + M], rq.k,
                       layout=nat.NAT_NEUMANN_PER_TRIANGLE)


def _solo(rq, R, sopts):
    M = rq.n_modes
    if rq.kind == "mc":
        o = nat.nat_mc_opts_default()
        p, rep = nat.nat_mcbem_estimate(R["mesh"], R["gv"][rq.m0:rq.m0 + M], rq.k,
                                        R["qt"][:rq.n_queries], R["qb"][:rq.n_queries],
                                        rq.n_samples, rq.seed, o, allow_noconv=True)
        return p, rep
    outs, reps = [], []
    for m in range(M):
        op = nat.nat_bem_assemble(R["mesh"], rq.k[m], True)
        p, rep = nat.nat_bem_solve(op, R["gt"][rq.m0 + m:rq.m0 + m + 1],
                                   layout=nat.NAT_NEUMANN_PER_TRIANGLE, tol=sopts.dense_tol,
                                   max_iter=sopts.dense_max_iter, allow_noconv=True)
        torch.cuda.synchronize()
        op.close()
        outs.append(p)
        reps += rep
    return torch.cat(outs), reps


def test_served_stream_accounting(ctx, stream_setup):
    meshes, reqs, res = stream_setup
    sopts = nat.nat_server_opts_default()
    sopts.n_slots = 3
    sopts.max_batch = 8
    sopts.hbm_budget = 2 << 30
    srv = nat.Server(ctx, sopts)
    _say(f"served stream: {len(reqs)} requests, "
         f"{sum(r.kind == 'dense' for r in reqs)} dense, meshes T = {[len(m.tris) for m in meshes]}")
    torch.cuda.synchronize()
    tickets = [nat.nat_server_submit(srv, _request(rq, res[rq.mesh])) for rq in reqs]
    for t, rq in zip(tickets, reqs):
        st, r, reps = nat.nat_server_wait(srv, t)
        assert st in (nat.NAT_OK, nat.NAT_E_NOCONV), (rq, nat.status_str(st))
        assert r["latency_ms"] >= r["run_ms"] > 0.0 and r["queue_ms"] >= 0.0
        assert abs(r["latency_ms"] - r["queue_ms"] - r["run_ms"]) < 1e-6
        assert r["max_iters"] == max(x["iters"] for x in reps)
        if rq.kind == "dense":
            assert r["batch_size"] == 1
    stats = nat.nat_server_stats_read(srv)
    _say(f"  stats {stats}")
    assert stats["completed"] == len(reqs) and stats["peak_bytes"] <= sopts.hbm_budget
    assert stats["max_batch_seen"] > 1
    srv.close()


def test_served_equal_solo_bitwise(ctx, stream_setup):
    meshes, reqs, res = stream_setup
    sopts = nat.nat_server_opts_default()
    sopts.n_slots = 3
    sopts.max_batch = 8
    sopts.hbm_budget = 2 << 30
    srv = nat.Server(ctx, sopts)
    torch.cuda.synchronize()
    built = [_request(rq, res[rq.mesh]) for rq in reqs]
    tickets = [nat.nat_server_submit(srv, b) for b in built]
    results = [nat.nat_server_wait(srv, t) for t in tickets]
    srv.close()
    n_batched = 0
    for rq, b, (st, r, reps) in zip(reqs, built, results):
        assert st in (nat.NAT_OK, nat.NAT_E_NOCONV)
        n_batched += r["batch_size"] > 1
        p_solo, rep_solo = _solo(rq, res[rq.mesh], sopts)
        torch.cuda.synchronize()
        assert torch.equal(b.p_out, p_solo), (rq.kind, rq.mesh, rq.n_modes)
        assert [x["iters"] for x in reps] == [x["iters"] for x in rep_solo]
    _say(f"  {n_batched} of {len(reqs)} requests ran in shared batches; all equal their solo runs")
    assert n_batched > 0


def test_served_results_match_oracle(ctx, stream_setup):
    """Every request of the mixed stream, served with continuous batching over
    three worker streams, against the FP64 oracle on the same inputs:
    Monte-Carlo requests at the same seed, GMRES tolerance 1e-6 and cap 200
    (bar 1e-3); dense requests solved to 1e-12 against the oracle's
    collocation assembly and solve (bar 1e-9)."""
    meshes, reqs, res = stream_setup
    sopts = nat.nat_server_opts_default()
    sopts.n_slots = 3
    sopts.max_batch = 8
    sopts.hbm_budget = 2 << 30
    sopts.dense_tol = 1e-12
    srv = nat.Server(ctx, sopts)
    torch.cuda.synchronize()
    built = [_request(rq, res[rq.mesh]) for rq in reqs]
    tickets = [nat.nat_server_submit(srv, b) for b in built]
    results = [nat.nat_server_wait(srv, t) for t in tickets]
    srv.close()
    n_mc = n_dense = 0
    for j, (rq, b, (st, r, reps)) in enumerate(zip(reqs, built, results)):
        assert st in (nat.NAT_OK, nat.NAT_E_NOCONV)
        m = meshes[rq.mesh]
        got = b.p_out.cpu().numpy()
        M = rq.n_modes
        if rq.kind == "mc":
            ref = O.mcbem(m.vertices, m.tris, m.g_vertex[rq.m0:rq.m0 + M], rq.k,
                          m.q_tri[:rq.n_queries], m.q_b[:rq.n_queries], rq.n_samples, rq.seed,
                          tol=1e-6, max_iter=200)["p"]
            check_modes(got, ref, 1e-3, f"request {j} mc M={M} Q={rq.n_queries} "
                        f"N={rq.n_samples} (batch {r['batch_size']})")
            n_mc += 1
        else:
            ref = []
            for a in range(M):
                A, B = O.bem_assemble(m.vertices, m.tris, rq.k[a], True)
                ref.append(O.bem_solve(A, B, m.g_tri[rq.m0 + a], tol=1e-12)[0])
            check_modes(got, ref, 1e-9, f"request {j} dense M={M} n={len(m.tris)}")
            n_dense += 1
    _say(f"  {n_mc} Monte-Carlo and {n_dense} dense served results match the oracle")
    assert n_mc > 0 and n_dense > 0


def test_budget_bounds_admission(ctx, stream_setup):
    meshes, reqs, res = stream_setup
    mc = [rq for rq in reqs if rq.kind == "mc"][:12]
    sopts = nat.nat_server_opts_default()
    sopts.n_slots = 4
    sopts.max_batch = 64
    # an arena that holds only a few of the requests at once
    sopts.hbm_budget = 40 << 20
    before = ctx.bytes_in_use()
    srv = nat.Server(ctx, sopts)
    assert ctx.bytes_in_use() - before == sopts.hbm_budget
    built = [_request(rq, res[rq.mesh]) for rq in mc]
    torch.cuda.synchronize()
    tickets = [nat.nat_server_submit(srv, b) for b in built]
    for t in tickets:
        st, r, _ = nat.nat_server_wait(srv, t)
        assert st in (nat.NAT_OK, nat.NAT_E_NOCONV)
    stats = nat.nat_server_stats_read(srv)
    _say(f"  small arena: {stats}")
    assert stats["peak_bytes"] <= sopts.hbm_budget
    assert ctx.bytes_in_use() - before == sopts.hbm_budget   # nothing allocated per request
    # a request that cannot fit the arena is refused at submission
    big = nat.Request(nat.NAT_REQ_DENSE, res[0]["mesh"], res[0]["gt"][:1], [5.0],
                      layout=nat.NAT_NEUMANN_PER_TRIANGLE)
    tiny = nat.nat_server_opts_default()
    tiny.hbm_budget = 1 << 20
    srv2 = nat.Server(ctx, tiny)
    with pytest.raises(nat.NatError) as e:
        nat.nat_server_submit(srv2, big)
    assert e.value.status == nat.NAT_E_BUDGET
    srv2.close()
    srv.close()
    assert ctx.bytes_in_use() == before


def test_bad_request_fails_alone_in_its_batch(ctx, stream_setup):
    meshes, reqs, res = stream_setup
    mc = [rq for rq in reqs if rq.kind == "mc"][:6]
    sopts = nat.nat_server_opts_default()
    sopts.n_slots = 1
    sopts.max_batch = 8
    sopts.hbm_budget = 1 << 30
    srv = nat.Server(ctx, sopts)
    built = [_request(rq, res[rq.mesh]) for rq in mc]
    # request 3 carries a non-finite Neumann value (checked on the device)
    bad_v = built[3].v_n.clone()
    bad_v[0, 0] = complex(float("nan"), 0.0)
    built[3].v_n = bad_v
    torch.cuda.synchronize()
    tickets = [nat.nat_server_submit(srv, b) for b in built]
    out = [nat.nat_server_wait(srv, t) for t in tickets]
    srv.close()
    assert out[3][0] == nat.NAT_E_INVALID
    for i, (rq, b, (st, r, reps)) in enumerate(zip(mc, built, out)):
        if i == 3:
            continue
        assert st in (nat.NAT_OK, nat.NAT_E_NOCONV)
        p_solo, _ = _solo(rq, res[rq.mesh], sopts)
        torch.cuda.synchronize()
        assert torch.equal(b.p_out, p_solo)
