"""Benchmark of the Monte-Carlo BEM hot path on one MI355X.

Headline (default): the batched form.  One step = one Monte-Carlo estimate of
256 cube-sphere instances at once (2k-40k triangles, 8-64 modes with their
own wavenumbers, 2k-16k queries, 512-2048 samples): sampling, right-hand
side, GMRES (tol 1e-6, <= 200 iterations) and surface evaluation for all
~9.4k (instance, mode) systems, FP32 form, inputs resident in HBM.
`value` = algorithmic pair evaluations per second, sum over systems of
N(N-1) + Q N per step.

Also reported on the same JSON line:
  roofline      the dominant kernel class, from HIP events attached to its
                dispatches during a second pass over the same steps;
  precision     the 20480-triangle, 32-mode precision-form workload in the FP32
                form and in the plain FP64 form ("FP32 vs plain");
  cpu_baseline  the FP64 oracle on a bounded sample of the headline workload,
                timed on the host cores, with the GPU's error on that sample;
  served        the request server on a Poisson stream of Monte-Carlo and
                dense solves over 64 resident meshes: p50/p99 latency and
                solves/s, against the plain per-solve form (the same requests
                one at a time, no batching, no graphs) on the same arrivals,
                whose results are bitwise those of the served run.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
METRIC = "MC-BEM kernel pair-evals/s (FP32 vs plain) + p50/p99 solve latency at fixed error"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_jobs(nat, torch, ctx, wls, dev):
    meshes, jobs = [], []
    for wl in wls:
        mesh = nat.Mesh(ctx, wl.vertices, wl.tris)
        meshes.append(mesh)
        jobs.append(nat.McJob(mesh, torch.from_numpy(wl.g).to(dev), wl.k,
                              torch.from_numpy(wl.q_tri).to(dev), torch.from_numpy(wl.q_b).to(dev),
                              wl.n_samples, wl.seed))
    return meshes, jobs


def roofline_from(prof, peak=FP32_VECTOR_PEAK_TFLOPS):
    sums = {k: v for k, v in prof.items() if k.startswith(("sum32", "sym32"))}
    dom_name = max(sums, key=lambda k: sums[k]["total_ms"])
    dom = sums[dom_name]
    achieved = dom["flops"] / (dom["total_ms"] * 1e-3) / 1e12
    kern = "k_sym32" if dom_name.startswith("sym32") else "k_sum32"
    return {"bound": "alu", "kernel": f"{kern} ({dom_name})", "achieved": round(achieved, 3),
            "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "avg_launch_ms": round(dom["avg_ms"], 5), "launches": dom["launches"],
            "flops_per_launch": dom["flops"] / dom["launches"]}


def method_matvec_credit(prof, roof, wls, reps, steps, peak=FP32_VECTOR_PEAK_TFLOPS):
    """Roofline of the GMRES matvec credited with the method's own work only:
    per step, the sum over systems of (GMRES iterations) x N(N-1) ordered
    sample pairs x 37 flops (the survey's counting convention; the symmetric
    form evaluates each unordered pair once, so this is an ordered-pair
    equivalent).  The library's own per-launch credit (every system on the
    host's running list, N^2 pairs, including systems that converged since the
    list was refreshed and the converged members of a live mode group) is
    kept beside it as the executed figure."""
    import numpy as np
    dom = prof[roof["kernel"].split("(")[1].rstrip(")")]
    secs = dom["total_ms"] * 1e-3
    it = np.array([r["iters"] for rr in reps for r in rr], dtype=np.float64)
    n = np.array([w.n_samples for w in wls for _ in range(w.n_modes)], dtype=np.float64)
    per_step = 37.0 * float(np.sum(it * n * (n - 1.0)))
    achieved = per_step * steps / secs / 1e12
    t64 = 64.0 * np.ceil(n / 64.0)
    return {"achieved": round(achieved, 3), "frac": round(achieved / peak, 4),
            "flops_per_launch": per_step * steps / dom["launches"],
            "credit": "method's own matvec work: sum over systems of GMRES iterations x N(N-1) x "
                      "37 flops per step, ordered-pair equivalent",
            "method_matvec_flops_per_step": per_step,
            "executed_incl_converged_riders_tflops": round(dom["flops"] / secs / 1e12, 3),
            "padded_lane_share": round(float(1.0 - np.sum(it * n * n) / np.sum(it * t64 * t64)), 4)}


def auto_parts(wls):
    """The part count nat_mcbem_estimate_batch picks for n_streams = 0: one part
    per 2e10 pair terms (M N (31 N + Q) per job), at most 3, at most one per job."""
    work = sum(w.n_modes * w.n_samples * (31.0 * w.n_samples + w.n_queries) for w in wls)
    return int(min(3, len(wls), max(1, work // 2e10)))


def run_batched(nat, torch, ctx, args, dev):
    import numpy as np
    import workloads as W
    t0 = time.perf_counter()
    wls = W.config_batched()
    log(f"batched workload generated in {time.perf_counter() - t0:.1f} s")
    meshes, jobs = make_jobs(nat, torch, ctx, wls, dev)
    alg = sum(w.pair_evals() for w in wls)
    opts = nat.nat_mc_opts_default()
    for _ in range(args.warmup):
        nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
    torch.cuda.synchronize()
    log("batched warm-up done")
    t0 = time.perf_counter()
    reps = None
    for _ in range(args.steps):
        reps = nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"batched timed region: {elapsed:.3f} s for {args.steps} steps")
    iters = np.array([r["iters"] for rr in reps for r in rr])
    n_s = np.array([w.n_samples for w in wls for _ in range(w.n_modes)], dtype=np.float64)
    executed = float(np.sum(n_s * n_s) + sum(w.n_modes * w.n_queries * w.n_samples for w in wls)
                     + np.sum(iters * n_s * n_s))
    # roofline pass: the same steps with events on the kernel dispatches, on
    # one stream (so no other part's kernels share the GPU with the one timed)
    opts1 = nat.nat_mc_opts_default()
    opts1.n_streams = 1
    nat.nat_profile_enable(ctx, True)
    for _ in range(args.steps):
        nat.nat_mcbem_estimate_batch(ctx, jobs, opts1, allow_noconv=True)
    torch.cuda.synchronize()
    prof = nat.nat_profile_read(ctx)
    nat.nat_profile_enable(ctx, False)
    roof = roofline_from(prof)
    roof["timing_pass"] = ("second pass over the same steps, one stream (n_streams = 1), eager "
                           "dispatch, events on each dispatch")
    kern = roof["kernel"].split()[0]
    if kern in MATVEC:
        roof.update(method_matvec_credit(prof, roof, wls, reps, args.steps))
    roof["traffic"] = traffic_from_profile(kern) if kern in MATVEC else None
    valu = valu_from_profile(kern) if kern in MATVEC else None
    roof["executed_fp32_tflops_counters"] = valu[0] if valu else None
    roof["valu_active_per_simd_cycle_counters"] = valu[1] if valu else None
    roof["traffic_unit"] = "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-kernel scaled)"
    out = {
        "value": alg * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
        "config": {"workload": "batched: 256 cube-sphere instances, 2k-40k tri, 8-64 modes, "
                               "Q 2k-16k, N 512-2048, 200 Hz-8 kHz",
                   "instances": len(wls), "systems": int(len(iters)),
                   "triangles_total": int(sum(len(w.tris) for w in wls)),
                   "algorithmic_pair_evals_per_step": alg, "form": "FP32 compensated, graph-replayed GMRES",
                   "n_streams": f"automatic: {auto_parts(wls)} concurrent parts on streams of "
                                f"their own (timed step); the roofline pass runs on one stream",
                   "gmres_tol": 1e-6, "gmres_max_iter": 200},
        "executed_pair_evals_per_s": executed * args.steps / elapsed,
        "gmres_iters": {"mean": float(iters.mean()), "p50": float(np.median(iters)),
                        "max": int(iters.max()), "not_converged": int(sum(not r["converged"]
                                                                         for rr in reps for r in rr))},
        "roofline": roof,
        "kernels": {k: {"launches": v["launches"], "avg_ms": round(v["avg_ms"], 5),
                        "total_ms": round(v["total_ms"], 3)} for k, v in prof.items()},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        # the oracle on the first 4 modes of each instance in order, until about
        # args.cpu_seconds of host time is spent (whole instances)
        n_modes = 4
        sample_pairs = 0
        t_cpu = 0.0
        per_mode = []
        n_inst = 0
        for i, wl in enumerate(wls):
            if t_cpu >= args.cpu_seconds:
                break
            m = min(n_modes, wl.n_modes)
            t0 = time.perf_counter()
            r = O.mcbem(wl.vertices, wl.tris, wl.g[:m], wl.k[:m], wl.q_tri, wl.q_b, wl.n_samples,
                        wl.seed, tol=1e-6)
            t_cpu += time.perf_counter() - t0
            n_inst += 1
            sample_pairs += m * (wl.n_samples * (wl.n_samples - 1) + wl.n_queries * wl.n_samples)
            got = jobs[i].p_out[:m].cpu().numpy()
            for q in range(m):
                per_mode.append((i, q, rel_l2(got[q], r["p"][q]), rel_max(got[q], r["p"][q])))
        cores = O.num_threads()
        # one thread, on the first instance of the sample
        wl = wls[0]
        m = min(n_modes, wl.n_modes)
        O.set_threads(1)
        t0 = time.perf_counter()
        O.mcbem(wl.vertices, wl.tris, wl.g[:m], wl.k[:m], wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                tol=1e-6)
        t_one = time.perf_counter() - t0
        O.set_threads(cores)
        pairs_one = m * (wl.n_samples * (wl.n_samples - 1) + wl.n_queries * wl.n_samples)
        out["cpu_baseline"] = {"value": sample_pairs / t_cpu, "unit": "pair-evals/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"first {n_inst} instances x first {n_modes} modes of the "
                                         "headline workload, FP64, tol 1e-6",
                               "seconds": round(t_cpu, 3), "cpu_model": cpu_model(),
                               "single_thread_value": pairs_one / t_one,
                               "single_thread_sample": f"first instance x first {m} modes"}
        out["vs_oracle"] = {
            "sample": f"first {n_modes} modes of the first {n_inst} instances ({len(per_mode)} systems)",
            "max_rel_l2": max(e[2] for e in per_mode),
            "max_elementwise": max(e[3] for e in per_mode),
            "bar": 1e-3,
            "per_mode": [[e[0], e[1], float(f"{e[2]:.3g}"), float(f"{e[3]:.3g}")] for e in per_mode],
            "per_mode_fields": ["instance", "mode", "rel_l2", "max_abs_err / max_abs_ref"]}
    for mesh in meshes:
        mesh.close()
    return out


def rel_l2(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / max(float(np.linalg.norm(b)), 1e-300))


def rel_max(a, b):
    import numpy as np
    if b.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(float(np.abs(b).max()), 1e-300))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _percentiles(x):
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    return {"p50_ms": round(float(np.percentile(x, 50)), 3), "p99_ms": round(float(np.percentile(x, 99)), 3),
            "mean_ms": round(float(x.mean()), 3), "max_ms": round(float(x.max()), 3)}


def run_served(nat, torch, ctx, args, dev):
    """The request server on a Poisson stream over 64 resident meshes, in
    three runs: (1) capacity, the whole stream submitted at once; (2) the
    stream at 70 % of the served capacity (latency at the served form's own
    operating point); (3) equal load: the first requests of the stream at
    70 % of the plain per-solve form's capacity, run by both forms, so both
    latencies are measured at one offered load below both capacities.  The
    plain per-solve form runs the same requests one at a time on one stream
    (FP32 compensated like the served form, direct launches, no batching, no
    graph); its service times give its capacity.  Results of the served run
    are compared with the plain ones bit for bit, and a sample of requests
    with the FP64 oracle."""
    import numpy as np
    import workloads as W
    t0 = time.perf_counter()
    meshes, reqs = W.config_served(n_requests=args.serve_requests)
    log(f"served workload generated in {time.perf_counter() - t0:.1f} s")
    R = []
    for m in meshes:
        R.append({"mesh": nat.Mesh(ctx, m.vertices, m.tris),
                  "gv": torch.from_numpy(m.g_vertex).to(dev), "gt": torch.from_numpy(m.g_tri).to(dev),
                  "qt": torch.from_numpy(m.q_tri).to(dev), "qb": torch.from_numpy(m.q_b).to(dev)})
    sopts = nat.nat_server_opts_default()
    sopts.n_slots = args.serve_slots
    sopts.max_batch = args.serve_max_batch
    sopts.hbm_budget = args.serve_budget_gib << 30

    def build(rq):
        r = R[rq.mesh]
        M = rq.n_modes
        if rq.kind == "mc":
            return nat.Request(nat.NAT_REQ_MCBEM, r["mesh"], r["gv"][rq.m0:rq.m0 + M], rq.k,
                               r["qt"][:rq.n_queries], r["qb"][:rq.n_queries], rq.n_samples, rq.seed)
        return nat.Request(nat.NAT_REQ_DENSE, r["mesh"], r["gt"][rq.m0:rq.m0 + M], rq.k,
                           layout=nat.NAT_NEUMANN_PER_TRIANGLE)

    def plain(rq, out):
        r = R[rq.mesh]
        M = rq.n_modes
        if rq.kind == "mc":
            o = nat.nat_mc_opts_default()
            o.flags = nat.NAT_MC_NO_GRAPH
            nat.nat_mcbem_estimate(r["mesh"], r["gv"][rq.m0:rq.m0 + M], rq.k, r["qt"][:rq.n_queries],
                                   r["qb"][:rq.n_queries], rq.n_samples, rq.seed, o, p_out=out,
                                   allow_noconv=True)
            return
        for m in range(M):
            op = nat.nat_bem_assemble(r["mesh"], rq.k[m], True)
            nat.nat_bem_solve(op, r["gt"][rq.m0 + m:rq.m0 + m + 1], layout=nat.NAT_NEUMANN_PER_TRIANGLE,
                              tol=sopts.dense_tol, max_iter=sopts.dense_max_iter, p_out=out[m:m + 1],
                              allow_noconv=True)
            op.close()

    def served_run(sub, rate):
        """Submit `sub` at Poisson times of the given rate (None: all at once);
        returns (latencies, queue times, batch sizes, max iterations, span)."""
        built = [build(rq) for rq in sub]
        torch.cuda.synchronize()
        arrive = np.cumsum([rq.gap for rq in sub]) / rate if rate else np.zeros(len(sub))
        lat, qms, bsz, itm = [], [], [], []
        t0 = time.perf_counter()
        tickets = []
        for i, b in enumerate(built):
            d = arrive[i] - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tickets.append(nat.nat_server_submit(srv, b))
        for t in tickets:
            st, r, _ = nat.nat_server_wait(srv, t)
            if st not in (nat.NAT_OK, nat.NAT_E_NOCONV):
                raise RuntimeError(f"served request failed: {nat.status_str(st)}")
            lat.append(r["latency_ms"])
            qms.append(r["queue_ms"])
            bsz.append(r["batch_size"])
            itm.append(r["max_iters"])
        return built, lat, qms, bsz, itm, time.perf_counter() - t0

    def plain_run(sub, rate, outs):
        """The plain form on the same arrivals (None: back to back); returns
        (latencies, service times, span)."""
        arrive = np.cumsum([rq.gap for rq in sub]) / rate if rate else None
        lat, svc = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, rq in enumerate(sub):
            if arrive is not None:
                d = arrive[i] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
            ts = time.perf_counter()
            plain(rq, outs[i])
            torch.cuda.synchronize()
            te = time.perf_counter()
            svc.append(1e3 * (te - ts))
            lat.append(1e3 * (te - t0 - (arrive[i] if arrive is not None else (ts - t0))))
        return lat, svc, time.perf_counter() - t0

    srv = nat.Server(ctx, sopts)
    # warm-up: the first 16 requests
    warm = [build(rq) for rq in reqs[:16]]
    torch.cuda.synchronize()
    for t in [nat.nat_server_submit(srv, b) for b in warm]:
        nat.nat_server_wait(srv, t)
    del warm
    # (1) served capacity
    _, _, _, _, _, cap_s = served_run(reqs, None)
    capacity = len(reqs) / cap_s
    log(f"served capacity: {len(reqs)} requests in {cap_s:.2f} s")
    # (2) the stream at 70 % of the served capacity
    rate = 0.7 * capacity
    built, lat, qms, bsz, itm, span = served_run(reqs, rate)
    stats = nat.nat_server_stats_read(srv)
    log(f"served Poisson run: {span:.2f} s")
    # the plain per-solve form back to back: service times and capacity, and
    # the served results against its outputs bit for bit
    outs = [torch.empty_like(b.p_out) for b in built]
    _, svc, pspan = plain_run(reqs, None, outs)
    plain_capacity = len(reqs) / pspan
    equal = all(torch.equal(b.p_out, o) for b, o in zip(built, outs))
    log(f"plain per-solve back to back: {pspan:.2f} s")
    # (3) equal load, below both capacities
    n_eq = min(len(reqs), args.serve_equal_load_requests)
    sub = reqs[:n_eq]
    rate_eq = 0.7 * plain_capacity
    _, lat_s, _, bsz_eq, _, _ = served_run(sub, rate_eq)
    lat_p, _, _ = plain_run(sub, rate_eq, [torch.empty_like(b.p_out) for b in built[:n_eq]])
    log(f"equal-load runs: {n_eq} requests at {rate_eq:.1f} req/s")
    srv.close()
    out = {
        "workload": f"{len(meshes)} resident cube-spheres T {min(len(m.tris) for m in meshes)}-"
                    f"{max(len(m.tris) for m in meshes)}, {len(reqs)} requests "
                    f"({sum(rq.kind == 'dense' for rq in reqs)} dense: meshes <= 8000 triangles, 1-4 "
                    f"modes), modes 1-64, Q 1-16k, N 512-2048",
        "server": {"slots": sopts.n_slots, "max_batch": sopts.max_batch, "budget_gib": args.serve_budget_gib},
        "forms": {"served": "FP32 compensated, continuous batching over worker streams, graph-replayed GMRES",
                  "plain_per_solve": "FP32 compensated, one request at a time on one stream, direct "
                                     "launches, no batching, no graph"},
        "capacity_req_per_s": round(capacity, 2),
        "plain_capacity_req_per_s": round(plain_capacity, 2),
        "at_served_operating_point": {
            "arrival_rate_req_per_s": round(rate, 2), "latency": _percentiles(lat),
            "queue": _percentiles(qms), "solves_per_s": round(len(reqs) / span, 2),
            "batch_size_mean": round(float(np.mean(bsz)), 2), "gmres_iters_max": int(max(itm))},
        "equal_load": {
            "requests": n_eq, "arrival_rate_req_per_s": round(rate_eq, 2),
            "note": "70 % of the plain form's capacity, below both forms' capacities",
            "served_latency": _percentiles(lat_s), "plain_latency": _percentiles(lat_p),
            "served_batch_size_mean": round(float(np.mean(bsz_eq)), 2)},
        "plain_service_time": _percentiles(svc),
        "mc_pair_evals_per_s_at_capacity": sum(rq.pair_evals() for rq in reqs) / cap_s,
        "stats": stats,
        "results_bitwise_equal_to_plain": bool(equal),
    }
    if not args.no_cpu_baseline:
        # the first few Monte-Carlo requests of at most 3e8 pair evaluations
        # against the FP64 oracle (same seed, GMRES tol 1e-6, at most 200
        # iterations)
        from oracle import oracle as O
        errs = []
        for rq, b in zip(reqs, built):
            if rq.kind != "mc" or rq.pair_evals() > 3e8 or len(errs) >= args.serve_oracle_requests:
                continue
            m = meshes[rq.mesh]
            M = rq.n_modes
            ref = O.mcbem(m.vertices, m.tris, m.g_vertex[rq.m0:rq.m0 + M], rq.k, m.q_tri[:rq.n_queries],
                          m.q_b[:rq.n_queries], rq.n_samples, rq.seed, tol=1e-6)["p"]
            got = b.p_out.cpu().numpy()
            errs.append(max(max(rel_l2(got[q], ref[q]), rel_max(got[q], ref[q])) for q in range(M)))
        out["vs_oracle"] = {"requests": len(errs), "max_error_per_request": [float(f"{e:.3g}") for e in errs],
                            "bar": 1e-3, "error": "max over modes of rel L2 and element-wise"}
    for r in R:
        r["mesh"].close()
    return out


# ---------------------------------------------------------------- HBM traffic
# The counter passes are separate runs of this script under rocprofv3:
#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d D1 -o run -- python3 bench.py --pmc-pass
#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d D2 -o run -- python3 bench.py --pmc-pass
#   python3 bench.py --pmc-summarize D1 D2
# --pmc-pass copies a 1 GiB buffer (the calibration kernel of known traffic)
# and then runs one headline step with direct launches (--ordered: with the
# ordered matvec form); --pmc-summarize scales the matvec kernel's
# per-dispatch counters by the copy's measured / true bytes and writes the
# kernel's traffic file, stamped with a hash of the kernel source so the
# bench reports the figure only while the kernel is unchanged.
CSRC = os.path.join(ROOT, "paper_2506_06190_amd", "csrc")
MATVEC = {
    # symmetric form (default): k_sym32
    "k_sym32": {"src": os.path.join(CSRC, "k_sym32.hip"),
                "match": lambda k: "k_sym32" in k,
                "title": "k_sym32 (symmetric GMRES matvec)",
                "traffic": os.path.join(ROOT, "profiles", "k_sym32_matvec_batched_traffic.txt"),
                "valu": os.path.join(ROOT, "profiles", "k_sym32_matvec_valu_counters.txt")},
    # ordered form (NAT_MC_ORDERED_SUM): k_sum32<OP_MATVEC>
    "k_sum32": {"src": os.path.join(CSRC, "k_sum32.hip"),
                "match": lambda k: "k_sum32<1>" in k or "k_sum32ILi1E" in k,
                "title": "k_sum32<OP_MATVEC> (ordered GMRES matvec)",
                "traffic": os.path.join(ROOT, "profiles", "k_sum32_matvec_batched_traffic.txt"),
                "valu": os.path.join(ROOT, "profiles", "k_sum32_matvec_valu_counters.txt")},
}
COPY_BYTES = 1 << 30


def kernel_hash(kern):
    import hashlib
    with open(MATVEC[kern]["src"], "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def run_pmc_pass(nat, torch, ctx, args, dev):
    import workloads as W
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    wls = W.config_batched()
    meshes, jobs = make_jobs(nat, torch, ctx, wls, dev)
    opts = nat.nat_mc_opts_default()
    opts.flags = nat.NAT_MC_NO_GRAPH | (nat.NAT_MC_ORDERED_SUM if args.ordered else 0)
    opts.n_streams = 1
    nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
    torch.cuda.synchronize()
    for m in meshes:
        m.close()
    log("pmc pass done")


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def _matvec_in(rows):
    for kern, spec in MATVEC.items():
        if any(spec["match"](r["Kernel_Name"]) for r in rows):
            return kern
    raise SystemExit("no matvec kernel in the counter rows")


def pmc_summarize(d_fetch, d_write):
    kern = _matvec_in(_counter_rows(d_fetch))
    match = MATVEC[kern]["match"]
    out = {}
    for name, d in (("FETCH_SIZE", d_fetch), ("WRITE_SIZE", d_write)):
        per = {}
        for r in _counter_rows(d):
            if r.get("Counter_Name") != name:
                continue
            key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id")))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"]) * 1024.0  # KiB per dispatch
        copy = [v for (k, _), v in per.items() if "copy" in k.lower() or "elementwise" in k.lower()]
        mv = [v for (k, _), v in per.items() if match(k)]
        if not copy or not mv:
            raise SystemExit(f"{name}: copy kernel or matvec kernel not found")
        big = max(copy)
        out[name] = {"scale": COPY_BYTES / big, "copy_measured": big, "dispatches": len(mv),
                     "per_launch_raw": sum(mv) / len(mv)}
    f, w = out["FETCH_SIZE"], out["WRITE_SIZE"]
    fetch = f["per_launch_raw"] * f["scale"]
    write = w["per_launch_raw"] * w["scale"]
    lines = [
        f"# HBM traffic of {MATVEC[kern]['title']} (batched headline step, direct launches)",
        "# commands (run from the repository root, TMPDIR=/tmp):",
        f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d_fetch} -o run -- \\",
        f"#       python3 bench.py --pmc-pass{' --ordered' if kern == 'k_sum32' else ''}",
        f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d_write} -o run -- \\",
        f"#       python3 bench.py --pmc-pass{' --ordered' if kern == 'k_sum32' else ''}",
        f"#   python3 bench.py --pmc-summarize {d_fetch} {d_write}",
        "# The copy kernel (a 1 GiB device-to-device copy, 1 GiB read + 1 GiB written) gives",
        "# the scale of each counter; per-launch figures are averages over the matvec dispatches.",
        f"kernel_source_sha256_16: {kernel_hash(kern)}",
        f"matvec_dispatches: {f['dispatches']}",
        f"copy_bytes_true: {COPY_BYTES}",
        f"copy_fetch_measured_bytes: {f['copy_measured']:.0f}",
        f"copy_write_measured_bytes: {w['copy_measured']:.0f}",
        f"fetch_scale: {f['scale']:.4f}",
        f"write_scale: {w['scale']:.4f}",
        f"fetch_bytes_per_launch_scaled: {fetch:.0f}",
        f"write_bytes_per_launch_scaled: {write:.0f}",
        f"traffic_bytes_per_launch: {fetch + write:.0f}",
    ]
    path = MATVEC[kern]["traffic"]
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


VALU_COUNTERS = ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32",
                 "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_WAVES",
                 "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def pmc_valu_summarize(d):
    """Executed FP32 operations and VALU issue of the matvec from one counter
    pass (wave-level instruction counts; an FMA counts 2, a multiply, add or
    transcendental 1, times 64 lanes)."""
    tot = {c: 0.0 for c in VALU_COUNTERS}
    spans = {}
    rows = _counter_rows(d)
    kern = _matvec_in(rows)
    for r in rows:
        k = r["Kernel_Name"]
        if not MATVEC[kern]["match"](k):
            continue
        if r["Counter_Name"] in tot:
            tot[r["Counter_Name"]] += float(r["Counter_Value"])
        spans[r.get("Dispatch_Id")] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    if not spans:
        raise SystemExit("matvec kernel not found")
    secs = sum(spans.values()) * 1e-9
    flops = 64.0 * (2 * tot["SQ_INSTS_VALU_FMA_F32"] + tot["SQ_INSTS_VALU_MUL_F32"] +
                    tot["SQ_INSTS_VALU_ADD_F32"] + tot["SQ_INSTS_VALU_TRANS_F32"])
    # GRBM_GUI_ACTIVE is summed over the 8 XCDs; SQ_ACTIVE_INST_VALU counts,
    # per wave, the quad-cycles with a VALU instruction in flight, summed over
    # the waves: per SIMD cycle it can exceed 1 when the instructions of
    # several waves on one SIMD overlap, so it is a ratio, not a fraction
    xcd_cycles = tot["GRBM_GUI_ACTIVE"] / 8.0
    busy = 4.0 * tot["SQ_ACTIVE_INST_VALU"] / (1024.0 * xcd_cycles)
    ipc = tot["SQ_INSTS_VALU"] / (1024.0 * xcd_cycles)
    lines = [
        f"# VALU counters of {MATVEC[kern]['title']} (batched headline step, direct launches)",
        "# command (run from the repository root, TMPDIR=/tmp):",
        "#   rocprofv3 --pmc " + " ".join(VALU_COUNTERS) + " \\",
        f"#       --output-format csv -d {d} -o run -- python3 bench.py --pmc-pass"
        f"{' --ordered' if kern == 'k_sum32' else ''}",
        f"#   python3 bench.py --pmc-valu-summarize {d}",
        "# executed FP32 flops = 64 lanes x (2 FMA + MUL + ADD + TRANS) wave instructions;",
        "# valu_active_per_simd_cycle = 4 x SQ_ACTIVE_INST_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs)",
        "#   (per-wave VALU-active cycles summed over waves; can exceed 1 when waves overlap);",
        "# valu_insts_per_simd_cycle = SQ_INSTS_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE / 8 XCDs).",
        f"kernel_source_sha256_16: {kernel_hash(kern)}",
        f"matvec_dispatches: {len(spans)}",
        f"traced_seconds: {secs:.6f}",
    ] + [f"{c}: {tot[c]:.6g}" for c in VALU_COUNTERS] + [
        f"executed_fp32_flops: {flops:.6g}",
        f"executed_fp32_tflops: {flops / secs * 1e-12:.3f}",
        f"trans_share_of_valu: {tot['SQ_INSTS_VALU_TRANS_F32'] / tot['SQ_INSTS_VALU']:.4f}",
        f"valu_active_per_simd_cycle: {busy:.4f}",
        f"valu_insts_per_simd_cycle: {ipc:.4f}",
    ]
    with open(MATVEC[kern]["valu"], "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def valu_from_profile(kern):
    """(executed FP32 TFLOP/s, VALU-active cycles per SIMD cycle) of the matvec,
    or None when absent or stale."""
    path = MATVEC[kern]["valu"]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash(kern):
        return None
    if "valu_active_per_simd_cycle" not in kv:
        return None
    return float(kv["executed_fp32_tflops"]), float(kv["valu_active_per_simd_cycle"])


def traffic_from_profile(kern):
    """Scaled HBM bytes per matvec launch, or None when absent or stale."""
    path = MATVEC[kern]["traffic"]
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash(kern):
        return None
    return float(kv["traffic_bytes_per_launch"])


def run_dense(nat, torch, ctx, args, dev):
    """Dense Burton-Miller path on the 5120-triangle sphere at ka = 5: assembly,
    one solve, and 16 right-hand sides at once (FP64 matrix cores) against the
    same 16 as four 4-wide solves (GEMV passes)."""
    import numpy as np
    import workloads as W
    wl = W.config_oscillating_sphere(ka=(5.0,))
    v, f = wl.vertices, wl.tris
    u = wl.extra["u"]
    c = u[f].mean(axis=1)
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    mesh = nat.Mesh(ctx, v, f)
    g1 = torch.from_numpy(np.ascontiguousarray(c[None, :, 2].astype(np.complex128))).to(dev)
    g16 = torch.from_numpy(W.sh_neumann(c, 16, 5)).to(dev)
    torch.cuda.synchronize()
    op = nat.nat_bem_assemble(mesh, wl.k[0], True)       # warm-up
    torch.cuda.synchronize()
    op.close()
    t0 = time.perf_counter()
    op = nat.nat_bem_assemble(mesh, wl.k[0], True)
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    lay = nat.NAT_NEUMANN_PER_TRIANGLE
    nat.nat_bem_solve(op, g1, layout=lay, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep1 = nat.nat_bem_solve(op, g1, layout=lay, tol=1e-10)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    nat.nat_bem_solve(op, g16, layout=lay, tol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep16 = nat.nat_bem_solve(op, g16, layout=lay, tol=1e-10)
    torch.cuda.synchronize()
    t_mfma = time.perf_counter() - t0
    t0 = time.perf_counter()
    for r0 in range(0, 16, 4):
        nat.nat_bem_solve(op, g16[r0:r0 + 4].contiguous(), layout=lay, tol=1e-10)
    torch.cuda.synchronize()
    t_gemv = time.perf_counter() - t0
    n = len(f)
    op.close()
    mesh.close()
    return {"workload": f"icosphere {n} triangles, a = 0.1 m, ka = 5, Burton-Miller, tol 1e-10",
            "assembly_ms": round(1e3 * t_asm, 2), "assembly_pairs_per_s": n * n / t_asm,
            "solve_1rhs_ms": round(1e3 * t_one, 2), "iters_1rhs": rep1[0]["iters"],
            "solve_16rhs_matrix_cores_ms": round(1e3 * t_mfma, 2),
            "solve_16rhs_as_4x4_gemv_ms": round(1e3 * t_gemv, 2),
            "iters_16rhs_max": max(r["iters"] for r in rep16)}


def run_field(nat, torch, ctx, args, dev):
    """Exterior field of the precision workload (20480-triangle ellipsoid, 32
    modes, N = 1024): from the FP32 estimate's sample values, the pressure
    and |p| at 10,000 random shell points per mode (1.5-3 R, the training
    tuples) and on the 32 x 64 FFAT grid at 2 R.  Reports the field step's
    time and pair-evals/s, the evaluation kernel's roofline, and the error of
    each mode against the oracle on the first 500 shell points and the whole
    FFAT grid."""
    import numpy as np
    import workloads as W
    wl = W.config_precision()
    mesh = nat.Mesh(ctx, wl.vertices, wl.tris)
    g = torch.from_numpy(wl.g).to(dev)
    ps = torch.empty((wl.n_modes, wl.n_samples), dtype=torch.complex128, device=dev)
    nat.nat_mcbem_estimate(mesh, g, wl.k, torch.from_numpy(wl.q_tri).to(dev),
                           torch.from_numpy(wl.q_b).to(dev), wl.n_samples, wl.seed, p_samples=ps)
    P = 10000
    pts, co = nat.nat_field_points(mesh, nat.NAT_FIELD_SHELL, P, 1, 1.5, 3.0, 11)
    gpts, gco = nat.nat_field_points(mesh, nat.NAT_FIELD_FFAT_GRID, 32, 64, 2.0, 2.0, 0)
    p = torch.empty((wl.n_modes, P), dtype=torch.complex128, device=dev)
    a = torch.empty((wl.n_modes, P), dtype=torch.float64, device=dev)

    def step():
        nat.nat_field_points(mesh, nat.NAT_FIELD_SHELL, P, 1, 1.5, 3.0, 11, points=pts, coords=co)
        nat.nat_mcbem_field(mesh, g, wl.k, ps, wl.n_samples, wl.seed, pts, p_out=p, abs_out=a)

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    steps = max(args.steps, 10)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    pairs = wl.n_modes * P * wl.n_samples
    nat.nat_profile_enable(ctx, True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = nat.nat_profile_read(ctx)
    nat.nat_profile_enable(ctx, False)
    ev = prof.get("sum32_eval")
    out = {"workload": "exterior field of the precision workload: 32 modes, N 1024, 10,000 shell "
                       "points per mode at 1.5-3 R, and a 32 x 64 FFAT grid at 2 R",
           "ms_per_step": round(1e3 * t, 4), "pair_evals_per_s": pairs / t,
           "points_per_s": wl.n_modes * P / t}
    if ev:
        # one evaluation launch per step over all 32 modes
        flops_per_launch = 47.0 * pairs * steps / ev["launches"]
        achieved = flops_per_launch / (ev["avg_ms"] * 1e-3) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "k_sum32<OP_EVAL> + k_reduce32 (sum32_eval)",
                           "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                           "avg_launch_ms": round(ev["avg_ms"], 5), "launches": ev["launches"],
                           "flops_per_launch": flops_per_launch,
                           "credit": "47 flops per (point, sample, mode)"}
    pg, ag = nat.nat_mcbem_field(mesh, g, wl.k, ps, wl.n_samples, wl.seed, gpts, want_abs=True)
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        ref = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri[:0], wl.q_b[:0], wl.n_samples,
                      wl.seed, tol=1e-12, want_samples=True)
        xs = pts[:500].cpu().numpy()
        xo, _ = O.field_points(wl.vertices, 0, 500, seed=11)
        pts_ok = float(np.abs(xs - xo).max())
        po = O.mcbem_field(wl.vertices, wl.tris, wl.g, wl.k, wl.n_samples, wl.seed, xo,
                           ref["p_samples"])
        got = p[:, :500].cpu().numpy()
        xg, cg = O.field_points(wl.vertices, 1, 32, 64, r_lo=2.0)
        pgo = O.mcbem_field(wl.vertices, wl.tris, wl.g, wl.k, wl.n_samples, wl.seed, xg,
                            ref["p_samples"])
        ffat = ag.cpu().numpy() * cg[None, :, 0]
        ffat_o = np.abs(pgo) * cg[None, :, 0]
        out["vs_oracle"] = {
            "shell_points_max_coord_err": pts_ok,
            "shell_rel_l2_per_mode": [float(f"{rel_l2(got[m], po[m]):.3g}") for m in range(wl.n_modes)],
            "shell_elementwise_per_mode": [float(f"{rel_max(got[m], po[m]):.3g}")
                                           for m in range(wl.n_modes)],
            "ffat_map_rel_l2_per_mode": [float(f"{rel_l2(ffat[m], ffat_o[m]):.3g}")
                                         for m in range(wl.n_modes)]}
    mesh.close()
    return out


def run_poisson(nat, torch, ctx, args, dev):
    """Poisson-disk sample sets (Section 4.2, parallel Poisson-disk sampling;
    Section 6.1: Poisson-disk samples beat independent ones at the same N):
    the sampler's time per set on the precision workload's 20480-triangle
    ellipsoid and on a 40k-triangle cube-sphere at N = 1024-10240 (the
    paper's 1K-10K), the precision-form estimate with Poisson-disk samples
    against independent ones, and (with the oracle) the sets checked bit for
    bit, the oracle's time for the same sets and the estimate's error
    against the closed-form spheres both ways."""
    import numpy as np
    import workloads as W
    wl = W.config_precision()
    cube = W.cubesphere_ellipsoid(9, 40000)
    meshes = [("ellipsoid 20480 tri", wl.vertices, wl.tris), (f"cube-sphere {len(cube[1])} tri", cube[0], cube[1])]
    reps = max(args.steps, 10)
    sets = []
    handles = []
    for name, v, f in meshes:
        mesh = nat.Mesh(ctx, v, f)
        handles.append(mesh)
        for N in (1024, 4096, 10240):
            tri = torch.empty(N, dtype=torch.int32, device=dev)
            bary = torch.empty((N, 2), dtype=torch.float64, device=dev)
            nat.nat_mcbem_poisson_samples(mesh, N, wl.seed, tri, bary)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(reps):
                _, _, n_acc = nat.nat_mcbem_poisson_samples(mesh, N, wl.seed + r, tri, bary)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            sets.append({"mesh": name, "N": N, "ms_per_set": round(1e3 * t, 4), "samples_per_s": N / t,
                         "accepted": n_acc, "candidates": 16 * N})
    out = {"workload": "Poisson-disk sample sets: 20480-triangle ellipsoid and 40k-triangle cube-sphere, "
                       "N 1024 / 4096 / 10240, candidate pool 16 N",
           "sets": sets}
    # the precision-form estimate with independent and with Poisson-disk samples
    g = torch.from_numpy(wl.g).to(dev)
    qt, qb = torch.from_numpy(wl.q_tri).to(dev), torch.from_numpy(wl.q_b).to(dev)
    est = {}
    for label, flags in (("independent", 0), ("poisson", nat.NAT_MC_POISSON)):
        opts = nat.nat_mc_opts_default()
        opts.flags = flags
        nat.nat_mcbem_estimate(handles[0], g, wl.k, qt, qb, wl.n_samples, wl.seed, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            nat.nat_mcbem_estimate(handles[0], g, wl.k, qt, qb, wl.n_samples, wl.seed, opts)
        torch.cuda.synchronize()
        est[label] = round(1e3 * (time.perf_counter() - t0) / reps, 4)
    out["precision_form_estimate_ms"] = est
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        from oracle import closed_forms as CF
        N = 1024
        tri, bary, n_acc = nat.nat_mcbem_poisson_samples(handles[0], N, wl.seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_o, b_o, n_o = O.poisson_samples(wl.vertices, wl.tris, N, wl.seed)
        t_cpu = time.perf_counter() - t0
        out["vs_oracle"] = {"set": "ellipsoid, N 1024", "bit_exact": bool(
            n_acc == n_o and np.array_equal(tri.cpu().numpy(), t_o) and np.array_equal(bary.cpu().numpy(), b_o))}
        out["cpu_oracle"] = {"ms_per_set": round(1e3 * t_cpu, 3), "cores": 1, "kind": "oracle",
                             "sample": "ellipsoid 20480 tri, N 1024"}
        # error against the closed forms, FP32 GPU estimates, independent vs Poisson-disk samples
        acc = {}
        cases = [("pulsating sphere, ico3, k a = 2", W.config_pulsating_sphere(),
                  lambda w: np.full(w.n_queries, CF.pulsating_sphere(2.0, 1.0)), 4),
                 ("oscillating sphere, ico4, k a = 5", W.config_oscillating_sphere(ka=(5.0,)),
                  lambda w: CF.oscillating_sphere_factor(w.k[0], 0.1) * w.extra["u"][:, 2], 4)]
        for name, w, exact_of, n_seeds in cases:
            m = nat.Mesh(ctx, w.vertices, w.tris)
            ex = exact_of(w)
            gw = torch.from_numpy(w.g).to(dev)
            qtw, qbw = torch.from_numpy(w.q_tri).to(dev), torch.from_numpy(w.q_b).to(dev)
            row = {}
            for label, flags in (("independent", 0), ("poisson", nat.NAT_MC_POISSON)):
                opts = nat.nat_mc_opts_default()
                opts.flags = flags
                errs = []
                for sd in range(n_seeds):
                    p, _ = nat.nat_mcbem_estimate(m, gw, w.k, qtw, qbw, 1024, 300 + sd, opts)
                    errs.append(float(np.linalg.norm(p[0].cpu().numpy() - ex) / np.linalg.norm(ex)))
                row[label] = round(float(np.mean(errs)), 4)
            acc[name] = row
            m.close()
        out["rel_error_vs_closed_form_N1024_mean_of_4_seeds"] = acc
    for m in handles:
        m.close()
    return out


def run_scenes(nat, torch, ctx, args, dev):
    """Training-data generation for a family of scenes (Section 3.4): 16
    speaker-torus scenes (a speaker patch with g = 1 moving along the axis of
    a passive torus, per-triangle data, ~9.4k triangles each) x 8
    frequencies, N = 2048 samples and 4096 surface queries each, solved as
    one batch (FP32); then the field at 10,000 shell points per (scene,
    frequency) from each scene's sample values: the (theta, phi, r, |p|)
    tuples the neural field trains on."""
    import numpy as np
    import workloads as W
    wls = W.config_scenes()
    meshes, jobs, ps = [], [], []
    opts = nat.nat_mc_opts_default()
    opts.layout = nat.NAT_NEUMANN_PER_TRIANGLE
    for wl in wls:
        mesh = nat.Mesh(ctx, wl.vertices, wl.tris)
        meshes.append(mesh)
        p_s = torch.empty((wl.n_modes, wl.n_samples), dtype=torch.complex128, device=dev)
        ps.append(p_s)
        jobs.append(nat.McJob(mesh, torch.from_numpy(wl.g).to(dev), wl.k, torch.from_numpy(wl.q_tri).to(dev),
                              torch.from_numpy(wl.q_b).to(dev), wl.n_samples, wl.seed, p_samples=p_s,
                              layout=nat.NAT_NEUMANN_PER_TRIANGLE))
    P = 10000
    pc = [nat.nat_field_points(m, nat.NAT_FIELD_SHELL, P, 1, 1.5, 3.0, 100 + i) for i, m in enumerate(meshes)]
    pts = [a for a, _ in pc]
    coords = [c for _, c in pc]
    fout = [torch.empty((wl.n_modes, P), dtype=torch.complex128, device=dev) for wl in wls]
    fabs = [torch.empty((wl.n_modes, P), dtype=torch.float64, device=dev) for wl in wls]

    fjobs = [nat.FieldJob(m, jobs[i].v_n, wl.k, ps[i], wl.n_samples, wl.seed, pts[i], p_out=fout[i],
                          abs_out=fabs[i]) for i, (wl, m) in enumerate(zip(wls, meshes))]

    def step():
        reps = nat.nat_mcbem_estimate_batch(ctx, jobs, opts, allow_noconv=True)
        for i, m in enumerate(meshes):
            nat.nat_field_points(m, nat.NAT_FIELD_SHELL, P, 1, 1.5, 3.0, 100 + i, points=pts[i])
        nat.nat_mcbem_field_batch(ctx, fjobs, opts)
        return reps

    step()
    torch.cuda.synchronize()
    steps = max(args.steps, 3)
    t0 = time.perf_counter()
    for _ in range(steps):
        reps = step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    alg = sum(w.pair_evals() for w in wls) + sum(w.n_modes * P * w.n_samples for w in wls)
    iters = [r["iters"] for rr in reps for r in rr]
    out = {"workload": f"{len(wls)} speaker-torus scenes ({len(wls[0].tris)} triangles), "
                       f"{wls[0].n_modes} frequencies each, N {wls[0].n_samples}, Q {wls[0].n_queries}, "
                       f"{P} field points per (scene, frequency)",
           "ms_per_step": round(1e3 * t, 3), "pair_evals_per_s": alg / t,
           "training_tuples_per_s": sum(w.n_modes for w in wls) * P / t,
           "gmres_iters": {"mean": float(np.mean(iters)), "max": int(max(iters))}}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        errs = []
        for i in (0, len(wls) // 2):
            wl = wls[i]
            modes = [0, wl.n_modes - 1]
            ref = O.mcbem(wl.vertices, wl.tris, wl.g[modes], wl.k[modes], wl.q_tri, wl.q_b, wl.n_samples,
                          wl.seed, tol=1e-6, layout=1, want_samples=True)
            got = jobs[i].p_out[modes].cpu().numpy()
            xs = pts[i][:300].cpu().numpy()
            fo = O.mcbem_field(wl.vertices, wl.tris, wl.g[modes], wl.k[modes], wl.n_samples, wl.seed, xs,
                               ref["p_samples"], layout=1)
            fg = fout[i][modes][:, :300].cpu().numpy()
            for a, m in enumerate(modes):
                errs.append({"scene": i, "mode": m,
                             "surface_rel_l2": float(f"{rel_l2(got[a], ref['p'][a]):.3g}"),
                             "surface_elementwise": float(f"{rel_max(got[a], ref['p'][a]):.3g}"),
                             "field_elementwise": float(f"{rel_max(fg[a], fo[a]):.3g}")})
        out["vs_oracle"] = errs
    # the same tuples from independent sample sets (seed + 1000), and both
    # again with Poisson-disk samples (Section 4.2): how much of the field's
    # held-out error is the targets' own Monte-Carlo noise, and how much the
    # Poisson-disk sets lower it
    def tuples(seed_off, flags):
        o = nat.nat_mc_opts_default()
        o.layout = nat.NAT_NEUMANN_PER_TRIANGLE
        o.flags = flags
        jj, pp = [], []
        for i, (wl, m) in enumerate(zip(wls, meshes)):
            p_s = torch.empty((wl.n_modes, wl.n_samples), dtype=torch.complex128, device=dev)
            pp.append(p_s)
            jj.append(nat.McJob(m, jobs[i].v_n, wl.k, jobs[i].q_tri, jobs[i].q_bary, wl.n_samples,
                                wl.seed + seed_off, p_samples=p_s, layout=nat.NAT_NEUMANN_PER_TRIANGLE))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nat.nat_mcbem_estimate_batch(ctx, jj, o, allow_noconv=True)
        fj = [nat.FieldJob(m, jobs[i].v_n, wl.k, pp[i], wl.n_samples, wl.seed + seed_off, pts[i], want_abs=True)
              for i, (wl, m) in enumerate(zip(wls, meshes))]
        nat.nat_mcbem_field_batch(ctx, fj, o)
        fa = [j.abs_out for j in fj]
        torch.cuda.synchronize()
        return fa, time.perf_counter() - t0

    fabs2, _ = tuples(1000, 0)
    fabs_p, _ = tuples(0, nat.NAT_MC_POISSON)
    fabs_p2, t_p = tuples(1000, nat.NAT_MC_POISSON)  # the second call: workspace already grown
    out["poisson_disk_step_ms"] = round(1e3 * t_p, 3)
    out["neural_field_trained_on_these_tuples"] = train_on_scene_tuples(nat, torch, ctx, dev, wls, coords, fabs,
                                                                        fabs2=fabs2)
    out["neural_field_trained_on_poisson_disk_tuples"] = train_on_scene_tuples(
        nat, torch, ctx, dev, wls, coords, fabs_p, fabs2=fabs_p2)
    for m in meshes:
        m.close()
    return out


def scene_training_rows(torch, wls, coords, fabs):
    """Neural-field rows (theta, phi, r / R, v, f) and targets |p| from the
    scenes' shell points: R the scene's bounding radius, v the speaker height
    mapped to [0, 1], f the frequency on a log scale over 200 Hz - 8 kHz
    mapped to [0, 1]."""
    import numpy as np
    rows, tgt = [], []
    lo, hi = np.log(200.0), np.log(8000.0)
    for i, wl in enumerate(wls):
        R = 0.5 * float(np.linalg.norm(wl.vertices.max(0) - wl.vertices.min(0)))
        v = (wl.extra["speaker_y"] + 0.15) / 0.30
        fn = (np.log(np.asarray(wl.k) * 343.0 / (2.0 * np.pi)) - lo) / (hi - lo)
        c = coords[i]
        n = c.shape[0]
        for m in range(wl.n_modes):
            rows.append(torch.stack([c[:, 1], c[:, 2], c[:, 0] / R, torch.full_like(c[:, 0], v),
                                     torch.full_like(c[:, 0], float(fn[m]))], 1))
            tgt.append(fabs[i][m, :n])
    return torch.cat(rows).float().contiguous(), torch.cat(tgt).float()[:, None].contiguous()


def train_on_scene_tuples(nat, torch, ctx, dev, wls, coords, fabs, steps=3000, batch=1 << 16, fabs2=None):
    """The neural field (one condition variable: the speaker height) trained
    on the scenes' (theta, phi, r, v, f, |p|) tuples with Adam (Section 3.4),
    minibatches drawn uniformly from 90 % of the tuples; reports the loss and
    the relative RMS error of |p| on the held-out 10 % (every tenth tuple).
    Targets are divided by their RMS so the loss is relative.  With fabs2
    (the same tuples from an independent sample set) it also reports the
    targets' own noise, sqrt(1/2) |Y - Y2| / |Y|, and the held-out error
    against Y2 and against the mean of the two."""
    X, Y = scene_training_rows(torch, wls, coords, fabs)
    scale = float(Y.pow(2).mean().sqrt())
    Y = Y / scale
    held = torch.zeros(X.shape[0], dtype=torch.bool, device=dev)
    held[::10] = True
    Xtr, Ytr = X[~held].contiguous(), Y[~held].contiguous()
    Xte, Yte = X[held].contiguous(), Y[held].contiguous()
    nf = nat.NeuralField(ctx, 1, 1, 1.5, 3.0, seed=7)
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    first = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(steps):
        idx = torch.randint(0, Xtr.shape[0], (batch,), device=dev, generator=gen)
        loss = nf.train_step(Xtr[idx], Ytr[idx], s_, steps, want_loss=(s_ == 0))
        if s_ == 0:
            first = loss
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    last = nf.loss_grad(Xtr[:batch].contiguous(), Ytr[:batch].contiguous())
    pred = nf.infer(Xte)
    err = float((pred - Yte).norm() / Yte.norm())
    nf.close()
    out = {"tuples": int(X.shape[0]), "held_out": int(Xte.shape[0]), "steps": steps, "batch": batch,
           "seconds": round(t, 3), "train_rows_per_s_incl_sampling": steps * batch / t,
           "loss_first": first, "loss_last": last, "held_out_rel_rms_error_abs_p": round(err, 4),
           "target_rms": scale}
    if fabs2 is not None:
        _, Y2 = scene_training_rows(torch, wls, coords, fabs2)
        Y2te = (Y2 / scale)[held].contiguous()
        mean = 0.5 * (Yte + Y2te)
        out["held_out_target_noise_rel_rms"] = round(float((Yte - Y2te).norm() / Yte.norm()) / 2 ** 0.5, 4)
        out["held_out_rel_rms_error_vs_independent_targets"] = round(float((pred - Y2te).norm() / Y2te.norm()), 4)
        out["held_out_rel_rms_error_vs_mean_of_two"] = round(float((pred - mean).norm() / mean.norm()), 4)
    return out


def run_neural(nat, torch, ctx, args, dev):
    """Neural-field training and inference (Sections 3.2-3.4): one condition
    variable and the frequency, |p| as the one output, synthetic training
    rows of the paper's shell (directions uniform, 1.5-3 R) with a smooth
    target.  Training steps of 2^18 rows (loss, gradient of every parameter,
    Adam) and inference over 2^20 rows.  The credited work is the MLP's
    products (2 flops per multiply-add: forward, input gradient, weight
    gradient) against the bfloat16 matrix-core peak, and the step's
    algorithmic HBM bytes (each activation written and read in both
    layouts) against 8 TB/s."""
    import numpy as np
    import workloads as W
    n_v, n_out, B, B_inf = 1, 1, 1 << 18, 1 << 20

    def rows_of(n, seed):
        th, ph, r, v, f = W.nf_rows(n, n_v, seed)
        tgt = W.nf_smooth_target(th, ph, r, v, f, n_out)
        rows = np.concatenate([th[:, None], ph[:, None], r[:, None], v, f[:, None]], axis=1)
        return (torch.from_numpy(rows.astype(np.float32)).to(dev),
                torch.from_numpy(tgt.astype(np.float32)).to(dev), (th, ph, r, v, f, tgt))

    x, t, host = rows_of(B, 21)
    xi, _, _ = rows_of(B_inf, 22)
    nf = nat.NeuralField(ctx, n_v, n_out, 1.5, 3.0, seed=5)
    D = nf.input_dim
    steps = max(args.steps, 20)
    warm = max(args.warmup, 2)
    total = warm + steps + 1
    first = nf.train_step(x, t, 0, total)
    for s in range(1, warm):
        nf.train_step(x, t, s, total, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        nf.train_step(x, t, warm + s, total, want_loss=False)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    last = nf.train_step(x, t, total - 1, total)
    y = nf.infer(xi)
    torch.cuda.synchronize()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        nf.infer(xi, out=y)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    H = 128
    fwd = 2 * (D * H + 3 * H * H + H * n_out)
    bwd_in = 2 * (3 * H * H + H * 32 + H * n_out)
    wgrad = 2 * (D * H + 3 * H * H + H * n_out)
    flops_step = B * (fwd + bwd_in + wgrad)
    # HBM bytes per row of the step as built (bfloat16 = 2 B): the fused
    # forward pass reads the 5 FP32 inputs and writes the input row (2 D) and
    # the 4 hidden activations (4 x 256); the output step reads A_4 (256) and
    # the target and writes dZ_3 (256); each fused backward pass reads dZ_i
    # and A_i and writes dZ_{i-1} (3 x 768), the first-layer pass reads dZ_0
    # and the input (256 + 2 D) and writes the 16 FP32 grid columns (64); the
    # grid gradient reads the inputs and those columns (84).  The grid
    # tables (1.6 MB) stay in L2.
    per_row = 20 + 2 * D + 4 * 2 * H + (2 * H + 4 + 2 * H) + 3 * 3 * 2 * H + (2 * H + 2 * D + 64) + 84
    bytes_step = B * per_row
    tf = flops_step / t_step / 1e12
    bw = bytes_step / t_step / 1e9
    out = {"workload": f"neural field (grid 4 levels x 4 features, PE 6 freqs, MLP 4x128), n_v {n_v}, "
                       f"D {D}, training batch {B} rows, inference {B_inf} rows",
           "train_ms_per_step": round(1e3 * t_step, 4), "train_rows_per_s": B / t_step,
           "infer_ms": round(1e3 * t_inf, 4), "infer_rows_per_s": B_inf / t_inf,
           "loss_first": first, "loss_after": last, "steps_trained": total,
           "mfma": {"achieved": round(tf, 3), "peak": 2500.0, "unit": "TFLOP/s",
                    "frac": round(tf / 2500.0, 5), "flops_per_step": flops_step},
           "hbm": {"achieved": round(bw, 1), "peak": 8000.0, "unit": "GB/s", "frac": round(bw / 8000.0, 4),
                   "bytes_per_step": bytes_step}}
    if not args.no_cpu_baseline:
        from oracle import neural as NF
        th, ph, r, v, f, tgt = host
        n = 16384
        p = NF.init_params(n_v, n_out, 5)
        t0 = time.perf_counter()
        loss, g = NF.loss_and_grad(th[:n], ph[:n], r[:n], v[:n], f[:n], tgt[:n], p, 1.5, 3.0, bf=True)
        NF.adam_step(p, g, {}, 0, 10)
        t_cpu = time.perf_counter() - t0
        out["cpu_oracle"] = {"rows_per_s": n / t_cpu, "sample": f"one training step of {n} rows",
                             "kind": "oracle"}
    nf.close()
    return out


def run_precision(nat, torch, ctx, args, dev, with_plain=True):
    import numpy as np
    import workloads as W
    wl = W.config_precision()
    mesh = nat.Mesh(ctx, wl.vertices, wl.tris)
    g = torch.from_numpy(wl.g).to(dev)
    qt = torch.from_numpy(wl.q_tri).to(dev)
    qb = torch.from_numpy(wl.q_b).to(dev)
    p = torch.empty((wl.n_modes, wl.n_queries), dtype=torch.complex128, device=dev)
    alg = wl.pair_evals()

    def step(prec, flags=0):
        o = nat.nat_mc_opts_default()
        o.precision = prec
        o.flags = flags
        return nat.nat_mcbem_estimate(mesh, g, wl.k, qt, qb, wl.n_samples, wl.seed, o, p_out=p)

    for _ in range(max(1, args.warmup)):
        step(nat.NAT_PREC_FP32)
    torch.cuda.synchronize()
    steps = max(args.steps, 5)
    t0 = time.perf_counter()
    for _ in range(steps):
        _, reps = step(nat.NAT_PREC_FP32)
    torch.cuda.synchronize()
    t32 = (time.perf_counter() - t0) / steps
    p32 = p.cpu().numpy()
    out = {"workload": wl.name, "fp32": {"value": alg / t32, "ms_per_step": 1e3 * t32},
           "gmres_iters": [r["iters"] for r in reps]}
    # the same with the phase formed from FP64 positions and reduced in FP64
    step(nat.NAT_PREC_FP32, nat.NAT_MC_FP64_PHASE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, reps_ph = step(nat.NAT_PREC_FP32, nat.NAT_MC_FP64_PHASE)
    torch.cuda.synchronize()
    tph = (time.perf_counter() - t0) / steps
    pph = p.cpu().numpy()
    out["fp32_fp64_phase"] = {"value": alg / tph, "ms_per_step": 1e3 * tph,
                              "gmres_iters": [r["iters"] for r in reps_ph]}
    if with_plain:
        step(nat.NAT_PREC_FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(nat.NAT_PREC_FP64)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        p64 = p.cpu().numpy()
        out["plain_fp64"] = {"form": "plain FP64, one thread per target, no tiling",
                             "value": alg / t64, "ms_per_step": 1e3 * t64}
        out["fp32_speedup_vs_plain"] = t64 / t32
        out["fp32_max_rel_l2_vs_plain"] = max(rel_l2(p32[m], p64[m]) for m in range(wl.n_modes))
    mesh.close()
    if not args.no_cpu_baseline:
        # error of each mode against the FP64 oracle (same seed and samples,
        # GMRES to 1e-12 on the oracle's side)
        from oracle import oracle as O
        t0 = time.perf_counter()
        ref = O.mcbem(wl.vertices, wl.tris, wl.g, wl.k, wl.q_tri, wl.q_b, wl.n_samples, wl.seed,
                      tol=1e-12)["p"]
        out["oracle_seconds"] = round(time.perf_counter() - t0, 2)
        out["fp32_vs_oracle_per_mode"] = {
            "rel_l2": [float(f"{rel_l2(p32[m], ref[m]):.3g}") for m in range(wl.n_modes)],
            "elementwise": [float(f"{rel_max(p32[m], ref[m]):.3g}") for m in range(wl.n_modes)]}
        out["fp32_fp64_phase_vs_oracle_per_mode"] = {
            "rel_l2": [float(f"{rel_l2(pph[m], ref[m]):.3g}") for m in range(wl.n_modes)],
            "elementwise": [float(f"{rel_max(pph[m], ref[m]):.3g}") for m in range(wl.n_modes)]}
        if with_plain:
            out["plain_fp64_vs_oracle_per_mode"] = {
                "rel_l2": [float(f"{rel_l2(p64[m], ref[m]):.3g}") for m in range(wl.n_modes)],
                "elementwise": [float(f"{rel_max(p64[m], ref[m]):.3g}") for m in range(wl.n_modes)]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["batched", "precision", "served", "dense", "field", "scenes", "neural",
                                           "poisson"],
                    default="batched")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true")
    ap.add_argument("--ordered", action="store_true",
                    help="with --pmc-pass: the ordered matvec form (NAT_MC_ORDERED_SUM)")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--pmc-valu-summarize", metavar="DIR")
    ap.add_argument("--tune", choices=["cache", "default"], default="cache",
                    help="kernel-sum tiling: the autotuner's table (cache, else a sweep) or the defaults")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2506_06190_amd", "tune",
                                                         "kernel_sum_tiles.json"))
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-equal-load-requests", type=int, default=400)
    ap.add_argument("--serve-oracle-requests", type=int, default=8)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="host time the oracle's sample of the headline workload may take")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args()
    if args.pmc_summarize:
        pmc_summarize(*args.pmc_summarize)
        return
    if args.pmc_valu_summarize:
        pmc_valu_summarize(args.pmc_valu_summarize)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is "
              "described in the design notes but not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_06190_amd import nat

    dev = "cuda:0"
    ctx = nat.Context(0)
    os.makedirs(os.path.dirname(args.tune_cache), exist_ok=True)
    if args.pmc_pass:
        nat.nat_autotune(ctx, args.tune_cache)
        run_pmc_pass(nat, torch, ctx, args, dev)
        ctx.close()
        return
    had_cache = os.path.exists(args.tune_cache)
    t0 = time.perf_counter()
    if args.tune == "cache":
        table = nat.nat_autotune(ctx, args.tune_cache)
        source = "cache" if had_cache else "sweep"
    else:
        table = nat.nat_tune_get(ctx)
        source = "defaults"
    form = nat.nat_tune_get_form(ctx, with_rates=True)
    tune = {"cache": os.path.relpath(args.tune_cache, ROOT), "source": source,
            "seconds": round(time.perf_counter() - t0, 2), "items_a": table["items_a"],
            "items_b": table["items_b"], "matvec_assembled": form["assembled"]}
    if any(form["rate_matrix_free"]):
        tune["matvec_rate_matrix_free"] = [float(f"{x:.3g}") for x in form["rate_matrix_free"]]
        tune["matvec_rate_assembled"] = [float(f"{x:.3g}") for x in form["rate_assembled"]]
    log(f"kernel-sum tiling from {tune['source']} in {tune['seconds']} s")
    out = {"metric": METRIC, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "autotune": tune}
    if args.workload == "batched":
        res = run_batched(nat, torch, ctx, args, dev)
        out.update({k: res.pop(k) for k in ("value", "ms_per_step", "config")})
        out.update(res)
        out["precision"] = run_precision(nat, torch, ctx, args, dev, with_plain=not args.no_plain)
        out["dense"] = run_dense(nat, torch, ctx, args, dev)
        out["field"] = run_field(nat, torch, ctx, args, dev)
        out["scenes"] = run_scenes(nat, torch, ctx, args, dev)
        out["neural"] = run_neural(nat, torch, ctx, args, dev)
        out["poisson"] = run_poisson(nat, torch, ctx, args, dev)
        if not args.no_serve:
            out["served"] = run_served(nat, torch, ctx, args, dev)
    elif args.workload == "served":
        res = run_served(nat, torch, ctx, args, dev)
        out["metric"] = "served solves/s with p50/p99 latency"
        out["unit"] = "solves/s"
        out["value"] = res["at_served_operating_point"]["solves_per_s"]
        out["ms_per_step"] = None
        out["config"] = {"workload": res["workload"]}
        out["served"] = res
    elif args.workload == "dense":
        res = run_dense(nat, torch, ctx, args, dev)
        out["metric"] = "dense Burton-Miller solve, 16 right-hand sides"
        out["unit"] = "solves/s"
        out["value"] = 16e3 / res["solve_16rhs_matrix_cores_ms"]
        out["ms_per_step"] = res["solve_16rhs_matrix_cores_ms"]
        out["dtype"] = "f64"
        out["config"] = {"workload": res["workload"]}
        out["dense"] = res
    elif args.workload == "scenes":
        res = run_scenes(nat, torch, ctx, args, dev)
        out["value"] = res["pair_evals_per_s"]
        out["ms_per_step"] = res["ms_per_step"]
        out["config"] = {"workload": res["workload"]}
        out["scenes"] = res
    elif args.workload == "neural":
        res = run_neural(nat, torch, ctx, args, dev)
        out["metric"] = "neural-field training rows/s"
        out["unit"] = "rows/s"
        out["value"] = res["train_rows_per_s"]
        out["ms_per_step"] = res["train_ms_per_step"]
        out["dtype"] = "bf16"
        out["config"] = {"workload": res["workload"]}
        out["neural"] = res
    elif args.workload == "poisson":
        res = run_poisson(nat, torch, ctx, args, dev)
        out["metric"] = "Poisson-disk samples/s"
        out["unit"] = "samples/s"
        big = res["sets"][2]
        out["value"] = big["samples_per_s"]
        out["ms_per_step"] = big["ms_per_set"]
        out["dtype"] = "f64"
        out["config"] = {"workload": res["workload"]}
        out["poisson"] = res
    elif args.workload == "field":
        res = run_field(nat, torch, ctx, args, dev)
        out["metric"] = "exterior field pair-evals/s"
        out["value"] = res["pair_evals_per_s"]
        out["ms_per_step"] = res["ms_per_step"]
        out["config"] = {"workload": res["workload"]}
        out["field"] = res
    else:
        res = run_precision(nat, torch, ctx, args, dev, with_plain=not args.no_plain)
        out["value"] = res["fp32"]["value"]
        out["ms_per_step"] = res["fp32"]["ms_per_step"]
        out["config"] = {"workload": res["workload"], "form": "FP32 compensated"}
        out["precision"] = res
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
