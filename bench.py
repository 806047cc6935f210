"""Benchmark: time-to-1e-10 of the FP64 p-multigrid-preconditioned CG on the 3D warped,
variable-coefficient problem (16^3 hexes, p = 8, 2,146,689 nodes; mu = exp(4.6 sx sy sz),
cyclic sine warp a = 0.05, f = 1), with the hierarchy resident in HBM.

One step = one complete solve from x = 0 to ||r|| <= 1e-10 ||b|| (every row of the hot path:
products, Chebyshev smoothing, transfers, coarse solve, V-cycle, PCG). value = nodes solved per
second (N / time-to-solution), in GDOF/s. The JSON line also carries the operator-apply rate
and its HBM roofline fraction, measured with HIP events on the stream the kernels run on, and
the CPU oracle timed on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per operator product read by the FETCH_SIZE / WRITE_SIZE counters (calibrated on a
# plain copy kernel), with the hash of the apply kernels' source they were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_warped_16cubed_p8_hbm_traffic.txt")
# the sources the operator-product kernels are compiled from
APPLY_SOURCES = [os.path.join(ROOT, "paper_1402_5938_amd", "csrc", f)
                 for f in ("k_apply.hip", "dev_apply.h", "epilogue.h")]


def apply_source_sha():
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()
CALIB_COPY_BYTES = 256 * 2 ** 20


def measured_traffic(nelem, order):
    """HBM bytes per product from the committed counter runs, or None when they were taken on
    another problem size or the apply kernels' source has changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("apply_sources_sha256") != apply_source_sha() or kv.get("problem") != f"{nelem}^3 hexes p={order}":
        return None
    try:
        return float(kv["hbm_bytes_per_apply"])
    except (KeyError, ValueError):
        return None


def apply_bytes(dim, ne, p, N, s):
    """Algorithmic bytes of one operator product: every stored geometric factor once
    (6 words per GLL point in 3D, 3 in 2D) plus x read once and y written once."""
    n = p + 1
    E = 1
    for v in ne:
        E *= v
    g = 6 if dim == 3 else 3
    return s * (g * E * n ** dim + 2 * N)


def apply_flops(dim, ne, p):
    n = p + 1
    E = 1
    for v in ne:
        E *= v
    return E * (12 * n ** 4 + 15 * n ** 3) if dim == 3 else E * (8 * n ** 3 + 6 * n ** 2)


def stream_copy_gbs(nbytes=1 << 30, reps=10):
    """Bandwidth of the library's own streaming copy kernel (gllmg_stream_copy) over nbytes
    read and nbytes written, HIP events on the launch stream: the achievable HBM rate."""
    import torch

    from paper_1402_5938_amd import gllmg
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        gllmg.stream_copy(src, dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gllmg.stream_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def apply_beyond_cache(ne=32, p=8, reps=20):
    """One FP64 product of the warped workload on ne^3 hexes at order p (32^3 at p = 8: 35.9M
    nodes, 1.42 GB of algorithmic bytes, beyond the 256 MB Infinity Cache): the median of reps
    HIP-event-timed products after 5 warm-ups."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    cfg = gllmg.make_config(3, (ne,) * 3, p, "p", max_levels=1, eig_steps=1)
    G = gllmg.Problem(cfg, inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(4.6))
    N = G.nnodes(0)
    x = torch.from_numpy(inputs.uniform_nodal(99, N)).cuda()
    y = torch.empty_like(x)
    for _ in range(5):
        G.apply(x, y)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        G.apply(x, y)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    ts.sort()
    t = ts[len(ts) // 2]
    nb = apply_bytes(3, (ne,) * 3, p, N, 8)
    G.close()
    del x, y
    torch.cuda.empty_cache()
    return {"problem": f"{ne}^3 hexes p={p}", "nodes": N, "algorithmic_bytes": nb,
            "apply_us": t * 1e6, "achieved": nb / t / 1e9}


def cpu_baseline():
    """The oracle's PCG (FP64, assembled factored sparse operator, single thread) on a bounded
    sample of the same workload: the same warp, coefficient, hierarchy (orders 8, 4, 2, 1, the
    exact solve on the first-order level) and smoother on 4^3 hexes at p = 8 (35,937 nodes);
    setup excluded as on the GPU side."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fem, mg
    from paper_1402_5938_amd import inputs
    prob = inputs.warped_var3d(nelem=4, order=8)
    with threadpool_limits(limits=1):
        H = mg.Hierarchy(3, prob.nelem, prob.order, prob.map, prob.mu, hierarchy="p", nu=4,
                         coarse_unknowns=inputs.COARSE_UNKNOWNS)
        b = fem.load_vector(H.fine.mesh, fem.nodal_field(H.fine.mesh, prob.f))
        reps = 0
        t0 = time.perf_counter()
        while True:
            res = mg.pcg(H, b, rtol=1e-10)
            reps += 1
            el = time.perf_counter() - t0
            if el > 10.0 or reps >= 80:  # about 10 s of host work
                break
    N = H.fine.mesh.N
    return {"value": N * reps / el / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle PCG to 1e-10 on 4^3 hexes p=8 (N={N}, {res.iters} iterations), "
                      f"{reps} solves in {el:.1f} s, setup excluded"}


def _solve_timed(G, b, steps, warmup, rtol, maxit, mode="pcg"):
    import torch
    x = torch.zeros_like(b)
    for _ in range(warmup):
        x.zero_()
        G.solve(b, x, mode=mode, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        r = G.solve(b, x, mode=mode, rtol=rtol, maxit=maxit)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, r, x


IR_INNER = 12   # FP32 CG steps of the first refinement step (at most, in later ones)


def workload_mixed(a):
    """Mixed precision on the 3D warped problem with 8^3 hexes at p = 16 (2,146,689 nodes),
    f ~ U[-1,1] (seed 0), all to 1e-10: the all-FP64 PCG, the FP32 V-cycle inside FP64 PCG, and
    iterative refinement (FP64 residuals, IR_INNER steps of FP32 CG with the FP32 V-cycle per
    refinement step). Errors against a tight (1e-13) FP64 solve on the GPU and against the
    oracle's tight solution at its sample nodes."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    out = {}
    sols = {}
    for name, prec, mode in (("f64", "f64", "pcg"), ("f32", "f32", "pcg"), ("f32_ir", "f32", "ir")):
        # order halving 16 -> 1, the exact solve on the first-order level (8^3: 343 unknowns)
        prob = inputs.warped_var3d(nelem=8, order=16, vcycle_prec=prec, f_seed=0,
                                   coarse_unknowns=inputs.COARSE_UNKNOWNS)
        G = gllmg.Problem.from_inputs(prob, ir_inner=IR_INNER if mode == "ir" else 0)
        b = G.rhs(torch.from_numpy(prob.nodal_rhs()).cuda())
        t, r, x = _solve_timed(G, b, a.steps, a.warmup, 1e-10, 500, mode)
        out[name] = {"time_to_solution_ms": t * 1e3, "pcg_iterations": r.iters,
                     "relres_true": r.relres_true}
        if mode == "ir":
            out[name]["refinement_steps"] = len(r.history) - 1
            out[name]["inner_cg_steps_first_refinement"] = IR_INNER
        sols[name] = x.clone()
        if name == "f64":
            xt = torch.zeros_like(b)
            G.solve(b, xt, rtol=1e-13, maxit=500)
            sols["tight"] = xt
        G.close()
    u = sols["tight"]
    # the oracle's tight (rtol 1e-13) FP64 solution at its seeded sample nodes, written by
    # tests/golden/make_golden.py from the CPU oracle
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                                       "golden", "warped_8cubed_p16.json")))
    idx = torch.tensor(gold["sample_nodes"], device="cuda")
    xo = torch.tensor(gold["x_tight_sample"], dtype=torch.float64, device="cuda")
    for name in ("f64", "f32", "f32_ir"):
        out[name]["rel_error_vs_fp64_tight"] = float(torch.linalg.norm(sols[name] - u) /
                                                     torch.linalg.norm(u))
        xs = sols[name][idx]
        out[name]["rel_error_vs_oracle_samples"] = float(torch.linalg.norm(xs - xo) / torch.linalg.norm(xo))
        out[name]["rel_error_vs_oracle_norm2"] = abs(float(torch.linalg.norm(sols[name])) -
                                                     gold["x_tight_norm2"]) / gold["x_tight_norm2"]
    out["speedup_mixed_over_fp64"] = out["f64"]["time_to_solution_ms"] / out["f32"]["time_to_solution_ms"]
    out["speedup_ir_over_fp64"] = out["f64"]["time_to_solution_ms"] / out["f32_ir"]["time_to_solution_ms"]
    return {"workload": "mixed: 3D warped var 8^3 p=16, N=2146689, p-multigrid 16->8->4->2->1 "
                        "with the exact solve on 8^3 at p=1, to 1e-10", **out}


def workload_batch(a):
    """256 independent 3D problems on 4^3 hexes, p uniform in {2,4,8,16}, mu = exp(random
    Fourier field), f ~ U[-1,1], FP32 V-cycle + FP64 PCG, all solved by one batched call."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    probs = inputs.batched_problems(seed=0, count=a.batch_count)
    t0 = time.perf_counter()
    Gs, bs = [], []
    for pr in probs:
        G = gllmg.Problem.from_inputs(pr)
        Gs.append(G)
        bs.append(G.rhs(torch.from_numpy(pr.nodal_rhs()).cuda()))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(Gs, bs, xs, rtol=1e-10)
    torch.cuda.synchronize()
    best = None
    for _ in range(max(1, a.steps)):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = gllmg.batch_solve(Gs, bs, xs, rtol=1e-10)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
    nodes = sum(G.nnodes(0) for G in Gs)
    ok = sum(r.converged for r in res)
    for G in Gs:
        G.close()
    return {"workload": f"batch: {len(probs)} x 3D 4^3 hexes, p in {{2,4,8,16}}, FP32 V-cycle + FP64 PCG to 1e-10",
            "batch_time_ms": best * 1e3, "solves_per_s": len(probs) / best,
            "gdof_solves_per_s": nodes / best / 1e9, "total_nodes": nodes, "converged": ok,
            "setup_s": t_setup, "max_iters": max(r.iters for r in res)}


def workload_serve(a):
    """Poisson-arrival stream (mean a.serve_rate req/s; 200 by default, the serving workload's
    rate, which is beyond the measured capacity of about 150 solves/s, so the queue grows) of
    mixed 2D/3D solves to 1e-8 under an HBM budget; p50/p99 latency and solves/s over the first
    a.serve_s seconds of arrivals."""
    from paper_1402_5938_amd import inputs
    from paper_1402_5938_amd.serve import Server
    trace = inputs.serving_trace(seed=0, rate=a.serve_rate, duration_s=a.serve_s)
    if a.warmup > 0:
        # not reported: the first launch of each kernel in a process loads its code and the
        # allocator's pools grow, so 1 s of another trace (seed 1) runs first, on its own server
        ws = Server(hbm_budget=int(a.hbm_gb * 2 ** 30), max_active=64)
        ws.run(inputs.serving_trace(seed=1, rate=a.serve_rate, duration_s=1.0), time_scale=1.0,
               max_wall_s=80.0)
        ws.close()
    srv = Server(hbm_budget=int(a.hbm_gb * 2 ** 30), max_active=64)
    rep = srv.run(trace, time_scale=1.0, max_wall_s=a.serve_s * 20 + 60)
    srv.close()
    return {"workload": f"serve: {len(trace)} requests over {a.serve_s} s at {a.serve_rate:g} req/s, "
                        f"budget {a.hbm_gb} GiB", **rep}


def workload_requests(a):
    """The serving stream's requests (seed 0, 200 req/s) one at a time, without the server: the
    first a.requests of them set up, then solved alone (FP32 V-cycle in FP64 PCG to 1e-8), after
    one untimed pass over the same requests (set up, solved, destroyed) so that every kernel's
    code is loaded. Per-request setup (hierarchy, geometry, diagonal, Lanczos bounds, coarse
    inverse) and solve times: the GPU work a served request costs when nothing overlaps it."""
    import numpy as np
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    probs = [r.problem for r in inputs.serving_trace(seed=0, rate=200.0, duration_s=60.0,
                                                     max_requests=a.requests)]

    def rhs(G, p):
        return G.rhs(torch.from_numpy(p.nodal_rhs()).cuda())

    for p in probs:
        G = gllmg.Problem.from_inputs(p)
        G.solve(rhs(G, p), rtol=p.rtol, maxit=p.maxit)
        G.close()
    torch.cuda.synchronize()
    Gs, t_set, t_sol, its = [], [], [], []
    for p in probs:
        t0 = time.perf_counter()
        Gs.append(gllmg.Problem.from_inputs(p))
        torch.cuda.synchronize()
        t_set.append(time.perf_counter() - t0)
    for G, p in zip(Gs, probs):
        b = rhs(G, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = G.solve(b, rtol=p.rtol, maxit=p.maxit)
        torch.cuda.synchronize()
        t_sol.append(time.perf_counter() - t0)
        its.append(r.iters)
        assert r.converged, (p.name, r)
    nodes = [G.nnodes(0) for G in Gs]
    for G in Gs:
        G.close()
    ms = lambda v: round(1e3 * float(v), 3)  # noqa: E731
    return {"workload": f"requests: the first {len(probs)} requests of the serving stream, set up "
                        "and solved one at a time", "requests": len(probs),
            "total_nodes": int(sum(nodes)), "setup_total_s": float(sum(t_set)),
            "solve_total_s": float(sum(t_sol)), "setup_mean_ms": ms(np.mean(t_set)),
            "setup_median_ms": ms(np.median(t_set)), "setup_max_ms": ms(np.max(t_set)),
            "solve_mean_ms": ms(np.mean(t_sol)), "solve_median_ms": ms(np.median(t_sol)),
            "solve_max_ms": ms(np.max(t_sol)), "mean_iters": float(np.mean(its))}


SMOOTHER_CASES = {"chebyshev": (4, 4), "jacobi": (3, 3), "ssor": (2, 1), "l1jacobi": (3, 3),
                  "blockjacobi": (3, 3)}


def workload_smoothers(a):
    """The benchmark problem (3D warped, mu = exp(4.6 sx sy sz), f = 1, a.nelem^3 hexes at
    p = a.order) solved to 1e-10 by FP64 PCG with the p-multigrid V-cycle and each smoother the
    paper compares (§4.3, §4.4.3: Chebyshev(4,4) of the workload, Jacobi(3,3), SSOR(2,1),
    l1-Jacobi(3,3), block Jacobi(3,3)): time to solution, iterations, the time of one
    fine-level smoothing step (HIP events on the launch stream) and of one V-cycle."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    prob = inputs.warped_var3d(nelem=a.nelem, order=a.order)
    rows = []
    for name in a.smoothers.split(","):
        pre, post = SMOOTHER_CASES[name]
        cfg = gllmg.make_config(3, prob.nelem, prob.order, "p", name, pre, nu_post=post)
        t0 = time.perf_counter()
        G = gllmg.Problem(cfg, prob.map, prob.mu)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        b = G.rhs(G.eval_field(prob.f))
        t, r, x = _solve_timed(G, b, a.steps, a.warmup, prob.rtol, prob.maxit)
        # one smoothing step on the finest level and one V-cycle
        xs = torch.zeros_like(b)
        z = torch.empty_like(b)
        G.smooth(b, xs, 1, 0, zero_guess=False)
        G.vcycle(b, z)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        G.smooth(b, xs, 1, 0, zero_guess=False)
        e[1].record()
        G.vcycle(b, z)
        e[2].record()
        torch.cuda.synchronize()
        rows.append({"smoother": name, "nu_pre": pre, "nu_post": post, "pcg_iterations": r.iters,
                     "converged": r.converged, "time_to_solution_ms": t * 1e3,
                     "smoothing_step_us": e[0].elapsed_time(e[1]) * 1e3,
                     "vcycle_ms": e[1].elapsed_time(e[2]), "setup_s": t_setup,
                     "relres_true": r.relres_true})
        G.close()
        torch.cuda.empty_cache()
    return {"workload": f"smoothers: 3D warped var {a.nelem}^3 hexes p={a.order}, FP64 PCG to 1e-10",
            "nodes": inputs.node_count(prob.nelem, prob.order), "cases": rows}


def workload_lowprec(a):
    """The benchmark problem (3D warped, a.nelem^3 hexes at p = a.order, f = 1) solved to 1e-10
    by FP64 PCG preconditioned by the p-multigrid V-cycle and by the first-order hierarchy's
    preconditioner (k sweeps of the V-cycle of first-order cells on the order-p nodes, k = 1, 2,
    4): iterations, time to solution, time of one preconditioner application."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    prob = inputs.warped_var3d(nelem=a.nelem, order=a.order)
    rows = []
    for hier, k in (("p", 1), ("low", 1), ("low", 2), ("low", 4)):
        cfg = gllmg.make_config(3, prob.nelem, prob.order, hier, "chebyshev", 4, low_cycles=k)
        t0 = time.perf_counter()
        G = gllmg.Problem(cfg, prob.map, prob.mu)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        b = G.rhs(G.eval_field(prob.f))
        t, r, _ = _solve_timed(G, b, a.steps, a.warmup, prob.rtol, prob.maxit)
        z = torch.empty_like(b)
        G.vcycle(b, z)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        G.vcycle(b, z)
        e1.record()
        torch.cuda.synchronize()
        rows.append({"hierarchy": hier, "low_cycles": k if hier == "low" else None,
                     "levels": G.nlevels, "pcg_iterations": r.iters, "converged": r.converged,
                     "time_to_solution_ms": t * 1e3, "precond_ms": e0.elapsed_time(e1),
                     "setup_s": t_setup})
        G.close()
        torch.cuda.empty_cache()
    return {"workload": f"hierarchies: 3D warped var {a.nelem}^3 hexes p={a.order}, FP64 PCG to 1e-10",
            "cases": rows}


def apply_flops_gauss(dim, ne, p):
    """Flops of one Gauss-quadrature product (q = p + 1 points): the five sum-factorized passes
    take 16 n^4 (3D) or 6 n^3 (2D) multiply-adds per element, the pointwise factors 9 n^3 (4 n^2)."""
    n = p + 1
    E = 1
    for v in ne:
        E *= v
    return E * (32 * n ** 4 + 18 * n ** 3) if dim == 3 else E * (12 * n ** 3 + 8 * n ** 2)


def workload_gauss(a):
    """The warped variable-coefficient problem (16^3 hexes at p = 8 and 8^3 at p = 16, f = 1)
    with the collocated GLL and the Gauss-quadrature operator: FP64 PCG time to 1e-10,
    iterations, and one fine-level product (median of 50, HIP events) against the HBM
    roofline (algorithmic bytes: 6 factors per quadrature point, x and y once)."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    rows = []
    for ne, p in ((16, 8), (8, 16)):
        prob = inputs.warped_var3d(nelem=ne, order=p)
        for quad in ("gll", "gauss"):
            cfg = gllmg.make_config(3, prob.nelem, p, "p", "chebyshev", 4, quadrature=quad)
            G = gllmg.Problem(cfg, prob.map, prob.mu)
            b = G.rhs(G.eval_field(prob.f))
            t, r, _ = _solve_timed(G, b, a.steps, a.warmup, prob.rtol, prob.maxit)
            N = G.nnodes(0)
            x = torch.from_numpy(inputs.uniform_nodal(99, N)).cuda()
            y = torch.empty_like(x)
            us = _median_apply_us(G, x, y, 50)
            nb = apply_bytes(3, prob.nelem, p, N, 8)
            fl = apply_flops_gauss(3, prob.nelem, p) if quad == "gauss" else apply_flops(3, prob.nelem, p)
            rows.append({"nelem": ne, "order": p, "quadrature": quad, "nodes": N,
                         "pcg_iterations": r.iters, "time_to_solution_ms": t * 1e3,
                         "apply_us": us, "achieved_gbs": nb / (us * 1e-6) / 1e9,
                         "frac_hbm": nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                         "tflops": fl / (us * 1e-6) / 1e12})
            G.close()
            torch.cuda.empty_cache()
    return {"workload": "quadrature: 3D warped var, GLL collocation vs Gauss (p+1 points), FP64 PCG to 1e-10",
            "cases": rows}


SWEEP_CASES = [(3, 256, 1), (3, 128, 2), (3, 64, 4), (3, 40, 6), (3, 32, 8), (3, 20, 12), (3, 16, 16),
               (2, 512, 8)]


def _median_apply_us(G, x, y, reps):
    import torch
    for _ in range(10):
        G.apply(x, y)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        G.apply(x, y)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    ts.sort()
    return ts[len(ts) // 2]


def workload_sweep(a):
    """Operator products at working sets of about 1 GB and more (beyond the 256 MB Infinity
    Cache), FP64 and FP32, against the 8 TB/s nominal and the bandwidth of the library's own
    streaming copy (gllmg_stream_copy, 1 GiB):
    the median of 50 HIP-event-timed products after 10 warm-ups, per case."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    copy_gbs = stream_copy_gbs()
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(4.6)
    rows = []
    for dim, ne, p in SWEEP_CASES:
        for prec in ("f64", "f32"):
            cfg = gllmg.make_config(dim, (ne,) * dim, p, "p", max_levels=1, vcycle_prec=prec,
                                    eig_steps=1)
            G = gllmg.Problem(cfg, mp, mu)
            N = G.nnodes(0)
            dt = torch.float64 if prec == "f64" else torch.float32
            x = torch.from_numpy(inputs.uniform_nodal(99, N)).to(device="cuda", dtype=dt)
            y = torch.empty_like(x)
            us = _median_apply_us(G, x, y, 50)
            nb = apply_bytes(dim, (ne,) * dim, p, N, 8 if prec == "f64" else 4)
            gbs = nb / (us * 1e-6) / 1e9
            rows.append({"dim": dim, "nelem": ne, "order": p, "prec": prec, "nodes": N,
                         "algorithmic_bytes": nb, "apply_us": us, "gdof_s": N / us * 1e-3,
                         "achieved_gbs": gbs, "frac_nominal": gbs / HBM_PEAK_GBS,
                         "frac_copy": gbs / copy_gbs})
            G.close()
            del x, y
            torch.cuda.empty_cache()
    return {"workload": "apply sweep at >= 1 GB working sets (3D p = 1..16, 2D 512^2 p = 8)",
            "copy_gbs": copy_gbs, "cases": rows}


def workload_apply(a):
    """Operator products alone on the benchmark problem, for counter runs: 5 untimed products,
    a.apply_reps products timed with HIP events on the launch stream, then 3 plain device
    copies of 256 MiB (the calibration kernel for the HBM byte counters)."""
    import torch

    from paper_1402_5938_amd import gllmg, inputs
    prob = inputs.warped_var3d(nelem=a.nelem, order=a.order, vcycle_prec=a.prec)
    G = gllmg.Problem.from_inputs(prob)
    N = G.nnodes(0)
    dt = torch.float64 if a.prec == "f64" else torch.float32
    xr = torch.from_numpy(inputs.uniform_nodal(99, N)).cuda().to(dt)
    y = torch.empty_like(xr)
    for _ in range(5):
        G.apply(xr, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.apply_reps):
        G.apply(xr, y)
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / a.apply_reps * 1e-3
    src = torch.ones(CALIB_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    nbytes = apply_bytes(3, prob.nelem, prob.order, N, 8 if a.prec == "f64" else 4)
    G.close()
    return {"workload": f"apply: 3D warped var {a.nelem}^3 hexes p={a.order} {a.prec}, N={N}, "
                        f"{a.apply_reps} timed products, then 3 copies of {CALIB_COPY_BYTES} bytes",
            "apply_us": t_apply * 1e6, "algorithmic_bytes": nbytes,
            "achieved_gbs": nbytes / t_apply / 1e9}


def extra_workloads(a):
    """The other workloads measured in the same run, in summary: the 8^3 p = 16 solve in FP64,
    mixed precision and iterative refinement (errors against the oracle's samples), the batch
    of 256 problems, and the Poisson-arrival server at 200 req/s. A workload that fails is
    reported with its error instead of its figures."""
    import torch
    out = {}
    for name, fn, keep in (
            ("mixed_8cubed_p16", workload_mixed,
             lambda r: {k: r[k] for k in ("f64", "f32", "f32_ir", "speedup_mixed_over_fp64",
                                          "speedup_ir_over_fp64") if k in r}),
            ("batch_256_4cubed", workload_batch,
             lambda r: {k: r[k] for k in ("batch_time_ms", "solves_per_s", "converged", "max_iters")}),
            ("serve_200rps", workload_serve,
             lambda r: {k: r[k] for k in r if k != "workload"})):
        t0 = time.perf_counter()
        try:
            out[name] = keep(fn(a))
        except Exception as e:  # reported, not raised: the headline line is printed regardless
            out[name] = {"error": f"{type(e).__name__}: {e}"}
        out[name]["wall_s"] = time.perf_counter() - t0
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="config2", choices=["config2", "mixed", "batch", "serve", "apply", "sweep",
                                                          "smoothers", "gauss", "lowprec", "requests"])
    ap.add_argument("--smoothers", default="chebyshev,jacobi,ssor")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--serve-s", type=float, default=2.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--requests", type=int, default=150, help="requests workload: how many requests")
    ap.add_argument("--hbm-gb", type=float, default=64.0)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=50)
    ap.add_argument("--prec", default="f64", choices=["f64", "f32"], help="apply workload: product precision")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="config2: leave out the mixed-precision, batched and serving workloads")
    ap.add_argument("--nelem", type=int, default=16)
    ap.add_argument("--order", type=int, default=8)
    ap.add_argument("--levels", type=int, default=0, help="config2: keep the finest k levels (0: all)")
    ap.add_argument("--coarse-unknowns", type=int, default=4096,
                    help="config2: stop at the first first-order level with at most this many "
                         "interior unknowns (0: coarsen to the bottom)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported: the solver and "
              "its benchmarks use a single device", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1402_5938_amd import gllmg, inputs

    torch.cuda.set_device(0)
    if a.workload != "config2":
        fn = {"mixed": workload_mixed, "batch": workload_batch, "serve": workload_serve,
              "apply": workload_apply, "sweep": workload_sweep,
              "smoothers": workload_smoothers, "gauss": workload_gauss,
              "lowprec": workload_lowprec, "requests": workload_requests}[a.workload]
        print(json.dumps(fn(a)))
        return
    # the configuration's order sequence 8 -> 4 -> 2 -> 1, the exact solve on the first-order
    # level (16^3 hexes: 3375 unknowns)
    prob = inputs.warped_var3d(nelem=a.nelem, order=a.order, max_levels=a.levels,
                               coarse_unknowns=a.coarse_unknowns)
    t_setup = time.perf_counter()
    G = gllmg.Problem.from_inputs(prob)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    N = G.nnodes(0)
    f = G.eval_field(prob.f)
    b = G.rhs(f)
    x = torch.zeros_like(b)

    for _ in range(a.warmup):
        x.zero_()
        G.solve(b, x, rtol=prob.rtol, maxit=prob.maxit)
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        x.zero_()
        r = G.solve(b, x, rtol=prob.rtol, maxit=prob.maxit)
        iters.append(r.iters)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / a.steps * 1e3
    assert r.converged and r.relres_true < 1e-9, r

    # operator product on the finest level, HIP events on the launch stream
    xr = torch.from_numpy(inputs.uniform_nodal(99, N)).cuda()
    y = torch.empty_like(xr)
    for _ in range(5):
        G.apply(xr, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.apply_reps):
        G.apply(xr, y)
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / a.apply_reps * 1e-3
    nbytes = apply_bytes(3, prob.nelem, prob.order, N, 8)
    achieved = nbytes / t_apply / 1e9
    copy_gbs = stream_copy_gbs()
    big = apply_beyond_cache()
    big["frac"] = big["achieved"] / HBM_PEAK_GBS
    big["frac_copy"] = big["achieved"] / copy_gbs

    out = {
        "metric": "GDOF/s operator apply; time-to-1e-10 residual; solves/s + p99 latency",
        "value": N / (ms * 1e-3) / 1e9,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D warped var-coefficient Poisson, {a.nelem}^3 hexes, p={a.order}, "
                               f"N={N}; FP64 p-multigrid "
                               + "->".join(str(lv.order) for lv in G.levels)
                               + f" with the exact solve on {a.nelem}^3 at p={G.levels[-1].order} "
                               f"({G.levels[-1].ninterior} unknowns), Chebyshev(4,4), PCG to 1e-10; "
                               "value = N / time-to-solution",
                   "levels": G.nlevels,
                   "nodes": N, "pcg_iterations": iters[-1], "time_to_solution_ms": ms,
                   "solves_per_s": 1e3 / ms, "setup_s": t_setup,
                   "apply_gdof_s": N / t_apply / 1e9, "apply_us": t_apply * 1e6},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(a.nelem, a.order),
                     "kernel": "operator apply (element kernel + face-sum kernel), finest level",
                     "algorithmic_bytes": nbytes, "flops": apply_flops(3, prob.nelem, prob.order),
                     "copy_gbs": copy_gbs, "frac_copy": achieved / copy_gbs,
                     "beyond_cache": big},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    G.close()
    if not a.no_extra:
        out["workloads"] = extra_workloads(a)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
