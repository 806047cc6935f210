"""Continuous-batching server: admission ledger on the CPU; on the GPU, every request's result
is bitwise the same alone and in the mix, and admission never exceeds the HBM budget."""

import numpy as np
import pytest

from paper_1402_5938_amd import inputs


def test_ledger_admission():
    from paper_1402_5938_amd.serve import HbmLedger
    L = HbmLedger(100)
    assert L.try_reserve(60)
    assert not L.try_reserve(50)
    assert L.try_reserve(40)
    assert L.peak == 100
    L.release(60)
    assert L.try_reserve(50) and L.used == 90
    with pytest.raises(AssertionError):
        L.release(1000)


def test_footprint_is_plan_plus_vectors():
    from paper_1402_5938_amd import gllmg
    from paper_1402_5938_amd.serve import request_config, request_footprint
    prob = inputs.serving_trace(seed=3, rate=200, duration_s=0.1)[0].problem
    _, ws = gllmg.plan(request_config(prob))
    assert request_footprint(prob) == ws + 256 + 24 * prob.nnodes


def test_trace_is_seeded_and_poisson():
    a = inputs.serving_trace(seed=5, rate=200.0, duration_s=5.0)
    b = inputs.serving_trace(seed=5, rate=200.0, duration_s=5.0)
    assert [r.problem.name for r in a] == [r.problem.name for r in b]
    gaps = np.diff([r.arrival_s for r in a])
    assert abs(gaps.mean() - 1 / 200.0) < 0.25 / 200.0
    assert {r.problem.dim for r in a} == {2, 3}
    assert {r.problem.order for r in a} <= {4, 6, 8, 12, 16}


def _small_trace(n=10, seed=7, max_nodes=120_000):
    out = []
    for r in inputs.serving_trace(seed=seed, rate=200.0, duration_s=30.0):
        if r.problem.nnodes <= max_nodes:
            out.append(r)
        if len(out) == n:
            break
    return out


@pytest.mark.gpu
def test_server_same_alone_and_in_mix():
    import torch
    from paper_1402_5938_amd import gllmg
    from paper_1402_5938_amd.serve import Server, request_config, request_footprint
    trace = _small_trace()
    fps = sorted(request_footprint(r.problem) for r in trace)
    budget = sum(fps[-3:])                      # forces requests to wait for memory
    srv = Server(hbm_budget=budget, max_active=6, keep_solutions=True)
    rep = srv.run(trace, time_scale=0.05)
    srv.close()
    assert rep["completed"] == len(trace), rep
    assert srv.ledger.peak <= budget
    assert srv.ledger.used == 0
    for req in trace:
        rec = srv.records[req.rid]
        P = gllmg.Problem(request_config(req.problem), req.problem.map, req.problem.mu)
        b = P.rhs(req.problem.nodal_rhs_device())
        x = torch.zeros_like(b)
        res = P.solve(b, x, rtol=req.problem.rtol, maxit=req.problem.maxit)
        assert res.iters == rec.iters and res.converged
        assert torch.equal(x, srv.solutions[req.rid]), req.rid
        P.close()
    assert rep["p99_latency_s"] >= rep["p50_latency_s"] > 0


def _same_shape_trace():
    """Three copies (own right-hand side, own coefficient phase) of each of three small served
    shapes, all arriving at once, and two requests of other shapes."""
    import dataclasses
    base = [r for r in inputs.serving_trace(seed=11, rate=200.0, duration_s=30.0)
            if r.problem.nnodes <= 60_000]
    shapes, seen = [], set()
    for r in base:
        key = (r.problem.dim, r.problem.nelem, r.problem.order)
        if key not in seen:
            seen.add(key)
            shapes.append(r.problem)
    out, rid = [], 0
    for pb in shapes[:3]:
        for k in range(3):
            mu = dict(pb.mu)
            mu["param"] = list(pb.mu["param"])
            mu["param"][1] = (mu["param"][1] + 0.1 * k) % 1.0
            prob = dataclasses.replace(pb, name=f"{pb.name}#{k}", mu=mu, f_seed=pb.f_seed + k)
            out.append(inputs.Request(rid=rid, arrival_s=0.0, problem=prob))
            rid += 1
    for pb in shapes[3:5]:
        out.append(inputs.Request(rid=rid, arrival_s=0.0, problem=pb))
        rid += 1
    return out


@pytest.mark.gpu
def test_server_groups_same_shape_requests():
    """Same-shape requests ready together are solved as one launch group; every result is
    bitwise the one the request gets alone."""
    import torch
    from paper_1402_5938_amd import gllmg
    from paper_1402_5938_amd.serve import Server, request_config
    trace = _same_shape_trace()
    srv = Server(hbm_budget=64 << 30, max_active=32, keep_solutions=True, group_window_s=30.0)
    rep = srv.run(trace)
    srv.close()
    assert rep["completed"] == len(trace), rep
    assert rep["grouped_requests"] == 9, rep
    assert sorted(srv.records[r.rid].grouped for r in trace) == [1, 1] + [3] * 9
    for req in trace:
        rec = srv.records[req.rid]
        P = gllmg.Problem(request_config(req.problem), req.problem.map, req.problem.mu)
        b = P.rhs(req.problem.nodal_rhs_device())
        x = torch.zeros_like(b)
        res = P.solve(b, x, rtol=req.problem.rtol, maxit=req.problem.maxit)
        assert res.iters == rec.iters and res.converged
        assert torch.equal(x, srv.solutions[req.rid]), req.rid
        P.close()
