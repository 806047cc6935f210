"""The batched and served workloads against the CPU oracle (expected values written by
tests/golden/make_golden.py from the oracle alone).

Batched: one problem of each order class p in {2, 4, 8, 16} of the 256-problem batch (4^3 hexes,
random-Fourier mu), each with a partner of the same class so that every class runs as a launch
group of two through gllmg_batch_solve, in the batch's own mode (FP32 V-cycle inside FP64 PCG,
rtol 1e-10). Served: four requests of a seeded serving trace (3D 2^3 p = 8, 2D 12^2 p = 16,
3D 8^3 p = 6, 3D 3^3 p = 12; FP32 V-cycle, rtol 1e-8) taken through the continuous-batching
server among other requests.

Bars for a mixed-precision solve against the oracle's FP64 solves: the recursive residual
reaches rtol and the true FP64 residual 2 rtol; at most 3 iterations more than the oracle's
FP64 V-cycle PCG; the solution's error against the oracle's tight solution (rtol 1e-13), over
the stored sample nodes, at most 100 times the oracle's own error at rtol (and at most 1e-8 /
1e-6 at rtol 1e-10 / 1e-8). The same problems with the FP64 V-cycle must reproduce the oracle
exactly as the parity bar states: lambda_max per level 1e-10, equal iteration counts, residual
history 1e-8, solution samples 1e-8."""

import glob
import json
import os

import numpy as np
import pytest

from paper_1402_5938_amd import inputs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BATCH_SEED, BATCH_COUNT = 0, 256
SERVE_SEED, SERVE_RATE, SERVE_SPAN = 7, 200.0, 30.0


def _gold(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    return json.load(open(path))


def _check_mixed(res, x, gold, rtol):
    idx = np.array(gold["sample_nodes"])
    xt = np.array(gold["x_tight_sample"])
    err = np.linalg.norm(x.cpu().numpy()[idx] - xt) / np.linalg.norm(xt)
    cap = 1e-8 if rtol <= 1e-10 else 1e-6
    assert res.converged and res.relres <= rtol and res.relres_true <= 2 * rtol, res
    assert res.iters <= gold["iters"] + 3, (res.iters, gold["iters"])
    assert err <= min(max(100 * gold["err_vs_tight"], 1e-12), cap), (err, gold["err_vs_tight"])
    return err


def _check_fp64(G, res, x, gold):
    for l, lam in enumerate(gold["lmax"]):
        assert abs(G.levels[l].lmax - lam) <= 1e-10 * lam, (l, G.levels[l].lmax, lam)
    assert res.converged and res.iters == gold["iters"], (res.iters, gold["iters"])
    h, hg = np.array(res.history), np.array(gold["history"])
    assert np.max(np.abs(h - hg) / hg) <= 1e-8
    idx = np.array(gold["sample_nodes"])
    xg = np.array(gold["x_sample"])
    assert np.max(np.abs(x.cpu().numpy()[idx] - xg)) <= 1e-8 * np.max(np.abs(xg))


def _batch_pairs():
    probs = inputs.batched_problems(seed=BATCH_SEED, count=BATCH_COUNT)
    names = sorted(os.path.basename(p)[:-5] for p in glob.glob(os.path.join(GOLDEN, "batch_4cubed_p*_i*.json")))
    out = []
    for name in names:
        i = int(name.rsplit("_i", 1)[1])
        partner = next(j for j in range(i + 1, len(probs)) if probs[j].order == probs[i].order)
        out.append((name, i, partner))
    return probs, out


def test_batch_classes_against_oracle():
    import torch

    from paper_1402_5938_amd import gllmg
    probs, pairs = _batch_pairs()
    if not pairs:
        pytest.skip("no batch goldens")
    handles, bs, which = [], [], []
    for name, i, j in pairs:
        for k in (i, j):
            pb = probs[k]
            P = gllmg.Problem.from_inputs(pb)
            handles.append(P)
            bs.append(P.rhs(torch.from_numpy(pb.nodal_rhs()).cuda()))
            which.append(name if k == i else None)
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(handles, bs, xs, rtol=1e-10, maxit=500)
    torch.cuda.synchronize()
    for k, name in enumerate(which):
        assert res[k].converged, (k, res[k])
        if name is None:
            continue
        gold = _gold(name)
        assert handles[k].nnodes(0) == gold["nnodes"]
        assert [[list(lv.nelem), lv.order] for lv in handles[k].levels] == gold["levels"]
        err = _check_mixed(res[k], xs[k], gold, 1e-10)
        print(f"{name}: batch (FP32 V-cycle) iters {res[k].iters} (oracle FP64 {gold['iters']}), "
              f"error vs tight {err:.2e} (oracle {gold['err_vs_tight']:.2e})")
    for P in handles:
        P.close()


@pytest.mark.parametrize("name", ["batch_4cubed_p2_i4", "batch_4cubed_p4_i6", "batch_4cubed_p8_i1",
                                  "batch_4cubed_p16_i0"])
def test_batch_problem_fp64_vcycle_equals_oracle(name):
    """The same problem with the FP64 V-cycle: the oracle's algorithm exactly."""
    import torch

    from paper_1402_5938_amd import gllmg
    gold = _gold(name)
    i = int(name.rsplit("_i", 1)[1])
    pb = inputs.batched_problems(seed=BATCH_SEED, count=BATCH_COUNT)[i]
    pb.vcycle_prec = "f64"
    G = gllmg.Problem.from_inputs(pb)
    b = G.rhs(torch.from_numpy(pb.nodal_rhs()).cuda())
    assert abs(torch.linalg.norm(b).item() - gold["b_norm2"]) <= 1e-13 * gold["b_norm2"]
    x = torch.zeros_like(b)
    r = G.solve(b, x, rtol=1e-10, maxit=500)
    _check_fp64(G, r, x, gold)
    G.close()


SERVE_NAMES = ["serve_req1", "serve_req4", "serve_req7", "serve_req39"]


def test_served_requests_against_oracle():
    """The golden requests, served among the other requests of the trace up to the last golden
    one (small ones only), with host-drawn right-hand sides."""
    from paper_1402_5938_amd.serve import Server, request_footprint
    golds = {n: _gold(n) for n in SERVE_NAMES}
    rids = [int(n[len("serve_req"):]) for n in SERVE_NAMES]
    full = inputs.serving_trace(seed=SERVE_SEED, rate=SERVE_RATE, duration_s=SERVE_SPAN)
    trace = [r for r in full[:max(rids) + 1] if r.rid in rids or r.problem.nnodes <= 60_000]
    budget = sum(sorted(request_footprint(r.problem) for r in trace)[-4:])
    srv = Server(hbm_budget=budget, max_active=8, keep_solutions=True, host_rhs=True)
    rep = srv.run(trace, time_scale=0.05)
    srv.close()
    assert rep["completed"] == len(trace), rep
    for n, rid in zip(SERVE_NAMES, rids):
        rec = srv.records[rid]
        gold = golds[n]
        assert rec.nnodes == gold["nnodes"]
        x = srv.solutions[rid]
        idx = np.array(gold["sample_nodes"])
        xt = np.array(gold["x_tight_sample"])
        err = np.linalg.norm(x.cpu().numpy()[idx] - xt) / np.linalg.norm(xt)
        assert rec.converged and rec.relres_true <= 2e-8, (n, rec)
        assert rec.iters <= gold["iters"] + 3, (n, rec.iters, gold["iters"])
        assert err <= min(max(100 * gold["err_vs_tight"], 1e-12), 1e-6), (n, err, gold["err_vs_tight"])
        print(f"{n}: served iters {rec.iters} (oracle FP64 {gold['iters']}), error vs tight "
              f"{err:.2e} (oracle {gold['err_vs_tight']:.2e})")


@pytest.mark.parametrize("name", SERVE_NAMES)
def test_served_request_fp64_vcycle_equals_oracle(name):
    import torch

    from paper_1402_5938_amd import gllmg
    gold = _gold(name)
    rid = int(name[len("serve_req"):])
    pb = inputs.serving_trace(seed=SERVE_SEED, rate=SERVE_RATE, duration_s=SERVE_SPAN)[rid].problem
    pb.vcycle_prec = "f64"
    G = gllmg.Problem.from_inputs(pb)
    b = G.rhs(torch.from_numpy(pb.nodal_rhs()).cuda())
    x = torch.zeros_like(b)
    r = G.solve(b, x, rtol=pb.rtol, maxit=pb.maxit)
    _check_fp64(G, r, x, gold)
    G.close()
