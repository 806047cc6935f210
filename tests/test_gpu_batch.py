"""Mixed precision, the non-blocking solve and batched solves, on the GPU through the C ABI.

* FP32 V-cycle pieces against the FP64 oracle at FP32 tolerance; the mixed-precision PCG
  (FP32 V-cycle, FP64 outer) converges to 1e-10 and its solution matches the oracle's tight
  FP64 solve to the accuracy the tolerance allows.
* gllmg_solve_begin/_poll/_end gives bitwise the same iterates as gllmg_solve.
* A batch of problems of mixed dimension, order and precision gives, for every problem,
  bitwise the result of the same problem solved alone.
"""

import numpy as np
import pytest

from gpu_helpers import build_pair, rel_err, random_vec, to_dev, to_np
from oracle import fem, mg
from paper_1402_5938_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p", [8, 12])
def test_fp32_vcycle_pieces_against_oracle(p):
    import torch
    G, H = build_pair(3, (2, 2, 2), p, hierarchy="p", vcycle_prec="f32")
    for l, lv in enumerate(H.levels[:-1]):
        G.set_lmax(l, lv.lmax)
    m = H.fine.mesh
    b = random_vec(m.N, 1) * m.interior
    x = to_dev(np.zeros(m.N), torch.float32)
    G.smooth(to_dev(b, torch.float32), x, 4, 0, zero_guess=True)
    assert rel_err(to_np(x), H.smooth(0, b, None, steps=4)) <= 1e-5
    e = to_np(G.vcycle(to_dev(b, torch.float32)))
    assert rel_err(e, H.vcycle(b)) <= 1e-5
    for l in range(len(H.levels) - 1):
        c = H.levels[l + 1]
        xc = random_vec(c.mesh.N, 30 + l)
        xf = to_np(G.prolong(to_dev(xc, torch.float32), l))
        assert rel_err(xf, H.levels[l].to_coarse.prolong(xc)) <= 1e-6
    G.close()


@pytest.mark.parametrize("dim,ne,p", [(3, (2, 2, 2), 8), (3, (4, 4, 4), 4), (2, (6, 6), 16)])
def test_mixed_precision_pcg(dim, ne, p):
    """FP32 V-cycle inside FP64 PCG reaches 1e-10; the solution agrees with the oracle's FP64
    solve to 1e-13 within the error that a 1e-10 residual allows."""
    import torch
    G, H = build_pair(dim, ne, p, hierarchy="p", vcycle_prec="f32")
    m = H.fine.mesh
    f = np.random.default_rng(11).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    ref = mg.pcg(H, b, rtol=1e-13)
    ref64 = mg.pcg(H, b, rtol=1e-10)
    bg = G.rhs(to_dev(f))
    x = torch.zeros_like(bg)
    r = G.solve(bg, x, rtol=1e-10)
    assert r.converged and r.relres_true <= 2e-10
    assert r.iters <= ref64.iters + 3
    u = ref.x
    err = np.linalg.norm(to_np(x) - u) / np.linalg.norm(u)
    err64 = np.linalg.norm(ref64.x - u) / np.linalg.norm(u)
    assert err <= max(100 * err64, 1e-8), (err, err64)
    G.close()


def test_async_solve_equals_blocking():
    import torch
    G, H = build_pair(3, (2, 2, 2), 4, hierarchy="p")
    f = np.random.default_rng(4).uniform(-1, 1, H.fine.mesh.N)
    b = G.rhs(to_dev(f))
    x1 = torch.zeros_like(b)
    r1 = G.solve(b, x1, rtol=1e-10)
    x2 = torch.zeros_like(b)
    a = G.solve_async(b, x2, rtol=1e-10)
    polls = 0
    while not a.poll():
        polls += 1
    r2 = a.finish()
    assert r2.iters == r1.iters and r2.history == r1.history
    assert torch.equal(x1, x2)
    assert r2.relres_true == r1.relres_true
    G.close()


def _mix():
    return [(3, (2, 2, 2), 4, "f64"), (2, (4, 4), 8, "f32"), (3, (2, 2, 2), 8, "f32"),
            (2, (8, 8), 2, "f64"), (3, (4, 4, 4), 2, "f32"), (3, (2, 2, 2), 16, "f32"),
            (2, (4, 6), 6, "f64"), (3, (4, 4, 4), 1, "f64")]


def test_batch_equals_alone():
    """On the stream path every problem of a mixed batch gives bitwise the result it gives
    alone."""
    import torch
    from paper_1402_5938_amd import gllmg
    probs, bs, alone = [], [], []
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    for k, (dim, ne, p, prec) in enumerate(_mix()):
        cfg = gllmg.make_config(dim, ne, p, "p", vcycle_prec=prec)
        P = gllmg.Problem(cfg, mp, mu)
        P.set_persistent(False)
        f = torch.from_numpy(np.random.default_rng(100 + k).uniform(-1, 1, P.nnodes(0))).cuda()
        b = P.rhs(f)
        x = torch.zeros_like(b)
        alone.append((P.solve(b, x, rtol=1e-10), x.clone()))
        probs.append(P)
        bs.append(b)
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(probs, bs, xs, rtol=1e-10)
    torch.cuda.synchronize()
    for k, (r, (ra, xa)) in enumerate(zip(res, alone)):
        assert r.converged and r.iters == ra.iters and r.history == ra.history, k
        assert torch.equal(xs[k], xa), k
    # interleaved begin/poll from Python as a server would drive it, on separate streams
    xs2 = [torch.zeros_like(b) for b in bs]
    streams = [torch.cuda.Stream() for _ in probs]
    for s_, b in zip(streams, bs):
        s_.wait_stream(torch.cuda.current_stream())
    act = [P.solve_async(b, x, stream=s_) for P, b, x, s_ in zip(probs, bs, xs2, streams)]
    while not all(a.poll() for a in act):
        pass
    torch.cuda.synchronize()
    for k, a in enumerate(act):
        assert a.result.iters == alone[k][0].iters
        assert torch.equal(xs2[k], alone[k][1]), k
    for P in probs:
        P.close()


def _persistent_set(modes=("pcg",)):
    """3D problems with an FP32 V-cycle (the persistent solver's), with a few 2D and FP64 ones
    mixed in (stream path, run concurrently)."""
    return [(3, (2, 2, 2), 4, "f32", "p", 0), (3, (4, 4, 4), 2, "f32", "p", 0),
            (3, (2, 2, 2), 8, "f32", "p", 0), (3, (2, 2, 2), 16, "f32", "p", 0),
            (3, (4, 4, 4), 1, "f32", "p", 0), (3, (2, 2, 4), 3, "f32", "p", 0),
            (3, (4, 2, 2), 4, "f32", "h", 0), (3, (2, 2, 2), 6, "f32", "p", 0),
            (3, (1, 1, 1), 16, "f32", "p", 4), (3, (1, 2, 1), 12, "f32", "p", 4),
            (2, (4, 4), 8, "f32", "p", 0), (3, (2, 2, 2), 4, "f64", "p", 0)]


@pytest.mark.parametrize("mode", ["pcg", "mg"])
def test_persistent_batch_matches_stream_path(mode):
    """The persistent solver (one workgroup per problem) against gllmg_solve on the stream
    path: the workgroup adds every FP64 reduction in the stream path's order, so status,
    iteration and product counts, residual histories and solutions are equal bit for bit."""
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    probs, bs, alone = [], [], []
    for k, (dim, ne, p, prec, hier, ml) in enumerate(_persistent_set()):
        cfg = gllmg.make_config(dim, ne, p, hier, vcycle_prec=prec, max_levels=ml)
        P = gllmg.Problem(cfg, mp, mu)
        f = torch.from_numpy(np.random.default_rng(300 + k).uniform(-1, 1, P.nnodes(0))).cuda()
        b = P.rhs(f)
        x = torch.zeros_like(b)
        alone.append((P.solve(b, x, mode=mode, rtol=1e-10, maxit=200), x.clone()))
        probs.append(P)
        bs.append(b)
    for rep in range(2):  # twice: the descriptors are refilled per call
        xs = [torch.zeros_like(b) for b in bs]
        res = gllmg.batch_solve(probs, bs, xs, mode=mode, rtol=1e-10, maxit=200)
        torch.cuda.synchronize()
        for k, (r, (ra, xa)) in enumerate(zip(res, alone)):
            assert r.status == ra.status and r.iters == ra.iters, (k, r.iters, ra.iters)
            assert r.converged
            assert r.history == ra.history, k
            assert torch.equal(xs[k], xa), k
            assert r.relres_true == ra.relres_true, k
            assert r.applies == ra.applies, (k, r.applies, ra.applies)
    for P in probs:
        P.close()


def test_persistent_batch_failures_are_per_problem():
    """maxit reached and a NaN right-hand side end only their own problem's solve (three
    shapes, so that no two problems form a launch group and all take the persistent solver)."""
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    probs, bs = [], []
    for k, ne in enumerate([(2, 2, 2), (2, 2, 3), (3, 2, 2)]):
        cfg = gllmg.make_config(3, ne, 4, "p", vcycle_prec="f32")
        P = gllmg.Problem(cfg, mp, mu)
        b = P.rhs(torch.from_numpy(inputs.uniform_nodal(k, P.nnodes(0))).cuda())
        if k == 1:
            b[P.nnodes(0) // 2] = float("nan")
        probs.append(P)
        bs.append(b)
    import ctypes as C
    n = 3
    xs = [torch.zeros_like(b) for b in bs]
    status = (C.c_int * n)()
    st = gllmg.lib().gllmg_batch_solve((C.c_void_p * n)(*[p.h for p in probs]),
                                       (C.c_void_p * n)(*[b.data_ptr() for b in bs]),
                                       (C.c_void_p * n)(*[x.data_ptr() for x in xs]),
                                       n, gllmg.MODE_PCG, C.c_double(1e-10), 3, None, status, None)
    torch.cuda.synchronize()
    assert st == gllmg.EBREAKDOWN
    assert list(status) == [gllmg.ENOTCONV, gllmg.EBREAKDOWN, gllmg.ENOTCONV]
    res = gllmg.batch_solve([probs[0], probs[2]], [bs[0], bs[2]],
                            [torch.zeros_like(bs[0]), torch.zeros_like(bs[2])], rtol=1e-10)
    assert all(r.converged for r in res)
    for P in probs:
        P.close()
