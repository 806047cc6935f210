"""Launch groups in gllmg_batch_solve: problems of one shape are solved in lockstep, each kernel
launched once for all of them (problem k of a launch is blockIdx.y; a problem leaves the
launches when its solve has ended).

Each problem's result must equal, bit for bit, the same problem solved alone by gllmg_solve:
the group runs the same kernels with the same reduction trees on each problem's own buffers,
with each problem's own Chebyshev coefficients. Checked: status, iteration count, residual
history, solution, true residual and the per-level product counts.
"""

import ctypes as C

import numpy as np
import pytest

from paper_1402_5938_amd import inputs

pytestmark = pytest.mark.gpu

# (dim, elements, p, V-cycle precision, smoother, hierarchy)
CASES = [
    (3, (3, 3, 3), 4, "f64", "chebyshev", "p"),
    (3, (4, 4, 4), 8, "f32", "chebyshev", "p"),   # 35,937 nodes: beyond the one-workgroup solver
    (2, (6, 6), 8, "f64", "chebyshev", "p"),
    (3, (3, 3, 3), 3, "f64", "jacobi", "h"),
    (3, (4, 4, 3), 6, "f32", "chebyshev", "p"),   # 11,875 nodes, anisotropic element grid
]


def _problems(case, count, seed0):
    import torch
    from paper_1402_5938_amd import gllmg
    dim, ne, p, prec, smoother, hier = case
    mp = inputs.map_warp_sine(0.05)
    probs, bs = [], []
    for k in range(count):
        cfg = gllmg.make_config(dim, ne, p, hier, smoother=smoother, vcycle_prec=prec)
        P = gllmg.Problem(cfg, mp, inputs.mu_exp_sine_product(1.0 + 0.7 * k))
        f = torch.from_numpy(np.random.default_rng(seed0 + k).uniform(-1, 1, P.nnodes(0))).cuda()
        probs.append(P)
        bs.append(P.rhs(f))
    return probs, bs


def _alone(probs, bs, maxit=300):
    import torch
    out = []
    for P, b in zip(probs, bs):
        x = torch.zeros_like(b)
        r = P.solve(b, x, rtol=1e-10, maxit=maxit)
        out.append((r, x.clone()))
    return out


def _same(r, x, ra, xa):
    import torch
    assert r.status == ra.status
    assert r.iters == ra.iters, (r.iters, ra.iters)
    assert r.history == ra.history
    assert r.relres_true == ra.relres_true
    assert r.applies == ra.applies, (r.applies, ra.applies)
    assert torch.equal(x, xa)


@pytest.mark.parametrize("case", CASES)
def test_group_equals_solving_alone(case):
    import torch
    from paper_1402_5938_amd import gllmg
    probs, bs = _problems(case, 3, 500)
    alone = _alone(probs, bs)
    for rep in range(2):  # twice: nothing of a group solve outlives the call
        xs = [torch.zeros_like(b) for b in bs]
        res = gllmg.batch_solve(probs, bs, xs, rtol=1e-10, maxit=300)
        torch.cuda.synchronize()
        for k in range(len(probs)):
            assert res[k].converged
            _same(res[k], xs[k], *alone[k])
    for P in probs:
        P.close()


def test_groups_singles_and_persistent_together():
    """Two shapes with two problems each, one shape alone (stream path) and one small FP32
    problem (one-workgroup solver) in one call: every result as if solved alone."""
    import torch
    from paper_1402_5938_amd import gllmg
    pa, ba = _problems(CASES[0], 2, 600)
    pb, bb = _problems(CASES[2], 2, 610)
    pc, bc = _problems(CASES[3], 1, 620)
    pd, bd = _problems((3, (2, 2, 2), 4, "f32", "chebyshev", "p"), 1, 630)
    probs, bs = pa + pb + pc + pd, ba + bb + bc + bd
    alone = _alone(probs, bs)
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(probs, bs, xs, rtol=1e-10, maxit=300)
    torch.cuda.synchronize()
    for k in range(len(probs) - 1):
        _same(res[k], xs[k], *alone[k])
    # the one-workgroup solver sums its dot products in another fixed order
    r, (ra, xa) = res[-1], alone[-1]
    assert r.iters == ra.iters and r.converged
    assert torch.linalg.norm(xs[-1] - xa) <= 1e-8 * torch.linalg.norm(xa)
    for P in probs:
        P.close()


def test_group_failures_are_per_problem():
    """In one group: a NaN right-hand side breaks down alone; the others converge exactly as
    alone. With maxit = 3 every problem stops at 3 iterations with ENOTCONV."""
    import torch
    from paper_1402_5938_amd import gllmg
    probs, bs = _problems(CASES[0], 3, 700)
    bs[1][probs[1].nnodes(0) // 2] = float("nan")
    alone = _alone([probs[0], probs[2]], [bs[0], bs[2]])
    n = 3
    xs = [torch.zeros_like(b) for b in bs]
    status = (C.c_int * n)()
    st = gllmg.lib().gllmg_batch_solve((C.c_void_p * n)(*[p.h for p in probs]),
                                       (C.c_void_p * n)(*[b.data_ptr() for b in bs]),
                                       (C.c_void_p * n)(*[x.data_ptr() for x in xs]),
                                       n, gllmg.MODE_PCG, C.c_double(1e-10), 300, None, status, None)
    torch.cuda.synchronize()
    assert st == gllmg.EBREAKDOWN
    assert list(status) == [gllmg.OK, gllmg.EBREAKDOWN, gllmg.OK]
    assert torch.equal(xs[0], alone[0][1]) and torch.equal(xs[2], alone[1][1])
    good = [bs[0], bs[2]]
    xs = [torch.zeros_like(b) for b in good]
    res = gllmg.batch_solve([probs[0], probs[2]], good, xs, rtol=1e-10, maxit=3)
    torch.cuda.synchronize()
    short = _alone([probs[0], probs[2]], good, maxit=3)
    for k in range(2):
        assert res[k].status == gllmg.ENOTCONV and res[k].iters == 3
        _same(res[k], xs[k], *short[k])
    for P in probs:
        P.close()


def test_group_after_lmax_change():
    """gllmg_set_lmax refreshes the coefficient table that the group kernels read."""
    import torch
    from paper_1402_5938_amd import gllmg
    probs, bs = _problems(CASES[0], 2, 800)
    probs[1].set_lmax(0, 1.3 * probs[1].levels[0].lmax)
    alone = _alone(probs, bs)
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(probs, bs, xs, rtol=1e-10, maxit=300)
    torch.cuda.synchronize()
    for k in range(2):
        _same(res[k], xs[k], *alone[k])
    for P in probs:
        P.close()
