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


def test_fp32_vcycle_pieces_against_oracle():
    import torch
    G, H = build_pair(3, (2, 2, 2), 8, hierarchy="p", vcycle_prec="f32")
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
    """Every problem of a mixed batch gives bitwise the result it gives alone."""
    import torch
    from paper_1402_5938_amd import gllmg
    probs, bs, alone = [], [], []
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    for k, (dim, ne, p, prec) in enumerate(_mix()):
        cfg = gllmg.make_config(dim, ne, p, "p", vcycle_prec=prec)
        P = gllmg.Problem(cfg, mp, mu)
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
