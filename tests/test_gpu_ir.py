"""Iterative refinement (GLLMG_MODE_IR): FP64 residuals outside, CG in FP32 with the FP32
V-cycle as preconditioner inside, FP64 dot products (the mixed-precision pattern with an
iterative-refinement outer loop). Checked against the oracle's tight FP64 solve: the FP64
residual reaches the tolerance and the solution is as close to the oracle's as that residual
allows; the refinement-step residuals fall; the mode's argument and setup errors."""

import numpy as np
import pytest

from gpu_helpers import to_dev, to_np
from oracle import fem, mg
from paper_1402_5938_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,ne,p,k", [((3), (2, 2, 2), 8, 8), (3, (4, 4, 4), 4, 6), (2, (6, 6), 16, 10),
                                        (3, (2, 3, 2), 12, 12)])
def test_ir_against_oracle(dim, ne, p, k):
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    cfg = gllmg.make_config(dim, ne, p, "p", vcycle_prec="f32", ir_inner=k)
    G = gllmg.Problem(cfg, mp, mu)
    H = mg.Hierarchy(dim, ne, p, mp, mu, hierarchy="p")
    m = H.fine.mesh
    f = np.random.default_rng(21).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    ref = mg.pcg(H, b, rtol=1e-13)
    ref64 = mg.pcg(H, b, rtol=1e-10)
    bg = G.rhs(to_dev(f))
    x = torch.zeros_like(bg)
    r = G.solve(bg, x, mode="ir", rtol=1e-10, maxit=200)
    assert r.converged and r.relres_true <= 1e-10, r
    h = np.array(r.history)
    steps = len(h) - 1  # refinement steps: k CG steps in the first, at most k in each later one
    assert steps >= 1 and np.all(np.diff(h) < 0), h
    assert k + steps - 1 <= r.iters <= steps * k or r.iters == 200, (r.iters, steps)
    # the true residual, recomputed independently of the solve
    res = to_np(bg) - to_np(G.apply(x))
    assert np.linalg.norm(res * m.interior) <= 1.01e-10 * np.linalg.norm(to_np(bg))
    u = ref.x
    err = np.linalg.norm(to_np(x) - u) / np.linalg.norm(u)
    err64 = np.linalg.norm(ref64.x - u) / np.linalg.norm(u)
    assert err <= max(100 * err64, 1e-12), (err, err64)
    G.close()


def test_ir_argument_errors():
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    with pytest.raises(gllmg.GllmgError) as e:   # refinement runs the FP32 V-cycle
        gllmg.plan(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f64", ir_inner=5))
    assert e.value.status == gllmg.EINVAL
    with pytest.raises(gllmg.GllmgError) as e:
        gllmg.plan(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f32", ir_inner=101))
    assert e.value.status == gllmg.EINVAL
    G = gllmg.Problem(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f32"), mp, mu)
    b = G.rhs(torch.ones(G.nnodes(0), dtype=torch.float64, device="cuda"))
    with pytest.raises(gllmg.GllmgError) as e:   # no refinement vectors without ir_inner
        G.solve(b, mode="ir")
    assert e.value.status == gllmg.EUNSUPPORTED
    G.close()
    G = gllmg.Problem(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f32", ir_inner=4), mp, mu)
    with pytest.raises(gllmg.GllmgError) as e:
        G.solve_async(b, torch.zeros_like(b), mode="ir")
    assert e.value.status == gllmg.EUNSUPPORTED
    with pytest.raises(gllmg.GllmgError) as e:
        gllmg.batch_solve([G], [b], [torch.zeros_like(b)], mode="ir")
    assert e.value.status == gllmg.EUNSUPPORTED
    # the refinement vectors share the region of the setup temporaries: the footprint grows
    # by at most their size
    _, w0 = gllmg.plan(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f32"))
    _, w1 = gllmg.plan(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f32", ir_inner=4))
    assert w0 <= w1 <= w0 + 5 * 4 * G.nnodes(0) + 256
    G.close()


def test_ir_maxit_below_the_inner_length():
    """maxit < k: one refinement step of maxit CG steps, ENOTCONV (not raised by default), the
    history holding the two residual norms and the iteration count maxit."""
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    G = gllmg.Problem(gllmg.make_config(3, (2, 2, 2), 4, "p", vcycle_prec="f32", ir_inner=8), mp, mu)
    b = G.rhs(torch.ones(G.nnodes(0), dtype=torch.float64, device="cuda"))
    x = torch.zeros_like(b)
    r = G.solve(b, x, mode="ir", rtol=1e-14, maxit=3)
    assert r.status == gllmg.ENOTCONV and not r.converged
    assert r.iters == 3 and len(r.history) == 2 and r.history[1] < r.history[0]
    G.close()
