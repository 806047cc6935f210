"""GPU (through the C ABI) versus the CPU FP64 oracle for the multicolor SSOR smoother (§3.2.1,
§4.3 "SSOR(2,1)", omega = 1): smoothing steps from zero and non-zero guesses at orders 1..16 in
2D and 3D (FP64 to the 1e-12 bar, FP32 to 1e-5), V-cycles with SSOR(2,1) (1e-10), and PCG / MG
solves with equal iteration counts. Batched solves of SSOR problems equal solving alone."""

import numpy as np
import pytest

from gpu_helpers import build_pair, fp64_close, rel_err, random_vec, to_dev, to_np
from oracle import fem, mg

pytestmark = pytest.mark.gpu

SSOR_SMOOTH_CASES = [(2, (3, 2), 3), (2, (2, 3), 1), (2, (2, 2), 16), (3, (2, 1, 2), 4),
                     (3, (1, 2, 1), 8), (3, (3, 2, 2), 1), (3, (2, 2, 1), 2), (3, (1, 1, 1), 13),
                     (3, (1, 1, 1), 16)]


@pytest.mark.parametrize("dim,ne,p", SSOR_SMOOTH_CASES)
def test_ssor_smoother_fp64(dim, ne, p):
    G, H = build_pair(dim, ne, p, smoother="ssor", nu=2, nu_post=1, max_levels=2)
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 5) * lv.mesh.interior
    x0 = random_vec(lv.mesh.N, 6)          # boundary entries are ignored on input
    for k in (1, 2):
        for zero in (True, False):
            xg = to_dev(x0.copy())
            G.smooth(to_dev(b), xg, k, 0, zero_guess=zero)
            xo = H.smooth(0, b, None if zero else x0 * lv.mesh.interior, steps=k)
            ok, e = fp64_close(to_np(xg), xo)
            assert ok, (k, zero, e)
    G.close()


@pytest.mark.parametrize("dim,ne,p", [(3, (2, 1, 2), 4), (2, (2, 2), 12), (3, (1, 1, 1), 16)])
def test_ssor_smoother_fp32(dim, ne, p):
    import torch
    G, H = build_pair(dim, ne, p, smoother="ssor", nu=2, nu_post=1, max_levels=2,
                      vcycle_prec="f32")
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 15) * lv.mesh.interior
    x = torch.zeros(lv.mesh.N, dtype=torch.float32, device="cuda")
    G.smooth(to_dev(b, torch.float32), x, 2, 0, zero_guess=True)
    assert rel_err(to_np(x), H.smooth(0, b, None, steps=2)) <= 1e-5
    G.close()


SSOR_VCYCLE_CASES = [(2, (4, 4), 4, "h"), (2, (4, 4), 3, "p"), (3, (2, 2, 2), 4, "p"),
                     (3, (2, 2, 2), 8, "p"), (3, (4, 2, 2), 2, "h")]


@pytest.mark.parametrize("dim,ne,p,hier", SSOR_VCYCLE_CASES)
def test_ssor_vcycle(dim, ne, p, hier):
    G, H = build_pair(dim, ne, p, hierarchy=hier, smoother="ssor", nu=2, nu_post=1)
    m = H.fine.mesh
    r = random_vec(m.N, 9) * m.interior
    e = to_np(G.vcycle(to_dev(r)))
    assert rel_err(e, H.vcycle(r)) <= 1e-10
    G.close()


@pytest.mark.parametrize("dim,ne,p,mode", [(3, (2, 2, 2), 4, "pcg"), (2, (8, 6), 8, "pcg"),
                                           (3, (2, 2, 2), 8, "pcg"), (2, (4, 4), 4, "mg")])
def test_ssor_solve_iteration_counts(dim, ne, p, mode):
    G, H = build_pair(dim, ne, p, hierarchy="p", smoother="ssor", nu=2, nu_post=1)
    m = H.fine.mesh
    f = np.random.default_rng(3).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    ro = mg.pcg(H, b, rtol=1e-10) if mode == "pcg" else mg.mg_solve(H, b, rtol=1e-10)
    rg = G.solve(G.rhs(to_dev(f)), mode=mode, rtol=1e-10)
    assert rg.converged and ro.converged
    assert rg.iters == ro.iters, (rg.iters, ro.iters)
    assert rel_err(rg.history, ro.history) <= 1e-8
    G.close()


def test_ssor_batch_equals_alone():
    import torch
    from paper_1402_5938_amd import gllmg, inputs
    probs, bs = [], []
    for s in range(3):
        mu = inputs.mu_exp_sine_product(1.0 + s, (0.1 * s, 0.0, 0.2))
        cfg = gllmg.make_config(3, (2, 2, 2), 4, "p", "ssor", 2, nu_post=1, vcycle_prec="f32")
        P = gllmg.Problem(cfg, inputs.map_warp_sine(0.05), mu)
        f = torch.from_numpy(np.random.default_rng(s).uniform(-1, 1, P.nnodes(0))).cuda()
        probs.append(P)
        bs.append(P.rhs(f))
    alone = []
    for P, b in zip(probs, bs):
        x = torch.zeros_like(b)
        r = P.solve(b, x, rtol=1e-10)
        alone.append((r, x))
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(probs, bs, xs, rtol=1e-10)
    for (r, x), rb, xb in zip(alone, res, xs):
        assert rb.converged and rb.iters == r.iters
        assert torch.equal(xb, x)
    for P in probs:
        P.close()


# ------------------------------------------------------------------ l1-Jacobi (§3.2.3, §4.4.3)
L1_CASES = [(2, (3, 2), 3), (2, (2, 2), 16), (3, (2, 1, 2), 4), (3, (1, 2, 1), 8),
            (3, (3, 2, 2), 1), (3, (2, 2, 1), 2), (3, (1, 1, 1), 16)]


@pytest.mark.parametrize("dim,ne,p", L1_CASES)
def test_l1_jacobi_smoother_fp64(dim, ne, p):
    G, H = build_pair(dim, ne, p, smoother="l1jacobi", nu=3, max_levels=2)
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 25) * lv.mesh.interior
    x0 = random_vec(lv.mesh.N, 26) * lv.mesh.interior
    for k in (1, 3):
        for zero in (True, False):
            xg = to_dev(x0.copy())
            G.smooth(to_dev(b), xg, k, 0, zero_guess=zero)
            xo = H.smooth(0, b, None if zero else x0.copy(), steps=k)
            ok, e = fp64_close(to_np(xg), xo)
            assert ok, (k, zero, e)
    G.close()


@pytest.mark.parametrize("dim,ne,p,hier", [(2, (4, 4), 4, "h"), (3, (2, 2, 2), 4, "p"),
                                           (3, (2, 2, 2), 8, "p")])
def test_l1_jacobi_vcycle_and_pcg(dim, ne, p, hier):
    G, H = build_pair(dim, ne, p, hierarchy=hier, smoother="l1jacobi", nu=3)
    m = H.fine.mesh
    r = random_vec(m.N, 29) * m.interior
    assert rel_err(to_np(G.vcycle(to_dev(r))), H.vcycle(r)) <= 1e-10
    f = np.random.default_rng(4).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    ro = mg.pcg(H, b, rtol=1e-10)
    rg = G.solve(G.rhs(to_dev(f)), rtol=1e-10)
    assert rg.converged and ro.converged and rg.iters == ro.iters, (rg.iters, ro.iters)
    assert rel_err(rg.history, ro.history) <= 1e-8
    G.close()


def test_l1_jacobi_fp32_and_launch_group():
    import torch
    from paper_1402_5938_amd import gllmg, inputs
    G, H = build_pair(3, (2, 1, 2), 4, smoother="l1jacobi", nu=3, max_levels=2, vcycle_prec="f32")
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 31) * lv.mesh.interior
    x = torch.zeros(lv.mesh.N, dtype=torch.float32, device="cuda")
    G.smooth(to_dev(b, torch.float32), x, 3, 0, zero_guess=True)
    assert rel_err(to_np(x), H.smooth(0, b, None, steps=3)) <= 1e-5
    G.close()
    # two problems of one shape form a launch group: results equal solving alone, bit for bit
    probs, bs = [], []
    for s in range(2):
        cfg = gllmg.make_config(3, (2, 2, 2), 4, "p", "l1jacobi", 3, vcycle_prec="f32")
        P = gllmg.Problem(cfg, inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(1.0 + s))
        f = torch.from_numpy(np.random.default_rng(s).uniform(-1, 1, P.nnodes(0))).cuda()
        probs.append(P)
        bs.append(P.rhs(f))
    alone = []
    for P, b in zip(probs, bs):
        xa = torch.zeros_like(b)
        alone.append((P.solve(b, xa, rtol=1e-10), xa))
    xs = [torch.zeros_like(b) for b in bs]
    res = gllmg.batch_solve(probs, bs, xs, rtol=1e-10)
    for (r, xa), rb, xb in zip(alone, res, xs):
        assert rb.converged and rb.iters == r.iters
        assert torch.equal(xb, xa)
    for P in probs:
        P.close()


# ------------------------------------------------------------------ element block Jacobi
BJ_CASES = [(2, (3, 2), 3), (2, (2, 2), 16), (3, (2, 1, 2), 4), (3, (1, 2, 1), 8),
            (3, (3, 2, 2), 1), (3, (2, 2, 1), 2), (3, (2, 1, 1), 10)]


@pytest.mark.parametrize("dim,ne,p", BJ_CASES)
def test_block_jacobi_smoother_fp64(dim, ne, p):
    G, H = build_pair(dim, ne, p, smoother="blockjacobi", nu=3, max_levels=2)
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 35) * lv.mesh.interior
    x0 = random_vec(lv.mesh.N, 36)
    for k in (1, 3):
        for zero in (True, False):
            xg = to_dev(x0.copy())
            G.smooth(to_dev(b), xg, k, 0, zero_guess=zero)
            xo = H.smooth(0, b, None if zero else x0 * lv.mesh.interior, steps=k)
            ok, e = fp64_close(to_np(xg), xo)
            assert ok, (k, zero, e)
    G.close()


@pytest.mark.parametrize("dim,ne,p,hier", [(2, (4, 4), 4, "h"), (3, (2, 2, 2), 4, "p"),
                                           (3, (2, 2, 2), 8, "p")])
def test_block_jacobi_vcycle_and_pcg(dim, ne, p, hier):
    G, H = build_pair(dim, ne, p, hierarchy=hier, smoother="blockjacobi", nu=3)
    m = H.fine.mesh
    r = random_vec(m.N, 39) * m.interior
    assert rel_err(to_np(G.vcycle(to_dev(r))), H.vcycle(r)) <= 1e-10
    f = np.random.default_rng(5).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    for mode in ("pcg", "mg"):
        ro = mg.pcg(H, b, rtol=1e-10) if mode == "pcg" else mg.mg_solve(H, b, rtol=1e-10)
        rg = G.solve(G.rhs(to_dev(f)), mode=mode, rtol=1e-10)
        assert rg.converged and ro.converged and rg.iters == ro.iters, (mode, rg.iters, ro.iters)
        assert rel_err(rg.history, ro.history) <= 1e-8
    G.close()


def test_block_jacobi_fp32_and_limits():
    import torch
    from paper_1402_5938_amd import gllmg, inputs
    G, H = build_pair(3, (2, 1, 2), 4, smoother="blockjacobi", nu=3, max_levels=2,
                      vcycle_prec="f32")
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 41) * lv.mesh.interior
    x = torch.zeros(lv.mesh.N, dtype=torch.float32, device="cuda")
    G.smooth(to_dev(b, torch.float32), x, 3, 0, zero_guess=True)
    assert rel_err(to_np(x), H.smooth(0, b, None, steps=3)) <= 1e-5
    G.close()
    # element blocks beyond 1024 unknowns (3D p = 11: 1331) are refused at planning
    cfg = gllmg.make_config(3, (1, 1, 1), 11, "p", "blockjacobi", 3)
    with pytest.raises(gllmg.GllmgError) as e:
        gllmg.plan(cfg)
    assert e.value.status == gllmg.EUNSUPPORTED
