"""GPU (HIP, through the C ABI) versus the CPU FP64 oracle, element by element, on seeded
inputs that span several elements per axis, ragged (non-cubic) element counts and all orders
1..16. Tolerances: FP64 products, diagonal, transfers and smoothing <= 1e-12 relative in the
2-norm and 5e-12 in the max-norm (the observed plain errors stay below 1e-13; the oracle's
rounding scale |B|^T|G||B||x| of each product is reported beside them); V-cycle <= 1e-10; FP32
paths <= 2e-5 relative; iteration counts equal."""

import numpy as np
import pytest

from gpu_helpers import build_pair, fp64_close, rel_err, random_vec, to_dev, to_np
from oracle import fem, mg, transfer
from paper_1402_5938_amd import inputs

pytestmark = pytest.mark.gpu

APPLY_CASES = [
    (2, (3, 4), 1), (2, (3, 2), 2), (2, (2, 3), 4), (2, (3, 1), 7), (2, (2, 2), 12), (2, (1, 2), 16),
    (3, (2, 3, 2), 1), (3, (2, 2, 3), 2), (3, (3, 1, 2), 3), (3, (2, 1, 2), 4), (3, (1, 2, 1), 5),
    (3, (1, 1, 2), 8), (3, (2, 1, 1), 9), (3, (1, 1, 1), 13), (3, (1, 2, 1), 16),
    # every high-order branch of the 3D element pass: n = 11 (register column), n = 12, 13
    # (column read back from LDS in FP64), n = 15, 16 (register copy)
    (3, (1, 1, 1), 10), (3, (1, 2, 1), 11), (3, (2, 1, 1), 12), (3, (1, 1, 1), 14),
    (3, (1, 1, 1), 15), (3, (2, 1, 2), 6), (3, (1, 1, 1), 7),
]


@pytest.mark.parametrize("dim,ne,p", APPLY_CASES)
def test_apply_diag_coords_fp64(dim, ne, p):
    import torch
    G, H = build_pair(dim, ne, p, max_levels=1)
    lv = H.levels[0]
    m = lv.mesh
    assert G.nnodes(0) == m.N
    np.testing.assert_allclose(to_np(G.node_coords(0)), m.x, rtol=0, atol=1e-14)
    x = random_vec(m.N, 11)
    y = to_np(G.apply(to_dev(x)))
    ok, e = fp64_close(y, lv.op.apply(x), lv.op.apply_abs(x))
    assert ok, e
    yn = to_np(G.apply(to_dev(x), neumann=True))
    ok, e = fp64_close(yn, lv.op.apply(x, neumann=True), lv.op.apply_abs(x, neumann=True))
    assert ok, e
    d = to_np(G.diag(0))
    ok, e = fp64_close(d, lv.op.diag())
    assert ok, e
    # determinism: a second product is bitwise identical
    y2 = to_np(G.apply(to_dev(x)))
    assert np.array_equal(y, y2)
    torch.cuda.synchronize()
    G.close()


FP32_CASES = [(2, (3, 2), 4), (2, (2, 2), 12), (3, (2, 1, 2), 4), (3, (1, 2, 1), 8),
              (3, (2, 1, 1), 12), (3, (1, 1, 1), 13), (3, (1, 1, 1), 14), (3, (1, 1, 1), 15),
              (3, (1, 1, 1), 16)]


@pytest.mark.parametrize("dim,ne,p", FP32_CASES)
def test_apply_fp32(dim, ne, p):
    import torch
    G, H = build_pair(dim, ne, p, max_levels=1, vcycle_prec="f32")
    lv = H.levels[0]
    x = random_vec(lv.mesh.N, 12)
    y32 = to_np(G.apply(to_dev(x, torch.float32)))
    assert rel_err(y32, lv.op.apply(x)) <= 2e-5
    G.close()


@pytest.mark.parametrize("ne,prec", [((28, 27, 26), "f64"), ((41, 41, 40), "f32")])
def test_apply_order1_large_levels(ne, prec):
    """3D order-1 levels above the one-kernel product's size limit (16,384 nodes in FP64,
    65,536 in FP32) take the element kernel and gather: the same bar against the oracle's
    operator (built alone: a one-level oracle hierarchy would factor a dense coarse matrix)."""
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    G = gllmg.Problem(gllmg.make_config(3, ne, 1, "p", max_levels=1, vcycle_prec=prec), mp, mu)
    op = fem.LevelOperator(fem.Mesh(3, ne, 1, mp, mu))
    assert G.nnodes(0) > (16384 if prec == "f64" else 65536)
    x = random_vec(G.nnodes(0), 13)
    if prec == "f64":
        y = to_np(G.apply(to_dev(x)))
        ok, e = fp64_close(y, op.apply(x), op.apply_abs(x))
        assert ok, e
    else:
        y32 = to_np(G.apply(to_dev(x, torch.float32)))
        assert rel_err(y32, op.apply(x)) <= 2e-5
    G.close()


@pytest.mark.parametrize("ne,prec", [((7, 5, 9), "f64"), ((17, 16, 15), "f64"), ((9, 1, 6), "f32"),
                                     ((41, 40, 23), "f64")])
def test_apply_order2_levels(ne, prec):
    """3D order-2 levels up to 65,536 nodes take the one-kernel box product (boxes of 2^3
    owned elements, partial boxes at odd element counts); the last case, above that size, takes
    the element kernel and gather. Dirichlet and Neumann products against the oracle's
    operator."""
    import torch
    from paper_1402_5938_amd import gllmg
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    G = gllmg.Problem(gllmg.make_config(3, ne, 2, "p", max_levels=1, vcycle_prec=prec), mp, mu)
    op = fem.LevelOperator(fem.Mesh(3, ne, 2, mp, mu))
    x = random_vec(G.nnodes(0), 17)
    for neu in (False, True):
        if prec == "f64":
            y = to_np(G.apply(to_dev(x), neumann=neu))
            ok, e = fp64_close(y, op.apply(x, neumann=neu), op.apply_abs(x, neumann=neu))
            assert ok, e
        else:
            y32 = to_np(G.apply(to_dev(x, torch.float32), neumann=neu))
            assert rel_err(y32, op.apply(x, neumann=neu)) <= 2e-5
    G.close()


def test_rhs_and_fields():
    import torch
    prob = inputs.poisson2d_manufactured()
    G, H = build_pair(2, (4, 4), 4, inputs.map_identity(), inputs.field_const(1.0), "h")
    m = H.fine.mesh
    f = to_np(G.eval_field(prob.f))
    np.testing.assert_allclose(f, fem.nodal_field(m, prob.f), rtol=1e-14, atol=1e-13)
    b = to_np(G.rhs(to_dev(f)))
    assert rel_err(b, fem.load_vector(m, f)) <= 1e-13
    G.close()


TRANSFER_CASES = [
    (2, (4, 4), 4, "h"), (2, (4, 2), 3, "p"), (3, (4, 2, 2), 4, "p"), (3, (2, 2, 2), 2, "h"),
    (3, (2, 2, 2), 8, "p"), (2, (6, 4), 6, "p"), (2, (4, 2), 5, "p"), (3, (2, 1, 2), 7, "p"),
    (3, (2, 2, 2), 16, "p"), (3, (2, 2, 2), 8, "h"), (2, (2, 4), 16, "h"), (3, (2, 2, 2), 16, "h"),
]


@pytest.mark.parametrize("dim,ne,p,hier", TRANSFER_CASES)
def test_transfers_and_lmax(dim, ne, p, hier):
    G, H = build_pair(dim, ne, p, hierarchy=hier)
    assert len(G.levels) == len(H.levels)
    for l in range(len(H.levels) - 1):
        f, c = H.levels[l], H.levels[l + 1]
        assert G.levels[l].order == f.mesh.p and G.levels[l].nelem == f.mesh.nelem
        xc = random_vec(c.mesh.N, 20 + l)
        rf = random_vec(f.mesh.N, 40 + l)
        xf = to_np(G.prolong(to_dev(xc), l))
        rc = to_np(G.restrict(to_dev(rf), l))
        assert fp64_close(xf, f.to_coarse.prolong(xc))[0]
        assert fp64_close(rc, f.to_coarse.restrict(rf))[0]
        assert abs(G.levels[l].lmax - f.lmax) <= 1e-10 * f.lmax
    G.close()


@pytest.mark.parametrize("smoother", ["chebyshev", "jacobi"])
@pytest.mark.parametrize("dim,ne,p", [(2, (3, 2), 5), (3, (2, 1, 2), 4)])
def test_smoother(smoother, dim, ne, p):
    G, H = build_pair(dim, ne, p, smoother=smoother, hierarchy="p")
    G.set_lmax(0, H.levels[0].lmax)
    lv = H.levels[0]
    b = random_vec(lv.mesh.N, 5) * lv.mesh.interior
    x0 = random_vec(lv.mesh.N, 6) * lv.mesh.interior
    for k in (1, 2, 3, 4):  # 3 and 4: the deferred x updates
        for zero in (True, False):
            xg = to_dev(x0.copy())
            G.smooth(to_dev(b), xg, k, 0, zero_guess=zero)
            xo = H.smooth(0, b, None if zero else x0.copy(), steps=k)
            ok, e = fp64_close(to_np(xg), xo)
            assert ok, (k, zero, e)
    G.close()


VCYCLE_CASES = [
    (2, (4, 4), 4, "h", "chebyshev", 2), (2, (4, 4), 4, "p", "chebyshev", 3),
    (3, (2, 2, 2), 4, "p", "chebyshev", 4), (3, (4, 2, 2), 2, "h", "jacobi", 3),
    (3, (2, 2, 2), 8, "p", "chebyshev", 4), (3, (2, 2, 2), 12, "p", "chebyshev", 4),
]


@pytest.mark.parametrize("dim,ne,p,hier,smoother,nu", VCYCLE_CASES)
def test_vcycle(dim, ne, p, hier, smoother, nu):
    G, H = build_pair(dim, ne, p, hierarchy=hier, smoother=smoother, nu=nu)
    for l, lv in enumerate(H.levels[:-1]):
        G.set_lmax(l, lv.lmax)
    m = H.fine.mesh
    r = random_vec(m.N, 9) * m.interior
    e = to_np(G.vcycle(to_dev(r)))
    assert rel_err(e, H.vcycle(r)) <= 1e-10
    G.close()


def test_config1_solver_iteration_counts():
    """2D 4x4 p=4, mu=1, manufactured f, h-multigrid, Chebyshev degree 2: MG solver and PCG."""
    prob = inputs.poisson2d_manufactured()
    G, H = build_pair(2, (4, 4), 4, prob.map, prob.mu, "h", nu=2)
    m = H.fine.mesh
    f = fem.nodal_field(m, prob.f)
    b = fem.load_vector(m, f)
    bg = G.rhs(to_dev(f))
    for mode in ("mg", "pcg"):
        ro = mg.mg_solve(H, b, rtol=1e-10) if mode == "mg" else mg.pcg(H, b, rtol=1e-10)
        rg = G.solve(bg, mode=mode, rtol=1e-10)
        assert rg.converged and ro.converged
        assert rg.iters == ro.iters, (mode, rg.iters, ro.iters)
        assert rel_err(rg.history, ro.history) <= 1e-9
    G.close()


@pytest.mark.parametrize("dim,ne,p", [(3, (2, 2, 2), 4), (3, (4, 4, 4), 2), (2, (8, 6), 8)])
def test_pcg_iteration_counts_warped(dim, ne, p):
    G, H = build_pair(dim, ne, p, hierarchy="p", nu=4)
    m = H.fine.mesh
    f = np.random.default_rng(3).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    ro = mg.pcg(H, b, rtol=1e-10)
    rg = G.solve(G.rhs(to_dev(f)), rtol=1e-10)
    assert rg.converged and rg.iters == ro.iters
    assert rel_err(rg.history, ro.history) <= 1e-8
    G.close()


@pytest.mark.parametrize("vprec", ["f64", "f32"])
def test_graph_replays_match_eager(vprec):
    """The captured V-cycle graph, replayed in several solves with eager work and
    synchronizations in between, gives bitwise the same iterates as eager launches."""
    import torch
    G, H = build_pair(3, (2, 2, 2), 4, hierarchy="p", vcycle_prec=vprec)
    f = np.random.default_rng(8).uniform(-1, 1, H.fine.mesh.N)
    b = G.rhs(to_dev(f))
    G.set_graphs(False)
    xe = torch.zeros_like(b)
    re_ = G.solve(b, xe, rtol=1e-10)
    G.set_graphs(True)
    for rep in range(3):
        xg = torch.zeros_like(b)
        rg = G.solve(b, xg, rtol=1e-10)
        torch.cuda.synchronize()
        G.apply(to_dev(f))                      # unrelated eager work between replays
        torch.cuda.synchronize()
        assert rg.iters == re_.iters and rg.history == re_.history
        assert torch.equal(xg, xe), rep
        assert rg.applies == re_.applies
    G.close()
