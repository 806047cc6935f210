"""The Gauss-quadrature operator (§2.3: p+1 Gauss points per axis, geometry and mu at the Gauss
points) on the GPU through the C ABI against the oracle's assembled Gauss discretization: the
product (FP64 to the 1e-12 bar, FP32 to 2e-5) at orders 1..16 in 2D and 3D, Dirichlet and
Neumann, the diagonal, the consistent-mass load vector, V-cycles and PCG iteration counts."""

import numpy as np
import pytest

from gpu_helpers import build_pair, fp64_close, rel_err, random_vec, to_dev, to_np
from oracle import fem, mg

pytestmark = pytest.mark.gpu

CASES = [(2, (3, 2), 1), (2, (2, 3), 2), (2, (2, 2), 5), (2, (1, 2), 16), (3, (2, 2, 2), 1),
         (3, (2, 1, 2), 2), (3, (1, 2, 1), 4), (3, (1, 1, 2), 7), (3, (1, 1, 1), 8),
         (3, (1, 1, 1), 12), (3, (1, 1, 1), 15), (3, (1, 1, 1), 16)]


def _gauss_level(dim, ne, p, vcycle_prec="f64"):
    """The GPU problem (two levels, so that the finest takes no dense coarse solve) and the
    oracle's operator of its finest level."""
    from paper_1402_5938_amd import gllmg, inputs
    mp, mu = inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0)
    cfg = gllmg.make_config(dim, ne, p, "p", max_levels=2, vcycle_prec=vcycle_prec,
                            quadrature="gauss")
    G = gllmg.Problem(cfg, mp, mu)

    class Lv:
        pass
    lv = Lv()
    lv.mesh = fem.Mesh(dim, ne, p, mp, mu, "gauss")
    lv.op = fem.LevelOperator(lv.mesh)
    return G, lv


@pytest.mark.parametrize("dim,ne,p", CASES)
def test_gauss_apply_diag_rhs(dim, ne, p):
    G, lv = _gauss_level(dim, ne, p)
    m = lv.mesh
    x = random_vec(m.N, 13)
    ok, e = fp64_close(to_np(G.apply(to_dev(x))), lv.op.apply(x), lv.op.apply_abs(x))
    assert ok, e
    ok, e = fp64_close(to_np(G.apply(to_dev(x), neumann=True)), lv.op.apply(x, neumann=True),
                       lv.op.apply_abs(x, neumann=True))
    assert ok, e
    ok, e = fp64_close(to_np(G.diag(0)), lv.op.diag())
    assert ok, e
    f = np.random.default_rng(4).uniform(-1, 1, m.N)
    ok, e = fp64_close(to_np(G.rhs(to_dev(f))), fem.load_vector(m, f))
    assert ok, e
    G.close()


@pytest.mark.parametrize("dim,ne,p", [(2, (2, 2), 6), (3, (2, 1, 2), 3), (3, (1, 1, 1), 9),
                                      (3, (1, 1, 1), 16)])
def test_gauss_apply_fp32(dim, ne, p):
    import torch
    G, lv = _gauss_level(dim, ne, p, "f32")
    x = random_vec(lv.mesh.N, 17)
    y = to_np(G.apply(to_dev(x, torch.float32)))
    assert rel_err(y, lv.op.apply(x)) <= 2e-5
    G.close()


@pytest.mark.parametrize("dim,ne,p,hier,smoother", [(2, (4, 4), 4, "h", "chebyshev"),
                                                    (3, (2, 2, 2), 4, "p", "chebyshev"),
                                                    (3, (2, 2, 2), 8, "p", "jacobi"),
                                                    (2, (4, 2), 8, "p", "chebyshev")])
def test_gauss_vcycle_and_pcg(dim, ne, p, hier, smoother):
    G, H = build_pair(dim, ne, p, hierarchy=hier, smoother=smoother, nu=3 if smoother == "jacobi" else 4,
                      quadrature="gauss")
    for l, lv in enumerate(H.levels[:-1]):
        assert abs(G.levels[l].lmax - lv.lmax) <= 1e-10 * lv.lmax
    m = H.fine.mesh
    r = random_vec(m.N, 19) * m.interior
    assert rel_err(to_np(G.vcycle(to_dev(r))), H.vcycle(r)) <= 1e-10
    f = np.random.default_rng(6).uniform(-1, 1, m.N)
    b = fem.load_vector(m, f)
    ro = mg.pcg(H, b, rtol=1e-10)
    rg = G.solve(G.rhs(to_dev(f)), rtol=1e-10)
    assert rg.converged and ro.converged and rg.iters == ro.iters, (rg.iters, ro.iters)
    assert rel_err(rg.history, ro.history) <= 1e-8
    G.close()


def test_gauss_rejects_collocation_smoothers():
    from paper_1402_5938_amd import gllmg
    for sm in ("ssor", "l1jacobi", "blockjacobi"):
        cfg = gllmg.make_config(3, (2, 2, 2), 4, "p", sm, 2, quadrature="gauss")
        with pytest.raises(gllmg.GllmgError) as e:
            gllmg.plan(cfg)
        assert e.value.status == gllmg.EUNSUPPORTED
