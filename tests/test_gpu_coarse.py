"""The exact coarse solve (§3, the coarsest level's direct solve) against the oracle: the
coarsest operator assembled from colored matrix-free products, its dense inverse, and the
kernel that applies it; at the size of the literal 16^3 first-order coarse level (3375
interior unknowns) inside a V-cycle and PCG, and as a whole one-level solve at orders 1-3,
2D and 3D, GLL and Gauss quadrature."""

import numpy as np
import pytest

from gpu_helpers import build_pair, random_vec, rel_err, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_literal_first_order_coarse_level():
    """16^3 hexes at p = 2 over 16^3 at p = 1: the coarsest level has 15^3 = 3375 interior
    unknowns, the size the 16^3 p = 8 hierarchy stopped at p = 1 would have."""
    G, H = build_pair(3, (16, 16, 16), 2, max_levels=2)
    assert G.nlevels == 2 and G.nnodes(1) == 17 ** 3
    G.set_lmax(0, H.levels[0].lmax)
    m = H.fine.mesh
    r = random_vec(m.N, 9) * m.interior
    assert rel_err(to_np(G.vcycle(to_dev(r))), H.vcycle(r)) <= 1e-10
    from oracle import mg
    b = random_vec(m.N, 4) * m.interior
    ro = mg.pcg(H, b, rtol=1e-10)
    rg = G.solve(to_dev(b), rtol=1e-10)
    assert rg.converged and rg.iters == ro.iters, (rg.iters, ro.iters)
    assert rel_err(rg.history, ro.history) <= 1e-9
    G.close()


@pytest.mark.parametrize("dim,ne,p,quad", [
    (3, (3, 3, 3), 3, "gll"),      # 8^3 interior unknowns, 7 colors per axis
    (3, (6, 5, 4), 2, "gll"),      # 11 x 9 x 7, 5 colors per axis, fewer nodes than colors on z
    (3, (9, 7, 8), 1, "gll"),      # 3 colors per axis
    (2, (30, 21), 1, "gll"),
    (2, (7, 6), 3, "gll"),
    (3, (4, 3, 3), 2, "gauss"),
    (2, (9, 8), 2, "gauss"),
])
def test_one_level_exact_solve(dim, ne, p, quad):
    """A one-level hierarchy's V-cycle is the exact solve: equal to the oracle's Cholesky solve,
    and A x = r on the interior nodes."""
    G, H = build_pair(dim, ne, p, max_levels=1, quadrature=quad)
    assert G.nlevels == 1
    m = H.fine.mesh
    r = random_vec(m.N, 5) * m.interior
    x = to_np(G.vcycle(to_dev(r)))
    assert rel_err(x, H.vcycle(r)) <= 1e-10
    assert np.all(x[~m.interior.astype(bool)] == 0.0)
    Ax = to_np(G.apply(to_dev(x)))
    assert rel_err(Ax * m.interior, r) <= 1e-10
    G.close()


@pytest.mark.parametrize("dim,ne,p,hier,k", [
    (3, (4, 4, 4), 4, "p", 64),      # 4^3 at p = 4, 2, 1: the exact solve on 27 unknowns
    (2, (16, 16), 2, "p", 300),      # 16^2 at p = 2, 1: 225 unknowns
    (3, (2, 2, 2), 4, "low", 4096),  # the order-4 level and its first-order level, solved exactly
    (3, (4, 4, 4), 2, "h", 4096),    # order 2 throughout: no level is cut
])
def test_coarse_unknowns_rule_against_oracle(dim, ne, p, hier, k):
    """Stopping at the first first-order level with at most k interior unknowns: the same plan,
    V-cycle (1e-10) and PCG iteration counts as the oracle."""
    from oracle import mg
    G, H = build_pair(dim, ne, p, hierarchy=hier, coarse_unknowns=k)
    assert [[list(lv.nelem)[:dim], lv.order] for lv in G.levels] == \
        [[list(n), q] for n, q in H.plan]
    m = H.fine.mesh
    b = random_vec(m.N, 13) * m.interior
    if hier != "low":
        for l, lv in enumerate(H.levels[:-1]):
            G.set_lmax(l, lv.lmax)
        assert rel_err(to_np(G.vcycle(to_dev(b))), H.vcycle(b)) <= 1e-10
    ro = mg.pcg(H, b, rtol=1e-10)
    rg = G.solve(to_dev(b), rtol=1e-10)
    assert rg.converged and rg.iters == ro.iters, (rg.iters, ro.iters)
    assert rel_err(rg.history, ro.history) <= 1e-9
    G.close()
