"""Pins of the oracle's Gauss-quadrature discretization (§2.3: Gauss quadrature at p+1 points
per axis, isoparametric geometry at the Gauss points, consistent mass) against what the rule and
the mathematics fix: the Gauss-Legendre closed forms and exactness degree, the derivative at the
Gauss points, exact stiffness and mass for Q_p polynomials on affine meshes (where collocated
GLL quadrature is not exact), symmetry, the constant null space, the linear-function energy on
warped meshes and spectral convergence."""

import math

import numpy as np
import pytest

from oracle import fem, mg
from paper_1402_5938_amd import inputs

WARP = inputs.map_warp_sine(0.05)
MU = inputs.mu_exp_sine_product(2.0)


def test_gauss_points_closed_forms_and_exactness():
    m = fem.Mesh(2, (1, 1), 1, inputs.map_identity(), inputs.field_const(1.0), "gauss")
    assert np.allclose(m.eta, [-1 / math.sqrt(3), 1 / math.sqrt(3)], rtol=0, atol=1e-15)
    assert np.allclose(m.wg, [1.0, 1.0], rtol=0, atol=1e-15)
    for p in (2, 5, 8, 16):
        m = fem.Mesh(2, (1, 1), p, inputs.map_identity(), inputs.field_const(1.0), "gauss")
        q = p + 1
        for k in range(2 * q):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(np.dot(m.wg, m.eta ** k) - exact) <= 1e-13
        # degree 2q is not integrated exactly
        assert abs(np.dot(m.wg, m.eta ** (2 * q)) - 2.0 / (2 * q + 1)) > 1e-11
        # interpolation and derivative at the Gauss points reproduce x^k, k <= p
        for k in range(p + 1):
            assert np.abs(m.Iq @ m.xi ** k - m.eta ** k).max() <= 1e-12
            if k:
                assert np.abs(m.Dq @ m.xi ** k - k * m.eta ** (k - 1)).max() <= 1e-11 * p * p


def _poly_energy(p, dim, quad):
    """u = prod_a x_a^p on [0,1]^d: returns (u^T K u, exact int |grad u|^2, u^T M u, exact int u^2)."""
    m = fem.Mesh(dim, (2,) * dim, p, inputs.map_identity(), inputs.field_const(1.0), quad)
    u = np.prod(m.x ** p, axis=1)
    K = fem.Stiffness(m).csr()
    # int_0^1 x^(2p) = 1/(2p+1); int (p x^(p-1))^2 = p^2/(2p-1)
    one = 1.0 / (2 * p + 1)
    der = p * p / (2 * p - 1)
    exact_k = dim * der * one ** (dim - 1)
    exact_m = one ** dim
    M = m.mass_matrix() if quad == "gauss" else None
    um = float(u @ (M @ u)) if M is not None else float(np.sum(m.lumped_mass() * u * u))
    return float(u @ (K @ u)), exact_k, um, exact_m


@pytest.mark.parametrize("dim,p", [(2, 3), (2, 6), (3, 2), (3, 4)])
def test_gauss_exact_for_qp_polynomials_where_gll_is_not(dim, p):
    ek, xk, em, xm = _poly_energy(p, dim, "gauss")
    assert abs(ek - xk) <= 1e-13 * xk and abs(em - xm) <= 1e-13 * xm
    gk, _, gm, _ = _poly_energy(p, dim, "gll")
    assert abs(gk - xk) > 1e-11 * xk and abs(gm - xm) > 1e-11 * xm


@pytest.mark.parametrize("dim,ne,p", [(2, (3, 2), 4), (3, (2, 1, 2), 3)])
def test_gauss_stiffness_invariants(dim, ne, p):
    m = fem.Mesh(dim, ne, p, WARP, MU, "gauss")
    K = fem.Stiffness(m).csr().toarray()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(K @ np.ones(m.N)).max() <= 1e-12 * np.abs(K).max()
    idx = np.nonzero(m.interior)[0]
    assert np.linalg.eigvalsh(K[np.ix_(idx, idx)]).min() > 0
    # element blocks are dense: every pair of an element's nodes couples (unlike collocation)
    e0 = m.conn[0]
    assert np.count_nonzero(np.abs(K[np.ix_(e0, e0)]) > 0) == len(e0) ** 2
    # a function linear in the physical coordinates: u^T K u = |a|^2 sum_q w detJ mu
    a = np.array([0.3, -1.1, 0.7][:dim])
    u = m.x @ a
    _, wdet, mu, _ = m.geometry()
    assert abs(u @ K @ u - (a @ a) * np.sum(wdet * mu)) <= 1e-11 * (a @ a) * np.sum(wdet * mu)
    # the operator through the factored form equals the assembled matrix
    x = np.random.default_rng(0).standard_normal(m.N)
    op = fem.LevelOperator(m)
    assert np.abs(op.apply(x, neumann=True) - K @ x).max() <= 1e-12 * np.abs(K @ x).max()
    # the diagonal
    assert np.abs(op.diag() - np.diag(K) * m.interior).max() <= 1e-13 * np.abs(np.diag(K)).max()


def test_gauss_consistent_mass_volume():
    m = fem.Mesh(3, (2, 2, 1), 3, WARP, MU, "gauss")
    M = m.mass_matrix()
    _, wdet, _, _ = m.geometry()
    one = np.ones(m.N)
    assert abs(one @ (M @ one) - wdet.sum()) <= 1e-13
    # the warp moves the boundary but keeps the volume (mean of the sine terms is 0)
    assert abs(wdet.sum() - 1.0) <= 1e-6


def test_gauss_discretization_converges_spectrally():
    errs = []
    for p in (2, 4, 6, 8):
        prob = inputs.poisson2d_manufactured(nelem=2, order=p)
        m = fem.Mesh(2, (2, 2), p, prob.map, prob.mu, "gauss")
        op = fem.LevelOperator(m)
        b = fem.load_vector(m, fem.nodal_field(m, prob.f))
        A, idx = op.dense_interior()
        u = np.zeros(m.N)
        u[idx] = np.linalg.solve(A, b[idx])
        exact = np.sin(np.pi * m.x[:, 0]) * np.sin(np.pi * m.x[:, 1])
        errs.append(np.abs(u - exact).max())
    assert errs[-1] < 1e-6 and all(errs[i + 1] < errs[i] / 5 for i in range(len(errs) - 1))


def test_gauss_multigrid_solves():
    H = mg.Hierarchy(3, (2, 2, 2), 4, WARP, MU, hierarchy="p", quadrature="gauss")
    m = H.fine.mesh
    b = fem.load_vector(m, np.ones(m.N))
    A, idx = H.fine.op.dense_interior()
    xs = np.linalg.solve(A, b[idx])
    res = mg.pcg(H, b, rtol=1e-10)
    assert res.converged and np.abs(res.x[idx] - xs).max() <= 1e-8 * np.abs(xs).max()
