"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

Each group targets mistakes that could hide in one oracle function (a dropped term, a wrong
sign or index, a transposed operand): closed forms, printed values of the paper, exactness of
the quadrature, invariants, special cases that reduce to textbook stencils, and dense brute
force on tiny meshes. CPU only.
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem, gll, mg, splitmix, transfer
from oracle.fields import eval_map
from paper_1402_5938_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------- GLL rule
def test_gll_closed_forms():
    s37 = math.sqrt(3.0 / 7.0)
    cases = {
        1: ([-1, 1], [1, 1]),
        2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
        3: ([-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
        4: ([-1, -s37, 0, s37, 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
    }
    for p, (xs, ws) in cases.items():
        x, w = gll.gll(p)
        np.testing.assert_allclose(x, xs, atol=1e-15)
        np.testing.assert_allclose(w, ws, atol=1e-15)


def test_gll_matches_paper_figure1():
    """Figure 1 draws the p = 4 GLL points of an element of [0, 1] at 0, .1727, .5, .8273, 1."""
    printed = np.loadtxt(os.path.join(GOLDEN, "fig1_gll_p4.txt"))
    x, _ = gll.gll(4)
    np.testing.assert_allclose((x + 1) / 2, printed, atol=5e-5)
    # the h-coarsened element of Fig. 1 carries the same points scaled by 2 (on [0, 2])
    np.testing.assert_allclose(2 * (x + 1) / 2, 2 * printed, atol=1e-4)


@pytest.mark.parametrize("p", list(range(1, 17)))
def test_gll_exactness(p):
    x, w = gll.gll(p)
    assert abs(w.sum() - 2) < 1e-14
    for k in range(0, 2 * p):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) < 1e-13, (p, k)
    # Lobatto, not Gauss: degree 2p is not integrated exactly
    assert abs(np.sum(w * x ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-10
    # interior nodes are the roots of P_p'
    P, Pm1 = gll.legendre(p, x[1:-1])
    assert np.all(np.abs(p * (Pm1 - x[1:-1] * P)) < 1e-12)


# ---------------------------------------------------------------------------- derivative / interpolation
def test_deriv_matrix_p2_closed_form():
    D = gll.deriv_matrix(gll.gll(2)[0])
    np.testing.assert_allclose(D, [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 8, 12, 16])
def test_deriv_matrix_differentiates_polynomials(p):
    x, _ = gll.gll(p)
    D = gll.deriv_matrix(x)
    np.testing.assert_allclose(D @ np.ones(p + 1), 0, atol=1e-12)
    for k in range(1, p + 1):
        np.testing.assert_allclose(D @ x ** k, k * x ** (k - 1), atol=1e-10 * k * k)
    # closed-form endpoint entries D_00 = -p(p+1)/4, D_pp = p(p+1)/4
    assert abs(D[0, 0] + p * (p + 1) / 4) < 1e-10 * p * p
    assert abs(D[p, p] - p * (p + 1) / 4) < 1e-10 * p * p


@pytest.mark.parametrize("pc,pf", [(1, 2), (2, 4), (4, 8), (8, 16), (3, 6), (6, 12)])
def test_interpolation_reproduces_polynomials(pc, pf):
    xc, _ = gll.gll(pc)
    xf, _ = gll.gll(pf)
    M = gll.lagrange_eval(xc, xf)
    np.testing.assert_allclose(M.sum(axis=1), 1, atol=1e-13)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(pc + 1)
    np.testing.assert_allclose(M @ np.polyval(c, xc), np.polyval(c, xf), atol=1e-11)
    # h-children: the coarse interpolant evaluated on each half
    for ch in (0, 1):
        Mh = gll.lagrange_eval(xc, (xc + 2 * ch - 1) / 2)
        np.testing.assert_allclose(Mh @ np.polyval(c, xc), np.polyval(c, (xc + 2 * ch - 1) / 2),
                                   atol=1e-11)


# ---------------------------------------------------------------------------- geometry
@pytest.mark.parametrize("dim,ne,p", [(2, 3, 4), (3, 2, 3)])
def test_geometry_unit_box(dim, ne, p):
    m = fem.Mesh(dim, (ne,) * dim, p, inputs.map_identity(), inputs.field_const(1.0))
    G, wdet, mu, detJ = m.geometry()
    _, w = gll.gll(p)
    wq = w
    for _ in range(dim - 1):
        wq = np.multiply.outer(w, wq)
    expect = wq.ravel()[None, :] * (2.0 * ne) ** (2 - dim)
    for a in range(dim):
        np.testing.assert_allclose(G[:, :, a, a], np.broadcast_to(expect, G.shape[:2]), rtol=1e-13)
        for b in range(dim):
            if a != b:
                assert np.max(np.abs(G[:, :, a, b])) < 1e-14
    np.testing.assert_allclose(detJ, (2.0 * ne) ** (-dim), rtol=1e-13)
    assert abs(wdet.sum() - 1.0) < 1e-13


def test_geometry_affine_volume():
    M = np.array([[1.3, 0.2, -0.1], [0.1, 0.9, 0.3], [0.0, -0.2, 1.1]])
    m = fem.Mesh(3, (2, 3, 2), 3, inputs.map_affine(M, [0.5, -1.0, 2.0]), inputs.field_const(1.0))
    _, wdet, _, _ = m.geometry()
    assert abs(wdet.sum() - abs(np.linalg.det(M))) < 1e-13


def test_warped_volume_is_one():
    """det(grad Phi) of the cyclic sine warp integrates to exactly 1 over the unit cube, and
    every non-constant term of it is odd under a reflection of the uniform mesh, so the
    isoparametric GLL volume is 1 to rounding at every order."""
    for p in (1, 2, 3, 4, 6, 8):
        m = fem.Mesh(3, (2, 2, 2), p, inputs.map_warp_sine(0.05), inputs.field_const(1.0))
        _, wdet, _, _ = m.geometry()
        assert abs(wdet.sum() - 1.0) < 1e-13


def test_coefficient_integral_converges_spectrally():
    """sum_q w_q detJ_q mu_q -> int_Omega mu: differences between successive orders shrink
    exponentially on a fixed mesh."""
    vals = []
    for p in (2, 4, 6, 8, 10):
        m = fem.Mesh(2, (3, 3), p, inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0))
        _, wdet, mu, _ = m.geometry()
        vals.append(np.sum(wdet * mu))
    diffs = [abs(vals[i + 1] - vals[i]) for i in range(len(vals) - 1)]
    assert diffs[-1] < 1e-7
    assert all(diffs[i + 1] < 0.2 * diffs[i] for i in range(len(diffs) - 1)), diffs


def test_exp_sine_product_values_fixed_by_the_workload():
    """The 3D workload's coefficient exp(4.6 sx sy sz) (sW = sin 2 pi W): its maximum e^4.6 sits
    at (1/4, 1/4, 1/4), its minimum e^-4.6 at (3/4, 1/4, 1/4), it is exactly 1 on every plane
    x_i = 0 or 1/2, so the contrast max/min over any point set containing the two extrema is
    e^9.2 ~ 9.9e3 (the stated contrast of about 1e4). A phase shifts the extremum to
    (1/4 - phase). A wrong amplitude, a missing 2 pi or a wrong phase sign fails one of these."""
    from oracle.fields import eval_scalar
    mu = inputs.mu_exp_sine_product(4.6)
    pts = np.array([[0.25, 0.25, 0.25], [0.75, 0.25, 0.25], [0.25, 0.75, 0.75]])
    np.testing.assert_allclose(eval_scalar(mu, pts), [math.exp(4.6), math.exp(-4.6), math.exp(4.6)],
                               rtol=1e-14)
    rng = np.random.default_rng(5)
    for axis in range(3):
        for plane in (0.0, 0.5):
            q = rng.uniform(0, 1, (50, 3))
            q[:, axis] = plane
            np.testing.assert_allclose(eval_scalar(mu, q), 1.0, atol=1e-14)
    # contrast over the nodes of an unwarped 4^3 mesh at p = 2 (nodes on the quarter planes)
    m = fem.Mesh(3, (4, 4, 4), 2, inputs.map_identity(), mu)
    v = eval_scalar(mu, m.x)
    assert abs(v.max() / v.min() - math.exp(9.2)) < 1e-9 * math.exp(9.2)
    # phases: the maximum moves to 1/4 - phase (2D: two factors)
    ph = (0.1, 0.3, 0.05)
    mu3 = inputs.mu_exp_sine_product(2.0, ph)
    assert abs(eval_scalar(mu3, np.array([[0.15, -0.05, 0.2]]))[0] - math.exp(2.0)) < 1e-13
    mu2 = inputs.mu_exp_sine_product(1.5, ph[:2])
    assert abs(eval_scalar(mu2, np.array([[0.15, -0.05]]))[0] - math.exp(1.5)) < 1e-13
    assert abs(eval_scalar(mu2, np.array([[0.65, -0.05]]))[0] - math.exp(-1.5)) < 1e-13


def test_exp_fourier_single_modes_closed_form():
    """One mode (J = 1): g = sqrt(2) a cos(2 pi k.x + phi). With k = e_axis, phi = pi/2 this is
    -sqrt(2) a sin(2 pi x_axis): the values at x_axis = 0, 1/4, 3/4 are 1, e^{-sqrt2 a},
    e^{+sqrt2 a}, and the other coordinates do not matter. A diagonal k = (1, 1, -1) with phi = 0
    is periodic along (1, -1, 0) and equals e^{sqrt2 a} wherever x + y - z is an integer."""
    from oracle.fields import eval_scalar
    rng = np.random.default_rng(1)
    for axis in range(3):
        k = [0.0, 0.0, 0.0]
        k[axis] = 1.0
        a = 0.8
        mu = inputs.mu_exp_fourier(np.array([k + [a, math.pi / 2]]))
        q = rng.uniform(0, 1, (3, 3))
        q[:, axis] = [0.0, 0.25, 0.75]
        np.testing.assert_allclose(eval_scalar(mu, q),
                                   [1.0, math.exp(-math.sqrt(2) * a), math.exp(math.sqrt(2) * a)],
                                   rtol=1e-14)
    mu = inputs.mu_exp_fourier(np.array([[1.0, 1.0, -1.0, 0.5, 0.0]]))
    q = rng.uniform(0, 1, (20, 2))
    pts = np.stack([q[:, 0], q[:, 1], q[:, 0] + q[:, 1] - 1.0], axis=1)
    np.testing.assert_allclose(eval_scalar(mu, pts), math.exp(math.sqrt(2) * 0.5), rtol=1e-13)


def test_exp_fourier_batch_field_is_standard_normal_and_mean_free():
    """The batched workload's log-coefficient g = sqrt(2/J) sum_j a_j cos(2 pi k_j.x + phi_j),
    a_j ~ N(0,1), phi_j ~ U[0, 2 pi), is N(0,1) at every point over the draws: across the 256
    problems' spawned seeds ln mu at a fixed point has sample mean ~ 0 (standard error 1/16)
    and sample variance ~ 1 (standard error ~0.09). Every k_j is a nonzero integer vector, so
    each draw's g integrates to exactly 0 over the unit cube (checked by high-order GLL
    quadrature). A wrong sqrt(2/J), a missing 2 pi or a non-integer frequency fails."""
    from oracle.fields import eval_scalar
    probs = inputs.batched_problems(seed=0, count=256)
    pts = np.array([[0.1, 0.2, 0.3], [0.5, 0.5, 0.5], [0.9, 0.35, 0.65], [0.0, 0.0, 0.0]])
    L = np.array([np.log(eval_scalar(pb.mu, pts)) for pb in probs])     # (256, npts)
    for j in range(pts.shape[0]):
        assert abs(L[:, j].mean()) < 0.25, (j, L[:, j].mean())
        assert abs(L[:, j].var() - 1.0) < 0.3, (j, L[:, j].var())
    assert abs(L.mean()) < 0.15 and abs(L.var() - 1.0) < 0.2
    m = fem.Mesh(3, (2, 2, 2), 12, inputs.map_identity(), inputs.field_const(1.0))
    _, wdet, _, _ = m.geometry()
    for pb in probs[:8]:
        _, _, mu, _ = fem.Mesh(3, (2, 2, 2), 12, inputs.map_identity(), pb.mu).geometry()
        assert abs(np.sum(wdet * np.log(mu))) < 1e-9


def test_warp_map_values_and_jacobian():
    """Cyclic sine warp, a = 0.05: Phi(1/4,1/4,1/4) = (1/4 + a)(1,1,1) and Phi(3/4,1/4,1/4) moves
    y and z by -a and x by +a; on the face X = 0 only x moves (by a sY sZ); 2D: Phi(1/4,3/4) =
    (1/4 - a, 3/4 + a). The oracle's isoparametric detJ at p = 12 agrees with central
    differences of the map to the interpolation error of the degree-12 geometry."""
    a = 0.05
    P = eval_map(inputs.map_warp_sine(a), np.array([[0.25, 0.25, 0.25], [0.75, 0.25, 0.25]]))
    np.testing.assert_allclose(P, [[0.25 + a] * 3, [0.75 + a, 0.25 - a, 0.25 - a]], atol=1e-15)
    q = np.random.default_rng(2).uniform(0, 1, (10, 3))
    q[:, 0] = 0.0
    P = eval_map(inputs.map_warp_sine(a), q)
    np.testing.assert_allclose(P[:, 1:], q[:, 1:], atol=1e-15)
    np.testing.assert_allclose(P[:, 0], a * np.sin(2 * math.pi * q[:, 1]) * np.sin(2 * math.pi * q[:, 2]),
                               atol=1e-15)
    P2 = eval_map(inputs.map_warp_sine(a), np.array([[0.25, 0.75]]))
    np.testing.assert_allclose(P2, [[0.25 - a, 0.75 + a]], atol=1e-15)
    m = fem.Mesh(3, (1, 1, 1), 12, inputs.map_warp_sine(a), inputs.field_const(1.0))
    detJ = m.geometry()[3].reshape(-1)        # element-local points, z slowest, x fastest
    h = 1e-6
    xi, _ = gll.gll(12)
    Z, Y, Xg = np.meshgrid((xi + 1) / 2, (xi + 1) / 2, (xi + 1) / 2, indexing="ij")
    ref = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], axis=1)
    J = np.zeros((ref.shape[0], 3, 3))
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        J[:, :, b] = (eval_map(inputs.map_warp_sine(a), ref + e) - eval_map(inputs.map_warp_sine(a), ref - e)) / (2 * h)
    det_fd = np.linalg.det(J) / 8.0          # reference element [-1,1]^3 -> [0,1]^3
    # degree-12 interpolation of one full sine period per element: ~5e-7 relative
    np.testing.assert_allclose(detJ, det_fd, rtol=2e-6)
    assert np.ptp(det_fd) * 8 > 0.15             # the warp really varies the Jacobian


def test_sin_product_and_cos2_sum_values():
    """sin_product: amp at the centre, 0 on the boundary; cos2_sum (the paper's coefficient form
    1 + 1e6 sum cos^2(2 pi x_i)): c0 + d c1 at the origin and c0 where every 2 pi x_i = pi/2."""
    from oracle.fields import eval_scalar
    f = inputs.f_sin_product(3.0, 1.0)
    np.testing.assert_allclose(eval_scalar(f, np.array([[0.5, 0.5], [0.0, 0.3], [0.7, 1.0]])),
                               [3.0, 0.0, 0.0], atol=1e-15)
    c = inputs.mu_cos2_sum(1.0, 1e6, 2.0)
    v = eval_scalar(c, np.array([[0.0, 0.0, 0.0], [0.25, 0.75, 0.25], [0.25, 0.5, 0.75]]))
    np.testing.assert_allclose(v, [1.0 + 3e6, 1.0, 1.0 + 1e6], rtol=1e-12)


def test_geometry_rejects_folded_map():
    with pytest.raises(ValueError):
        m = fem.Mesh(2, (2, 2), 2, inputs.map_warp_sine(0.5), inputs.field_const(1.0))
        m.geometry()


# ---------------------------------------------------------------------------- stiffness
def _mesh(dim, ne, p, warped=True, mu=None):
    mp = inputs.map_warp_sine(0.05) if warped else inputs.map_identity()
    return fem.Mesh(dim, (ne,) * dim, p, mp, mu or inputs.mu_exp_sine_product(2.0))


@pytest.mark.parametrize("dim,ne,p", [(2, 3, 3), (2, 2, 5), (3, 2, 2), (3, 1, 4)])
def test_stiffness_symmetric_nullspace_spd(dim, ne, p):
    m = _mesh(dim, ne, p)
    K = fem.Stiffness(m)
    A = K.csr().toarray()
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    np.testing.assert_allclose(A @ np.ones(m.N), 0, atol=1e-11 * np.abs(A).max())
    idx = np.nonzero(m.interior)[0]
    sla.cholesky(A[np.ix_(idx, idx)])        # raises if not SPD
    x = np.random.default_rng(0).standard_normal(m.N)
    np.testing.assert_allclose(K.matvec(x), A @ x, rtol=1e-12, atol=1e-12 * np.abs(A).max())
    np.testing.assert_allclose(K.diagonal(), np.diag(A), rtol=1e-13)


def test_abs_product_bounds_product():
    """|B|^T|G||B||x| >= |A x| entrywise, with equality for x >= 0 on a mesh where every
    factor is nonnegative (unit box, mu = 1, p = 1: D has one negative column, so compare
    with the dense absolute-value product instead)."""
    m = _mesh(3, 2, 4)
    op = fem.LevelOperator(m)
    x = np.random.default_rng(3).standard_normal(m.N)
    ya, y = op.apply_abs(x, neumann=True), op.apply(x, neumann=True)
    assert np.all(ya >= np.abs(y) - 1e-12 * ya.max())
    K = fem.Stiffness(m)
    dense = sum(abs(K.B[a]).T.toarray() @ np.diag(np.abs(K.G[:, a, b])) @ abs(K.B[b]).toarray()
                for a in range(3) for b in range(3))
    np.testing.assert_allclose(ya, dense @ np.abs(x), rtol=1e-12)


@pytest.mark.parametrize("dim,ne,p", [(2, 3, 3), (3, 2, 3)])
def test_energy_of_linear_functions(dim, ne, p):
    """grad u = a exactly for u = a.x + c (linear functions lie in the isoparametric space),
    so u^T A u = |a|^2 sum_q w_q detJ_q mu_q on any mesh and coefficient."""
    m = _mesh(dim, ne, p)
    K = fem.Stiffness(m)
    a = np.array([0.7, -1.3, 0.4][:dim])
    u = m.x @ a + 0.25
    _, wdet, mu, _ = m.geometry()
    expect = (a @ a) * np.sum(wdet * mu)
    assert abs(u @ K.matvec(u) - expect) < 1e-12 * expect


@pytest.mark.parametrize("dim,p", [(2, 4), (3, 3), (2, 7)])
def test_energy_of_monomials_unit_box(dim, p):
    """mu = 1 on the unit box: int |grad x^k|^2 = k^2 / (2k-1) for k <= p, computed exactly by
    the GLL rule (integrand degree 2k-2 <= 2p-1 in x, constant in the other variables)."""
    m = fem.Mesh(dim, (2,) * dim, p, inputs.map_identity(), inputs.field_const(1.0))
    K = fem.Stiffness(m)
    for k in range(1, p + 1):
        for axis in range(dim):
            u = m.x[:, axis] ** k
            assert abs(u @ K.matvec(u) - k * k / (2 * k - 1)) < 1e-12, (k, axis)


def test_p1_is_finite_difference_laplacian():
    """p = 1 with nodal quadrature on a uniform grid gives the 5-point Laplacian in 2D and
    h times the 7-point Laplacian in 3D."""
    for dim, ne in ((2, 5), (3, 4)):
        m = fem.Mesh(dim, (ne,) * dim, 1, inputs.map_identity(), inputs.field_const(1.0))
        op = fem.LevelOperator(m)
        A, idx = op.dense_interior()
        h = 1.0 / ne
        scale = 1.0 if dim == 2 else h
        G = m.grid[:, idx].T
        dist = np.abs(G[:, None, :] - G[None, :, :]).sum(axis=2)
        expect = np.where(dist == 0, 2 * dim, np.where(dist == 1, -1.0, 0.0)) * scale
        np.testing.assert_allclose(A, expect, atol=1e-14)


def test_element_matrix_brute_force():
    """Dense element matrices from the quadrature sum written out with loops:
    K_e[i,j] = sum_q sum_ab dphi_i/dxi_a(q) G_ab(q) dphi_j/dxi_b(q)."""
    for dim, ne, p in ((2, 2, 2), (3, 1, 2)):
        m = _mesh(dim, ne, p)
        G, _, _, _ = m.geometry()
        n, nl = m.n, m.nloc
        D = m.D
        loc = m.local
        A = np.zeros((m.N, m.N))
        for e in range(m.E):
            Ke = np.zeros((nl, nl))
            for q in range(nl):
                grad = np.zeros((dim, nl))     # dphi_i/dxi_a at q
                for i in range(nl):
                    for a in range(dim):
                        others = all(loc[c][i] == loc[c][q] for c in range(dim) if c != a)
                        if others:
                            grad[a, i] = D[loc[a][q], loc[a][i]]
                Ke += grad.T @ G[e, q] @ grad
            A[np.ix_(m.conn[e], m.conn[e])] += Ke
        np.testing.assert_allclose(fem.Stiffness(m).csr().toarray(), A, atol=1e-12 * np.abs(A).max())


def test_load_vector_integrates_f():
    """b = M_L f: sum of b over all nodes (unmasked) is the GLL quadrature of f."""
    m = fem.Mesh(2, (3, 3), 4, inputs.map_identity(), inputs.field_const(1.0))
    f = np.sin(math.pi * m.x[:, 0]) * np.sin(math.pi * m.x[:, 1])
    b = m.lumped_mass() * f
    assert abs(b.sum() - 4 / math.pi ** 2) < 1e-6


# ---------------------------------------------------------------------------- transfers
@pytest.mark.parametrize("dim,nef,pf,nec,pc", [(2, 4, 4, 2, 4), (2, 2, 4, 2, 2), (3, 2, 2, 1, 2),
                                               (3, 2, 4, 2, 2), (2, 3, 6, 3, 3), (3, 2, 1, 1, 1)])
def test_prolongation_definition_and_reproduction(dim, nef, pf, nec, pc):
    mp = inputs.map_warp_sine(0.05)
    mu = inputs.field_const(1.0)
    fine = fem.Mesh(dim, (nef,) * dim, pf, mp, mu)
    coarse = fem.Mesh(dim, (nec,) * dim, pc, mp, mu)
    Pd = transfer.prolongation_direct(fine, coarse)
    Pk = transfer.prolongation(fine, coarse)
    np.testing.assert_allclose(Pd.toarray(), Pk.toarray(), atol=1e-14)
    np.testing.assert_allclose(Pk @ np.ones(coarse.N), 1.0, atol=1e-13)
    # a polynomial of degree <= pc per axis in reference coordinates is reproduced
    rng = np.random.default_rng(3)
    coefs = [rng.standard_normal(pc + 1) for _ in range(dim)]

    def poly(X):
        v = np.ones(X.shape[0])
        for a in range(dim):
            v = v * np.polyval(coefs[a], X[:, a])
        return v
    np.testing.assert_allclose(Pk @ poly(coarse.X), poly(fine.X), atol=1e-11)
    # restriction is the exact transpose on interior unknowns
    T = transfer.Transfer(fine, coarse)
    r = rng.standard_normal(fine.N) * fine.interior
    e = rng.standard_normal(coarse.N) * coarse.interior
    assert abs(T.restrict(r) @ e - r @ T.prolong(e)) < 1e-12 * np.abs(r).sum()


def test_transfer_rejects_unrelated_levels():
    a = fem.Mesh(2, (4, 4), 2, inputs.map_identity(), inputs.field_const(1.0))
    b = fem.Mesh(2, (3, 3), 2, inputs.map_identity(), inputs.field_const(1.0))
    with pytest.raises(ValueError):
        transfer.relation(a, b)


# ---------------------------------------------------------------------------- hierarchy plan
def test_plan_levels():
    assert mg.plan_levels(2, (4, 4), 4, "h") == [((4, 4), 4), ((2, 2), 4), ((1, 1), 4)]
    assert mg.plan_levels(3, (16,) * 3, 8, "p") == [((16,) * 3, 8), ((16,) * 3, 4), ((16,) * 3, 2),
                                                    ((16,) * 3, 1), ((8,) * 3, 1), ((4,) * 3, 1),
                                                    ((2,) * 3, 1)]
    assert mg.plan_levels(3, (8,) * 3, 16, "p")[-1] == ((2,) * 3, 1)
    assert len(mg.plan_levels(3, (8,) * 3, 16, "p")) == 7
    # the paper's 2D p = 16 example: five orders on the fine mesh, then two h-levels (§4.3)
    lv = mg.plan_levels(2, (32, 32), 16, "p", max_levels=7)
    assert [q for _, q in lv] == [16, 8, 4, 2, 1, 1, 1] and lv[-1][0] == (8, 8)
    assert mg.plan_levels(3, (24,) * 3, 12, "p")[-1] == ((3,) * 3, 1)
    assert [q for _, q in mg.plan_levels(2, (8, 8), 12, "p")][:5] == [12, 6, 3, 2, 1]
    assert mg.plan_levels(3, (16,) * 3, 8, "p", max_levels=4)[-1] == ((16,) * 3, 1)


def test_plan_levels_coarse_unknowns():
    """Halving stops at the first first-order level with at most k interior unknowns."""
    full = mg.plan_levels(3, (16,) * 3, 8, "p")
    assert mg.plan_levels(3, (16,) * 3, 8, "p", coarse_unknowns=4096) == full[:4]   # 15^3 = 3375
    assert mg.plan_levels(3, (16,) * 3, 8, "p", coarse_unknowns=3375) == full[:4]
    assert mg.plan_levels(3, (16,) * 3, 8, "p", coarse_unknowns=3374) == full[:5]   # 7^3 = 343
    assert mg.plan_levels(3, (16,) * 3, 8, "p", coarse_unknowns=26) == full         # 1^3 at 2^3
    assert mg.plan_levels(3, (16,) * 3, 8, "p", coarse_unknowns=1) == full
    assert mg.plan_levels(3, (8,) * 3, 16, "p", coarse_unknowns=4096)[-1] == ((8,) * 3, 1)
    # levels of order > 1 are never cut short: the h-hierarchy at p = 4 keeps every level
    assert mg.plan_levels(2, (16, 16), 4, "h", coarse_unknowns=4096) == mg.plan_levels(2, (16, 16), 4, "h")
    # the first-order hierarchy: its first first-order level (on the order-p nodes) when small
    assert mg.plan_levels(3, (2, 2, 2), 4, "low", coarse_unknowns=4096) == [((2,) * 3, 4), ((8,) * 3, 1)]
    assert mg.plan_levels(2, (64, 64), 16, "p", coarse_unknowns=4096)[-1] == ((64, 64), 1)  # 63^2
    assert mg.plan_levels(2, (66, 66), 1, "h", coarse_unknowns=4096)[-1] == ((33, 33), 1)


# ---------------------------------------------------------------------------- smoothers
def _gen_eig(dim=2, ne=2, p=3):
    H = mg.Hierarchy(dim, (ne,) * dim, p, inputs.map_warp_sine(0.05), inputs.mu_exp_sine_product(2.0),
                     hierarchy="h", max_levels=1)
    lv = H.levels[0]
    A, idx = lv.op.dense_interior()
    Dg = np.diag(A)
    lam, V = sla.eigh(A, np.diag(Dg))
    return H, lv, A, idx, lam, V


def test_jacobi_error_factor():
    H, lv, A, idx, lam, V = _gen_eig()
    for j in (0, len(lam) // 2, len(lam) - 1):
        x0 = np.zeros(lv.mesh.N)
        x0[idx] = V[:, j]
        x = mg.jacobi(lv.op, lv.dinv, np.zeros(lv.mesh.N), x0, 3, 2.0 / 3.0)
        np.testing.assert_allclose(x[idx], (1 - 2.0 / 3.0 * lam[j]) ** 3 * V[:, j], atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6])
def test_chebyshev_error_factor(k):
    H, lv, A, idx, lam, V = _gen_eig()
    lmax = lam[-1]
    beta, alpha = lmax, lmax / 4
    theta, delta = (beta + alpha) / 2, (beta - alpha) / 2

    def T(kk, t):
        t = np.asarray(t, dtype=float)
        return np.where(np.abs(t) <= 1, np.cos(kk * np.arccos(np.clip(t, -1, 1))),
                        np.cosh(kk * np.arccosh(np.maximum(np.abs(t), 1))) * np.sign(t) ** kk)
    for j in (0, 3, len(lam) // 2, len(lam) - 1):
        x0 = np.zeros(lv.mesh.N)
        x0[idx] = V[:, j]
        x = mg.chebyshev(lv.op, lv.dinv, lmax, np.zeros(lv.mesh.N), x0, k, 0.25)
        fac = T(k, (theta - lam[j]) / delta) / T(k, theta / delta)
        np.testing.assert_allclose(x[idx], fac * V[:, j], atol=1e-11)


def test_chebyshev_zero_guess_matches_general_form():
    """With x = 0 on entry the smoother is the same polynomial (one apply saved)."""
    H, lv, A, idx, lam, V = _gen_eig()
    b = np.zeros(lv.mesh.N)
    b[idx] = np.random.default_rng(5).standard_normal(len(idx))
    x1 = mg.chebyshev(lv.op, lv.dinv, lam[-1], b, None, 4)
    x2 = mg.chebyshev(lv.op, lv.dinv, lam[-1], b, np.zeros_like(b), 4)
    np.testing.assert_allclose(x1, x2, atol=1e-13)


def test_lanczos_estimate():
    H, lv, A, idx, lam, V = _gen_eig(2, 2, 3)          # 25 interior unknowns
    v0 = splitmix.start_vector(7, 0, lv.mesh.N)
    est, al, be = mg.lanczos_lmax(lv.op, lv.dinv, v0, 10)
    assert est <= lam[-1] * (1 + 1e-12)
    assert est >= 0.9 * lam[-1]
    assert len(al) == 10
    # exact when the number of unknowns is <= the step count
    H2, lv2, A2, idx2, lam2, _ = _gen_eig(2, 1, 3)       # 4 interior unknowns
    v0 = splitmix.start_vector(7, 0, lv2.mesh.N)
    est2, al2, _ = mg.lanczos_lmax(lv2.op, lv2.dinv, v0, 10)
    assert abs(est2 - lam2[-1]) < 1e-12 * lam2[-1]
    assert len(al2) <= 4


def test_splitmix64_published_outputs():
    """First outputs of SplitMix64 seeded with 0 (state advances by the golden gamma)."""
    g = 0x9E3779B97F4A7C15
    assert int(splitmix.splitmix64(np.uint64(0))) == 0xE220A8397B1DCDAF
    assert int(splitmix.splitmix64(np.uint64(g))) == 0x6E789E6AA1B965F4
    assert int(splitmix.splitmix64(np.uint64((2 * g) % 2 ** 64))) == 0x06C45D188009454F


# ---------------------------------------------------------------------------- V-cycle and solvers
def _small_h(dim=2, ne=4, p=2, smoother="chebyshev", nu=3, **kw):
    return mg.Hierarchy(dim, (ne,) * dim, p, inputs.map_warp_sine(0.05),
                        inputs.mu_exp_sine_product(2.0), hierarchy=kw.pop("hierarchy", "h"),
                        smoother=smoother, nu=nu, **kw)


def _materialize(H, li=0):
    lv = H.levels[li]
    idx = np.nonzero(lv.mesh.interior)[0]
    Vm = np.zeros((len(idx), len(idx)))
    for j, g in enumerate(idx):
        r = np.zeros(lv.mesh.N)
        r[g] = 1.0
        Vm[:, j] = H.vcycle(r)[idx]
    return Vm, idx


@pytest.mark.parametrize("smoother,hier", [("chebyshev", "h"), ("jacobi", "h"), ("chebyshev", "p")])
def test_vcycle_symmetric_and_convergent(smoother, hier):
    H = _small_h(smoother=smoother, hierarchy=hier, ne=4, p=2)
    Vm, idx = _materialize(H)
    np.testing.assert_allclose(Vm, Vm.T, atol=1e-12 * np.abs(Vm).max())
    A, _ = H.fine.op.dense_interior()
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(len(idx)) - Vm @ A)))
    assert rho < 0.5


def test_one_level_vcycle_is_exact_solve():
    H = _small_h(max_levels=1, ne=2, p=3)
    A, idx = H.fine.op.dense_interior()
    r = np.zeros(H.fine.mesh.N)
    r[idx] = np.random.default_rng(2).standard_normal(len(idx))
    np.testing.assert_allclose(H.vcycle(r)[idx], np.linalg.solve(A, r[idx]), rtol=1e-10)


def test_solvers_match_dense_solve():
    H = _small_h(dim=2, ne=4, p=3, hierarchy="h")
    A, idx = H.fine.op.dense_interior()
    b = np.zeros(H.fine.mesh.N)
    b[idx] = np.random.default_rng(4).standard_normal(len(idx))
    u = np.linalg.solve(A, b[idx])
    kappa = np.linalg.cond(A)
    for res in (mg.pcg(H, b, rtol=1e-12), mg.mg_solve(H, b, rtol=1e-12)):
        assert res.converged
        assert np.linalg.norm(res.x[idx] - u) <= 1e-12 * kappa * np.linalg.norm(u)


def test_pcg_equals_textbook_cg_with_materialized_vcycle():
    H = _small_h(dim=2, ne=4, p=2, hierarchy="p")
    Vm, idx = _materialize(H)
    A, _ = H.fine.op.dense_interior()
    b = np.zeros(H.fine.mesh.N)
    b[idx] = np.random.default_rng(6).standard_normal(len(idx))
    res = mg.pcg(H, b, rtol=1e-10)
    # textbook PCG on dense arrays
    x = np.zeros(len(idx))
    r = b[idx].copy()
    z = Vm @ r
    p = z.copy()
    g = z @ r
    n0 = np.linalg.norm(r)
    it = 0
    while True:
        it += 1
        h = A @ p
        al = g / (p @ h)
        x += al * p
        r -= al * h
        if np.linalg.norm(r) <= 1e-10 * n0:
            break
        z = Vm @ r
        gn = z @ r
        p = z + gn / g * p
        g = gn
    assert it == res.iters
    np.testing.assert_allclose(res.x[idx], x, rtol=1e-8, atol=1e-12 * np.abs(x).max())


def test_cost_model_seven_fine_applies_per_iteration():
    """§4.3: with three smoothing steps before and three after, each PCG iteration costs one
    residual-type product plus six smoothing products on the finest level (7 N g_p)."""
    for smoother in ("chebyshev", "jacobi"):
        H = _small_h(smoother=smoother, nu=3, ne=4, p=2, hierarchy="p")
        b = np.zeros(H.fine.mesh.N)
        b[H.fine.mesh.interior] = 1.0
        H.fine.op.applies = 0                 # the setup's Lanczos products are not counted
        res = mg.pcg(H, b, rtol=1e-8)
        # per iteration: A p (1) + one V-cycle: pre-smoothing from zero (2) + residual (1) +
        # post-smoothing (3). The initial V-cycle stands in for the one skipped after
        # convergence; one more product checks the true residual.
        expected = 7 * res.iters + 1
        assert H.fine.op.applies == expected, (smoother, H.fine.op.applies, res.iters)


def test_spectral_convergence_manufactured():
    """-lap u = 2 pi^2 sin(pi x) sin(pi y) on the unit square: the nodal error of the discrete
    solution decays exponentially in p on a fixed 4 x 4 mesh."""
    errs = []
    for p in (2, 4, 6, 8):
        prob = inputs.poisson2d_manufactured(4, p)
        H, b, res = mg.solve(prob)
        assert res.converged
        m = H.fine.mesh
        ue = np.sin(math.pi * m.x[:, 0]) * np.sin(math.pi * m.x[:, 1])
        errs.append(np.abs(res.x - ue).max())
    assert errs[-1] < 1e-9
    rates = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(r > 20 for r in rates), errs


def test_config1_solver_converges():
    prob = inputs.poisson2d_manufactured()
    H, b, res = mg.solve(prob)
    assert res.converged and res.history[-1] <= 1e-10 * res.history[0]
    assert [lv.mesh.nelem for lv in H.levels] == [(4, 4), (2, 2), (1, 1)]
    assert len(H.levels[-1].idx) == 9
