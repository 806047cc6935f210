"""Pins of the oracle's multicolor SSOR, l1-Jacobi and element block-Jacobi smoothers (§3.2,
§4.3, §4.4.3) against what the definitions and textbook forms fix, not against the oracle itself:
* the coloring separates every coupled pair (so a color update is a Gauss-Seidel update);
* a color-by-color sweep equals the scalar node-by-node Gauss-Seidel loop;
* one SSOR step equals x + M^{-1}(b - A x) with the textbook splitting
  M = (D + omega L) D^{-1} (D + omega U) / (omega (2 - omega)) in the color order;
* SSOR(nu,nu) V-cycles are symmetric, SSOR(2,1) V-cycles contract;
* at p = 1 on a uniform 2D grid the sweep is the textbook five-point Gauss-Seidel loop;
* l1 row sums: closed form on the five-point stencil, D_l1 - A positive semidefinite;
* block Jacobi: blocks partition the unknowns, reduce to point Jacobi at p = 1 and to an exact
  solve on a one-element mesh."""

import numpy as np
import pytest

from oracle import fem, mg, relax
from paper_1402_5938_amd import inputs

WARP = inputs.map_warp_sine(0.05)
MU = inputs.mu_exp_sine_product(2.0)

MESHES = [(2, (3, 2), 3), (2, (4, 4), 1), (2, (2, 2), 4), (3, (2, 2, 1), 2), (3, (2, 1, 1), 3),
          (3, (3, 3, 2), 1)]


def _level(dim, ne, p, mp=WARP, mu=MU):
    m = fem.Mesh(dim, ne, p, mp, mu)
    op = fem.LevelOperator(m)
    dg = op.diag()
    dinv = np.zeros_like(dg)
    dinv[m.interior] = 1.0 / dg[m.interior]
    return m, op, dinv


@pytest.mark.parametrize("dim,ne,p", MESHES)
def test_coloring_separates_coupled_nodes(dim, ne, p):
    m, op, _ = _level(dim, ne, p)
    col = relax.node_colors(m)
    A = op.K.csr().tocoo()
    off = A.row != A.col
    assert np.all(col[A.row[off]] != col[A.col[off]])
    n = p + 1
    assert set(np.unique(col)) == set(range(n * n))
    # every element holds (p+1)^(d-2) nodes of each color
    for e in range(m.E):
        counts = np.bincount(col[m.conn[e]], minlength=n * n)
        assert np.all(counts == n ** (dim - 2))


def test_coloring_is_tight_and_needed():
    # a coloring with one color fewer per axis (mod p instead of mod p+1) puts coupled nodes
    # of one element into one color: the n^2 colors are needed
    m, op, _ = _level(3, (2, 1, 1), 3)
    g = m.grid
    bad = ((g[0] + g[2]) % m.p) + m.p * ((g[1] + g[2]) % m.p)
    A = op.K.csr().tocoo()
    off = A.row != A.col
    assert np.any(bad[A.row[off]] == bad[A.col[off]])


@pytest.mark.parametrize("dim,ne,p", [(2, (2, 2), 2), (3, (2, 1, 1), 2), (3, (1, 1, 1), 3)])
@pytest.mark.parametrize("omega", [1.0, 0.7])
def test_color_sweep_equals_scalar_gauss_seidel(dim, ne, p, omega):
    m, op, dinv = _level(dim, ne, p)
    S = relax.ColoredSSOR(op, dinv)
    A = op.K.csr().toarray()
    rng = np.random.default_rng(3)
    b = rng.standard_normal(m.N) * m.interior
    x0 = rng.standard_normal(m.N) * m.interior
    col = relax.node_colors(m)
    for order in (list(range(S.ncolors)), list(range(S.ncolors))[::-1]):
        x = x0.copy()
        for c in order:
            for i in range(m.N):
                if col[i] != c or not m.interior[i]:
                    continue
                r = b[i] - sum(A[i, j] * x[j] for j in range(m.N) if m.interior[j])
                x[i] = x[i] + omega * r / A[i, i]
        xs = S.sweep(b, x0.copy(), order, omega)
        assert np.abs(xs - x).max() <= 1e-13 * np.abs(x).max()


@pytest.mark.parametrize("dim,ne,p", [(2, (3, 2), 3), (3, (2, 1, 2), 2)])
@pytest.mark.parametrize("omega", [1.0, 0.7])
def test_ssor_step_is_the_textbook_splitting(dim, ne, p, omega):
    m, op, dinv = _level(dim, ne, p)
    S = relax.ColoredSSOR(op, dinv)
    idx = np.nonzero(m.interior)[0]
    A = op.K.csr().toarray()[np.ix_(idx, idx)]
    col = relax.node_colors(m)[idx]
    D = np.diag(np.diag(A))
    lower = col[None, :] < col[:, None]          # j visited before i in the forward sweep
    L = np.where(lower, A, 0.0)
    U = L.T
    M = (D + omega * L) @ np.linalg.inv(D) @ (D + omega * U) / (omega * (2.0 - omega))
    rng = np.random.default_rng(5)
    b = np.zeros(m.N)
    b[idx] = rng.standard_normal(len(idx))
    x0 = np.zeros(m.N)
    x0[idx] = rng.standard_normal(len(idx))
    x1 = S.ssor(b, x0, 1, omega)
    ref = x0[idx] + np.linalg.solve(M, b[idx] - A @ x0[idx])
    assert np.abs(x1[idx] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(x1[~m.interior] == 0)


def _dense_vcycle(H):
    N = H.fine.mesh.N
    idx = np.nonzero(H.fine.mesh.interior)[0]
    V = np.zeros((len(idx), len(idx)))
    for k, i in enumerate(idx):
        e = np.zeros(N)
        e[i] = 1.0
        V[:, k] = H.vcycle(e)[idx]
    return V, idx


@pytest.mark.parametrize("nu,nu_post", [(1, 1), (2, 2), (2, 1)])
def test_ssor_vcycle_symmetry_and_contraction(nu, nu_post):
    H = mg.Hierarchy(2, (4, 4), 2, WARP, MU, hierarchy="h", smoother="ssor", nu=nu, nu_post=nu_post)
    V, idx = _dense_vcycle(H)
    if nu == nu_post:
        assert np.abs(V - V.T).max() <= 1e-12 * np.abs(V).max()
    A = H.fine.op.K.csr().toarray()[np.ix_(idx, idx)]
    E = np.eye(len(idx)) - V @ A
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert rho < 0.2
    # a post-smoothing step that is not the adjoint of the pre-smoothing makes V non-symmetric
    if nu != nu_post:
        assert np.abs(V - V.T).max() > 1e-6 * np.abs(V).max()


def test_p1_sweep_is_the_five_point_gauss_seidel_loop():
    ne = 6
    m, op, dinv = _level(2, (ne, ne), 1, inputs.map_identity(), inputs.field_const(1.0))
    A = op.K.csr().toarray()
    nx = ne + 1
    # the collocated p = 1 stiffness on a uniform grid is the five-point Laplacian
    for i in np.nonzero(m.interior)[0]:
        row = np.zeros(m.N)
        row[i] = 4.0
        for j in (i - 1, i + 1, i - nx, i + nx):
            row[j] = -1.0
        assert np.abs(A[i] - row).max() <= 1e-14
    rng = np.random.default_rng(9)
    b = rng.standard_normal(m.N) * m.interior
    u = np.zeros((nx, nx))
    B = b.reshape(nx, nx)
    for cy in (0, 1):
        for cx in (0, 1):
            for gy in range(1, nx - 1):
                for gx in range(1, nx - 1):
                    if gx % 2 == cx and gy % 2 == cy:
                        u[gy, gx] = (B[gy, gx] + u[gy, gx - 1] + u[gy, gx + 1] + u[gy - 1, gx]
                                     + u[gy + 1, gx]) / 4.0
    S = relax.ColoredSSOR(op, dinv)
    x = S.sweep(b, np.zeros(m.N), list(range(4)), 1.0)
    assert np.abs(x - u.ravel()).max() <= 1e-13 * np.abs(u).max()


def test_l1_row_sums_five_point_closed_form():
    ne = 5
    m, op, _ = _level(2, (ne, ne), 1, inputs.map_identity(), inputs.field_const(1.0))
    s1 = relax.l1_row_sums(op)
    nx = ne + 1
    for i in np.nonzero(m.interior)[0]:
        gx, gy = i % nx, i // nx
        nb = sum(1 for (a, c) in ((gx - 1, gy), (gx + 1, gy), (gx, gy - 1), (gx, gy + 1))
                 if 0 < a < nx - 1 and 0 < c < nx - 1)
        assert abs(s1[i] - (4.0 + nb)) <= 1e-13


@pytest.mark.parametrize("dim,ne,p", [(2, (3, 2), 3), (3, (2, 2, 1), 2)])
def test_l1_jacobi_converges_without_damping(dim, ne, p):
    m, op, _ = _level(dim, ne, p)
    s1 = relax.l1_row_sums(op)
    idx = np.nonzero(m.interior)[0]
    A = op.K.csr().toarray()[np.ix_(idx, idx)]
    assert np.all(s1[idx] >= np.diag(A))
    ev = np.linalg.eigvalsh(np.diag(s1[idx]) - A)
    assert ev.min() >= -1e-12 * np.abs(A).max()
    lam = np.linalg.eigvals(np.diag(1.0 / s1[idx]) @ A).real
    assert lam.min() > 0 and lam.max() <= 1.0 + 1e-12


@pytest.mark.parametrize("dim,ne,p", [(2, (3, 4), 3), (3, (2, 3, 2), 2)])
def test_owned_blocks_partition_the_unknowns(dim, ne, p):
    m, _, _ = _level(dim, ne, p)
    blocks = relax.owned_blocks(m)
    allidx = np.sort(np.concatenate(blocks))
    assert np.array_equal(allidx, np.nonzero(m.interior)[0])
    # an element away from the upper faces owns p^d nodes
    sizes = [len(b) for b in blocks]
    assert max(sizes) <= (p + 1) ** dim


@pytest.mark.parametrize("dim,ne", [(2, (4, 3)), (3, (3, 2, 2))])
def test_block_jacobi_is_point_jacobi_at_order_one(dim, ne):
    m, op, dinv = _level(dim, ne, 1)
    BJ = relax.BlockJacobi(op)
    r = np.random.default_rng(2).standard_normal(m.N) * m.interior
    z = BJ.apply_inverse(r)
    assert np.abs(z - dinv * r).max() <= 1e-14 * np.abs(z).max()


def test_block_jacobi_single_element_is_exact():
    m, op, _ = _level(3, (1, 1, 1), 4)
    BJ = relax.BlockJacobi(op)
    b = np.random.default_rng(4).standard_normal(m.N) * m.interior
    x = relax.jacobi_type(op, BJ.apply_inverse, b, None, 1, 1.0)
    assert np.abs(op.apply(x) - b).max() <= 1e-11 * np.abs(b).max()


@pytest.mark.parametrize("smoother", ["ssor", "l1jacobi", "blockjacobi"])
def test_new_smoothers_solve_to_the_dense_solution(smoother):
    H = mg.Hierarchy(3, (2, 2, 2), 2, WARP, MU, hierarchy="p", smoother=smoother,
                     nu=2 if smoother == "ssor" else 3, nu_post=1 if smoother == "ssor" else 3)
    m = H.fine.mesh
    b = fem.load_vector(m, np.ones(m.N))
    idx = np.nonzero(m.interior)[0]
    A = H.fine.op.K.csr().toarray()[np.ix_(idx, idx)]
    xs = np.linalg.solve(A, b[idx])
    for solve in (mg.pcg, mg.mg_solve):
        res = solve(H, b, rtol=1e-10)
        assert res.converged
        assert np.abs(res.x[idx] - xs).max() <= 1e-8 * np.abs(xs).max()


# ------------------------------------------------------------------ first-order preconditioner
def test_low_order_level_is_order_one_on_the_high_order_nodes():
    H = mg.Hierarchy(2, (3, 2), 4, WARP, MU, hierarchy="low")
    m0, m1 = H.levels[0].mesh, H.levels[1].mesh
    assert m1.p == 1 and m1.nelem == (12, 8) and m1.N == m0.N
    assert np.array_equal(m1.x, m0.x)                     # the same physical nodes
    # at p = 1 the order-p level is already first order: the hierarchy is the h-hierarchy
    assert mg.plan_levels(3, (4, 4, 2), 1, "low") == mg.plan_levels(3, (4, 4, 2), 1, "h")
    # coarser first-order levels sit on every other node
    H2 = mg.Hierarchy(2, (2, 2), 4, WARP, MU, hierarchy="low")
    m2 = H2.levels[2].mesh
    sub = H2.levels[0].mesh.x.reshape(9, 9, 2)[::2, ::2].reshape(-1, 2)
    assert np.array_equal(m2.x, sub)


def _equivalence_band(dim, ne, p):
    H = mg.Hierarchy(dim, ne, p, WARP, MU, hierarchy="low")
    A0, idx = H.levels[0].op.dense_interior()
    A1, idx1 = H.levels[1].op.dense_interior()
    assert np.array_equal(idx, idx1)
    ev = np.linalg.eigvals(np.linalg.solve(A1, A0))
    assert np.abs(ev.imag).max() <= 1e-8 * np.abs(ev.real).max()
    return ev.real.min(), ev.real.max()


@pytest.mark.parametrize("dim,p,ne0,ne1", [(2, 4, (2, 2), (4, 4)), (3, 2, (2, 2, 2), (4, 4, 4))])
def test_low_order_operator_is_spectrally_equivalent(dim, p, ne0, ne1):
    """A_1^{-1} A_p has real positive eigenvalues in a bounded band (the finite-element /
    spectral-element equivalence) that refining the mesh leaves nearly unchanged."""
    lo0, hi0 = _equivalence_band(dim, ne0, p)
    lo1, hi1 = _equivalence_band(dim, ne1, p)
    assert 0.3 < lo1 and hi1 < 6.0, (lo1, hi1)
    assert hi1 / lo1 < 1.3 * hi0 / lo0, ((lo0, hi0), (lo1, hi1))


def test_low_order_sweeps_tend_to_the_exact_inverse():
    H = mg.Hierarchy(2, (4, 4), 4, WARP, MU, hierarchy="low", low_cycles=1)
    m = H.fine.mesh
    r = np.random.default_rng(7).standard_normal(m.N) * m.interior
    exact = H.low_order_exact(r)
    errs = []
    for k in (1, 3, 6, 12):
        H.low_cycles = k
        errs.append(np.abs(H.precond(r) - exact).max() / np.abs(exact).max())
    assert errs[-1] < 1e-8 and all(errs[i + 1] < errs[i] for i in range(3))
    # the preconditioner is symmetric (a polynomial in the symmetric V_1 A_1, times V_1)
    H.low_cycles = 3
    idx = np.nonzero(m.interior)[0]
    M = np.zeros((len(idx), len(idx)))
    for c, i in enumerate(idx):
        e = np.zeros(m.N)
        e[i] = 1.0
        M[:, c] = H.precond(e)[idx]
    assert np.abs(M - M.T).max() <= 1e-11 * np.abs(M).max()


def test_low_order_pcg_solves():
    H = mg.Hierarchy(3, (2, 2, 2), 4, WARP, MU, hierarchy="low", low_cycles=2)
    m = H.fine.mesh
    b = fem.load_vector(m, np.ones(m.N))
    A, idx = H.fine.op.dense_interior()
    xs = np.linalg.solve(A, b[idx])
    res = mg.pcg(H, b, rtol=1e-10)
    assert res.converged and np.abs(res.x[idx] - xs).max() <= 1e-8 * np.abs(xs).max()
    exact = mg.pcg(H, b, rtol=1e-10, precond=H.low_order_exact)
    assert exact.converged and exact.iters <= res.iters
