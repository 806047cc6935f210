"""Mesh, isoparametric geometry and the assembled Galerkin stiffness.

Test infrastructure only (see the package docstring).

Discretization (paper §2.1 and §2.3):
* the domain is Phi([0,1]^d) for a smooth map Phi, meshed by n_e elements per axis of a
  uniform reference grid; each element carries the tensor GLL nodes of order p;
* geometry is isoparametric: on every element the map is replaced by its degree-p interpolant
  through the mapped nodes, and the Jacobian J = dx/dxi is evaluated at every quadrature point;
* quadrature is the collocated (p+1)^d-point GLL rule (nodes = quadrature points), so the
  mass matrix is diagonal, or (quadrature="gauss", the paper's rule, §2.3) the (p+1)^d-point
  Gauss-Legendre rule, at whose points the basis is interpolated (I~_qi = l_i(eta_q)) and
  differentiated (D~ = I~ D, exact since l_i' has degree p); the geometry, mu and the weights
  are taken at the Gauss points and the mass matrix is the consistent one;
* the stiffness is (A)_ij = a(phi_i, phi_j) = int mu grad phi_i . grad phi_j, which under
  the quadrature is  A = sum_e sum_q B_q^T G_q B_q  with B_q the reference gradient of the
  element basis at q and G_q = w_q mu(x_q) detJ_q J^{-1} J^{-T};
* homogeneous Dirichlet data: the unknowns are the interior nodes.

Node numbering: lexicographic over the global (n_e p + 1)^d grid, x fastest. Element numbering
and element-local numbering are lexicographic with x fastest as well.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fields import eval_map, eval_scalar
from .gll import deriv_matrix, gll, lagrange_eval


def lex(shape):
    """Coordinates of all points of a grid of the given (x, y[, z]) shape, x fastest.
    Returns an int array of shape (d, count)."""
    d = len(shape)
    grids = np.indices(tuple(shape[::-1]))
    return np.stack([grids[d - 1 - a].ravel() for a in range(d)])


class Mesh:
    """A structured conforming mesh of order p and its geometry at the GLL points."""

    def __init__(self, dim, nelem, p, map_desc, mu_desc, quadrature="gll"):
        if quadrature not in ("gll", "gauss"):
            raise ValueError("quadrature must be 'gll' or 'gauss'")
        self.quadrature = quadrature
        self.dim = int(dim)
        self.nelem = tuple(int(v) for v in nelem)
        assert len(self.nelem) == self.dim
        self.p = int(p)
        self.n = self.p + 1
        self.map_desc = map_desc
        self.mu_desc = mu_desc
        self.nax = tuple(ne * self.p + 1 for ne in self.nelem)
        self.N = int(np.prod(self.nax))
        self.E = int(np.prod(self.nelem))
        self.nloc = self.n ** self.dim
        self.xi, self.w = gll(self.p)
        self.D = deriv_matrix(self.xi)
        if quadrature == "gauss":
            self.eta, self.wg = np.polynomial.legendre.leggauss(self.n)
            self.Iq = lagrange_eval(self.xi, self.eta)      # (q, n): l_i(eta_q)
            self.Dq = self.Iq @ self.D                      # (q, n): l_i'(eta_q)
        else:
            self.eta, self.wg = self.xi, self.w
            self.Iq = np.eye(self.n)
            self.Dq = self.D

        # reference coordinate of every global 1D grid index, per axis
        self.X1 = []
        for ne in self.nelem:
            g = np.arange(ne * self.p + 1)
            e = np.minimum(g // self.p, ne - 1)
            i = g - e * self.p
            self.X1.append((e + (self.xi[i] + 1.0) / 2.0) / ne)
        G = lex(self.nax)                       # (d, N) grid indices of every node
        self.grid = G
        self.X = np.stack([self.X1[a][G[a]] for a in range(self.dim)], axis=1)
        self.x = eval_map(map_desc, self.X)
        self.boundary = np.zeros(self.N, dtype=bool)
        for a in range(self.dim):
            self.boundary |= (G[a] == 0) | (G[a] == self.nax[a] - 1)
        self.interior = ~self.boundary

        # element -> global node map
        Ee = lex(self.nelem)                    # (d, E)
        Ll = lex((self.n,) * self.dim)          # (d, nloc)
        self.local = Ll
        stride = np.cumprod((1,) + self.nax[:-1])
        conn = np.zeros((self.E, self.nloc), dtype=np.int64)
        for a in range(self.dim):
            conn += (Ee[a][:, None] * self.p + Ll[a][None, :]) * stride[a]
        self.conn = conn
        self.elem_coords = Ee

    # ------------------------------------------------------------------ geometry
    def _contract(self, arr, mats):
        """Apply the 1D matrix mats[b] along reference direction b of arr (m, n_z, n_y, n_x,
        ...) for every b (array axis d - b holds direction b)."""
        d = self.dim
        for b in range(d):
            ax = d - b
            moved = np.moveaxis(arr, ax, 0)
            arr = np.moveaxis(np.tensordot(mats[b], moved, axes=([1], [0])), 0, ax)
        return arr

    def geometry(self, elems=None):
        """Per element and quadrature point: G = w mu detJ J^{-1} J^{-T} (m, nq, d, d), the
        quadrature weight times detJ (m, nq), mu (m, nq) and detJ (m, nq). The points are the GLL
        nodes (collocation) or the Gauss points, where the isoparametric interpolant of the
        mapped nodes gives both x_q and J."""
        if elems is None:
            elems = np.arange(self.E)
        d, n = self.dim, self.n
        m = len(elems)
        nq = len(self.eta)
        xe = self.x[self.conn[elems]].reshape((m,) + (n,) * d + (d,))
        J = np.empty((m,) + (nq,) * d + (d, d))
        for b in range(d):
            mats = [self.Dq if c == b else self.Iq for c in range(d)]
            J[..., :, b] = self._contract(xe, mats)
        xq = self._contract(xe, [self.Iq] * d)
        detJ = np.linalg.det(J)
        if not np.all(detJ > 0):
            raise ValueError("detJ <= 0: the map is not a diffeomorphism on this mesh")
        Jinv = np.linalg.inv(J)
        wq = self.wg
        for _ in range(d - 1):
            wq = np.multiply.outer(self.wg, wq)         # (nq,)*d, last axis = x
        mu = eval_scalar(self.mu_desc, xq.reshape(-1, d)).reshape((m,) + (nq,) * d)
        if not np.all(np.isfinite(mu)) or not np.all(mu > 0):
            raise ValueError("mu must be finite and positive")
        scale = wq[None] * mu * detJ
        G = scale[..., None, None] * np.einsum("...ac,...bc->...ab", Jinv, Jinv)
        npts = nq ** d
        return (G.reshape(m, npts, d, d), (wq[None] * detJ).reshape(m, npts),
                mu.reshape(m, npts), detJ.reshape(m, npts))

    # ------------------------------------------------------------------ operators
    def grad_matrices(self, elems=None):
        """Global reference-gradient matrices B_a, a < d: row (e, q) of B_a maps the global
        node vector to d u_e / d xi_a at quadrature point q of element e. Collocated GLL:
        sum_l D[q_a, l] u(local node q with coordinate a replaced by l); Gauss: the tensor
        product of D~ along a and I~ along the other axes (a dense row per element)."""
        if elems is None:
            elems = np.arange(self.E)
        d, n, nloc = self.dim, self.n, self.nloc
        m = len(elems)
        conn = self.conn[elems]
        mats = []
        if self.quadrature == "gll":
            rows = np.repeat(np.arange(m * nloc), n)
            for a in range(d):
                qa = self.local[a]
                base = np.arange(nloc) - qa * n ** a
                loc = base[:, None] + np.arange(n)[None, :] * n ** a        # (nloc, n)
                cols = conn[:, loc]                                          # (m, nloc, n)
                vals = np.broadcast_to(self.D[qa], (m, nloc, n))
                B = sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(m * nloc, self.N))
                mats.append(B)
            return mats
        nq = len(self.eta) ** d
        for a in range(d):
            K = np.ones((1, 1))
            for c in range(d):                  # local index x fastest: kron(M_z, M_y, M_x)
                K = np.kron(self.Dq if c == a else self.Iq, K)
            rows = np.repeat(np.arange(m * nq), nloc)
            cols = np.tile(conn[:, None, :], (1, nq, 1))
            vals = np.broadcast_to(K, (m, nq, nloc))
            B = sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(m * nq, self.N))
            mats.append(B)
        return mats

    def interp_matrix(self, elems=None):
        """Rows (e, q): the global node vector interpolated to quadrature point q of e."""
        if elems is None:
            elems = np.arange(self.E)
        d, nloc = self.dim, self.nloc
        m = len(elems)
        nq = len(self.eta) ** d
        K = np.ones((1, 1))
        for c in range(d):
            K = np.kron(self.Iq, K)
        rows = np.repeat(np.arange(m * nq), nloc)
        cols = np.tile(self.conn[elems][:, None, :], (1, nq, 1))
        vals = np.broadcast_to(K, (m, nq, nloc))
        return sp.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(m * nq, self.N))

    def lumped_mass(self):
        """M_L = diag of the GLL-quadrature mass matrix: sum over elements of w_q detJ_q."""
        if self.quadrature != "gll":
            raise ValueError("the mass matrix is diagonal only under GLL quadrature")
        _, wdet, _, _ = self.geometry()
        return np.bincount(self.conn.ravel(), weights=wdet.ravel(), minlength=self.N)

    def mass_matrix(self):
        """The mass matrix (phi_i, phi_j) under the mesh's quadrature: I^T diag(w detJ) I
        (diagonal, the lumped mass, under GLL collocation)."""
        _, wdet, _, _ = self.geometry()
        Iq = self.interp_matrix() if self.quadrature == "gauss" else None
        if Iq is None:
            return sp.diags(self.lumped_mass()).tocsr()
        return (Iq.T @ sp.diags(wdet.ravel()) @ Iq).tocsr()


class Stiffness:
    """A = sum_{a,b} B_a^T diag(G_ab) B_b, kept in this factored sparse form (B_a and G are
    stored, A itself is only multiplied out on request)."""

    def __init__(self, mesh: Mesh, elems=None):
        self.mesh = mesh
        self.B = mesh.grad_matrices(elems)
        G, _, _, _ = mesh.geometry(elems)
        d = mesh.dim
        self.G = G.reshape(-1, d, d)

    def matvec(self, x):
        """y = A x over all nodes (no boundary condition applied)."""
        d = self.mesh.dim
        u = [self.B[b] @ x for b in range(d)]
        y = np.zeros(self.mesh.N)
        for a in range(d):
            wa = np.zeros_like(u[0])
            for b in range(d):
                wa += self.G[:, a, b] * u[b]
            y += self.B[a].T @ wa
        return y

    def matvec_abs(self, x):
        """|B|^T |G| |B| |x|: every product of the factored sum taken in absolute value. It
        bounds |A x| entrywise and is the scale of the rounding error of any evaluation order
        of A x; it is a yardstick for comparisons, not part of the method."""
        d = self.mesh.dim
        ax = np.abs(x)
        u = [abs(self.B[b]) @ ax for b in range(d)]
        y = np.zeros(self.mesh.N)
        for a in range(d):
            wa = np.zeros_like(u[0])
            for b in range(d):
                wa += np.abs(self.G[:, a, b]) * u[b]
            y += abs(self.B[a]).T @ wa
        return y

    def csr(self):
        """The assembled stiffness as a CSR matrix."""
        d = self.mesh.dim
        A = None
        for a in range(d):
            for b in range(d):
                t = self.B[a].T @ (sp.diags(self.G[:, a, b]) @ self.B[b])
                A = t if A is None else A + t
        return A.tocsr()

    def diagonal(self):
        """diag(A)_g = sum_{a,b} sum_rows B_a[r, g] G_ab[r] B_b[r, g]."""
        d = self.mesh.dim
        out = np.zeros(self.mesh.N)
        for a in range(d):
            for b in range(d):
                t = self.B[a].multiply(sp.diags(self.G[:, a, b]) @ self.B[b])
                out += np.asarray(t.sum(axis=0)).ravel()
        return out


class LevelOperator:
    """The Dirichlet operator of one mesh acting on full-length node vectors: boundary
    entries of the input are ignored (treated as 0) and those of the output are 0."""

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        self.K = Stiffness(mesh)
        self.mask = mesh.interior.astype(np.float64)
        self.applies = 0

    def apply(self, x, neumann=False):
        self.applies += 1
        if neumann:
            return self.K.matvec(x)
        return self.mask * self.K.matvec(self.mask * x)

    def apply_abs(self, x, neumann=False):
        """The rounding scale |B|^T |G| |B| |x| of apply(x) (see Stiffness.matvec_abs)."""
        if neumann:
            return self.K.matvec_abs(x)
        return self.mask * self.K.matvec_abs(self.mask * x)

    def diag(self):
        return self.mask * self.K.diagonal()

    def dense_interior(self):
        """The interior block A_II as a dense array (small meshes only)."""
        A = self.K.csr()
        idx = np.nonzero(self.mesh.interior)[0]
        return A[idx][:, idx].toarray(), idx


def load_vector(mesh: Mesh, f_nodal):
    """b_j = (f_h, phi_j) under the mesh's quadrature for the nodal interpolant f_h of f: under
    GLL quadrature (lumped mass) * f at the node; under Gauss quadrature M f with the consistent
    mass. 0 on the boundary."""
    f = np.asarray(f_nodal, dtype=np.float64)
    if mesh.quadrature == "gll":
        b = mesh.lumped_mass() * f
    else:
        _, wdet, _, _ = mesh.geometry()
        Iq = mesh.interp_matrix()
        b = Iq.T @ (wdet.ravel() * (Iq @ f))
    b[mesh.boundary] = 0.0
    return b


def nodal_field(mesh: Mesh, desc):
    """A scalar field evaluated at the physical node coordinates."""
    return eval_scalar(desc, mesh.x)
