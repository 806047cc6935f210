"""Gauss-Seidel-type and modified-Jacobi smoothers on the assembled interior matrix.

Test infrastructure only (see the package docstring).

* Multicolor SSOR (§3.2.1, §4.3 "SSOR(2,1)", damping omega = 1). The paper orders the unknowns
  lexicographically, which is sequential; a parallel Gauss-Seidel needs a coloring of the
  unknowns (§3.2.1). The coloring used here (and by the GPU library) has n^2 colors, n = p + 1:
  with (gx, gy[, gz]) the global grid indices of a node,
      2D: color = (gx mod n) + n (gy mod n)
      3D: color = ((gx + gz) mod n) + n ((gy + gz) mod n).
  The collocated stiffness couples two nodes only if some element holds both and, in 3D, they
  share a grid coordinate; within one element distinct indices along an axis have distinct
  residues mod n, so coupled nodes always differ in color and each color is a set of mutually
  uncoupled unknowns. A forward Gauss-Seidel sweep visits the colors 0, 1, ..., C-1 and updates
  every interior node i of the color by
      x_i <- x_i + omega (b_i - (A x)_i) / A_ii,
  the backward sweep visits C-1, ..., 0; one SSOR step is a forward and a backward sweep, so it
  costs about two operator products (§4.3). Because the nodes of one color are uncoupled, the
  update of a whole color at once equals the node-by-node Gauss-Seidel update in any order
  within the color.
* l1-Jacobi (§3.2.3, §4.4.3; Baker, Falgout, Kolev and Yang 2011): the Jacobi iteration
  x <- x + omega D_l1^{-1} (b - A x) with (D_l1)_ii = sum_j |A_ij| over the interior row, which
  converges for every SPD A without an eigenvalue estimate (omega = 2/3 in the paper's table).
* Element block Jacobi (§3.2.3, §4.4.3): x <- x + omega B^{-1} (b - A x), B block diagonal with
  one block per element: the element's owned interior nodes (along each axis an element owns
  its local nodes 0..p-1, and the last element also p, so every node lies in exactly one
  block), B_e = A restricted to them, inverted exactly.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def node_colors(mesh):
    """Color of every node (see the module docstring); n^2 colors."""
    n = mesh.n
    g = mesh.grid
    if mesh.dim == 2:
        return (g[0] % n) + n * (g[1] % n)
    return ((g[0] + g[2]) % n) + n * ((g[1] + g[2]) % n)


class ColoredSSOR:
    """Multicolor Gauss-Seidel sweeps on the assembled Dirichlet operator A_II of one level."""

    def __init__(self, op, dinv):
        mesh = op.mesh
        self.A = op.K.csr()
        self.dinv = dinv
        self.ncolors = mesh.n ** 2
        col = node_colors(mesh)
        inter = mesh.interior
        self.idx = [np.nonzero(inter & (col == c))[0] for c in range(self.ncolors)]
        # rows of each color, restricted to interior columns (boundary entries of x are 0)
        mask = inter.astype(np.float64)
        self.rows = [(self.A[ix] @ sp.diags(mask)).tocsr() for ix in self.idx]

    def sweep(self, b, x, order, omega):
        for c in order:
            ix = self.idx[c]
            if len(ix) == 0:
                continue
            r = b[ix] - self.rows[c] @ x
            x[ix] = x[ix] + omega * self.dinv[ix] * r
        return x

    def ssor(self, b, x, steps, omega=1.0):
        """`steps` SSOR steps (forward then backward sweep each); x = None: zero guess."""
        x = np.zeros_like(b) if x is None else x.copy()
        fwd = list(range(self.ncolors))
        for _ in range(steps):
            self.sweep(b, x, fwd, omega)
            self.sweep(b, x, fwd[::-1], omega)
        return x


def l1_row_sums(op):
    """(D_l1)_ii = sum_j |A_ij| over the interior block (0 at boundary nodes)."""
    mesh = op.mesh
    A = op.K.csr()
    idx = np.nonzero(mesh.interior)[0]
    Aii = A[idx][:, idx]
    out = np.zeros(mesh.N)
    out[idx] = np.asarray(abs(Aii).sum(axis=1)).ravel()
    return out


def owned_blocks(mesh):
    """For every element, the interior nodes it owns (see the module docstring), ascending."""
    p = mesh.p
    owner = np.zeros(mesh.N, dtype=np.int64)
    stride = 1
    for a in range(mesh.dim):
        ga = mesh.grid[a]
        ea = np.minimum(ga // p, mesh.nelem[a] - 1)
        owner += ea * stride
        stride *= mesh.nelem[a]
    blocks = []
    for e in range(mesh.E):
        blocks.append(np.nonzero((owner == e) & mesh.interior)[0])
    return blocks


class BlockJacobi:
    """Element block Jacobi: exact inverses of the owned-node blocks of A."""

    def __init__(self, op):
        A = op.K.csr()
        self.blocks = owned_blocks(op.mesh)
        self.inv = []
        for ix in self.blocks:
            if len(ix) == 0:
                self.inv.append(None)
                continue
            Be = A[ix][:, ix].toarray()
            self.inv.append(sla.inv(Be))

    def apply_inverse(self, r):
        z = np.zeros_like(r)
        for ix, Bi in zip(self.blocks, self.inv):
            if Bi is not None:
                z[ix] = Bi @ r[ix]
        return z


def jacobi_type(op, minv_apply, b, x, nu, omega):
    """nu steps of x <- x + omega M^{-1} (b - A x); x = None means a zero initial guess."""
    for _ in range(nu):
        r = b.copy() if x is None else b - op.apply(x)
        x = (np.zeros_like(b) if x is None else x) + omega * minv_apply(r)
    return x
