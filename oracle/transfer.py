"""Prolongation P_ij = phi_j^{coarse}(p_i) and restriction R = P^T (paper §2.2, Eq. (Pstencil)).

Test infrastructure only (see the package docstring).

The coarse space is either the same mesh at a lower order (p-coarsening, §3.1.2) or the mesh
with half the elements per axis at the same order (h-coarsening, §3.1.1). The coarse basis is
evaluated at each fine node in reference coordinates: for a fine node with local coordinate
xi_f in a fine element, the containing coarse element is the same element (p) or its parent
e // 2 (h); in the latter case the coarse local coordinate is (xi_f + 2c - 1)/2 for the child
index c = e % 2. The restriction is the exact transpose (the adjoint w.r.t. the
mass-weighted inner product, §2.2). On the Dirichlet problem, P acts between interior
unknowns: coarse boundary values are 0 and fine boundary rows are dropped.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .gll import lagrange_eval


def relation(fine, coarse):
    if fine.nelem == coarse.nelem and coarse.p < fine.p:
        return "p"
    if coarse.p == fine.p and all(f == 2 * c for f, c in zip(fine.nelem, coarse.nelem)):
        return "h"
    raise ValueError("levels are not related by h- or p-coarsening")


def _coarse_local(fine, coarse, kind):
    """For every fine element and local 1D node, per axis: coarse element coordinate and the
    node's coordinate in the coarse element's reference interval."""
    out = []
    for a in range(fine.dim):
        ef = fine.elem_coords[a]                        # (E_f,)
        xi = fine.xi                                    # (n_f,)
        if kind == "p":
            ec = ef
            xc = np.broadcast_to(xi, (len(ef), fine.n))
        else:
            ec = ef // 2
            c = ef % 2
            xc = (xi[None, :] + 2.0 * c[:, None] - 1.0) / 2.0
        out.append((ec, xc))
    return out


def prolongation_direct(fine, coarse):
    """P (N_f x N_c) built node by node from the definition: for every fine node, take one
    fine element containing it, locate the coarse element and evaluate all of that coarse
    element's basis functions at the node."""
    kind = relation(fine, coarse)
    d = fine.dim
    loc = _coarse_local(fine, coarse, kind)
    gf = fine.conn.ravel()
    _, first = np.unique(gf, return_index=True)         # one (element, local node) per fine node
    e_idx = first // fine.nloc
    l_idx = first % fine.nloc
    stride_c = np.cumprod((1,) + coarse.nelem[:-1])
    ec_flat = np.zeros(len(first), dtype=np.int64)
    vals = np.ones((len(first), coarse.nloc))
    for a in range(d):
        ec, xc = loc[a]
        ec_flat += ec[e_idx] * stride_c[a]
        la = fine.local[a][l_idx]
        pts = xc[e_idx, la]                              # coarse reference coordinate, axis a
        L = lagrange_eval(coarse.xi, pts)                # (npts, n_c)
        vals *= L[:, coarse.local[a]]                    # basis j contributes l_{j_a}(pts)
    rows = np.repeat(gf[first], coarse.nloc)
    cols = coarse.conn[ec_flat].ravel()
    P = sp.csr_matrix((vals.ravel(), (rows, cols)), shape=(fine.N, coarse.N))
    P.eliminate_zeros()
    return P


def prolongation_1d(fine, coarse, a):
    """The 1D factor of axis a: the coarse 1D Lagrange basis at every fine 1D grid point."""
    kind = relation(fine, coarse)
    nf = fine.nax[a]
    Nc = coarse.nax[a]
    P1 = np.zeros((nf, Nc))
    for g in range(nf):
        ef = min(g // fine.p, fine.nelem[a] - 1)
        i = g - ef * fine.p
        if kind == "p":
            ec, xc = ef, fine.xi[i]
        else:
            ec, c = ef // 2, ef % 2
            xc = (fine.xi[i] + 2.0 * c - 1.0) / 2.0
        P1[g, ec * coarse.p:ec * coarse.p + coarse.n] = lagrange_eval(coarse.xi, xc)[0]
    return sp.csr_matrix(P1)


def prolongation(fine, coarse):
    """P as the Kronecker product of its 1D factors. The coarse basis is a tensor product of
    1D Lagrange functions and the fine nodes form a tensor grid, so phi_j(p_i) is the product
    of 1D values; equality with ``prolongation_direct`` is checked by the tests."""
    d = fine.dim
    P = prolongation_1d(fine, coarse, 0)
    for a in range(1, d):
        P = sp.kron(prolongation_1d(fine, coarse, a), P, format="csr")
    P.eliminate_zeros()
    return P.tocsr()


class Transfer:
    """P and R = P^T between interior unknowns, on full-length vectors."""

    def __init__(self, fine, coarse, direct=False):
        self.fine, self.coarse = fine, coarse
        self.kind = relation(fine, coarse)
        self.P = prolongation_direct(fine, coarse) if direct else prolongation(fine, coarse)
        self.mf = fine.interior.astype(np.float64)
        self.mc = coarse.interior.astype(np.float64)

    def prolong(self, xc):
        return self.mf * (self.P @ (self.mc * xc))

    def restrict(self, rf):
        return self.mc * (self.P.T @ (self.mf * rf))
