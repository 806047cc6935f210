"""Smoothers, eigenvalue estimate, hierarchy, V-cycle, multigrid solver and MG-preconditioned CG.

Test infrastructure only (see the package docstring).

* Jacobi: x <- x + omega D^{-1} (b - A x), omega = 2/3 (§3.2.2, §4.3).
* Chebyshev-accelerated Jacobi targeting [lambda/4, lambda] of D^{-1} A (§3.2.1, §3.2.2,
  §4.3). The paper gives no recurrence; this is the preconditioned Chebyshev iteration of
  Saad, Iterative Methods for Sparse Linear Systems (2nd ed.), Alg. 12.1, with D^{-1} as the
  preconditioner: after k steps the error is T_k((theta - lambda)/delta) / T_k(theta/delta)
  times its initial value on every generalized eigenpair A v = lambda D v.
* lambda_max of D^{-1} A from 10 Arnoldi steps in setup (§3.2.2, §4.3): Arnoldi on D^{-1} A in
  the D inner product is Lanczos on the symmetric D^{-1/2} A D^{-1/2}; full
  reorthogonalization, m = min(10, number of unknowns) steps, start vector from SplitMix64.
* Hierarchy (§3.1, §4.3): h-multigrid keeps p and halves the elements per axis; p-multigrid
  takes p -> ceil(p/2) down to 1 and then halves the elements; every level is rediscretized
  with its own mesh, order and mu at its own quadrature points (§2.3). A coarser level is
  added only while it keeps at least one interior unknown.
* V-cycle with zero initial guess, nu_pre pre- and nu_post post-smoothing steps per level,
  restriction P^T, exact (dense Cholesky) solve on the coarsest level.
* The other smoothers the paper compares (multicolor SSOR, l1-Jacobi, element block Jacobi,
  §3.2, §4.3, §4.4.3) are in ``relax``.
* Multigrid as solver: x <- x + V(b - A x). PCG: Algorithm 1 with one V-cycle per iteration.
  Both stop when ||r||_2 <= rtol ||r_0||_2 (§4.3: the discrete residual norm); the count is
  the number of V-cycles applied to update x.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .fem import LevelOperator, Mesh, load_vector, nodal_field
from .relax import BlockJacobi, ColoredSSOR, jacobi_type, l1_row_sums
from .splitmix import start_vector
from .transfer import Transfer


def plan_levels(dim, nelem, p, hierarchy="p", max_levels=0, coarse_unknowns=0):
    """List of (nelem, p) from fine to coarse. hierarchy "low": the order-p level, then the
    first-order level on the same nodes (n_e p cells of order 1 per axis), then h-coarsening.
    Halving goes on while every axis is even and the halved level keeps an interior node; with
    coarse_unknowns = k > 0 it stops at the first first-order level with at most k interior
    unknowns, the level then solved exactly (§3)."""
    nelem = tuple(int(v) for v in nelem)

    def interior(ne, q):
        return int(np.prod([v * q - 1 for v in ne]))

    levels = [(nelem, int(p))]
    ne, q = nelem, int(p)
    if hierarchy == "p":
        while q > 1:
            q = (q + 1) // 2
            levels.append((ne, q))
    elif hierarchy == "low":
        if q > 1:
            ne, q = tuple(v * q for v in ne), 1
            levels.append((ne, q))
    elif hierarchy != "h":
        raise ValueError("hierarchy must be 'h', 'p' or 'low'")
    while all(v % 2 == 0 for v in ne) and interior(tuple(v // 2 for v in ne), q) >= 1:
        if coarse_unknowns and q == 1 and interior(ne, q) <= coarse_unknowns:
            break
        ne = tuple(v // 2 for v in ne)
        levels.append((ne, q))
    if max_levels and max_levels > 0:
        levels = levels[:max_levels]
    return levels


def jacobi(op: LevelOperator, dinv, b, x, nu, omega=2.0 / 3.0):
    """nu damped-Jacobi sweeps; x = None means a zero initial guess."""
    for _ in range(nu):
        r = b.copy() if x is None else b - op.apply(x)
        x = (np.zeros_like(b) if x is None else x) + omega * dinv * r
    return x


def chebyshev(op: LevelOperator, dinv, lmax, b, x, k, lo=0.25):
    """Degree-k Chebyshev-Jacobi on [lo*lmax, lmax]; x = None means a zero initial guess."""
    beta = lmax
    alpha = lo * lmax
    theta = 0.5 * (beta + alpha)
    delta = 0.5 * (beta - alpha)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x is None:
        r = b.copy()
        x = np.zeros_like(b)
    else:
        r = b - op.apply(x)
    d = dinv * r / theta
    for i in range(1, k + 1):
        x = x + d
        if i < k:
            r = r - op.apply(d)
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * r
            rho = rho_new
    return x


def lanczos_lmax(op: LevelOperator, dinv, v0, steps=10, reorth_passes=2):
    """Largest Ritz value of S = D^{-1/2} A D^{-1/2} after m = min(steps, n) Lanczos steps
    with full reorthogonalization. Returns (lambda, alphas, betas)."""
    s = np.sqrt(dinv)
    nint = int(np.count_nonzero(dinv))
    m = min(steps, nint)
    v = v0 * (dinv != 0)
    v = v / np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    tnorm = 0.0
    for j in range(m):
        w = s * op.apply(s * V[j])
        a = float(V[j] @ w)
        w = w - a * V[j]
        if j > 0:
            w = w - betas[-1] * V[j - 1]
        for _ in range(reorth_passes):
            for vi in V:
                w = w - float(vi @ w) * vi
        alphas.append(a)
        bnext = float(np.linalg.norm(w))
        tnorm = max(tnorm, abs(a) + (betas[-1] if betas else 0.0) + bnext)
        if j == m - 1 or bnext <= 1e-14 * tnorm:
            break
        betas.append(bnext)
        V.append(w / bnext)
    T = np.diag(alphas)
    for i, bt in enumerate(betas[:len(alphas) - 1]):
        T[i, i + 1] = T[i + 1, i] = bt
    lam = float(np.max(np.linalg.eigvalsh(T)))
    return lam, alphas, betas[:len(alphas) - 1]


@dataclass
class Level:
    mesh: Mesh
    op: LevelOperator
    dinv: np.ndarray
    lmax: float = 0.0
    to_coarse: Optional[Transfer] = None     # transfer between this level and the next coarser
    chol: object = None                      # coarsest level: Cholesky factor of A_II
    idx: Optional[np.ndarray] = None
    relax: object = None                     # SSOR sweeps or block inverses (those smoothers)
    l1inv: Optional[np.ndarray] = None       # l1-Jacobi: 1 / sum_j |A_ij|


class Hierarchy:
    def __init__(self, dim, nelem, p, map_desc, mu_desc, hierarchy="p", max_levels=0,
                 smoother="chebyshev", nu=4, omega=None, cheb_lo=0.25, cheb_safety=1.0,
                 eig_steps=10, eig_seed=0, lmax_override=None, direct_transfer=False,
                 nu_post=None, quadrature="gll", low_cycles=1, coarse_unknowns=0):
        if smoother not in ("jacobi", "chebyshev", "ssor", "l1jacobi", "blockjacobi"):
            raise ValueError(f"unknown smoother {smoother!r}")
        if omega is None:
            omega = 1.0 if smoother == "ssor" else 2.0 / 3.0
        self.smoother, self.omega = smoother, omega
        self.nu = self.nu_pre = nu
        self.nu_post = nu if nu_post is None else nu_post
        self.cheb_lo, self.cheb_safety = cheb_lo, cheb_safety
        self.plan = plan_levels(dim, nelem, p, hierarchy, max_levels, coarse_unknowns)
        self.levels: List[Level] = []
        if quadrature != "gll" and smoother in ("ssor", "l1jacobi", "blockjacobi"):
            raise ValueError("the Gauss-Seidel, l1 and block smoothers are built for GLL collocation")
        self.quadrature = quadrature
        self.hierarchy, self.low_cycles = hierarchy, int(low_cycles)
        for li, (ne, q) in enumerate(self.plan):
            if hierarchy == "low" and li >= 1 and p > 1:
                # first-order cells whose vertices are the order-p nodes (every 2^(li-1)-th one
                # on the coarser first-order levels): the geometry comes from those nodes
                mesh = Mesh(dim, ne, q, _node_lookup(self.levels[0].mesh, ne), mu_desc, quadrature)
            else:
                mesh = Mesh(dim, ne, q, map_desc, mu_desc, quadrature)
            op = LevelOperator(mesh)
            dg = op.diag()
            dinv = np.zeros_like(dg)
            dinv[mesh.interior] = 1.0 / dg[mesh.interior]
            self.levels.append(Level(mesh=mesh, op=op, dinv=dinv))
        for li in range(len(self.levels) - 1):
            if hierarchy == "low" and li == 0:
                continue            # levels 0 and 1 share their nodes
            self.levels[li].to_coarse = Transfer(self.levels[li].mesh,
                                                 self.levels[li + 1].mesh, direct_transfer)
        for li, lv in enumerate(self.levels[:-1]):
            if lmax_override is not None:
                lv.lmax = float(lmax_override[li])
            else:
                v0 = start_vector(eig_seed, li, lv.mesh.N)
                lam, _, _ = lanczos_lmax(lv.op, lv.dinv, v0, eig_steps)
                lv.lmax = cheb_safety * lam
        for lv in self.levels:
            if smoother == "ssor":
                lv.relax = ColoredSSOR(lv.op, lv.dinv)
            elif smoother == "blockjacobi":
                lv.relax = BlockJacobi(lv.op)
            elif smoother == "l1jacobi":
                s1 = l1_row_sums(lv.op)
                lv.l1inv = np.zeros_like(s1)
                lv.l1inv[lv.mesh.interior] = 1.0 / s1[lv.mesh.interior]
        last = self.levels[-1]
        Ad, idx = last.op.dense_interior()
        last.idx = idx
        last.chol = sla.cho_factor(Ad, lower=True) if len(idx) else None

    @property
    def fine(self) -> Level:
        return self.levels[0]

    def apply(self, li, x):
        return self.levels[li].op.apply(x)

    def smooth(self, li, b, x, steps=None, post=False):
        """Pre-smoothing (nu_pre steps) or, with post, post-smoothing (nu_post steps); steps
        overrides the count. x = None means a zero initial guess."""
        lv = self.levels[li]
        k = (self.nu_post if post else self.nu_pre) if steps is None else steps
        if self.smoother == "jacobi":
            return jacobi(lv.op, lv.dinv, b, x, k, self.omega)
        if self.smoother == "ssor":
            return lv.relax.ssor(b, x, k, self.omega)
        if self.smoother == "l1jacobi":
            return jacobi_type(lv.op, lambda r: lv.l1inv * r, b, x, k, self.omega)
        if self.smoother == "blockjacobi":
            return jacobi_type(lv.op, lv.relax.apply_inverse, b, x, k, self.omega)
        return chebyshev(lv.op, lv.dinv, lv.lmax, b, x, k, self.cheb_lo)

    def coarse_solve(self, b):
        lv = self.levels[-1]
        x = np.zeros_like(b)
        if lv.chol is not None:
            x[lv.idx] = sla.cho_solve(lv.chol, b[lv.idx])
        return x

    def precond(self, r):
        """The preconditioner of the solvers: the V-cycle from the finest level, or (hierarchy
        "low", §3.1.3) low_cycles sweeps of x <- x + V_1 (r - A_1 x) from x = 0 with the
        first-order operator A_1 on the order-p nodes and its V-cycle V_1 (level 1 down): an
        approximation of A_1^{-1} r that tends to it as the sweeps grow. Levels 0 and 1 share
        their nodes, so r and the result are the same vectors on both."""
        if self.hierarchy != "low" or len(self.levels) == 1:
            return self.vcycle(r)
        op1 = self.levels[1].op
        x = self.vcycle(r, 1)
        for _ in range(self.low_cycles - 1):
            x = x + self.vcycle(r - op1.apply(x), 1)
        return x

    def low_order_exact(self, r):
        """A_1^{-1} r by a sparse direct factorization (the paper's experiments, §4.3)."""
        import scipy.sparse.linalg as spla
        lv = self.levels[1]
        A = lv.op.K.csr()
        idx = np.nonzero(lv.mesh.interior)[0]
        x = np.zeros_like(r)
        x[idx] = spla.spsolve(A[idx][:, idx].tocsc(), r[idx])
        return x

    def vcycle(self, r, li=0):
        """e = V r with zero initial guess on level li."""
        if li == len(self.levels) - 1:
            return self.coarse_solve(r)
        lv = self.levels[li]
        x = self.smooth(li, r, None)
        res = r - lv.op.apply(x)
        ec = self.vcycle(lv.to_coarse.restrict(res), li + 1)
        x = x + lv.to_coarse.prolong(ec)
        return self.smooth(li, r, x, post=True)

    def applies(self):
        return [lv.op.applies for lv in self.levels]


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    history: List[float] = field(default_factory=list)
    relres_true: float = float("nan")


def _node_lookup(fine_mesh, ne):
    """A map description placing the vertices of a first-order mesh of ne cells per axis on the
    physical nodes of fine_mesh (every (n_e p / ne)-th node per axis)."""
    stride = [fm // c for fm, c in zip([v * fine_mesh.p for v in fine_mesh.nelem], ne)]
    nax, x = fine_mesh.nax, fine_mesh.x

    def fn(X):
        idx = np.zeros(len(X), dtype=np.int64)
        mult = 1
        for a in range(X.shape[1]):
            g = np.rint(X[:, a] * ne[a]).astype(np.int64) * stride[a]
            idx += g * mult
            mult *= nax[a]
        return x[idx]
    return {"kind": "map_callback", "fn": fn}


def mg_solve(H: Hierarchy, b, x0=None, rtol=1e-10, maxit=1000):
    op = H.fine.op
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - op.apply(x) if x0 is not None else b.copy()
    n0 = float(np.linalg.norm(r))
    hist = [n0]
    if n0 == 0.0:
        return SolveResult(x, 0, True, hist, 0.0)
    for it in range(1, maxit + 1):
        x = x + H.precond(r)
        r = b - op.apply(x)
        nr = float(np.linalg.norm(r))
        hist.append(nr)
        if nr <= rtol * n0:
            return SolveResult(x, it, True, hist, nr / n0)
        if not math.isfinite(nr):
            break
    return SolveResult(x, len(hist) - 1, False, hist, hist[-1] / n0)


def pcg(H: Hierarchy, b, x0=None, rtol=1e-10, maxit=500, precond=None):
    """Algorithm 1: h = A p; alpha = (z, r) / (p, h); x += alpha p; r -= alpha h; test;
    z = V r; beta = (z, r)_new / (z, r)_old; p = z + beta p."""
    op = H.fine.op
    M = H.precond if precond is None else precond
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - op.apply(x) if x0 is not None else b.copy()
    n0 = float(np.linalg.norm(r))
    hist = [n0]
    if n0 == 0.0:
        return SolveResult(x, 0, True, hist, 0.0)
    z = M(r)
    p = z.copy()
    gamma = float(z @ r)
    for it in range(1, maxit + 1):
        h = op.apply(p)
        alpha = gamma / float(p @ h)
        x = x + alpha * p
        r = r - alpha * h
        nr = float(np.linalg.norm(r))
        hist.append(nr)
        if nr <= rtol * n0:
            rt = float(np.linalg.norm(b - op.apply(x))) / n0
            return SolveResult(x, it, True, hist, rt)
        if not math.isfinite(nr):
            break
        z = M(r)
        gnew = float(z @ r)
        beta = gnew / gamma
        gamma = gnew
        p = z + beta * p
    return SolveResult(x, len(hist) - 1, False, hist, hist[-1] / n0)


def build_problem(prob, **kw):
    """Hierarchy and right-hand side for a problem description from the seeded inputs."""
    H = Hierarchy(prob.dim, prob.nelem, prob.order, prob.map, prob.mu,
                  hierarchy=prob.hierarchy, max_levels=prob.max_levels,
                  smoother=prob.smoother, nu=prob.nu, nu_post=prob.nu_post,
                  eig_seed=prob.eig_seed, quadrature=prob.quadrature,
                  coarse_unknowns=prob.coarse_unknowns, **kw)
    fn = prob.nodal_rhs()
    if fn is None:
        fn = nodal_field(H.fine.mesh, prob.f)
    b = load_vector(H.fine.mesh, fn)
    return H, b


def solve(prob, **kw):
    H, b = build_problem(prob, **kw)
    if prob.mode == "mg":
        return H, b, mg_solve(H, b, rtol=prob.rtol, maxit=prob.maxit)
    return H, b, pcg(H, b, rtol=prob.rtol, maxit=prob.maxit)
