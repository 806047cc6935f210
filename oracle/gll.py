"""Reference element: GLL points and weights, Lagrange derivative and interpolation matrices.

Test infrastructure only (see the package docstring).

The paper uses tensorized nodal bases on Legendre-Gauss-Lobatto points (§1, §2.3; Fig. 1
shows the p = 4 points on [0, 1]). The nodes of order p are -1, 1 and the p-1 roots of the
derivative of the Legendre polynomial P_p; the weights are 2 / (p (p+1) P_p(xi_i)^2).
"""

from __future__ import annotations

import numpy as np


def legendre(p: int, x):
    """Return (P_p(x), P_{p-1}(x)) by the three-term (Bonnet) recurrence, p >= 1."""
    x = np.asarray(x, dtype=np.float64)
    prev = np.ones_like(x)
    cur = x.copy()
    for k in range(1, p):
        prev, cur = cur, ((2 * k + 1) * x * cur - k * prev) / (k + 1)
    return cur, prev


def gll(p: int):
    """GLL nodes (ascending, on [-1, 1]) and weights for polynomial order p >= 1.

    Interior nodes are the zeros of q(x) = (1 - x^2) P_p'(x) = p (P_{p-1}(x) - x P_p(x)).
    Since q'(x) = -p (p+1) P_p(x), Newton's step is x += (P_{p-1} - x P_p) / ((p+1) P_p);
    it starts from the Chebyshev-Lobatto points -cos(pi i / p).
    """
    if p < 1:
        raise ValueError("order must be >= 1")
    x = -np.cos(np.pi * np.arange(p + 1) / p)
    for _ in range(200):
        P, Pm1 = legendre(p, x)
        dx = (Pm1 - x * P) / ((p + 1) * P)
        dx[0] = 0.0
        dx[-1] = 0.0
        x = x + dx
        if np.max(np.abs(dx)) < 1e-17:
            break
    # the rule is symmetric about 0
    x = 0.5 * (x - x[::-1])
    if p % 2 == 0:
        x[p // 2] = 0.0
    P, _ = legendre(p, x)
    w = 2.0 / (p * (p + 1) * P * P)
    return x, w


def barycentric_weights(x):
    """lambda_j = 1 / prod_{k != j} (x_j - x_k)."""
    x = np.asarray(x, dtype=np.float64)
    diff = x[:, None] - x[None, :]
    np.fill_diagonal(diff, 1.0)
    return 1.0 / np.prod(diff, axis=1)


def deriv_matrix(x):
    """D_ij = l_j'(x_i) for the Lagrange basis l_j on the nodes x (barycentric form):
    D_ij = (lambda_j / lambda_i) / (x_i - x_j) for i != j, and D_ii = -sum_{j != i} D_ij
    (the derivative of the constant 1 = sum_j l_j vanishes)."""
    x = np.asarray(x, dtype=np.float64)
    lam = barycentric_weights(x)
    diff = x[:, None] - x[None, :]
    np.fill_diagonal(diff, 1.0)
    D = (lam[None, :] / lam[:, None]) / diff
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, -D.sum(axis=1))
    return D


def lagrange_eval(x, y):
    """M_ij = l_j(y_i) = prod_{k != j} (y_i - x_k) / (x_j - x_k): the Lagrange basis on the
    nodes x evaluated at the points y."""
    x = np.asarray(x, dtype=np.float64)
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    n = len(x)
    M = np.ones((len(y), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                M[:, j] *= (y - x[k]) / (x[j] - x[k])
    return M
