"""Domain maps and coefficient fields evaluated with numpy.

Test infrastructure only (see the package docstring).

The paper's domains are images of the unit square/cube under a diffeomorphism (§2.3), and the
coefficient mu is a known function, evaluated at whatever points need it (§2.3, §4.1). The field
families and their parameters are described (without arithmetic) in
``paper_1402_5938_amd.inputs``; this module gives them meaning for the oracle.
"""

from __future__ import annotations

import math

import numpy as np


def eval_map(desc: dict, X: np.ndarray) -> np.ndarray:
    """Physical coordinates x = Phi(X) for reference points X of shape (npts, d)."""
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    kind = desc["kind"]
    prm = list(desc.get("param") or [])
    if kind == "identity":
        return X.copy()
    if kind == "warp_sine":
        a = prm[0]
        s = np.sin(2.0 * math.pi * X)
        if d == 2:
            return np.stack([X[:, 0] + a * s[:, 1], X[:, 1] + a * s[:, 0]], axis=1)
        return np.stack([X[:, 0] + a * s[:, 1] * s[:, 2],
                         X[:, 1] + a * s[:, 2] * s[:, 0],
                         X[:, 2] + a * s[:, 0] * s[:, 1]], axis=1)
    if kind == "affine":
        M = np.array(prm[:d * d]).reshape(d, d)
        c = np.array(prm[d * d:d * d + d])
        return X @ M.T + c[None, :]
    if kind == "map_callback":          # a map the caller gives as a function (§2.3)
        return np.asarray(desc["fn"](X.copy()), dtype=np.float64).reshape(X.shape)
    raise ValueError(f"unknown map kind {kind!r}")


def eval_scalar(desc: dict, x: np.ndarray) -> np.ndarray:
    """A scalar field (coefficient or right-hand side) at physical points x (npts, d)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.shape[1]
    kind = desc["kind"]
    prm = list(desc.get("param") or [])
    if kind == "const":
        return np.full(x.shape[0], prm[0])
    if kind == "callback":              # a coefficient the caller gives as a function (§2)
        return np.asarray(desc["fn"](x.copy()), dtype=np.float64).reshape(x.shape[0])
    if kind == "exp_sine_product":
        amp = prm[0]
        prod = np.ones(x.shape[0])
        for i in range(d):
            prod = prod * np.sin(2.0 * math.pi * (x[:, i] + prm[1 + i]))
        return np.exp(amp * prod)
    if kind == "exp_fourier":
        modes = np.asarray(desc["modes"], dtype=np.float64)
        J = modes.shape[0]
        g = np.zeros(x.shape[0])
        for j in range(J):
            kx = np.zeros(x.shape[0])
            for i in range(d):
                kx = kx + modes[j, i] * x[:, i]
            g = g + modes[j, 3] * np.cos(2.0 * math.pi * kx + modes[j, 4])
        return np.exp(math.sqrt(2.0 / J) * g)
    if kind == "sin_product":
        amp, freq = prm[0], prm[1]
        prod = np.ones(x.shape[0])
        for i in range(d):
            prod = prod * np.sin(freq * math.pi * x[:, i])
        return amp * prod
    if kind == "cos2_sum":
        c0, c1, freq = prm[0], prm[1], prm[2]
        s = np.zeros(x.shape[0])
        for i in range(d):
            s = s + np.cos(freq * math.pi * x[:, i]) ** 2
        return c0 + c1 * s
    raise ValueError(f"unknown field kind {kind!r}")
