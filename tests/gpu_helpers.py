"""Shared helpers for the GPU parity tests: build the same problem on both sides."""

import numpy as np

from oracle import mg
from paper_1402_5938_amd import inputs


def to_np(t):
    return t.detach().cpu().numpy()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(a, b):
    """max |a - b| / max |b|"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / den


def rel2(a, b):
    """||a - b||_2 / ||b||_2"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# Every FP64 comparison made through fp64_close: (test, plain ||a-b||_2/||b||_2, plain
# max|a-b|/max|b|, the bar's share used). tests/conftest.py writes it out when
# GLLMG_PARITY_REPORT names a file, so the plain relative errors can be read beside the bar.
OBSERVED = []


def fp64_close(a, b, scale=None, tol=1e-12, tol_scale=1e-14):
    """The FP64 parity bar: ||a - b||_2 <= 1e-12 ||b||_2 and max|a - b| <= 5e-12 max|b|. With
    `scale` (the oracle's |B|^T|G||B||x|, the magnitude of the terms whose rounding the two
    evaluation orders differ by) the report also states the share of the wider bound
    1e-12 ||b||_2 + 1e-14 ||scale||_2 that the difference uses; the test itself applies the
    plain bound."""
    import os
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d2 = np.linalg.norm(a - b)
    e2, em = rel2(a, b), rel_err(a, b)
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    if scale is None:
        ok = e2 <= tol and em <= 5 * tol
        OBSERVED.append({"test": test, "rel2": e2, "relmax": em, "bar": "plain",
                         "used": max(e2 / tol, em / (5 * tol))})
        return ok, (e2, em)
    bound = tol * np.linalg.norm(b) + tol_scale * np.linalg.norm(scale)
    OBSERVED.append({"test": test, "rel2": e2, "relmax": em, "bar": "scaled",
                     "scaled_bound_rel2": bound / max(np.linalg.norm(b), 1e-300),
                     "used": max(e2 / tol, em / (5 * tol)),
                     "used_scaled": d2 / bound if bound > 0 else float("inf")})
    return e2 <= tol and em <= 5 * tol, (e2, em, d2 / bound if bound > 0 else float("inf"))


def build_pair(dim, nelem, p, map_desc=None, mu_desc=None, hierarchy="p", smoother="chebyshev",
               nu=4, max_levels=0, vcycle_prec="f64", eig_seed=0, nu_post=None,
               quadrature="gll", low_cycles=1, coarse_unknowns=0):
    from paper_1402_5938_amd import gllmg
    map_desc = map_desc or inputs.map_warp_sine(0.05)
    mu_desc = mu_desc or inputs.mu_exp_sine_product(2.0)
    cfg = gllmg.make_config(dim, nelem, p, hierarchy, smoother, nu, nu_post=nu_post,
                            vcycle_prec=vcycle_prec, max_levels=max_levels, eig_seed=eig_seed,
                            quadrature=quadrature, low_cycles=low_cycles,
                            coarse_unknowns=coarse_unknowns)
    G = gllmg.Problem(cfg, map_desc, mu_desc)
    H = mg.Hierarchy(dim, nelem, p, map_desc, mu_desc, hierarchy=hierarchy, max_levels=max_levels,
                     smoother=smoother, nu=nu, nu_post=nu_post, eig_seed=eig_seed,
                     quadrature=quadrature, low_cycles=low_cycles,
                     coarse_unknowns=coarse_unknowns)
    return G, H


def random_vec(n, seed):
    return np.random.default_rng(seed).standard_normal(n)
