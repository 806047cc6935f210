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


def fp64_close(a, b, tol=1e-12, tol_max=5e-12):
    """The FP64 parity bar: 2-norm relative error <= 1e-12, and max-norm error relative to the
    largest entry <= 5e-12 (rounding of the O(p) sums with |D| up to p(p+1)/4 grows with p)."""
    e2, em = rel2(a, b), rel_err(a, b)
    return e2 <= tol and em <= tol_max, (e2, em)


def build_pair(dim, nelem, p, map_desc=None, mu_desc=None, hierarchy="p", smoother="chebyshev",
               nu=4, max_levels=0, vcycle_prec="f64", eig_seed=0):
    from paper_1402_5938_amd import gllmg
    map_desc = map_desc or inputs.map_warp_sine(0.05)
    mu_desc = mu_desc or inputs.mu_exp_sine_product(2.0)
    cfg = gllmg.make_config(dim, nelem, p, hierarchy, smoother, nu, vcycle_prec=vcycle_prec,
                            max_levels=max_levels, eig_seed=eig_seed)
    G = gllmg.Problem(cfg, map_desc, mu_desc)
    H = mg.Hierarchy(dim, nelem, p, map_desc, mu_desc, hierarchy=hierarchy, max_levels=max_levels,
                     smoother=smoother, nu=nu, eig_seed=eig_seed)
    return G, H


def random_vec(n, seed):
    return np.random.default_rng(seed).standard_normal(n)
