"""Seeded synthetic inputs shared by the tests, the benchmark and the serving loop.

This module holds problem descriptions (mesh, order, the coefficient and map families with
their parameters) and every random draw the workloads need. It contains none of the
method's arithmetic: no basis, quadrature, operator, smoother or solver code. The CPU
oracle and the GPU library each evaluate the field families described here with their own
code.

Field descriptions are plain dicts ``{"kind": str, "param": [floats], "modes": ndarray|None}``.

Map kinds (the diffeomorphism of the unit square/cube onto the domain, paper §2.3):
  ``identity``    Phi(X) = X
  ``warp_sine``   3D: Phi = (X + a sY sZ, Y + a sZ sX, Z + a sX sY), sW = sin(2 pi W);
                  2D: Phi = (X + a sY, Y + a sX); param = [a]
  ``affine``      Phi(X) = M X + c; param = M row-major (d*d values) then c (d values)
Coefficient / right-hand-side kinds (evaluated at physical coordinates x = Phi(X)):
  ``const``             c; param = [c]
  ``exp_sine_product``  exp(amp * prod_i sin(2 pi (x_i + phase_i))); param = [amp, ph0, ph1, ph2]
  ``exp_fourier``       exp(sqrt(2/J) sum_j a_j cos(2 pi k_j . x + phi_j));
                        modes = (J, 5) rows [k0, k1, k2, a, phi]
  ``sin_product``       amp * prod_i sin(freq pi x_i); param = [amp, freq]
  ``cos2_sum``          c0 + c1 * sum_i cos^2(freq pi x_i); param = [c0, c1, freq]
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def field_const(c: float) -> dict:
    return {"kind": "const", "param": [float(c)], "modes": None}


def map_identity() -> dict:
    return {"kind": "identity", "param": [], "modes": None}


def map_warp_sine(a: float) -> dict:
    return {"kind": "warp_sine", "param": [float(a)], "modes": None}


def map_affine(M, c) -> dict:
    M = np.asarray(M, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    return {"kind": "affine", "param": list(M.ravel()) + list(c.ravel()), "modes": None}


def map_callback(fn) -> dict:
    """A map given as a function of reference points: fn(X) with X of shape (npts, d) returns the
    physical points (npts, d)."""
    return {"kind": "map_callback", "fn": fn}


def field_callback(fn) -> dict:
    """A coefficient given as a function of physical points: fn(x) with x of shape (npts, d)
    returns (npts,) values."""
    return {"kind": "callback", "fn": fn}


def mu_exp_sine_product(amp: float, phase=(0.0, 0.0, 0.0)) -> dict:
    ph = list(phase) + [0.0] * (3 - len(phase))
    return {"kind": "exp_sine_product", "param": [float(amp)] + [float(v) for v in ph],
            "modes": None}


def mu_exp_fourier(modes: np.ndarray) -> dict:
    return {"kind": "exp_fourier", "param": [], "modes": np.ascontiguousarray(modes, np.float64)}


def f_sin_product(amp: float, freq: float = 1.0) -> dict:
    return {"kind": "sin_product", "param": [float(amp), float(freq)], "modes": None}


def mu_cos2_sum(c0: float, c1: float, freq: float) -> dict:
    return {"kind": "cos2_sum", "param": [float(c0), float(c1), float(freq)], "modes": None}


# The exact coarse solve takes up to 4096 unknowns; one dense solve of that size costs less on
# the GPU than the launches of the levels below it. The single large solves of the benchmark
# stop coarsening at the first first-order level that small. Batched and served problems stop
# at 512: each request pays the host-side inverse (O(n^3)) and keeps the dense inverse
# resident (O(n^2) bytes), which at 4096 unknowns would cost a served request seconds of setup
# and 190 MB of device memory.
COARSE_UNKNOWNS = 4096
REQUEST_COARSE_UNKNOWNS = 512


@dataclass
class Problem:
    """One solve: mesh, order, fields, hierarchy and solver settings."""
    name: str
    dim: int
    nelem: tuple
    order: int
    map: dict
    mu: dict
    f: Optional[dict] = None            # a field evaluated at the nodes, or None if f_nodal given
    f_nodal: Optional[np.ndarray] = None
    f_seed: Optional[int] = None        # nodal f ~ U[-1,1] drawn on demand from this seed
    hierarchy: str = "p"                # "h" (fixed order) or "p" (order halving, then h)
    smoother: str = "chebyshev"         # "chebyshev", "jacobi", "ssor", "l1jacobi", "blockjacobi"
    nu: int = 4                         # Chebyshev degree / sweeps / SSOR steps, pre-smoothing
    nu_post: Optional[int] = None       # post-smoothing count (None: the same as nu)
    quadrature: str = "gll"             # "gll" (collocated) or "gauss" (p+1 Gauss points)
    mode: str = "pcg"                   # "pcg" or "mg"
    vcycle_prec: str = "f64"            # "f64" or "f32"
    rtol: float = 1e-10
    maxit: int = 500
    max_levels: int = 0
    coarse_unknowns: int = 0            # > 0: stop at the first first-order level this small
    eig_seed: int = 0

    @property
    def nnodes(self) -> int:
        return int(np.prod([ne * self.order + 1 for ne in self.nelem]))

    def nodal_rhs(self) -> Optional[np.ndarray]:
        """The nodal right-hand side if it is given by values rather than a field."""
        if self.f_nodal is not None:
            return self.f_nodal
        if self.f_seed is not None:
            return uniform_nodal(self.f_seed, self.nnodes)
        return None

    def nodal_rhs_device(self, device="cuda"):
        """Served requests: nodal f ~ U[-1,1] drawn on the device (torch's counter-based
        generator seeded with f_seed), as a client would hand over data already in GPU memory;
        None if f is a field."""
        import torch
        if self.f_seed is None:
            return None
        g = torch.Generator(device=device)
        g.manual_seed(self.f_seed & 0x7FFFFFFFFFFFFFFF)
        u = torch.rand(self.nnodes, dtype=torch.float64, device=device, generator=g)
        return u.mul_(2.0).sub_(1.0)


def node_count(nelem, order) -> int:
    return int(np.prod([ne * order + 1 for ne in nelem]))


def uniform_nodal(seed: int, n: int) -> np.ndarray:
    """f ~ U[-1, 1] at every node, from numpy's PCG64 stream for ``seed``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


# --------------------------------------------------------------------------------------
# The workloads. Each follows the structure of the paper's test problems (§4.1): a square or
# cube mapped by a smooth diffeomorphism, homogeneous Dirichlet data, a smooth coefficient.
# --------------------------------------------------------------------------------------

def poisson2d_manufactured(nelem=4, order=4) -> Problem:
    """2D unit square, mu = 1, f = 2 pi^2 sin(pi x) sin(pi y), h-multigrid, Chebyshev degree 2,
    multigrid as solver."""
    return Problem(name=f"2d-const {nelem}^2 p={order}", dim=2, nelem=(nelem, nelem),
                   order=order, map=map_identity(), mu=field_const(1.0),
                   f=f_sin_product(2.0 * math.pi ** 2, 1.0), hierarchy="h",
                   smoother="chebyshev", nu=2, mode="mg", maxit=1000)


def warped_var3d(nelem=16, order=8, vcycle_prec="f64", f_seed=None, max_levels=0,
                 coarse_unknowns=0) -> Problem:
    """3D unit cube under the cyclic sine warp (a = 0.05), mu = exp(4.6 sx sy sz), p-multigrid,
    Chebyshev degree 4, PCG. f = 1, or nodal U[-1,1] from ``f_seed``. Order halving to 1, then
    h-coarsening; coarse_unknowns = k > 0 stops at the first first-order level with at most k
    interior unknowns, max_levels = k > 0 keeps the finest k levels (at p = 8 on 16^3 hexes
    both k = 4096 and max_levels = 4 give the order sequence 8, 4, 2, 1 with the exact solve on
    the first-order level)."""
    ne = (nelem, nelem, nelem)
    p = Problem(name=f"3d-var {nelem}^3 p={order}" + (f" levels={max_levels}" if max_levels else "")
                + (f" coarse<={coarse_unknowns}" if coarse_unknowns else ""),
                dim=3, nelem=ne, order=order,
                map=map_warp_sine(0.05), mu=mu_exp_sine_product(4.6),
                hierarchy="p", smoother="chebyshev", nu=4, mode="pcg",
                vcycle_prec=vcycle_prec, max_levels=max_levels, coarse_unknowns=coarse_unknowns)
    if f_seed is None:
        p.f = field_const(1.0)
    else:
        p.f_seed = int(f_seed)
    return p


def fourier_modes(rng: np.random.Generator, J: int = 16, dim: int = 3) -> np.ndarray:
    """J random Fourier modes: k_j uniform in {-2..2}^d without 0, a_j ~ N(0,1),
    phi_j ~ U[0, 2 pi). Rows are [k0, k1, k2, a, phi] (unused k components are 0)."""
    rows = np.zeros((J, 5))
    for j in range(J):
        while True:
            k = rng.integers(-2, 3, size=dim)
            if np.any(k != 0):
                break
        rows[j, :dim] = k
    rows[:, 3] = rng.standard_normal(J)
    rows[:, 4] = rng.uniform(0.0, 2.0 * math.pi, size=J)
    return rows


def batched_problems(seed: int = 0, count: int = 256, nelem: int = 4,
                     orders=(2, 4, 8, 16),
                     coarse_unknowns: int = REQUEST_COARSE_UNKNOWNS) -> List[Problem]:
    """Independent 3D problems on 4^3 hex meshes, order uniform in ``orders``,
    mu = exp(random-Fourier field) and f ~ U[-1,1], each from its own spawned seed; the exact
    solve on the first first-order level with at most ``coarse_unknowns`` interior unknowns."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        p = int(rng.choice(orders))
        modes = fourier_modes(rng, 16, 3)
        prob = Problem(name=f"batch[{i}] 4^3 p={p}", dim=3, nelem=(nelem,) * 3, order=p,
                       map=map_identity(), mu=mu_exp_fourier(modes), hierarchy="p",
                       smoother="chebyshev", nu=4, mode="pcg", vcycle_prec="f32",
                       coarse_unknowns=coarse_unknowns)
        prob.f_seed = int(rng.integers(0, 2**63 - 1))
        out.append(prob)
    return out


@dataclass
class Request:
    rid: int
    arrival_s: float
    problem: Problem


def serving_trace(seed: int = 0, rate: float = 200.0, duration_s: float = 60.0,
                  max_requests: Optional[int] = None,
                  coarse_unknowns: int = REQUEST_COARSE_UNKNOWNS) -> List[Request]:
    """Poisson arrivals (exponential gaps of mean 1/rate) of mixed 2D/3D solves.
    dim in {2,3} equally likely; 2D n_e in {8,...,64}, 3D n_e in {2,...,24}; p in {4,6,8,12,16};
    mu = exp((ln C / 2) prod sin(2 pi (x_i + phi_i))) with C log-uniform in [1e2, 1e4]."""
    rng = np.random.default_rng(seed)
    ne2 = [8, 12, 16, 24, 32, 48, 64]
    ne3 = [2, 3, 4, 6, 8, 12, 16, 24]
    orders = [4, 6, 8, 12, 16]
    t = 0.0
    out = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s or (max_requests is not None and rid >= max_requests):
            break
        dim = int(rng.choice([2, 3]))
        ne = int(rng.choice(ne2 if dim == 2 else ne3))
        p = int(rng.choice(orders))
        C = float(10.0 ** rng.uniform(2.0, 4.0))
        phase = rng.uniform(0.0, 1.0, size=3)
        prob = Problem(name=f"req{rid} {dim}d {ne}^{dim} p={p}", dim=dim, nelem=(ne,) * dim,
                       order=p, map=map_identity(),
                       mu=mu_exp_sine_product(math.log(C) / 2.0, tuple(phase[:dim])),
                       hierarchy="p", smoother="chebyshev", nu=4, mode="pcg",
                       vcycle_prec="f32", rtol=1e-8, coarse_unknowns=coarse_unknowns)
        prob.f_seed = int(rng.integers(0, 2**63 - 1))
        out.append(Request(rid=rid, arrival_s=t, problem=prob))
        rid += 1
    return out
