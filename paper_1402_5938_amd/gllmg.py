"""Python binding of libgllmg (ctypes). Argument marshalling only: every step of the method
runs in the library's HIP kernels. PyTorch supplies device memory (tensors) and streams.

The binding never falls back to any other implementation: if the library is missing or a GPU
is not available, it raises.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GLLMG_LIB", os.path.join(HERE, "libgllmg.so"))

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, EUNSUPPORTED = range(7)
F64, F32 = 0, 1
HIER_H, HIER_P, HIER_LOW = 0, 1, 2
SMOOTH_JACOBI, SMOOTH_CHEBYSHEV, SMOOTH_SSOR, SMOOTH_L1_JACOBI, SMOOTH_BLOCK_JACOBI = 0, 1, 2, 3, 4
SMOOTHERS = {"jacobi": SMOOTH_JACOBI, "chebyshev": SMOOTH_CHEBYSHEV, "ssor": SMOOTH_SSOR,
             "l1jacobi": SMOOTH_L1_JACOBI, "blockjacobi": SMOOTH_BLOCK_JACOBI}
MODE_PCG, MODE_MG, MODE_IR = 0, 1, 2
MODES = {"pcg": MODE_PCG, "mg": MODE_MG, "ir": MODE_IR}

KINDS = {"identity": 0, "warp_sine": 1, "affine": 2, "map_callback": 3, "const": 10,
         "exp_sine_product": 11, "exp_fourier": 12, "sin_product": 13, "cos2_sum": 14,
         "callback": 20}

STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTCONV",
                5: "EBREAKDOWN", 6: "EUNSUPPORTED"}


class GllmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


FIELD_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.c_int32,
                       C.POINTER(C.c_double), C.c_void_p)


class Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nmodes", C.c_int32), ("param", C.c_double * 12),
                ("modes", C.POINTER(C.c_double)), ("fn", FIELD_FN), ("ctx", C.c_void_p)]


class Config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nelem", C.c_int32 * 3), ("order", C.c_int32),
                ("hierarchy", C.c_int32), ("max_levels", C.c_int32), ("smoother", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("omega", C.c_double),
                ("cheb_lo", C.c_double), ("cheb_safety", C.c_double), ("eig_steps", C.c_int32),
                ("vcycle_prec", C.c_int32), ("eig_seed", C.c_uint64), ("quadrature", C.c_int32),
                ("low_cycles", C.c_int32), ("coarse_unknowns", C.c_int32), ("ir_inner", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("relres_true", C.c_double), ("t_solve_s", C.c_double),
                ("applies", C.c_int64 * 16), ("history", C.POINTER(C.c_double))]


_lib = None

EXPORTS = ["gllmg_last_error", "gllmg_config_default", "gllmg_plan", "gllmg_setup",
           "gllmg_destroy", "gllmg_num_levels", "gllmg_level_info", "gllmg_set_lmax",
           "gllmg_set_graphs", "gllmg_set_persistent",
           "gllmg_node_coords", "gllmg_eval_field", "gllmg_rhs", "gllmg_diag", "gllmg_apply",
           "gllmg_apply_noalloc", "gllmg_smooth", "gllmg_prolong", "gllmg_restrict", "gllmg_vcycle", "gllmg_solve",
           "gllmg_solve_begin", "gllmg_solve_poll", "gllmg_solve_end", "gllmg_batch_solve",
           "gllmg_stream_copy"]


def lib():
    """Load libgllmg.so (built in-tree). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1402_5938_amd.build")
    # torch first: the library must resolve its HIP runtime to the one torch has loaded, since
    # it works on torch's device memory and streams (loaded first, the library would bring in
    # a second runtime that does not know them)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.gllmg_last_error.restype = C.c_char_p
    L.gllmg_config_default.argtypes = [C.POINTER(Config)]
    L.gllmg_config_default.restype = None
    L.gllmg_plan.argtypes = [C.POINTER(Config), C.POINTER(i32), C.POINTER(C.c_size_t)]
    L.gllmg_setup.argtypes = [C.POINTER(Config), C.POINTER(Field), C.POINTER(Field), vp,
                              C.c_size_t, vp, C.POINTER(vp)]
    L.gllmg_destroy.argtypes = [vp]
    L.gllmg_num_levels.argtypes = [vp, C.POINTER(i32)]
    L.gllmg_level_info.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32),
                                   C.POINTER(i32), C.POINTER(dbl)]
    L.gllmg_set_lmax.argtypes = [vp, i32, dbl]
    L.gllmg_set_graphs.argtypes = [vp, i32]
    L.gllmg_set_persistent.argtypes = [vp, i32]
    L.gllmg_node_coords.argtypes = [vp, i32, vp, vp]
    L.gllmg_eval_field.argtypes = [vp, i32, C.POINTER(Field), vp, vp]
    L.gllmg_rhs.argtypes = [vp, vp, vp, vp]
    L.gllmg_diag.argtypes = [vp, i32, i32, vp, vp]
    L.gllmg_apply.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    L.gllmg_apply_noalloc.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    L.gllmg_smooth.argtypes = [vp, i32, i32, vp, vp, i32, i32, vp]
    L.gllmg_prolong.argtypes = [vp, i32, i32, vp, vp, vp]
    L.gllmg_restrict.argtypes = [vp, i32, i32, vp, vp, vp]
    L.gllmg_vcycle.argtypes = [vp, i32, vp, vp, vp]
    L.gllmg_solve.argtypes = [vp, i32, vp, vp, dbl, i32, C.POINTER(SolveStats), vp]
    L.gllmg_solve_begin.argtypes = [vp, i32, vp, vp, dbl, i32, vp]
    L.gllmg_solve_poll.argtypes = [vp, C.POINTER(i32)]
    L.gllmg_solve_end.argtypes = [vp, C.POINTER(SolveStats)]
    L.gllmg_batch_solve.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), i32, i32, dbl,
                                    i32, C.POINTER(SolveStats), C.POINTER(C.c_int), vp]
    L.gllmg_stream_copy.argtypes = [vp, vp, C.c_size_t, vp]
    for name in EXPORTS[2:]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st):
    if st != OK:
        raise GllmgError(st, lib().gllmg_last_error().decode())


def make_field(desc: dict):
    """ctypes field from an input description dict; returns (Field, keepalive)."""
    f = Field()
    f.kind = KINDS[desc["kind"]]
    prm = list(desc.get("param") or [])
    assert len(prm) <= 12
    for i, v in enumerate(prm):
        f.param[i] = float(v)
    keep = None
    modes = desc.get("modes")
    if modes is not None:
        keep = np.ascontiguousarray(modes, dtype=np.float64)
        f.nmodes = keep.shape[0]
        f.modes = keep.ctypes.data_as(C.POINTER(C.c_double))
    if desc["kind"] in ("map_callback", "callback"):
        keep = _callback(desc["fn"], desc["kind"] == "map_callback")
        f.fn = keep
    return f, keep


def _callback(fn, is_map):
    """A C callback around fn(points) -> values: points is a (npts, dim) float64 array (reference
    coordinates for a map, physical ones for a coefficient); fn returns (npts, dim) or (npts,).
    An exception inside fn leaves NaN values, which setup then rejects."""
    def cb(pts, npts, dim, out, ctx):
        o = np.ctypeslib.as_array(out, shape=(npts, dim) if is_map else (npts,))
        try:
            X = np.ctypeslib.as_array(pts, shape=(npts, dim)).copy()
            o[...] = np.asarray(fn(X), dtype=np.float64).reshape(o.shape)
        except Exception:
            o[...] = np.nan
    return FIELD_FN(cb)


def make_config(dim, nelem, order, hierarchy="p", smoother="chebyshev", nu=4, nu_post=None,
                vcycle_prec="f64", max_levels=0, omega=None, cheb_lo=0.25,
                cheb_safety=1.0, eig_steps=10, eig_seed=0, quadrature="gll",
                low_cycles=1, coarse_unknowns=0, ir_inner=0) -> Config:
    c = Config()
    lib().gllmg_config_default(C.byref(c))
    c.dim = dim
    ne = list(nelem) + [1] * (3 - len(nelem))
    for a in range(3):
        c.nelem[a] = int(ne[a])
    c.order = order
    if hierarchy not in ("h", "p", "low"):
        raise ValueError(f"unknown hierarchy {hierarchy!r}")
    c.hierarchy = {"h": HIER_H, "p": HIER_P, "low": HIER_LOW}[hierarchy]
    c.low_cycles = low_cycles
    c.coarse_unknowns = coarse_unknowns
    c.ir_inner = ir_inner
    if smoother not in SMOOTHERS:
        raise ValueError(f"unknown smoother {smoother!r}")
    c.smoother = SMOOTHERS[smoother]
    if omega is None:   # the paper's damping: 1 for SSOR, 2/3 for the Jacobi smoothers
        omega = 1.0 if smoother == "ssor" else 2.0 / 3.0
    c.nu_pre = nu
    c.nu_post = nu if nu_post is None else nu_post
    c.vcycle_prec = F32 if vcycle_prec == "f32" else F64
    c.max_levels = max_levels
    c.omega, c.cheb_lo, c.cheb_safety = omega, cheb_lo, cheb_safety
    c.eig_steps, c.eig_seed = eig_steps, eig_seed
    if quadrature not in ("gll", "gauss"):
        raise ValueError(f"unknown quadrature {quadrature!r}")
    c.quadrature = 1 if quadrature == "gauss" else 0
    return c


def plan(cfg: Config):
    n = C.c_int32()
    b = C.c_size_t()
    _check(lib().gllmg_plan(C.byref(cfg), C.byref(n), C.byref(b)))
    return n.value, b.value


def _stream(stream):
    import torch
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(stream)


def _ptr(t):
    assert t.is_cuda and t.is_contiguous()
    return C.c_void_p(t.data_ptr())


@dataclass
class LevelInfo:
    nnodes: int
    ninterior: int
    order: int
    nelem: tuple
    lmax: float


@dataclass
class SolveResult:
    status: int
    iters: int
    converged: bool
    relres: float
    relres_true: float
    t_solve_s: float
    applies: List[int]
    history: List[float] = field(default_factory=list)


class Problem:
    """A set-up hierarchy on the current GPU. The workspace is a torch uint8 tensor (so torch's
    allocator accounts for it) unless ``workspace=False`` asks the library to allocate."""

    def __init__(self, cfg: Config, map_desc: dict, mu_desc: dict, stream=None, workspace=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("gllmg needs a GPU")
        self.cfg = cfg
        self.nlevels, self.bytes = plan(cfg)
        self.ws = None
        wsp, wsb = None, 0
        if workspace:
            self.ws = torch.empty(self.bytes + 256, dtype=torch.uint8, device="cuda")
            base = self.ws.data_ptr()
            wsp = (base + 255) // 256 * 256
            wsb = self.bytes
        fm, k1 = make_field(map_desc)
        fu, k2 = make_field(mu_desc)
        h = C.c_void_p()
        _check(lib().gllmg_setup(C.byref(cfg), C.byref(fm), C.byref(fu), C.c_void_p(wsp),
                                 C.c_size_t(wsb), _stream(stream), C.byref(h)))
        self.h = h
        self.dim = cfg.dim
        self.levels = [self.level_info(l) for l in range(self.nlevels)]

    @classmethod
    def from_inputs(cls, prob, stream=None, **kw):
        cfg = make_config(prob.dim, prob.nelem, prob.order, prob.hierarchy, prob.smoother,
                          prob.nu, nu_post=prob.nu_post, vcycle_prec=prob.vcycle_prec,
                          max_levels=prob.max_levels, eig_seed=prob.eig_seed,
                          quadrature=prob.quadrature, coarse_unknowns=prob.coarse_unknowns, **kw)
        return cls(cfg, prob.map, prob.mu, stream=stream)

    def close(self):
        if getattr(self, "h", None):
            lib().gllmg_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- info
    def level_info(self, l) -> LevelInfo:
        nn, ni = C.c_int64(), C.c_int64()
        o = C.c_int32()
        ne = (C.c_int32 * 3)()
        lm = C.c_double()
        _check(lib().gllmg_level_info(self.h, l, C.byref(nn), C.byref(ni), C.byref(o), ne,
                                      C.byref(lm)))
        return LevelInfo(nn.value, ni.value, o.value, tuple(ne[:self.dim]), lm.value)

    def set_lmax(self, l, v):
        _check(lib().gllmg_set_lmax(self.h, l, float(v)))
        self.levels[l].lmax = float(v)

    def set_graphs(self, enable: bool):
        _check(lib().gllmg_set_graphs(self.h, 1 if enable else 0))

    def set_persistent(self, enable: bool):
        _check(lib().gllmg_set_persistent(self.h, 1 if enable else 0))

    def nnodes(self, l=0):
        return self.levels[l].nnodes

    # ---------------------------------------------------------------- operations
    def node_coords(self, l=0, stream=None):
        import torch
        out = torch.empty(self.nnodes(l) * self.dim, dtype=torch.float64, device="cuda")
        _check(lib().gllmg_node_coords(self.h, l, _ptr(out), _stream(stream)))
        return out.view(-1, self.dim)

    def eval_field(self, desc, l=0, stream=None):
        import torch
        f, keep = make_field(desc)
        out = torch.empty(self.nnodes(l), dtype=torch.float64, device="cuda")
        _check(lib().gllmg_eval_field(self.h, l, C.byref(f), _ptr(out), _stream(stream)))
        return out

    def rhs(self, f_nodal, out=None, stream=None):
        import torch
        b = torch.empty_like(f_nodal) if out is None else out
        _check(lib().gllmg_rhs(self.h, _ptr(f_nodal), _ptr(b), _stream(stream)))
        return b

    def diag(self, l=0, prec=F64, stream=None):
        import torch
        dt = torch.float64 if prec == F64 else torch.float32
        d = torch.empty(self.nnodes(l), dtype=dt, device="cuda")
        _check(lib().gllmg_diag(self.h, l, prec, _ptr(d), _stream(stream)))
        return d

    def apply(self, x, y=None, l=0, prec=None, neumann=False, stream=None):
        import torch
        prec = _prec_of(x) if prec is None else prec
        y = torch.empty_like(x) if y is None else y
        _check(lib().gllmg_apply(self.h, l, prec, 1 if neumann else 0, _ptr(x), _ptr(y),
                                 _stream(stream)))
        return y

    def apply_noalloc(self, x, y, l=0, prec=None, neumann=False, stream=None):
        """gllmg_apply_noalloc: the product with the library's static element-vector buffer;
        y must be given (this call allocates nothing)."""
        prec = _prec_of(x) if prec is None else prec
        _check(lib().gllmg_apply_noalloc(self.h, l, prec, 1 if neumann else 0, _ptr(x), _ptr(y),
                                         _stream(stream)))
        return y

    def smooth(self, b, x, steps, l=0, zero_guess=False, stream=None):
        _check(lib().gllmg_smooth(self.h, l, _prec_of(b), _ptr(b), _ptr(x), steps,
                                  1 if zero_guess else 0, _stream(stream)))
        return x

    def prolong(self, xc, fine_level=0, out=None, stream=None):
        import torch
        xf = torch.empty(self.nnodes(fine_level), dtype=xc.dtype, device="cuda") if out is None else out
        _check(lib().gllmg_prolong(self.h, fine_level, _prec_of(xc), _ptr(xc), _ptr(xf),
                                   _stream(stream)))
        return xf

    def restrict(self, rf, fine_level=0, out=None, stream=None):
        import torch
        rc = torch.empty(self.nnodes(fine_level + 1), dtype=rf.dtype, device="cuda") if out is None else out
        _check(lib().gllmg_restrict(self.h, fine_level, _prec_of(rf), _ptr(rf), _ptr(rc),
                                    _stream(stream)))
        return rc

    def vcycle(self, r, out=None, stream=None):
        import torch
        e = torch.empty_like(r) if out is None else out
        _check(lib().gllmg_vcycle(self.h, _prec_of(r), _ptr(r), _ptr(e), _stream(stream)))
        return e

    def solve(self, b, x=None, mode="pcg", rtol=1e-10, maxit=500, stream=None,
              raise_on_notconv=False) -> SolveResult:
        import torch
        x = torch.zeros_like(b) if x is None else x
        hist = (C.c_double * (maxit + 1))()
        st = SolveStats()
        st.history = C.cast(hist, C.POINTER(C.c_double))
        m = MODES[mode]
        status = lib().gllmg_solve(self.h, m, _ptr(b), _ptr(x), float(rtol), int(maxit),
                                   C.byref(st), _stream(stream))
        if status not in (OK, ENOTCONV) or (status == ENOTCONV and raise_on_notconv):
            _check(status)
        res = _result(status, st, hist, self.nlevels)
        if m == MODE_IR:  # one residual norm per refinement step, then -1 (if there is room)
            n = next((i for i in range(maxit + 1) if hist[i] < 0.0), maxit + 1)
            res.history = list(hist[:n])
        return res

    def solve_async(self, b, x, mode="pcg", rtol=1e-10, maxit=500, stream=None) -> AsyncSolve:
        return AsyncSolve(self, b, x, mode, rtol, maxit, stream)


class AsyncSolve:
    """A solve in progress (gllmg_solve_begin / _poll / _end)."""

    def __init__(self, prob: "Problem", b, x, mode="pcg", rtol=1e-10, maxit=500, stream=None):
        self.prob, self.b, self.x, self.maxit = prob, b, x, maxit
        self.hist = (C.c_double * (maxit + 1))()
        m = MODES[mode]
        _check(lib().gllmg_solve_begin(prob.h, m, _ptr(b), _ptr(x), float(rtol), int(maxit),
                                       _stream(stream)))
        self.result = None

    def poll(self) -> bool:
        if self.result is not None:
            return True
        d = C.c_int32()
        _check(lib().gllmg_solve_poll(self.prob.h, C.byref(d)))
        if d.value:
            self.finish()
        return self.result is not None

    def finish(self) -> "SolveResult":
        if self.result is None:
            st = SolveStats()
            st.history = C.cast(self.hist, C.POINTER(C.c_double))
            status = lib().gllmg_solve_end(self.prob.h, C.byref(st))
            if status not in (OK, ENOTCONV):
                _check(status)
            self.result = _result(status, st, self.hist, self.prob.nlevels)
        return self.result


def _result(status, st, hist, nlevels):
    return SolveResult(status=status, iters=st.iters, converged=bool(st.converged),
                       relres=st.relres, relres_true=st.relres_true, t_solve_s=st.t_solve_s,
                       applies=list(st.applies[:nlevels]), history=list(hist[:st.iters + 1]))


def batch_solve(problems, bs, xs, mode="pcg", rtol=1e-10, maxit=500, stream=None):
    """gllmg_batch_solve over Problem objects with per-problem FP64 vectors."""
    n = len(problems)
    P = (C.c_void_p * n)(*[p.h for p in problems])
    B = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    X = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    stats = (SolveStats * n)()
    hists = [(C.c_double * (maxit + 1))() for _ in range(n)]
    for i in range(n):
        stats[i].history = C.cast(hists[i], C.POINTER(C.c_double))
    status = (C.c_int * n)()
    m = MODES[mode]
    st = lib().gllmg_batch_solve(P, B, X, n, m, float(rtol), int(maxit), stats, status,
                                 _stream(stream))
    if st not in (OK, ENOTCONV):
        _check(st)
    return [_result(status[i], stats[i], hists[i], problems[i].nlevels) for i in range(n)]


def stream_copy(src, dst, stream=None):
    """gllmg_stream_copy of a whole contiguous device tensor into another of the same size."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().gllmg_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)))
    return dst


def _prec_of(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("vectors must be float64 or float32")
