"""Write the full-size expected values in tests/golden/ from the CPU oracle only.

python tests/golden/make_golden.py [config2|config2lit|config3|batch|serve|all]

For the 3D warped variable-coefficient problem at its two full sizes (16^3 hexes at p = 8 and
8^3 hexes at p = 16, 2,146,689 nodes each), the oracle's FP64 p-multigrid PCG (Chebyshev
degree 4, rtol 1e-10) gives: lambda_max per level, the iteration count, the residual history,
the solution at seeded sample nodes and its norm; plus y = A x for a seeded x at sample nodes,
with the rounding scale |B|^T|G||B||x| at the same nodes. The 8^3, p = 16 problem also gets a
tight solve (rtol 1e-13) as the reference solution for the mixed-precision run.

For one problem of each order class of the batched workload (4^3 hexes, random-Fourier mu)
and for four requests of a seeded serving trace: the same quantities at the problem's own
tolerance, plus the tight reference solution at the sample nodes.
Inputs come from paper_1402_5938_amd.inputs (seeded, no arithmetic of the method); nothing
here calls the GPU library.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem, mg  # noqa: E402
from paper_1402_5938_amd import inputs  # noqa: E402

NSAMPLE = 2048


def sample_nodes(N, seed=1234):
    return np.sort(np.random.default_rng(seed).choice(N, size=NSAMPLE, replace=False))


def run(name, prob, tight=False):
    t0 = time.time()
    H, b = mg.build_problem(prob)
    t_setup = time.time() - t0
    m = H.fine.mesh
    idx = sample_nodes(m.N)
    xs = inputs.uniform_nodal(99, m.N)
    y = H.fine.op.apply(xs)
    ya = H.fine.op.apply_abs(xs)
    t1 = time.time()
    res = mg.pcg(H, b, rtol=prob.rtol, maxit=prob.maxit)
    t_solve = time.time() - t1
    out = {
        "problem": prob.name, "nnodes": int(m.N), "levels": [[list(lv.mesh.nelem), lv.mesh.p] for lv in H.levels],
        "lmax": [lv.lmax for lv in H.levels[:-1]], "iters": res.iters, "converged": bool(res.converged),
        "history": res.history, "relres_true": res.relres_true,
        "sample_nodes": idx.tolist(), "x_sample": res.x[idx].tolist(),
        "x_norm2": float(np.linalg.norm(res.x)), "b_norm2": float(np.linalg.norm(b)),
        "apply_input_seed": 99, "apply_sample": y[idx].tolist(), "apply_norm2": float(np.linalg.norm(y)),
        "apply_abs_sample": ya[idx].tolist(), "apply_abs_norm2": float(np.linalg.norm(ya)),
        "oracle_setup_s": t_setup, "oracle_solve_s": t_solve,
    }
    if tight:
        add_tight(out, H, b, res, idx)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f)
    print(name, "iters", res.iters, "setup", round(t_setup, 1), "s solve", round(t_solve, 1), "s", flush=True)


TIGHT_RTOL = 1e-13


def add_tight(out, H, b, res, idx):
    """The reference solution: the same PCG to rtol 1e-13, and the error of the
    problem-tolerance iterate against it."""
    ref = mg.pcg(H, b, rtol=TIGHT_RTOL, maxit=2000)
    assert ref.converged
    out["tight_rtol"] = TIGHT_RTOL
    out["tight_iters"] = ref.iters
    out["x_tight_sample"] = ref.x[idx].tolist()
    out["x_tight_norm2"] = float(np.linalg.norm(ref.x))
    out["err_vs_tight"] = float(np.linalg.norm(res.x - ref.x) / np.linalg.norm(ref.x))


def run_small(name, prob):
    """A problem of the batched or serving workload: level plan, lambda_max, iteration count and
    residual history at the problem's tolerance with the FP64 V-cycle, the tight reference."""
    t0 = time.time()
    H, b = mg.build_problem(prob)
    m = H.fine.mesh
    idx = sample_nodes(m.N, seed=4321) if m.N > NSAMPLE else np.arange(m.N)
    res = mg.pcg(H, b, rtol=prob.rtol, maxit=prob.maxit)
    out = {
        "problem": prob.name, "nnodes": int(m.N), "rtol": prob.rtol,
        "levels": [[list(lv.mesh.nelem), lv.mesh.p] for lv in H.levels],
        "lmax": [lv.lmax for lv in H.levels[:-1]], "iters": res.iters,
        "converged": bool(res.converged), "history": res.history,
        "relres_true": res.relres_true, "sample_nodes": idx.tolist(),
        "x_sample": res.x[idx].tolist(), "x_norm2": float(np.linalg.norm(res.x)),
        "b_norm2": float(np.linalg.norm(b)),
    }
    add_tight(out, H, b, res, idx)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f)
    print(name, "iters", res.iters, "tight", out["tight_iters"], "err", out["err_vs_tight"],
          round(time.time() - t0, 1), "s", flush=True)


BATCH_SEED, BATCH_COUNT = 0, 256
SERVE_SEED, SERVE_RATE, SERVE_SPAN = 7, 200.0, 30.0
SERVE_RIDS = (1, 4, 7, 39)


def batch_golden_indices(probs):
    """The first problem of each order class of the batch."""
    first = {}
    for i, pb in enumerate(probs):
        first.setdefault(pb.order, i)
    return sorted(first.values())


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("config2", "all"):
        run("warped_16cubed_p8", inputs.warped_var3d(nelem=16, order=8))
    if which in ("config2lit", "all"):
        # the order sequence 8, 4, 2, 1 with the exact solve on 16^3 at p = 1 (3375 unknowns)
        run("warped_16cubed_p8_levels4", inputs.warped_var3d(nelem=16, order=8, max_levels=4))
    if which in ("config3", "all"):
        run("warped_8cubed_p16", inputs.warped_var3d(nelem=8, order=16, f_seed=0), tight=True)
    if which in ("batch", "all"):
        probs = inputs.batched_problems(seed=BATCH_SEED, count=BATCH_COUNT)
        for i in batch_golden_indices(probs):
            run_small(f"batch_4cubed_p{probs[i].order}_i{i}", probs[i])
    if which in ("serve", "all"):
        trace = inputs.serving_trace(seed=SERVE_SEED, rate=SERVE_RATE, duration_s=SERVE_SPAN)
        for rid in SERVE_RIDS:
            run_small(f"serve_req{rid}", trace[rid].problem)


if __name__ == "__main__":
    main()
