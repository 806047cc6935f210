"""Continuous-batching solve server on one GPU.

Requests (problem descriptions with an arrival time) are admitted against an HBM budget by
their exact device footprint (gllmg_plan's workspace plus the request's own vectors). A setup
thread builds each admitted request's hierarchy, which then stays resident in HBM until its
solve finishes. The serving loop keeps every active solve moving iteration by iteration
(gllmg_solve_begin / _poll / _end): requests that arrive while others are on the GPU join as
soon as memory and a slot are free, and their iterations overlap on the device's queues.
Requests of one shape that are ready at the same moment are solved together as a launch group
(gllmg_batch_solve on a worker thread: every kernel launched once for all of them, each result
bit for bit the one it gets alone), the others one by one. Nothing here computes any part of
the method: every step runs in libgllmg.
"""

from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import queue
import threading
import time
from typing import Dict, List, Optional

import numpy as np

from . import gllmg
from .inputs import Problem, Request


class HbmLedger:
    """Bytes promised to admitted requests, against a fixed budget."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self._lock = threading.Lock()

    def try_reserve(self, nbytes: int) -> bool:
        with self._lock:
            if self.used + nbytes > self.budget:
                return False
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            return True

    def release(self, nbytes: int):
        with self._lock:
            self.used -= nbytes
            assert self.used >= 0


def request_config(prob: Problem) -> gllmg.Config:
    return gllmg.make_config(prob.dim, prob.nelem, prob.order, prob.hierarchy, prob.smoother,
                             prob.nu, vcycle_prec=prob.vcycle_prec, max_levels=prob.max_levels,
                             eig_seed=prob.eig_seed, coarse_unknowns=prob.coarse_unknowns)


def shape_key(prob: Problem):
    """Requests with equal keys can share a launch group: the same level plan, smoother and
    precision (coefficients, maps and right-hand sides may differ) and the same stopping rule."""
    return (prob.dim, tuple(prob.nelem), prob.order, prob.hierarchy, prob.smoother, prob.nu,
            prob.nu_post, prob.quadrature, prob.vcycle_prec, prob.max_levels,
            prob.coarse_unknowns, prob.mode, prob.rtol, prob.maxit)


def request_footprint(prob: Problem) -> int:
    """Device bytes of one request: the library workspace plus f, b and x (FP64)."""
    _, ws = gllmg.plan(request_config(prob))
    return ws + 256 + 3 * 8 * prob.nnodes


@dataclasses.dataclass
class Record:
    rid: int
    name: str
    nnodes: int
    footprint: int
    arrival: float
    admitted: float = float("nan")
    ready: float = float("nan")
    started: float = float("nan")
    finished: float = float("nan")
    iters: int = -1
    grouped: int = 1        # requests in the launch group that solved this one (1: alone)
    converged: bool = False
    relres_true: float = float("nan")
    status: int = -1
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    def __init__(self, hbm_budget: int, max_active: int = 64, nstreams: int = 8,
                 keep_solutions: bool = False, setup_threads: int = 6, host_rhs: bool = False,
                 group_requests: bool = True, group_threads: int = 2,
                 group_window_s: float = 0.002):
        """host_rhs: a request's nodal f is drawn on the host (numpy, the same values as
        Problem.nodal_rhs) and uploaded, instead of drawn on the device. group_requests: solve
        same-shape requests that are ready together as launch groups (group_threads worker
        threads drive them); a ready request whose shape has other requests still in setup
        waits for them up to group_window_s."""
        import torch
        self.host_rhs = host_rhs
        self.ledger = HbmLedger(hbm_budget)
        self.max_active = max_active
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.keep = keep_solutions
        self.solutions: Dict[int, object] = {}
        self.records: Dict[int, Record] = {}
        self._ready: "queue.Queue" = queue.Queue()
        self._todo: "queue.Queue" = queue.Queue()
        self._setup_threads = [threading.Thread(target=self._setup_worker, daemon=True)
                               for _ in range(setup_threads)]
        for t in self._setup_threads:
            t.start()
        self._t0 = 0.0
        self.group_requests = group_requests
        self.group_window_s = group_window_s
        self._groups = concurrent.futures.ThreadPoolExecutor(max_workers=group_threads)
        self._group_streams = [torch.cuda.Stream() for _ in range(group_threads)]

    def now(self) -> float:
        return time.perf_counter() - self._t0

    # ----------------------------------------------------------------- setup thread
    def _setup_worker(self):
        import torch
        s = torch.cuda.Stream()
        while True:
            item = self._todo.get()
            if item is None:
                return
            req, rec = item
            try:
                with torch.cuda.stream(s):
                    P = gllmg.Problem(request_config(req.problem), req.problem.map,
                                      req.problem.mu, stream=s)
                    if self.host_rhs and req.problem.f_seed is not None:
                        f = torch.from_numpy(req.problem.nodal_rhs()).to("cuda")
                    else:
                        f = req.problem.nodal_rhs_device()
                    if f is None:
                        f = P.eval_field(req.problem.f, stream=s)
                    b = P.rhs(f, stream=s)
                    x = torch.zeros_like(b)
                    del f
                s.synchronize()
                rec.ready = self.now()
                self._ready.put((req, rec, P, b, x))
            except Exception as e:  # reported per request; the ledger is released by the loop
                rec.error = str(e)
                self._ready.put((req, rec, None, None, None))

    def _solve_group(self, items, k):
        """One launch group: every request of `items` (same shape) in one gllmg_batch_solve on
        group stream k."""
        import torch
        s = self._group_streams[k % len(self._group_streams)]
        probs = [it[2] for it in items]
        req0 = items[0][0]
        with torch.cuda.stream(s):
            res = gllmg.batch_solve(probs, [it[3] for it in items], [it[4] for it in items],
                                    rtol=req0.problem.rtol, maxit=req0.problem.maxit, stream=s)
        s.synchronize()
        return res

    # ----------------------------------------------------------------- serving loop
    def run(self, trace: List[Request], time_scale: float = 1.0,
            max_wall_s: Optional[float] = None) -> dict:
        """Serve `trace` (arrival times multiplied by time_scale) until every request is done
        or max_wall_s has passed. Returns the report."""
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival_s))
        waiting: collections.deque = collections.deque()
        active = []  # (req, rec, P, b, x, async)
        groups = []  # (items, future)
        in_groups = 0
        ngroup = 0
        held = collections.OrderedDict()  # shape -> ready requests waiting for partners
        held_since = {}
        setup_keys = collections.Counter()  # shapes of the requests in setup
        in_setup = 0
        rr = 0
        self._t0 = time.perf_counter()
        for req in trace:
            self.records[req.rid] = Record(req.rid, req.problem.name, req.problem.nnodes,
                                           request_footprint(req.problem),
                                           req.arrival_s * time_scale)
        while pending or waiting or active or groups or held or in_setup:
            now = self.now()
            if max_wall_s is not None and now > max_wall_s:
                break
            progressed = False
            while pending and pending[0].arrival_s * time_scale <= now:
                waiting.append(pending.popleft())
            # FIFO admission by footprint and slots
            while waiting and len(active) + in_groups + in_setup + sum(map(len, held.values())) < self.max_active:
                req = waiting[0]
                rec = self.records[req.rid]
                if rec.footprint > self.ledger.budget:
                    rec.error = "request larger than the HBM budget"
                    rec.finished = now
                    waiting.popleft()
                    continue
                if not self.ledger.try_reserve(rec.footprint):
                    break
                waiting.popleft()
                rec.admitted = now
                in_setup += 1
                setup_keys[shape_key(req.problem)] += 1
                self._todo.put((req, rec))
                progressed = True
            # hierarchies that finished setting up start solving: same-shape requests ready
            # together as one launch group, the others alone
            while True:
                try:
                    req, rec, P, b, x = self._ready.get_nowait()
                except queue.Empty:
                    break
                in_setup -= 1
                setup_keys[shape_key(req.problem)] -= 1
                progressed = True
                if P is None:
                    rec.finished = self.now()
                    self.ledger.release(rec.footprint)
                    continue
                key = shape_key(req.problem) if self.group_requests and req.problem.mode == "pcg" \
                    else ("alone", req.rid)
                held.setdefault(key, []).append((req, rec, P, b, x))
                held_since.setdefault(key, self.now())
            ready = []
            for key in list(held):
                if setup_keys.get(key, 0) > 0 and self.now() - held_since[key] < self.group_window_s:
                    continue  # partners of this shape are still in setup
                ready.append(held.pop(key))
                del held_since[key]
            for items in ready:
                if len(items) >= 2:
                    t = self.now()
                    for it in items:
                        it[1].started = t
                        it[1].grouped = len(items)
                    groups.append((items, self._groups.submit(self._solve_group, items, ngroup)))
                    ngroup += 1
                    in_groups += len(items)
                    continue
                req, rec, P, b, x = items[0]
                st = self.streams[rr % len(self.streams)]  # setup already synchronized
                rr += 1
                a = P.solve_async(b, x, rtol=req.problem.rtol, maxit=req.problem.maxit, stream=st)
                rec.started = self.now()
                active.append((req, rec, P, b, x, a))
            # launch groups that have finished
            still_g = []
            for items, fut in groups:
                if not fut.done():
                    still_g.append((items, fut))
                    continue
                t = self.now()
                try:
                    results = fut.result()
                    err = ""
                except Exception as e:  # reported per request
                    results, err = [None] * len(items), str(e)
                for (req, rec, P, b, x), res in zip(items, results):
                    rec.finished = t
                    if res is not None:
                        rec.iters, rec.converged = res.iters, res.converged
                        rec.relres_true, rec.status = res.relres_true, res.status
                    else:
                        rec.error = err
                    if self.keep:
                        self.solutions[req.rid] = x.clone()
                    P.close()
                    self.ledger.release(rec.footprint)
                in_groups -= len(items)
                progressed = True
            groups = still_g
            # advance every active solve without blocking
            still = []
            for item in active:
                req, rec, P, b, x, a = item
                if a.poll():
                    res = a.result
                    rec.finished = self.now()
                    rec.iters, rec.converged = res.iters, res.converged
                    rec.relres_true, rec.status = res.relres_true, res.status
                    if self.keep:
                        self.solutions[req.rid] = x.clone()
                    P.close()
                    del b
                    self.ledger.release(rec.footprint)
                    progressed = True
                else:
                    still.append(item)
            active = still
            if not progressed:
                time.sleep(20e-6)
        return self.report()

    def close(self):
        for _ in self._setup_threads:
            self._todo.put(None)
        for t in self._setup_threads:
            t.join(timeout=60)
        self._groups.shutdown(wait=True)

    def report(self) -> dict:
        done = [r for r in self.records.values() if r.converged and np.isfinite(r.finished)]
        failed = [r for r in self.records.values() if r.error or (np.isfinite(r.finished) and not r.converged)]
        lat = np.array([r.latency for r in done]) if done else np.array([np.nan])
        t_first = min((r.arrival for r in self.records.values()), default=0.0)
        t_last = max((r.finished for r in done), default=0.0)
        span = max(t_last - t_first, 1e-9)
        dofs = sum(r.nnodes for r in done)
        return {
            "requests": len(self.records), "completed": len(done), "failed": len(failed),
            "solves_per_s": len(done) / span, "gdof_solves_per_s": dofs / span / 1e9,
            "p50_latency_s": float(np.nanpercentile(lat, 50)),
            "p99_latency_s": float(np.nanpercentile(lat, 99)),
            "mean_admission_wait_s": float(np.nanmean([r.admitted - r.arrival for r in done])) if done else float("nan"),
            "mean_setup_s": float(np.nanmean([r.ready - r.admitted for r in done])) if done else float("nan"),
            "mean_solve_s": float(np.nanmean([r.finished - r.started for r in done])) if done else float("nan"),
            "grouped_requests": sum(1 for r in done if r.grouped > 1),
            "hbm_budget": self.ledger.budget, "hbm_peak_reserved": self.ledger.peak,
            "span_s": span,
        }
