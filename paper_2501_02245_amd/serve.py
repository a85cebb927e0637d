"""Continuous-batching request loop for steady aGSIS solves on one GPU.

Requests (a mesh, a velocity grid, Kn and a starting field) arrive over time.
A request is admitted when its device footprint fits the memory budget next to
the cases already resident; its workspace, VDF and macroscopic state then stay
on the device until it converges.  Every tick advances all resident cases by
one outer iteration (Sec. 3.4): cases whose launches are compatible (same
precision, velocity dimension, sweep layout and forced wall layers) share one
batched kinetic-sweep launch and one batched launch per synthetic pseudo-time
step, so their work overlaps on the device.  Converged cases leave at once,
which frees memory for the queue.  Results do not depend on the mix: every
kernel computes each case's values exactly as when it runs alone.
"""
from __future__ import annotations

import dataclasses
import time
from collections import defaultdict, deque

import numpy as np

from . import (E_CAPACITY, F32, MODE_AGSIS, MODE_GSIS, Case, GsisError, Mesh, SolveParams, footprint, ns_init,
               step)


BATCH = 64   # cases per gsis_step call: the library's largest batched launch


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float               # seconds after the start of the run
    mesh: dict                   # gsis_inputs mesh dictionary
    grid: dict                   # velocity grid
    Kn: float
    W0: np.ndarray               # starting field [n_cells, 5]
    layers: int = 0              # forced kinetic wall layers
    capacity: float = 1.0        # kinetic capacity as a fraction of the cells
    kind: str = ""
    mode: str = "agsis"          # "agsis": NS start, then adaptive steps; "gsis": every cell kinetic
    cfl: float = 0.5             # synthetic pseudo-time step (< 0: one global step)
    fields: tuple = (0, 1, 2)    # residuals (rho, u, T) that must fall below tol
    solo: bool = False           # run the NS start alone (after a failed batched start)

    @classmethod
    def from_spec(cls, d):
        """From a gsis_inputs.serving_requests entry; flows with no mean velocity
        (stationary walls) converge on rho and T only."""
        still = d["kind"] == "fourier"
        return cls(d["rid"], d["arrival"], d["mesh"], d["grid"], d["Kn"], d["W0"], d["layers"], d["capacity"],
                   d["kind"], d["mode"], d["cfl"], (0, 2) if still else (0, 1, 2))


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    admitted: float
    finished: float
    iterations: int
    eps: np.ndarray
    n_kinetic: int
    status: str                  # "ok", "noconv" or the error text
    W: np.ndarray | None = None

    @property
    def latency(self):
        return self.finished - self.arrival


class _Active:
    def __init__(self, req, case, fp, t_admit):
        self.req, self.case, self.fp, self.t_admit = req, case, fp, t_admit
        self.it = 0
        self.eps = np.full(3, np.inf)

    def key(self):
        c, r = self.case, self.req
        return (c.dtype, c.vdim, c.points, c.sweep_layout()[0], r.mode, r.cfl, r.layers)


class Server:
    """FIFO admission by footprint, one batched outer iteration per tick."""

    def __init__(self, budget_bytes, dtype=F32, Kn_ref=0.01, tol=1e-6, max_iter=400, n_inner=400,
                 ns_chunks=50, max_active=256, keep_fields=True, min_iter=5, step_graphs=False, source_half=False):
        self.budget = int(budget_bytes)
        # replay each group's outer iteration from a HIP graph between region
        # updates (GSIS_STEP_GRAPHS; results are bitwise those of eager launches)
        self.step_graphs = step_graphs
        # source of the synthetic equations at the half step (f^{n+1/2},
        # W^{n+1/2}) rather than at f^n, W^n: same fixed point, fewer iterations
        self.source_half = int(bool(source_half))
        self.min_iter = min_iter     # a first small change is not convergence
        self.dtype, self.Kn_ref, self.tol, self.max_iter = dtype, Kn_ref, tol, max_iter
        self.n_inner, self.ns_chunks = n_inner, ns_chunks
        self.max_active, self.keep_fields = max_active, keep_fields
        self.peak_active = 0
        self.peak_bytes = 0
        self.requeued = 0

    def _params(self, mode, cfl, layers, **kw):
        return params_for(mode, cfl, layers, self.Kn_ref, self.tol, self.n_inner, **kw)

    def _bind(self, r, fp, t0):
        """Bind the case and set W0; aGSIS cases start every cell NS (Step 1 follows)."""
        M = Mesh(r.mesh)
        cap = max(1, int(round(r.capacity * M.n_cells)))
        case = Case(M, r.grid, r.Kn, dtype=self.dtype, capacity=cap)
        if r.mode == "agsis":
            case.set_state(r.W0, flags=np.zeros(M.n_cells, np.uint8))
        else:
            case.set_state(r.W0)
        return _Active(r, case, fp, time.perf_counter() - t0)

    def _ns_starts(self, fresh):
        """Steps 1-2 for newly bound aGSIS cases, batched by launch compatibility;
        returns [(active, outcome)]: None (started), "grow" (its region outgrew
        the reservation in a batched start), "retry" (the batched start failed:
        restart alone), or the error of a start run alone."""
        out = []
        groups = defaultdict(list)
        for k, a in enumerate(fresh):
            if a.req.mode == "agsis":
                groups[(a.case.dtype, a.req.cfl, a.req.layers, k if a.req.solo else -1)].append(a)
            else:
                out.append((a, None))
        for (_, cfl, layers, _), grp in groups.items():
            p = self._params("agsis", cfl, layers, max_iter=0, ns_init=1, ns_init_max_chunks=self.ns_chunks)
            try:
                ns_init([a.case for a in grp], p)
                out += [(a, None) for a in grp]
            except GsisError as e:
                ch = getattr(e, "chunks", None)
                if len(grp) > 1 and ch is not None and min(ch) < 0 and e.code == E_CAPACITY:
                    # the cases whose first flagging failed restart with a larger
                    # reservation (alone if they hold the whole mesh); the rest started
                    out += [(a, None if c >= 0 else "grow") for a, c in zip(grp, ch)]
                else:
                    out += [(a, "retry" if len(grp) > 1 else e) for a in grp]
        return out

    def _retire(self, a, status, t0):
        W = a.case.get_state()[0].cpu().numpy() if (self.keep_fields and status in ("ok", "noconv")) else None
        res = Result(a.req.rid, a.req.kind, a.req.arrival, a.t_admit, time.perf_counter() - t0, a.it,
                     a.eps.copy(), a.case.n_kin, status, W)
        a.case.close()
        a.case.mesh.close()
        return res

    def run(self, requests, log=None):
        import os
        old = os.environ.get("GSIS_STEP_GRAPHS")
        os.environ["GSIS_STEP_GRAPHS"] = "1" if self.step_graphs else "0"
        try:
            return self._run(requests, log)
        finally:
            if old is None:
                os.environ.pop("GSIS_STEP_GRAPHS", None)
            else:
                os.environ["GSIS_STEP_GRAPHS"] = old

    def _run(self, requests, log=None):
        import torch
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue, active, results = deque(), [], []
        used = 0
        t0 = time.perf_counter()
        while pending or queue or active:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            # admission: FIFO while the head fits; the new aGSIS cases then run
            # their NS starts together
            fresh = []
            while queue and len(active) + len(fresh) < self.max_active:
                r = queue[0]
                M = Mesh(r.mesh)
                cap = max(1, int(round(r.capacity * M.n_cells)))
                fp = footprint(M, r.grid, r.Kn, self.dtype, cap)
                M.close()
                if used + fp > self.budget:
                    if not active and not fresh:
                        queue.popleft()
                        results.append(Result(r.rid, r.kind, r.arrival, now, now, 0, np.full(3, np.inf), 0,
                                              "rejected: footprint %d B > budget" % fp))
                        continue
                    break
                queue.popleft()
                try:
                    fresh.append(self._bind(r, fp, t0))
                except GsisError as e:
                    results.append(Result(r.rid, r.kind, r.arrival, now, time.perf_counter() - t0, 0,
                                          np.full(3, np.inf), 0, "error: %s" % e))
                    continue
                used += fp
            for a, err in self._ns_starts(fresh):
                if err is None:
                    active.append(a)
                    continue
                used -= a.fp
                a.case.close()
                a.case.mesh.close()
                r = a.req
                if err == "grow" and r.capacity < 1.0:
                    queue.appendleft(dataclasses.replace(r, capacity=min(1.0, 2.0 * r.capacity)))
                    self.requeued += 1
                elif err in ("retry", "grow"):
                    queue.appendleft(dataclasses.replace(r, solo=True))
                    self.requeued += 1
                elif err.code == E_CAPACITY and r.capacity < 1.0:
                    # region larger than the reservation: retry with twice the reservation
                    queue.appendleft(dataclasses.replace(r, capacity=min(1.0, 2.0 * r.capacity)))
                    self.requeued += 1
                else:
                    results.append(Result(r.rid, r.kind, r.arrival, a.t_admit, time.perf_counter() - t0, 0,
                                          np.full(3, np.inf), 0, "error: %s" % err))
            self.peak_active = max(self.peak_active, len(active))
            self.peak_bytes = max(self.peak_bytes, used)
            if not active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                continue
            # one outer iteration for every resident case, batched by launch compatibility
            groups = defaultdict(list)
            for a in active:
                groups[a.key()].append(a)
            done = []
            for key, grp in groups.items():
                # a batch lists the case with the largest velocity axes first
                grp.sort(key=lambda a: -a.case.nv)
                for j0 in range(0, len(grp), BATCH):
                    part = grp[j0:j0 + BATCH]
                    try:
                        eps = step([a.case for a in part],
                                   self._params(key[4], key[5], key[6], source_half=self.source_half))
                        err = None
                    except GsisError as e:
                        eps, err = e.eps, e
                    for a, e in zip(part, eps):
                        a.it += 1
                        if np.isnan(e).any():
                            # a region that outgrew its reservation restarts with twice the reservation
                            requeue = err.code == E_CAPACITY and a.req.capacity < 1.0
                            done.append((a, "requeue" if requeue else "error: %s" % err))
                            continue
                        a.eps = e
                        if a.it >= self.min_iter and np.max(e[list(a.req.fields)]) < self.tol:
                            done.append((a, "ok"))
                        elif a.it >= self.max_iter:
                            done.append((a, "noconv"))
            for a, status in done:
                active.remove(a)
                used -= a.fp
                if status == "requeue":
                    a.case.close()
                    a.case.mesh.close()
                    queue.appendleft(dataclasses.replace(a.req, capacity=min(1.0, 2.0 * a.req.capacity)))
                    self.requeued += 1
                    continue
                results.append(self._retire(a, status, t0))
                if log:
                    log("request %d (%s) %s after %d iterations, %.3f s, eps %s" % (
                        a.req.rid, a.req.kind, status, a.it, results[-1].latency,
                        " ".join("%.2e" % x for x in a.eps)))
        torch.cuda.synchronize()
        return sorted(results, key=lambda r: r.rid)


def params_for(mode, cfl, layers, Kn_ref=0.01, tol=1e-6, n_inner=400, **kw):
    return SolveParams(mode=MODE_AGSIS if mode == "agsis" else MODE_GSIS, Kn_ref=Kn_ref, tol=tol,
                       n_macro_inner=n_inner, cfl=cfl, region_update_every=-5, force_wall_layers=layers, **kw)


def start_case(r: Request, dtype, Kn_ref=0.01, tol=1e-6, n_inner=400, ns_chunks=50):
    """Bind a case for the request and set its start: aGSIS requests run Steps
    1-2 of Sec. 3.4 (NS start, first flagging); GSIS requests start kinetic
    everywhere from the conservation-fixed Maxwellian of W0."""
    M = Mesh(r.mesh)
    cap = max(1, int(round(r.capacity * M.n_cells)))
    case = Case(M, r.grid, r.Kn, dtype=dtype, capacity=cap)
    try:
        if r.mode == "agsis":
            case.set_state(r.W0, flags=np.zeros(M.n_cells, np.uint8))
            case.solve(params_for(r.mode, r.cfl, r.layers, Kn_ref, tol, n_inner, max_iter=0, ns_init=1,
                                  ns_init_max_chunks=ns_chunks))
        else:
            case.set_state(r.W0)
    except GsisError:
        case.close()
        M.close()
        raise
    return case


def solve_alone(r: Request, dtype, Kn_ref=0.01, tol=1e-6, max_iter=400, n_inner=400, ns_chunks=50, min_iter=5,
                source_half=False):
    """One request on its own, with the same steps, stopping rule and
    reservation doubling as the server."""
    while True:
        try:
            case = start_case(r, dtype, Kn_ref, tol, n_inner, ns_chunks)
        except GsisError as e:
            if e.code == E_CAPACITY and r.capacity < 1.0:
                r = dataclasses.replace(r, capacity=min(1.0, 2.0 * r.capacity))
                continue
            return 0, np.full(3, np.inf), 0, None, "error: %s" % e
        p = params_for(r.mode, r.cfl, r.layers, Kn_ref, tol, n_inner, source_half=int(bool(source_half)))
        it, eps, status = 0, np.full(3, np.inf), "noconv"
        try:
            while it < max_iter:
                eps = case.step(p)
                it += 1
                if it >= min_iter and np.max(eps[list(r.fields)]) < tol:
                    status = "ok"
                    break
        except GsisError as e:
            if e.code == E_CAPACITY and r.capacity < 1.0:
                case.close()
                case.mesh.close()
                r = dataclasses.replace(r, capacity=min(1.0, 2.0 * r.capacity))
                continue
            status = "error: %s" % e
        W = case.get_state()[0].cpu().numpy() if status in ("ok", "noconv") else None
        nk = case.n_kin
        case.close()
        case.mesh.close()
        return it, eps, nk, W, status


def summarize(results, wall_s):
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    return {"requests": len(results), "solved": len(ok), "solves_per_s": len(ok) / wall_s if wall_s > 0 else 0.0,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "failed": [(r.rid, r.status) for r in results if r.status != "ok"]}
