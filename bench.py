"""Benchmark of the adaptive-GSIS kinetic hot path on one MI355X.

One step = one outer aGSIS iteration (Sec. 3.4): relaxation parameters, the
implicit kinetic sweep with fused moments, high-order terms and the
synthetic macroscopic solve, the GSIS correction, the convergence measure and
the local-Kn region update with compaction.  Workload: Mach-5 flow past a
sphere on a seeded ~200k-tetrahedron mesh, 32^3 stretched velocity grid on
[-15, 15]^3, FP32 VDF, FP64 macroscopic side; inputs already resident in HBM
when the timed region starts.

Beside the headline number the same JSON line carries the roofline of the
sweep kernel (HIP events around its launches), the plain FP64 sweep on the
same GPU, and the FP64 CPU oracle timed on a bounded sample of the workload.

Prints one JSON line (see the repository's benchmark contract); progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KN, KN_REF, MACH = 0.005, 0.01, 5.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_sphere32.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--capacity", type=float, default=0.7, help="kinetic capacity as a fraction of the cells")
    ap.add_argument("--ns-chunks", type=int, default=100, help="max chunks of n_inner steps for the NS start")
    ap.add_argument("--n-inner", type=int, default=400)
    ap.add_argument("--nv1d", type=int, default=32)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--region-every", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-sweep", action="store_true")
    ap.add_argument("--no-point-grid", action="store_true", help="skip the non-tensor velocity-grid sweep leg")
    ap.add_argument("--no-order2", action="store_true", help="skip the second-order sweep leg")
    ap.add_argument("--no-poly", action="store_true", help="skip the polyatomic-gas sweep leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="length of the oracle sample")
    ap.add_argument("--sweep-only", action="store_true", help="time kinetic sweeps only (diagnostic)")
    ap.add_argument("--serve-requests", type=int, default=12, help="requests in the serving leg (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate of the serving leg (1/s)")
    ap.add_argument("--serve-max-iter", type=int, default=150)
    ap.add_argument("--serve-tol", type=float, default=1e-4,
                    help="served solves stop at this residual (the explicit synthetic solver converges slowly in "
                         "transitional closed boxes)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain streaming kernel over MIB MiB (scale for HBM counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(nv1d):
    """Mesh, velocity grid and the synthetic starting field (no kinetic cells)."""
    import gsis_inputs as gi
    mesh, grid, W = gi.sphere_workload(nv1d, MACH)
    return mesh, grid, W, np.zeros(mesh["n_cells"], np.uint8)


def sweep_source_hash():
    h = hashlib.sha256()
    for name in ("gsis_sweep.hip", "gsis_impl.hpp"):
        with open(os.path.join(ROOT, "paper_2501_02245_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(n_kin_mean, nv):
    """HBM bytes per sweep launch from the committed counter summary, scaled to
    this launch's kinetic count; None if the kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("source_hash") != sweep_source_hash():
        return None
    return float(t["bytes_per_point"]) * n_kin_mean * nv


def cpu_baseline(mesh, grid, W, flags, seconds):
    """Oracle (FP64, OpenMP) sweep + moments of a chunk of kinetic cells, with
    their kinetic neighbours' rows present, repeated for `seconds`."""
    import gsis_inputs as gi
    import oracle
    O = oracle.Oracle(mesh, grid, KN)
    kin = np.nonzero(flags)[0]
    chunk = kin[: min(64, len(kin))]
    fc = mesh["face_cells"].reshape(-1, 2)
    inchunk = np.zeros(mesh["n_cells"], bool)
    inchunk[chunk] = True
    a_, b_ = fc[:, 0], fc[:, 1]
    touch = (b_ >= 0) & (inchunk[a_] | inchunk[np.maximum(b_, 0)])
    nb = np.union1d(chunk, np.concatenate([a_[touch], b_[touch]]))
    rows = nb[flags[nb] != 0].astype(np.int64)
    slot = -np.ones(mesh["n_cells"], np.int32)
    slot[rows] = np.arange(len(rows), dtype=np.int32)
    f0 = gi.gaussian_rows(grid, W[rows], seed=4, dtype=np.float64)
    ghost = O.ghost_params(W)
    O.sweep(f0, chunk, slot, ghost)       # first touch
    reps, t0 = 0, time.perf_counter()
    while True:
        fn = O.sweep(f0, chunk, slot, ghost)
        O.moments(fn[slot[chunk]])
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    nv = O.nv
    return {"value": reps * len(chunk) * nv / el, "unit": "updates/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "%d x (FP64 oracle sweep + moments of %d kinetic cells of this workload, "
                      "%d velocities, kinetic neighbours' rows present) in %.1f s" % (reps, len(chunk), nv, el)}


def serving(g, n, rate, max_iter, tol, seed=7):
    """Continuous-batching FP32 server on a seeded request stream, against the
    same requests solved one after another by the plain per-case FP64 path."""
    import gsis_inputs as gi
    import paper_2501_02245_amd.serve as sv
    reqs = [sv.Request.from_spec(d) for d in gi.serving_requests(n, rate, seed=seed)]
    budget = 64 << 30
    srv = sv.Server(budget, dtype=g.F32, max_iter=max_iter, tol=tol)
    t = time.perf_counter()
    res = srv.run(reqs, log=log)
    wall = time.perf_counter() - t
    out = sv.summarize(res, wall)
    out.update({"wall_s": wall, "peak_active": srv.peak_active, "peak_bytes": srv.peak_bytes,
                "requeued": srv.requeued, "dtype": "f32", "tol": srv.tol, "max_iter": max_iter,
                "mix": "seed %d: %d requests, Poisson rate %g/s, 1D Couette/Fourier 32-512 cells 16^3/32^3, "
                       "2D cylinder 2k-20k cells 32^2/64^2, Kn log-uniform [1e-3, 1], Mach [1, 8], Kn_ref 0.01"
                       % (seed, n, rate)})
    # the plain per-case FP64 path on the same requests, one at a time
    t = time.perf_counter()
    base, diff = [], []
    for r, rr in zip(reqs, res):
        it, eps, nk, W, status = sv.solve_alone(r, g.F64, max_iter=max_iter, tol=tol)
        base.append(status)
        if status == "ok" and rr.status == "ok":
            scale = np.maximum(np.abs(W).max(axis=0), 1e-3)
            diff.append(float((np.abs(W - rr.W).max(axis=0) / scale).max()))
        log("fp64 alone: request %d %s after %d iterations" % (r.rid, status, it))
    wall64 = time.perf_counter() - t
    n64 = sum(1 for b in base if b == "ok")
    out["fp64_per_case"] = {"solved": n64, "wall_s": wall64, "solves_per_s": n64 / wall64}
    out["speedup_vs_fp64_per_case"] = out["solves_per_s"] / (n64 / wall64) if n64 else None
    out["max_field_diff_vs_fp64"] = max(diff) if diff else None
    return out


def fp64_sweep(g, torch, M, grid, W, flags, steps=3):
    """Plain FP64 sweeps of the initial region on the same GPU."""
    cap = int(flags.sum()) + 64
    case = g.Case(M, grid, KN, dtype=g.F64, capacity=cap)
    case.set_state(W, flags=flags)
    case.sweep(1)
    torch.cuda.synchronize()
    ms = []
    t = time.perf_counter()
    for _ in range(steps):
        case.sweep(1)
        ms.append(case.last_sweep_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    n, nv = case.n_kin, case.nv
    out = {"updates_per_s": steps * n * nv / dt, "kernel_ms": float(np.mean(ms)),
           "achieved_gbs": 16.0 * n * nv / (np.mean(ms) / 1e3) / 1e9, "kinetic_cells": n}
    case.close()
    return out


def point_grid_sweep(g, torch, M, nv1d, W, flags, steps=3):
    """The same region on a non-tensor velocity set: the nv1d^3 stretched grid
    cropped to the ball |xi| <= 15 (a point set with its own weights; one exp
    per node and source, generic kernel), FP32 sweeps on the same GPU."""
    import gsis_inputs as gi
    grid = gi.ball_grid(nv1d, 15.0, "stretched")
    cap = int(flags.sum()) + 64
    case = g.Case(M, grid, KN, dtype=g.F32, capacity=cap)
    case.set_state(W, flags=flags)
    case.sweep(1)
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        case.sweep(1)
        ms.append(case.last_sweep_ms())
    torch.cuda.synchronize()
    n, nv = case.n_kin, case.nv
    kms = float(np.mean(ms))
    out = {"velocities": nv, "of_tensor": nv1d ** 3, "kinetic_cells": n, "kernel_ms": kms,
           "updates_per_s": n * nv / (kms / 1e3), "achieved_gbs": 8.0 * n * nv / (kms / 1e3) / 1e9}
    case.close()
    return out


def order2_sweep(g, torch, M, grid, W, flags, dim, steps=3):
    """Second-order face values on the same region and tensor grid (FP32):
    per sweep the slope kernel and the row sweep with the deferred correction.
    Algorithmic bytes per cell-velocity, counted for a slope of dim components:
    slope kernel 4 (read f) + 4 dim (write), sweep 4 (read f) + 4 dim (own
    slope) + 4 (write f); the library stores one increment per face instead."""
    cap = int(flags.sum()) + 64
    case = g.Case(M, grid, KN, dtype=g.F32, capacity=cap, order=2)
    case.set_state(W, flags=flags)
    case.sweep(1)
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        case.sweep(1)
        ms.append(case.last_sweep_ms())
    torch.cuda.synchronize()
    n, nv = case.n_kin, case.nv
    kms = float(np.mean(ms))
    bpp = 4.0 * (1 + dim) + 4.0 * (2 + dim)
    out = {"kinetic_cells": n, "velocities": nv, "slope_plus_sweep_ms": kms,
           "updates_per_s": n * nv / (kms / 1e3), "bytes_per_update": bpp,
           "achieved_gbs": bpp * n * nv / (kms / 1e3) / 1e9,
           "frac": bpp * n * nv / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, "damp2": 2.0}
    case.close()
    return out


def poly_sweep(g, torch, M, grid, W, flags, steps=3):
    """The polyatomic gas (two VDFs, nitrogen parameters: d_r 2, Z_r 2.667,
    omega 0.74, the A matrix of the thermal relaxation rates) on the same
    region and grid, FP32: sweeps of (f0, f1) with per-node Gaussians at T_t
    and T.  Algorithmic bytes per cell-velocity: 2 x (4 read + 4 write)."""
    cap = int(flags.sum()) + 64
    case = g.Case(M, grid, KN, omega=0.74, Pr=0.786, dtype=g.F32, capacity=cap,
                  dr=2.0, Zr=2.667, A=(0.786, -0.201, -0.059, 0.842))
    case.set_state(W, flags=flags)
    case.sweep(1)
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        case.sweep(1)
        ms.append(case.last_sweep_ms())
    torch.cuda.synchronize()
    n, nv = case.n_kin, case.nv
    kms = float(np.mean(ms))
    out = {"kinetic_cells": n, "velocities": nv, "kernel_ms": kms, "updates_per_s": n * nv / (kms / 1e3),
           "bytes_per_update": 16.0, "achieved_gbs": 16.0 * n * nv / (kms / 1e3) / 1e9,
           "frac": 16.0 * n * nv / (kms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "gas": "N2: d_r 2, Z_r 2.667, omega 0.74, A (0.786, -0.201, -0.059, 0.842)"}
    case.close()
    return out


def surface_leg(g, torch, case, mesh, es):
    """Surface quantities on the sphere (stress, pressure, heat flux per wall face,
    force and heat totals) at the state after the timed steps: kernel time over
    3 calls, the bytes of the kinetic wall rows it reads, and the coefficients
    (reference area: the sphere's cross-section)."""
    faces, out, tot = case.surface()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        faces, out, tot = case.surface()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    _, fl = case.get_state()
    fl = fl.cpu().numpy()
    f = faces.cpu().numpy()
    kin_walls = int(fl[mesh["face_cells"][f, 0]].sum())
    u_inf = mesh["patches"][[p["kind"] for p in mesh["patches"]].index("far")]["u"]
    coef = g.force_coefficients(tot.cpu().numpy(), 1.0, u_inf, np.pi / 4)
    return {"ms": ms, "wall_faces": int(len(f)), "kinetic_wall_faces": kin_walls,
            "read_gbs": kin_walls * case.nv * es / (ms / 1e3) / 1e9, **coef,
            "state": "after the timed steps (not converged)"}


def synthetic_leg(torch, case, mesh, n_inner, reps=2):
    """The synthetic macroscopic solve alone (eq. macro, FP64): n_inner
    pseudo-time steps over every cell from the state after the timed steps,
    zero HoT and source, local steps (cfl 0.5).  Timed with events on the
    stream the library launches on; one untimed solve first."""
    Wd, _ = case.get_state()
    n = mesh["n_cells"]
    hot = torch.zeros((n, 9), dtype=torch.float64, device="cuda")
    Ws = [Wd.clone() for _ in range(reps + 1)]
    case.macro_solve(Ws[0], hot, None, n_inner, 0.5)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        case.macro_solve(Ws[1 + r], hot, None, n_inner, 0.5)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"cells": n, "faces": int(len(mesh["face_cells"])), "inner_steps": n_inner, "ms": ms,
            "us_per_inner_step": 1e3 * ms / n_inner, "cell_steps_per_s": n * n_inner / (ms / 1e3)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2501_02245_amd as g

    t0 = time.time()
    mesh, grid, W, flags = workload(a.nv1d)
    n_cells = mesh["n_cells"]
    dtype = g.F32 if a.dtype == "f32" else g.F64
    cap = min(n_cells, int(a.capacity * n_cells))
    M = g.Mesh(mesh)
    case = g.Case(M, grid, KN, dtype=dtype, capacity=cap)
    case.set_state(W, flags=flags)
    params = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, tol=1e-12, n_macro_inner=a.n_inner, cfl=0.5,
                           region_update_every=a.region_every, force_wall_layers=2)
    # Steps 1-2 of Sec. 3.4 (untimed): NS solve to eps < 1e-6, first flagging, Grad-13 rows
    init = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, tol=1e-6, max_iter=0, n_macro_inner=a.n_inner,
                         cfl=0.5, force_wall_layers=2, ns_init=1, ns_init_max_chunks=a.ns_chunks)
    case.solve(init)
    Wd, fd = case.get_state()
    W, flags = Wd.cpu().numpy(), fd.cpu().numpy()
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    nv = case.nv
    log("setup %.1f s: %d cells, %d kinetic after the NS start, capacity %d, %d velocities, layout %s"
        % (setup_s, n_cells, case.n_kin, cap, nv, case.sweep_layout()))

    def one():
        if a.sweep_only:
            case.sweep(1)
            return None
        return case.step(params)

    for i in range(a.warmup):
        e = one()
        log("warmup %d n_kin %d eps %s" % (i, case.n_kin, e))
    torch.cuda.synchronize()
    kin_counts, sweep_ms = [], []
    t = time.perf_counter()
    for i in range(a.steps):
        kin_counts.append(case.n_kin)
        e = one()
        sweep_ms.append(case.last_sweep_ms())
        log("step %d n_kin %d sweep %.3f ms eps %s" % (i, kin_counts[-1], sweep_ms[-1], e))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    updates = float(sum(kin_counts)) * nv
    es = 4 if dtype == g.F32 else 8
    sweep_s = float(np.mean(sweep_ms)) / 1e3
    n_kin_mean = float(np.mean(kin_counts))
    alg_bytes = 2 * es * n_kin_mean * nv          # read f^n, write f^{n+1/2}
    achieved = alg_bytes / sweep_s / 1e9
    traffic = measured_traffic(n_kin_mean, nv) if dtype == g.F32 else None
    surface = surface_leg(g, torch, case, mesh, es)
    log("surface", surface)
    synthetic = None if a.sweep_only else synthetic_leg(torch, case, mesh, a.n_inner)
    log("synthetic solve", synthetic)
    case.close()

    if a.calibrate_copy > 0:
        # plain streaming kernel of known traffic: reads and writes MIB MiB each
        n = a.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 2.0, out=y)
        torch.cuda.synchronize()
        del x, y

    fp64 = None
    if not a.no_fp64_sweep and dtype == g.F32:
        fp64 = fp64_sweep(g, torch, M, grid, W, flags)
        log("fp64 sweep", fp64)
    points = None
    if not a.no_point_grid and not a.sweep_only:
        points = point_grid_sweep(g, torch, M, a.nv1d, W, flags)
        log("point-grid sweep", points)
    order2 = None
    if not a.no_order2 and not a.sweep_only and dtype == g.F32:
        order2 = order2_sweep(g, torch, M, grid, W, flags, mesh["dim"])
        log("second-order sweep", order2)
    poly = None
    if not a.no_poly and not a.sweep_only and dtype == g.F32:
        poly = poly_sweep(g, torch, M, grid, W, flags)
        log("polyatomic sweep", poly)

    out = {
        "metric": "kinetic cell-velocity updates/s",
        "value": updates / dt,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == g.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": "3D Mach-5 sphere, %d tetrahedra, %d^3 stretched velocities on [-15,15]^3, "
                               "aGSIS Kn=%g Kn_ref=%g" % (n_cells, a.nv1d, KN, KN_REF),
                   "kinetic_cells_mean": n_kin_mean, "kinetic_fraction": n_kin_mean / n_cells,
                   "start": "NS solve to eps<1e-6, then Kn_Gll flagging", "n_macro_inner": a.n_inner,
                   "sweep_only": bool(a.sweep_only)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_sweep_fast",
                     "kernel_ms": 1e3 * sweep_s},
        "sweep_updates_per_s": n_kin_mean * nv / sweep_s,
        "fp64_sweep": fp64,
        "point_grid_sweep": points,
        "order2_sweep": order2,
        "poly_sweep": poly,
        "surface": surface,
        "synthetic_solve": synthetic,
        "setup_s": setup_s,
    }
    if a.serve_requests > 0 and not a.sweep_only:
        t1 = time.time()
        out["serving"] = serving(g, a.serve_requests, a.serve_rate, a.serve_max_iter, a.serve_tol)
        log("serving leg %.1f s" % (time.time() - t1))
    if not a.no_cpu_baseline:
        t1 = time.time()
        out["cpu_baseline"] = cpu_baseline(mesh, grid, W, flags, a.cpu_seconds)
        log("cpu baseline %.1f s" % (time.time() - t1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
