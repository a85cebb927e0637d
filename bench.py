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
    ap.add_argument("--no-poly", action="store_true", help="skip the polyatomic-gas (nitrogen) aGSIS leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the Couette, cavity and cylinder legs")
    ap.add_argument("--poly-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="length of the oracle sample")
    ap.add_argument("--sweep-only", action="store_true", help="time kinetic sweeps only (diagnostic)")
    ap.add_argument("--serve-requests", type=int, default=170,
                    help="requests per arrival rate (0: skip serving); 170 give about 55 solved per rate for the p99")
    ap.add_argument("--serve-rates", default="5,20,80", help="Poisson arrival rates of the serving leg (1/s)")
    ap.add_argument("--serve-max-iter", type=int, default=300)
    ap.add_argument("--serve-tol", type=float, default=1e-6, help="served solves stop at this residual (Sec. 4)")
    ap.add_argument("--serve-source-half", type=int, default=1, choices=[0, 1],
                    help="served solves take the synthetic source at the half step (0: at f^n, W^n)")
    ap.add_argument("--serve-fp64-check", type=int, default=12,
                    help="requests of the middle rate also solved alone by the FP64 per-case path")
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


def sweep_kernel_name():
    """The plane sweep kernel the library launches for this workload's 32^3
    tensor grid: 16-byte rows (k_sweep_v4) unless GSIS_SWEEP_V4=0."""
    return "k_sweep_fast" if os.environ.get("GSIS_SWEEP_V4", "1") == "0" else "k_sweep_v4"


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


def cpu_model():
    """The host CPU's model name and logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def _oracle_sample(O, mesh, grid, W, flags, n_cells, seconds):
    """Repeated oracle sweeps + moments of the first n_cells kinetic cells
    (their kinetic neighbours' rows present) for `seconds`: (updates/s, text)."""
    import gsis_inputs as gi
    kin = np.nonzero(flags)[0]
    chunk = kin[: min(n_cells, len(kin))]
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
    return reps * len(chunk) * O.nv / el, "%d x (sweep + moments of %d cells) in %.1f s" % (reps, len(chunk), el)


def _oracle_sweep_ms(O, f, n):
    """Median of 3 oracle sweeps of every cell (all kinetic), ms."""
    kin = np.arange(n, dtype=np.int32)
    ts = []
    for _ in range(3):
        t = time.perf_counter()
        O.sweep(f, kin, kin)
        ts.append(time.perf_counter() - t)
    return 1e3 * float(np.median(ts))


def cpu_baseline(mesh, grid, W, flags, seconds):
    """The oracle (FP64, OpenMP) on this host: a bounded sample of the sphere
    workload with every thread and with one, one oracle sweep of C1 and C2
    (every cell kinetic), and the time of a C1 GSIS outer iteration."""
    import gsis_inputs as gi
    import oracle
    model, ncpu = cpu_model()
    O = oracle.Oracle(mesh, grid, KN)
    nt = oracle.threads()
    v, txt = _oracle_sample(O, mesh, grid, W, flags, 256, seconds)
    oracle.set_threads(1)
    v1, txt1 = _oracle_sample(O, mesh, grid, W, flags, 16, max(2.0, seconds / 4))
    oracle.set_threads(nt)
    out = {"value": v, "unit": "updates/s", "cores": nt, "kind": "oracle",
           "sample": "FP64 oracle on the sphere workload (%d velocities, the kinetic region after the NS "
                     "start): %s" % (O.nv, txt),
           "cpu_model": model, "logical_cpus": ncpu,
           "one_core": {"value": v1, "unit": "updates/s", "sample": txt1}}
    # C1 and C2: one sweep of every cell
    m1 = gi.couette_1d(64, 0.1)
    g1 = gi.velocity_grid(3, 16, 5.0)
    O1 = oracle.Oracle(m1, g1, 0.1)
    W1 = gi.couette_initial_W(64, seed=0)
    f1 = np.stack([O1.feq(w) for w in W1])
    ms1 = _oracle_sweep_ms(O1, f1, 64)
    m2 = gi.quad_cavity_2d(64, 64, 0.1)
    g2 = gi.velocity_grid(2, 32, 6.0, "stretched")
    O2 = oracle.Oracle(m2, g2, 0.1)
    f2 = gi.gaussian_rows(g2, gi.uniform_W(m2["n_cells"]), seed=4, dtype=np.float64)
    ms2 = _oracle_sweep_ms(O2, f2, m2["n_cells"])
    S = oracle.SteadySolver(O1, mode="gsis", n_inner=400, cfl=0.5)
    S.set_state(W1)
    t = time.perf_counter()
    for _ in range(10):
        S.step()
    c1 = (time.perf_counter() - t) / 10
    out["configs"] = {"C1_sweep_ms": ms1, "C1_updates_per_s": 64 * O1.nv / (ms1 / 1e3),
                      "C2_sweep_ms": ms2, "C2_updates_per_s": m2["n_cells"] * O2.nv / (ms2 / 1e3),
                      "C1_gsis_ms_per_iteration": 1e3 * c1,
                      "note": "C1 GSIS: 10 oracle iterations timed (the GPU leg gives the iterations to 1e-8); "
                              "full C2-C4 solves are not timed on the CPU (minutes to hours)"}
    return out


def serving(g, n, rates, max_iter, tol, n_check, source_half, seed=7):
    """Continuous-batching FP32 server on seeded request streams, one per
    Poisson arrival rate (the same seed: the same requests, arriving faster),
    and `n_check` requests of the middle rate solved one after another by the
    plain per-case FP64 path (the same steps and stopping rule)."""
    import gsis_inputs as gi
    import paper_2501_02245_amd.serve as sv
    out = {"dtype": "f32", "tol": tol, "max_iter": max_iter,
           "synthetic_source": "half step (f^{n+1/2}, W^{n+1/2})" if source_half else "f^n, W^n",
           "mix": "seed %d: %d requests per rate, 1D Couette/Fourier 32-512 cells 16^3/32^3 (GSIS), 2D cylinder "
                  "2k-20k cells 32^2/64^2 (aGSIS from the NS start), Kn log-uniform [1e-3, 1], Mach [1, 8], "
                  "Kn_ref 0.01" % (seed, n), "rates": []}
    mid = sorted(rates)[len(rates) // 2]
    for rate in rates:
        reqs = [sv.Request.from_spec(d) for d in gi.serving_requests(n, rate, seed=seed)]
        srv = sv.Server(64 << 30, dtype=g.F32, max_iter=max_iter, tol=tol, source_half=source_half)
        t = time.perf_counter()
        res = srv.run(reqs, log=log)
        wall = time.perf_counter() - t
        r = sv.summarize(res, wall)
        r.update({"rate_per_s": rate, "wall_s": wall, "peak_active": srv.peak_active,
                  "peak_bytes": srv.peak_bytes, "requeued": srv.requeued})
        log("serving rate %g: %d of %d solved in %.1f s, p50 %.3f s p99 %.3f s" % (
            rate, r["solved"], r["requests"], wall, r["p50_s"], r["p99_s"]))
        if rate == mid and n_check > 0:
            t = time.perf_counter()
            n64, diff = 0, []
            for q, rr in list(zip(reqs, res))[:n_check]:
                it, eps, nk, W, status = sv.solve_alone(q, g.F64, max_iter=max_iter, tol=tol, source_half=source_half)
                if status == "ok":
                    n64 += 1
                if status == "ok" and rr.status == "ok":
                    # per field, relative to its largest value; u (a vector) to
                    # max(|u|, 0.1), since the boxes' flows are nearly at rest
                    d = np.abs(W - rr.W)
                    diff.append(max(d[:, 0].max() / np.abs(W[:, 0]).max(),
                                    d[:, 1:4].max() / max(np.abs(W[:, 1:4]).max(), 0.1),
                                    d[:, 4].max() / np.abs(W[:, 4]).max()))
                    log("served vs fp64: request %d (%s) %.2e" % (q.rid, q.kind, diff[-1]))
                log("fp64 alone: request %d %s after %d iterations" % (q.rid, status, it))
            wall64 = time.perf_counter() - t
            r["fp64_per_case"] = {"requests": n_check, "solved": n64, "wall_s": wall64,
                                  "solves_per_s": n64 / wall64 if wall64 > 0 else 0.0}
            r["served_fields_vs_fp64_max"] = max(diff) if diff else None
            r["served_fields_vs_fp64_compared"] = len(diff)
        out["rates"].append(r)
    return out


def stream_rate(torch, mib=1024, reps=5):
    """A plain streaming kernel on this GPU (torch mul: reads and writes `mib`
    MiB each), timed with events on its stream; the best of `reps`, in GB/s.
    It is the attainable HBM rate the sweep's bytes are set against, beside
    the published peak."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(reps):
        e0.record()
        torch.mul(x, 2.0, out=y)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    torch.cuda.synchronize()
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


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


def _timed_steps(torch, case, params, steps, warmup=1):
    """warmup + timed outer iterations; returns (ms per step, mean sweep ms,
    mean kinetic cells, last eps)."""
    for _ in range(warmup):
        case.step(params)
    torch.cuda.synchronize()
    kin, sw = [], []
    e = None
    t = time.perf_counter()
    for _ in range(steps):
        kin.append(case.n_kin)
        e = case.step(params)
        sw.append(case.last_sweep_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    return 1e3 * dt / steps, float(np.mean(sw)), float(np.mean(kin)), e


def c1_couette(g, torch):
    """C1: 1D planar Couette (64 cells on [0,1], walls at T 1 moving -+0.1,
    16^3 uniform velocities on [-5,5], Kn 0.1, hard spheres, density
    perturbation 1e-3 N(0,1) from seed 0), FP64, full-kinetic: the plain
    iteration (DVM) and GSIS, each to eps < 1e-8."""
    import gsis_inputs as gi
    m = gi.couette_1d(64, 0.1)
    grid = gi.velocity_grid(3, 16, 5.0)
    W = gi.couette_initial_W(64, seed=0)
    out = {}
    for name, mode in (("dvm", g.MODE_DVM), ("gsis", g.MODE_GSIS)):
        case = g.Case(g.Mesh(m), grid, 0.1, dtype=g.F64)
        case.set_state(W)
        p = g.SolveParams(mode=mode, tol=1e-8, max_iter=20000, n_macro_inner=400, cfl=0.5)
        torch.cuda.synchronize()
        t = time.perf_counter()
        it, eps, _ = case.solve(p, allow_noconv=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        sweep_ms = case.last_sweep_ms()
        out[name] = {"iterations": int(it), "eps": [float(x) for x in eps], "converged": bool(max(eps) < 1e-8),
                     "solve_s": dt, "ms_per_iteration": 1e3 * dt / max(it, 1), "sweep_ms": sweep_ms,
                     "sweep_updates_per_s": 64 * case.nv / (sweep_ms / 1e3)}
        case.close()
    return out


def c2_cavity(g, torch):
    """C2: lid-driven cavity (64x64 quads as an unstructured mesh, lid +0.1,
    walls at T 1), reduced 2D distributions on a 32^2 stretched grid on
    [-6,6]^2, uniform start, FP32, full-kinetic GSIS at Kn 0.01, 0.1 and 1:
    per-sweep time (the plane kernel) and time per GSIS outer iteration."""
    import gsis_inputs as gi
    m = gi.quad_cavity_2d(64, 64, 0.1)
    grid = gi.velocity_grid(2, 32, 6.0, "stretched")
    W = gi.uniform_W(m["n_cells"])
    M = g.Mesh(m)
    out = {}
    for Kn in (0.01, 0.1, 1.0):
        case = g.Case(M, grid, Kn, dtype=g.F32)
        case.set_state(W)
        case.sweep(1)
        ms = []
        for _ in range(5):
            case.sweep(1)
            ms.append(case.last_sweep_ms())
        case.set_state(W)
        p = g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=400, cfl=0.5)
        step_ms, _, nk, e = _timed_steps(torch, case, p, 5)
        kms = float(np.median(ms))
        pts = nk * case.nv * 2
        out["Kn=%g" % Kn] = {"sweep_ms": kms, "sweep_updates_per_s": nk * case.nv / (kms / 1e3),
                             "achieved_gbs": 8.0 * pts / (kms / 1e3) / 1e9, "ms_per_gsis_iteration": step_ms,
                             "eps_after_6": [float(x) for x in e], "layout": list(case.sweep_layout())}
        case.close()
    return out


def c3_cylinder(g, torch, steps=5):
    """C3: Mach-5 flow past a unit cylinder (seeded Delaunay, ~20k
    triangles), reduced 2D distributions on a 64^2 stretched grid on
    [-15,15]^2, Kn 0.01, aGSIS with Kn_ref 0.01 and two forced wall layers
    from the NS start, FP32: time per outer iteration, per sweep, kinetic
    cells."""
    import gsis_inputs as gi
    u = MACH * np.sqrt(5.0 / 6.0)
    m = gi.cylinder_tri_2d(free=(1.0, (u, 0.0, 0.0), 1.0))
    grid = gi.velocity_grid(2, 64, 15.0, "stretched")
    W = gi.hypersonic_field(m)
    W[:, 3] = 0.0
    n = m["n_cells"]
    case = g.Case(g.Mesh(m), grid, 0.01, dtype=g.F32, capacity=int(0.6 * n))
    case.set_state(W, flags=np.zeros(n, np.uint8))
    t = time.perf_counter()
    case.solve(g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, tol=1e-6, max_iter=0, n_macro_inner=400, cfl=0.5,
                             force_wall_layers=2, ns_init=1, ns_init_max_chunks=50))
    torch.cuda.synchronize()
    ns_s = time.perf_counter() - t
    p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, n_macro_inner=400, cfl=0.5, region_update_every=1,
                      force_wall_layers=2)
    step_ms, kms, nk, e = _timed_steps(torch, case, p, steps)
    pts = nk * case.nv * 2
    out = {"cells": n, "velocities": case.nv, "ns_start_s": ns_s, "kinetic_cells_mean": nk,
           "kinetic_fraction": nk / n, "ms_per_step": step_ms, "sweep_ms": kms,
           "sweep_updates_per_s": nk * case.nv / (kms / 1e3), "achieved_gbs": 8.0 * pts / (kms / 1e3) / 1e9,
           "eps_last": [float(x) for x in e], "layout": list(case.sweep_layout())}
    case.close()
    return out


def poly_agsis(g, torch, M, grid, W0, cap, steps):
    """The paper's own gas on the sphere workload: nitrogen as a two-VDF gas
    (d_r 2, Z_r 2.667, omega 0.74, A = (0.786, -0.201, -0.059, 0.842)), FP32,
    aGSIS from the NS start (synthetic equations with the internal energy):
    time per outer iteration, per sweep of (f0, f1) (kernel k_sweep_poly,
    algorithmic bytes per cell-velocity 2 x (4 read + 4 write)), kinetic
    cells."""
    case = g.Case(M, grid, KN, omega=0.74, Pr=0.786, dtype=g.F32, capacity=cap,
                  dr=2.0, Zr=2.667, A=(0.786, -0.201, -0.059, 0.842))
    case.set_state(W0, flags=np.zeros(M.n_cells, np.uint8))
    t = time.perf_counter()
    case.solve(g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, tol=1e-6, max_iter=0, n_macro_inner=400, cfl=0.5,
                             force_wall_layers=2, ns_init=1, ns_init_max_chunks=100))
    torch.cuda.synchronize()
    ns_s = time.perf_counter() - t
    p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, n_macro_inner=400, cfl=0.5, region_update_every=1,
                      force_wall_layers=2)
    step_ms, kms, nk, e = _timed_steps(torch, case, p, steps)
    nv = case.nv
    gbs = 16.0 * nk * nv / (kms / 1e3) / 1e9
    out = {"kinetic_cells_mean": nk, "velocities": nv, "ns_start_s": ns_s, "ms_per_step": step_ms,
           "sweep_ms": kms, "sweep_updates_per_s": nk * nv / (kms / 1e3), "bytes_per_update": 16.0,
           "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS, "kernel": "k_sweep_poly",
           "eps_last": [float(x) for x in e], "limiters": case.limiter_stats(),
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


def step_graph_leg(g, torch, case, n_inner, steps=4):
    """Whole outer iterations with the region held (no re-flagging): eager
    launches, then replays of whole-step HIP graphs (GSIS_STEP_GRAPHS=1; the
    first two steps capture one graph per buffer parity)."""
    p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=KN_REF, n_macro_inner=n_inner, cfl=0.5, region_update_every=0,
                      force_wall_layers=2)
    out = {}
    for name, env, warm in (("eager", "0", 1), ("graphs", "1", 2)):
        os.environ["GSIS_STEP_GRAPHS"] = env
        try:
            for _ in range(warm):
                case.step(p)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                case.step(p)
            torch.cuda.synchronize()
            out[name + "_ms_per_step"] = 1e3 * (time.perf_counter() - t) / steps
        finally:
            os.environ.pop("GSIS_STEP_GRAPHS", None)
    out["kinetic_cells"] = case.n_kin
    return out


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
    W_start = W.copy()
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
    step_graphs = None if a.sweep_only else step_graph_leg(g, torch, case, a.n_inner)
    log("whole-step graphs", step_graphs)
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

    copy_gbs = stream_rate(torch)
    log("plain streaming kernel %.0f GB/s" % copy_gbs)

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
        poly = poly_agsis(g, torch, M, grid, W_start, cap, a.poly_steps)
        log("nitrogen aGSIS", poly)
    configs = None
    if not a.no_configs and not a.sweep_only:
        configs = {}
        configs["C1_couette_fp64"] = c1_couette(g, torch)
        log("C1", configs["C1_couette_fp64"])
        configs["C2_cavity_fp32"] = c2_cavity(g, torch)
        log("C2", configs["C2_cavity_fp32"])
        configs["C3_cylinder_fp32"] = c3_cylinder(g, torch)
        log("C3", configs["C3_cylinder_fp32"])

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": sweep_kernel_name(),
                     "kernel_ms": 1e3 * sweep_s, "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs if copy_gbs else None},
        "sweep_updates_per_s": n_kin_mean * nv / sweep_s,
        "fp64_sweep": fp64,
        "point_grid_sweep": points,
        "order2_sweep": order2,
        "nitrogen_agsis": poly,
        "configs": configs,
        "surface": surface,
        "synthetic_solve": synthetic,
        "step_graphs": step_graphs,
        "setup_s": setup_s,
    }
    if a.serve_requests > 0 and not a.sweep_only:
        t1 = time.time()
        rates = [float(x) for x in a.serve_rates.split(",") if x]
        out["serving"] = serving(g, a.serve_requests, rates, a.serve_max_iter, a.serve_tol, a.serve_fp64_check,
                                 a.serve_source_half)
        log("serving leg %.1f s" % (time.time() - t1))
    if not a.no_cpu_baseline:
        t1 = time.time()
        out["cpu_baseline"] = cpu_baseline(mesh, grid, W, flags, a.cpu_seconds)
        log("cpu baseline %.1f s" % (time.time() - t1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
