"""Benchmark of the adaptive-GSIS kinetic hot path on one MI355X.

One step = one outer aGSIS iteration (Sec. 3.4): relaxation parameters, the
implicit kinetic sweep with fused moments, high-order terms and the
synthetic macroscopic solve, the GSIS correction, the convergence measure and
the local-Kn region update with compaction.  Workload: Mach-5 flow past a
sphere on a seeded ~200k-tetrahedron mesh, 32^3 stretched velocity grid on
[-15, 15]^3, FP32 VDF, FP64 macroscopic side; inputs already resident in HBM
when the timed region starts.

Prints one JSON line (see the repository's benchmark contract).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fraction", type=float, default=0.2, help="kinetic fraction of the synthetic region")
    ap.add_argument("--n-inner", type=int, default=400)
    ap.add_argument("--nv1d", type=int, default=32)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--region-every", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-only", action="store_true", help="time kinetic sweeps only (diagnostic)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import gsis_inputs as gi
    import paper_2501_02245_amd as g

    t0 = time.time()
    mach = 5.0
    u_inf = mach * np.sqrt(5.0 / 6.0)
    mesh = gi.sphere_tet_3d(free=(1.0, (u_inf, 0.0, 0.0), 1.0))
    grid = gi.velocity_grid(3, a.nv1d, 15.0, "stretched")
    W = gi.hypersonic_field(mesh)
    flags = gi.synthetic_region(mesh, a.fraction, seed=11)
    n_cells = mesh["n_cells"]
    Kn = 0.005
    dtype = g.F32 if a.dtype == "f32" else g.F64
    cap = min(n_cells, int(flags.sum() * 1.5) + 64)
    M = g.Mesh(mesh)
    case = g.Case(M, grid, Kn, dtype=dtype, capacity=cap)
    case.set_state(W, flags=flags)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    nv = case.nv
    params = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, tol=1e-12, n_macro_inner=a.n_inner, cfl=0.5,
                           region_update_every=a.region_every, force_wall_layers=2)

    def one():
        if a.sweep_only:
            case.sweep(1)
        else:
            case.step(params)

    for _ in range(a.warmup):
        one()
    torch.cuda.synchronize()
    kin_counts, sweep_ms = [], []
    t = time.perf_counter()
    for _ in range(a.steps):
        kin_counts.append(case.n_kin)
        one()
        sweep_ms.append(case.last_sweep_ms())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    updates = float(sum(kin_counts)) * nv
    ms_step = 1e3 * dt / a.steps
    es = 4 if dtype == g.F32 else 8
    sweep_s = np.mean(sweep_ms) / 1e3
    n_kin_mean = float(np.mean(kin_counts))
    alg_bytes = 2 * es * n_kin_mean * nv          # read f^n, write f^{n+1/2}
    achieved = alg_bytes / sweep_s / 1e9
    out = {
        "metric": "kinetic cell-velocity updates/s",
        "value": updates / dt,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == g.F32 else "f64",
        "data": "synthetic",
        "config": {"workload": "3D Mach-5 sphere, %d tetrahedra, %d^3 stretched velocities on [-15,15]^3, "
                               "aGSIS Kn=0.005 Kn_ref=0.01" % (n_cells, a.nv1d),
                   "kinetic_cells_mean": n_kin_mean, "n_macro_inner": a.n_inner,
                   "sweep_only": bool(a.sweep_only)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sweep",
                     "kernel_ms": 1e3 * sweep_s},
        "sweep_updates_per_s": n_kin_mean * nv / sweep_s,
        "setup_s": setup_s,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
