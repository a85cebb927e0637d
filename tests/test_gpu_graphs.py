"""The synthetic solve replayed from a captured HIP graph gives bitwise the
eager results, step after step (eager sweeps, corrections and host reads
between the replays)."""
import os

import numpy as np
import pytest

from _cases import make_case, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


@pytest.mark.parametrize("name,mode", [("cylinder_fast", "agsis"), ("couette", "gsis")])
def test_graph_replays_equal_eager(g, name, mode):
    m, grid, Kn, W, flags = workload(name)
    out = {}
    for graphs in ("0", "1"):
        os.environ["GSIS_GRAPHS"] = graphs
        try:
            case = make_case(g, name, m, grid, Kn, g.F32)
            if mode == "agsis":
                case.set_state(W, flags=flags)
                p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, n_macro_inner=50, cfl=0.5, region_update_every=2,
                                  force_wall_layers=2)
            else:
                case.set_state(W)
                p = g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=50, cfl=-0.5)
            eps = [case.step(p) for _ in range(5)]
            Wg, fl = case.get_state()
            out[graphs] = (np.array(eps), Wg.cpu().numpy(), fl.cpu().numpy(), case.get_vdf().cpu().numpy())
            case.close()
        finally:
            os.environ.pop("GSIS_GRAPHS", None)
    for a, b in zip(out["0"], out["1"]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,mode,half", [("cylinder_fast", "agsis", 0), ("couette", "gsis", 0),
                                            ("sphere_fast", "agsis", 0), ("cylinder_fast", "agsis", 1),
                                            ("couette", "gsis", 1)])
def test_step_graph_replays_equal_eager(g, name, mode, half):
    """Whole outer iterations from HIP graphs (GSIS_STEP_GRAPHS=1): sweep,
    moments, HoT, synthetic solve, correction and residual captured per batch
    composition, counts and buffer parity, replayed between region updates
    (re-flagging once, after two iterations, then a fixed region: the later
    steps replay the graphs of the same parity).  Eight iterations with host
    reads between them are bitwise the eager ones, with the synthetic source
    at f^n, W^n and at the half step (its balance pass captured too)."""
    m, grid, Kn, W, flags = workload(name)
    out = {}
    for graphs in ("0", "1"):
        os.environ["GSIS_STEP_GRAPHS"] = graphs
        try:
            case = make_case(g, name, m, grid, Kn, g.F32)
            if mode == "agsis":
                case.set_state(W, flags=flags)
                p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, n_macro_inner=50, cfl=0.5, region_update_every=-2,
                                  force_wall_layers=2, source_half=half)
            else:
                case.set_state(W)
                p = g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=50, cfl=-0.5, source_half=half)
            eps, Ws = [], []
            for _ in range(8):
                eps.append(case.step(p))
                Ws.append(case.get_state()[0].cpu().numpy())
            Wg, fl = case.get_state()
            out[graphs] = (np.array(eps), np.array(Ws), fl.cpu().numpy(), case.get_vdf().cpu().numpy(),
                           case.moments()[0].cpu().numpy())
            case.close()
        finally:
            os.environ.pop("GSIS_STEP_GRAPHS", None)
    for a, b in zip(out["0"], out["1"]):
        assert np.array_equal(a, b)
