"""Binding to the library's static device workspace (gsis_case_bind_static)
against the ordinary binding to a caller-owned workspace: the same outer
iterations on the same inputs give the same fields, VDF and residuals, on two
bindings in a row (the second case smaller), and the first static case is
released when the second takes the workspace."""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    import paper_2501_02245_amd as g
    assert torch.cuda.is_available()
    return g


def _run(g, m, grid, Kn, W, flags, dtype, params, steps, static):
    print("bind", "static" if static else "workspace", m["n_cells"], "cells", flush=True)
    case = g.Case(g.Mesh(m), grid, Kn, dtype=dtype, static=static)
    if params.mode == g.MODE_AGSIS:
        kin = np.nonzero(flags)[0]
        f0 = gi.gaussian_rows(grid, W[kin], seed=2).astype(np.float64)
        case.set_state(W, vdf=f0, flags=flags)
    else:
        case.set_state(W)
    eps = np.array([case.step(params) for _ in range(steps)])
    Wd, fl = case.get_state()
    out = {"eps": eps, "W": Wd.cpu().numpy(), "flags": fl.cpu().numpy(), "f": case.get_vdf().cpu().numpy(),
           "mom": case.moments()[0].cpu().numpy(), "lim": case.limiter_stats()}
    return case, out


def _same(a, b):
    for k in a:
        if k == "lim":
            assert a[k] == b[k], (a[k], b[k])
        else:
            assert a[k].shape == b[k].shape and np.array_equal(a[k], b[k]), k


def test_static_binding_matches_workspace_binding(g):
    m, grid, Kn, W, flags = workload("cylinder_small")
    pa = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, n_macro_inner=100, cfl=0.5, region_update_every=1,
                       force_wall_layers=2)
    ref, a = _run(g, m, grid, Kn, W, flags, g.F32, pa, 3, static=False)
    ref.close()
    st1, b = _run(g, m, grid, Kn, W, flags, g.F32, pa, 3, static=True)
    _same(a, b)
    # second binding in a row, a smaller case: takes the workspace over
    m2 = gi.couette_1d(16, 0.1)
    grid2 = gi.velocity_grid(3, 12, 5.0)
    W2 = gi.couette_initial_W(16, seed=1)
    pg = g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=200, cfl=-0.5)
    ref2, c = _run(g, m2, grid2, 0.1, W2, None, g.F64, pg, 3, static=False)
    ref2.close()
    st2, d = _run(g, m2, grid2, 0.1, W2, None, g.F64, pg, 3, static=True)
    _same(c, d)
    assert st2.footprint < st1.footprint
    # the first static case was released: its calls fail until it is bound again
    with pytest.raises(g.GsisError) as e:
        st1.sweep(1)
    assert e.value.code == g.E_STATE
    st1.close()
    st2.close()


def test_static_binding_refuses_oversized_case(g):
    """A case whose footprint exceeds the 256 MiB workspace is refused before
    anything touches the device."""
    m, grid, Kn, W, flags = workload("cavity")
    big = gi.velocity_grid(2, 128, 6.0, "stretched")
    with pytest.raises(g.GsisError) as e:
        g.Case(g.Mesh(m), big, Kn, dtype=g.F64, static=True)
    assert e.value.code == g.E_NOMEM and "static workspace" in str(e.value)
