"""GPU parity of the second-order kinetic face values against the FP64 oracle:
limited least-squares slopes of every discrete-velocity value (slope kernel),
the deferred correction and pseudo-time term in the generic sweep, and the
wall densities fixed by the reconstructed outgoing values.

Cases: one sweep on the Couette slab (1D, walls), the cavity (reduced 2D,
walls, 64^2 cells), the Mach-5 cylinder and sphere with partial kinetic
regions (NS neighbours, ghosts, far field, walls), a grid whose rows span two
velocity tiles with a ragged tail, and a point-set grid; two sweeps in a row
on walled slabs (the second reads the first's slopes and wall sums); GSIS and
aGSIS outer iterations; layout, footprint and call-order checks.
Tolerances: FP32 1e-5 per sweep, FP64 1e-11.
"""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import f_error, moment_errors, workload

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


def _load(name):
    if name == "points":
        m = gi.couette_1d(16, 0.1)
        grid = gi.ball_grid(16, 5.0)
        W = gi.random_W(16, seed=3, u_scale=0.2)
        return m, grid, 0.05, W, np.ones(16, np.uint8)
    return workload(name)


@pytest.mark.parametrize("name", ["couette", "couette_ragged", "cavity", "cylinder_small", "sphere_small", "points",
                                  "hexbox"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_order2_one_sweep(g, oracle_mod, name, dtype):
    m, grid, Kn, W, flags = _load(name)
    print("order2 sweep", name, "dtype", dtype, flush=True)
    O = oracle_mod.Oracle(m, grid, Kn, order=2)
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    f0 = gi.gaussian_rows(grid, W[kin], seed=1, amp=0.2,
                          dtype=np.float32 if dtype == g.F32 else np.float64).astype(np.float64)
    W = W.copy()
    W[kin] = O.moments(f0)[:, :5]
    case = g.Case(g.Mesh(m), grid, Kn, dtype=dtype, order=2)
    assert case.sweep_layout()[0] == 0
    case.set_state(W, vdf=f0, flags=flags)
    ghost = O.ghost_params(W) if len(kin) < m["n_cells"] else None
    fo = O.sweep(f0, kin, slot, ghost)
    case.sweep(1)
    fg = case.get_vdf().cpu().numpy()
    mg, kc = case.moments()
    assert np.array_equal(kc.cpu().numpy(), kin)
    ef = f_error(fg, fo, O.w)
    em = moment_errors(mg.cpu().numpy(), O.moments(fo), u_scale=1.0)
    # the second-order sweep differs from the first-order one by far more than the tolerance
    d12 = f_error(oracle_mod.Oracle(m, grid, Kn).sweep(f0, kin, slot, ghost), fo, O.w)
    print("order2", name, dtype, "nv", case.nv, "f", ef, "moments", em, "vs order 1", d12, flush=True)
    assert d12 > 100 * TOL[0]
    assert ef < TOL[dtype]
    for k, v in em.items():
        assert v < TOL[dtype], (k, v)


@pytest.mark.parametrize("dtype", [0, 1])
def test_order2_generic_kernel_3d(g, oracle_mod, dtype, monkeypatch):
    """The generic kernel's second-order path on a 3D grid (selected by
    GSIS_ORDER2_GENERIC=1) against the oracle, on the sphere's partial region."""
    monkeypatch.setenv("GSIS_ORDER2_GENERIC", "1")
    m, grid, Kn, W, flags = workload("sphere_small")
    O = oracle_mod.Oracle(m, grid, Kn, order=2)
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    f0 = gi.gaussian_rows(grid, W[kin], seed=5, amp=0.2,
                          dtype=np.float32 if dtype == g.F32 else np.float64).astype(np.float64)
    W = W.copy()
    W[kin] = O.moments(f0)[:, :5]
    case = g.Case(g.Mesh(m), grid, Kn, dtype=dtype, order=2)
    case.set_state(W, vdf=f0, flags=flags)
    ghost = O.ghost_params(W)
    fo = O.sweep(f0, kin, slot, ghost)
    case.sweep(1)
    ef = f_error(case.get_vdf().cpu().numpy(), fo, O.w)
    print("order2 generic 3D", dtype, ef, flush=True)
    assert ef < TOL[dtype]


@pytest.mark.parametrize("name", ["couette", "cavity"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_order2_two_sweeps(g, oracle_mod, name, dtype):
    """Two sweeps in a row on walled domains: the second uses slopes and wall
    sums recomputed from the first's output."""
    m, grid, Kn, W, flags = workload(name)
    print("order2 two sweeps", name, "dtype", dtype, flush=True)
    O = oracle_mod.Oracle(m, grid, Kn, order=2, damp2=1.5)
    kin = np.arange(m["n_cells"])
    f0 = gi.gaussian_rows(grid, W, seed=4, amp=0.2,
                          dtype=np.float32 if dtype == g.F32 else np.float64).astype(np.float64)
    W = W.copy()
    W[:] = O.moments(f0)[:, :5]
    case = g.Case(g.Mesh(m), grid, Kn, dtype=dtype, order=2, damp2=1.5)
    case.set_state(W, vdf=f0)
    fo = O.sweep(O.sweep(f0, kin, kin), kin, kin)
    case.sweep(2)
    ef = f_error(case.get_vdf().cpu().numpy(), fo, O.w)
    print("order2 two sweeps", name, dtype, ef, flush=True)
    assert ef < 2 * TOL[dtype]


@pytest.mark.parametrize("half", [0, 1])
@pytest.mark.parametrize("dtype", [1, 0])
def test_order2_gsis_steps(g, oracle_mod, dtype, half):
    """Three GSIS outer iterations (sweep, synthetic solve, correction) at
    second order on the Couette slab (source of eq. macro at f^n and at the
    half step, whose balance pass takes the slopes of f^{n+1/2})."""
    m, grid, Kn, W, flags = workload("couette")
    O = oracle_mod.Oracle(m, grid, Kn, order=2)
    S = oracle_mod.SteadySolver(O, mode="gsis", n_inner=50, cfl=-0.5, source_half=bool(half))
    case = g.Case(g.Mesh(m), grid, Kn, dtype=dtype, order=2)
    if dtype == g.F32:
        f0 = gi.gaussian_rows(grid, W, seed=2).astype(np.float64)
        S.set_state(W, f=f0)
        case.set_state(W, vdf=f0)
    else:
        S.set_state(W)
        case.set_state(W)
    p = g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=50, cfl=-0.5, source_half=half)
    tol = 1e-9 if dtype == g.F64 else 1e-5
    for it in range(3):
        eo = S.step()
        eg = case.step(p)
        Wg = case.get_state()[0].cpu().numpy()
        err = np.abs(Wg - S.W).max() / np.abs(S.W).max()
        print("gsis order2", dtype, it, eo, eg, err, flush=True)
        assert err < tol
    fo = S.f[S.slot[S.kin]]
    assert f_error(case.get_vdf().cpu().numpy(), fo, O.w) < (1e-9 if dtype == g.F64 else 1e-5)


def test_order2_agsis_steps(g, oracle_mod):
    """aGSIS at second order on the sphere (FP64): two outer iterations with
    region updates (new cells start from Grad-13 rows; slopes are taken over
    the new region)."""
    m, grid, Kn, W, flags = workload("sphere_small")
    O = oracle_mod.Oracle(m, grid, Kn, order=2)
    S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=0.01, n_inner=40, cfl=0.5, force_wall_layers=2)
    S.set_state(W, flags=flags)
    case = g.Case(g.Mesh(m), grid, Kn, dtype=g.F64, order=2)
    case.set_state(W, flags=flags)
    p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, n_macro_inner=40, cfl=0.5, force_wall_layers=2)
    for it in range(2):
        eo = S.step()
        eg = case.step(p)
        Wg, fl = case.get_state()
        Wg, fl = Wg.cpu().numpy(), fl.cpu().numpy()
        err = np.abs(Wg - S.W).max() / np.abs(S.W).max()
        print("agsis order2", it, eo, eg, err, "n_kin", len(S.kin), case.n_kin, flush=True)
        assert np.array_equal(fl, S.flags)
        assert err < 1e-9


def test_order2_layout_footprint_and_call_order(g):
    """Order 2 forces the generic sweep, adds dim * row * capacity elements of
    slopes to the footprint, and is refused once the case is bound."""
    m, grid, Kn, W, flags = workload("sphere_fast")
    c1 = g.Case(g.Mesh(m), grid, Kn, dtype=g.F32)
    c2 = g.Case(g.Mesh(m), grid, Kn, dtype=g.F32, order=2)
    assert c1.sweep_layout()[0] == 1 and c2.sweep_layout()[0] == 0
    slope_bytes = 4 * m["dim"] * c2.capacity * c2.nv
    assert c2.footprint - c1.footprint >= slope_bytes
    with pytest.raises(g.GsisError):
        g._check(g.lib().gsis_set_spatial_order(c1.handle, 2, 2.0))
    import ctypes as C
    mesh = g.Mesh(gi.couette_1d(8))
    for order, damp in ((3, 2.0), (0, 2.0), (2, -1.0), (2, float("nan"))):
        hh = C.c_void_p()
        g._check(g.lib().gsis_create_case(mesh.handle, C.byref(g._Gas(0.1, 0.5, 2 / 3)), g.F32, C.byref(hh)))
        with pytest.raises(g.GsisError):
            g._check(g.lib().gsis_set_spatial_order(hh, order, damp))
        g._check(g.lib().gsis_destroy_case(hh))
