"""Edge cases of the GPU path against the FP64 oracle: an empty kinetic region
(every cell NS), the smallest mesh (one cell between two walls), the largest
velocity axis (128 nodes, 2D and 3D plane kernels), and a region that outgrows
the bound capacity (the error and the invalidated state)."""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import f_error, make_case, moment_errors, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_empty_region_step(g, oracle_mod):
    """Every cell NS and no re-flagging: the sweep has nothing to do and an aGSIS
    step is the synthetic solve alone (FP64 on both sides)."""
    m, grid, Kn, W, _ = workload("cylinder_small")
    flags = np.zeros(m["n_cells"], np.uint8)
    O = oracle_mod.Oracle(m, grid, Kn)
    S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=0.01, n_inner=50, cfl=0.5, region_every=0)
    S.set_state(W, flags=flags)
    case = make_case(g, "cylinder_small", m, grid, Kn, g.F64)
    case.set_state(W, flags=flags)
    case.sweep(1)
    mg, kc = case.moments()
    assert kc.numel() == 0 and case.n_kin == 0
    p = g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, n_macro_inner=50, cfl=0.5, region_update_every=0)
    eo = S.step()
    eg = case.step(p)
    Wg = case.get_state()[0].cpu().numpy()
    print("empty region: W", _rel(Wg, S.W), "eps", eo, eg, flush=True)
    assert _rel(Wg, S.W) < 1e-10
    assert np.allclose(eg, eo, rtol=1e-7)


@pytest.mark.parametrize("dtype", [0, 1])
def test_single_cell_slab(g, oracle_mod, dtype):
    """One cell between two diffuse walls moving -+0.1: one sweep and its moments."""
    m = gi.couette_1d(1, 0.1)
    grid = gi.velocity_grid(3, 16, 5.0)
    W = gi.random_W(1, seed=9, u_scale=0.1)
    O = oracle_mod.Oracle(m, grid, Kn=0.05)
    f0 = gi.gaussian_rows(grid, W, seed=3, dtype=np.float32 if dtype == g.F32 else np.float64).astype(np.float64)
    W = W.copy()
    W[:, :5] = O.moments(f0)[:, :5]
    case = make_case(g, "single", m, grid, 0.05, dtype)
    case.set_state(W, vdf=f0, flags=np.ones(1, np.uint8))
    fo = O.sweep(f0, np.arange(1), np.zeros(1, np.int32))
    case.sweep(1)
    fg = case.get_vdf().cpu().numpy()
    mg, _ = case.moments()
    tol = 1e-5 if dtype == g.F32 else 1e-11
    ef = f_error(fg, fo, O.w)
    mo = O.moments(fo)
    mgn = mg.cpu().numpy()
    em = moment_errors(mgn, mo, u_scale=0.1)
    # one cell: sigma and q are small numbers of their own, compared on the
    # scales p = rho T and p sqrt(T) of the cell
    p_ = mo[0, 0] * mo[0, 4]
    em["sigma"] = np.abs(mgn[0, 5:11] - mo[0, 5:11]).max() / p_
    em["q"] = np.abs(mgn[0, 11:14] - mo[0, 11:14]).max() / (p_ * np.sqrt(mo[0, 4]))
    print("single cell", dtype, ef, em, flush=True)
    assert ef < tol and max(em.values()) < tol


@pytest.mark.parametrize("vdim", [2, 3])
def test_largest_axis(g, oracle_mod, vdim):
    """128 nodes on the x axis (the library's maximum): reduced 128^2 on the
    cylinder and 128 x 16 x 16 in a slab, plane kernel, FP32 one-sweep parity."""
    if vdim == 2:
        m, _, Kn, W, flags = workload("cylinder_small")
        grid = gi.velocity_grid(2, 128, 15.0, "stretched")
        W = W.copy()
        W[:, 3] = 0.0
    else:
        m = gi.couette_1d(8, 0.1)
        grid = gi.velocity_grid(3, (128, 16, 16), (8.0, 5.0, 5.0))
        W = gi.random_W(8, seed=4, u_scale=0.2)
        flags = np.ones(8, np.uint8)
        Kn = 0.05
    O = oracle_mod.Oracle(m, grid, Kn)
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    f0 = gi.gaussian_rows(grid, W[kin], seed=5).astype(np.float64)
    W = W.copy()
    W[kin] = O.moments(f0)[:, :5]
    case = make_case(g, "largest", m, grid, Kn, g.F32)
    assert case.sweep_layout()[0] == 1
    case.set_state(W, vdf=f0, flags=flags)
    ghost = O.ghost_params(W)
    fo = O.sweep(f0, kin, slot, ghost)
    case.sweep(1)
    fg = case.get_vdf().cpu().numpy()
    mg, kc = case.moments()
    assert np.array_equal(kc.cpu().numpy(), kin)
    ef = f_error(fg, fo, O.w)
    em = moment_errors(mg.cpu().numpy(), O.moments(fo), u_scale=1.0)
    print("largest axis", vdim, ef, em, flush=True)
    assert ef < 1e-5 and max(em.values()) < 1e-5


def test_capacity_overflow(g, oracle_mod):
    """A re-flagging that needs more kinetic cells than the bound capacity fails
    with E_CAPACITY (the oracle's solver refuses it too) and leaves the case
    needing set_state; set_state with a fitting region recovers it."""
    m, grid, Kn, W, flags = workload("cylinder_small")
    kin = np.nonzero(flags)[0]
    small = np.zeros_like(flags)
    small[kin[:10]] = 1
    cap = 20
    O = oracle_mod.Oracle(m, grid, Kn)
    S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=1e-6, force_wall_layers=2, capacity=cap)
    S.set_state(W, flags=small)
    with pytest.raises(MemoryError):
        S.update_regions()
    case = make_case(g, "cylinder_small", m, grid, Kn, g.F32, capacity=cap)
    case.set_state(W, flags=small)
    with pytest.raises(g.GsisError) as e:
        case.update_regions(1e-6, 2)
    assert e.value.code == g.E_CAPACITY
    with pytest.raises(g.GsisError) as e:
        case.sweep(1)
    assert e.value.code == g.E_STATE
    case.set_state(W, flags=small)
    case.sweep(1)
    assert case.n_kin == 10
