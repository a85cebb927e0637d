"""GPU parity of the polyatomic gas (the two-VDF model of Sec. 2, nitrogen
parameters of Sec. 4) against the FP64 oracle: one sweep of both VDFs on the
Couette slab (walls), on a grid whose rows span two velocity tiles with a
ragged tail, and on the Mach-5 sphere's partial region (NS neighbours,
Grad-13 ghosts, far field, walls); the state filled from W; DVM outer
iterations; and the calls the polyatomic gas refuses.
Tolerances: FP32 1e-5 per sweep, FP64 1e-11.
"""
import ctypes as C

import numpy as np
import pytest

import gsis_inputs as gi
from _cases import f_error, moment_errors, workload

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}
N2 = dict(dr=2.0, Zr=2.667, omega=0.74, A=(0.786, -0.201, -0.059, 0.842))


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


def _pair(O, g, m, grid, Kn, dtype, capacity=None):
    Og = O(m, grid, Kn, omega=N2["omega"], Pr=N2["A"][0], dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    case = g.Case(g.Mesh(m), grid, Kn, omega=N2["omega"], Pr=N2["A"][0], dtype=dtype, capacity=capacity,
                  dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    return Og, case


def _rows(grid, W, seed, dtype):
    """f0: perturbed local Gaussians; f1 = (d_r T_r / 4) f0 times independent
    factors, with T_r = 0.8 T (internal modes out of equilibrium, q_r != 0)."""
    f0 = gi.gaussian_rows(grid, W, seed=seed, amp=0.2, dtype=np.float64)[:, 0]
    th = 0.25 * N2["dr"] * 0.8 * W[:, 4]
    f1 = th[:, None] * f0 * gi.perturbation(f0.shape, seed=seed + 1, amp=0.2)
    f = np.stack([f0, f1], axis=1)
    return f.astype(np.float32 if dtype == 0 else np.float64).astype(np.float64)


@pytest.mark.parametrize("name", ["couette", "couette_ragged", "sphere_small"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_poly_one_sweep(g, oracle_mod, name, dtype):
    m, grid, Kn, W, flags = workload(name)
    print("poly sweep", name, "dtype", dtype, flush=True)
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, dtype)
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    f0 = _rows(grid, W[kin], 3, dtype)
    mo = O.moments(f0)
    W = W.copy()
    W[kin] = mo[:, :5]
    assert case.sweep_layout()[0] == 0
    case.set_state(W, vdf=f0, flags=flags)
    # the filled state's moments, internal ones included
    mg0, _ = case.moments()
    ig0 = case.internal_moments().cpu().numpy()
    assert np.abs(ig0[:, 0] / mo[:, 14] - 1).max() < TOL[dtype]
    ghost = O.ghost_params(W) if len(kin) < m["n_cells"] else None
    fo = O.sweep(f0, kin, slot, ghost)
    case.sweep(1)
    fg = case.get_vdf().cpu().numpy()
    assert fg.shape == fo.shape == (len(kin), 2, O.nv)
    ef = f_error(fg, fo, O.w)
    mg, _ = case.moments()
    m_o = O.moments(fo)
    em = moment_errors(mg.cpu().numpy(), m_o[:, :14], u_scale=1.0)
    ig = case.internal_moments().cpu().numpy()
    eTr = np.abs(ig[:, 0] - m_o[:, 14]).max() / np.abs(m_o[:, 14]).max()
    # q_r = 2 sum w c f1 is a first moment of f1 about u, a small difference of
    # terms of size rho T_r sqrt(T) (the internal energy carried at the thermal
    # speed): each cell's error is measured on that scale, as sigma and q are
    # on p and p sqrt(T)
    scale = m_o[:, 0] * m_o[:, 14] * np.sqrt(m_o[:, 4])
    eqr = float((np.abs(ig[:, 1:] - m_o[:, 15:]).max(axis=1) / scale).max())
    print("poly", name, dtype, "f", ef, "moments", em, "T_r", eTr, "q_r", eqr, flush=True)
    assert ef < TOL[dtype]
    for k, v in em.items():
        assert v < TOL[dtype], (k, v)
    assert eTr < TOL[dtype] and eqr < TOL[dtype]


@pytest.mark.parametrize("dtype", [0, 1])
def test_poly_filled_state(g, oracle_mod, dtype):
    """set_state without rows: f0 = conservation-fixed Maxwellian of W, f1 =
    (d_r T / 4) f0, as the oracle's f_eq."""
    m, grid, Kn, W, flags = workload("sphere_small")
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, dtype)
    kin = np.nonzero(flags)[0]
    case.set_state(W, flags=flags)
    fg = case.get_vdf().cpu().numpy()
    fo = np.stack([O.feq(W[c]) for c in kin])
    assert f_error(fg, fo, O.w) < (1e-7 if dtype == 0 else 1e-11)
    ig = case.internal_moments().cpu().numpy()
    assert np.abs(ig[:, 0] / W[kin, 4] - 1).max() < (1e-6 if dtype == 0 else 1e-12)


@pytest.mark.parametrize("dtype", [1, 0])
def test_poly_dvm_steps(g, oracle_mod, dtype):
    """Three DVM outer iterations (gsis_step in DVM mode) on the Couette slab:
    W, the residuals and the rows against the oracle's plain iteration."""
    m, grid, Kn, W, flags = workload("couette")
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, dtype)
    S = oracle_mod.SteadySolver(O, mode="dvm")
    f0 = _rows(grid, W, 7, dtype)
    S.set_state(W, f=f0)
    case.set_state(S.W, vdf=f0)
    p = g.SolveParams(mode=g.MODE_DVM)
    tol = 1e-10 if dtype == g.F64 else 1e-5
    for it in range(3):
        eo = S.step()
        eg = case.step(p)
        Wg = case.get_state()[0].cpu().numpy()
        err = np.abs(Wg - S.W).max() / np.abs(S.W).max()
        print("poly dvm", dtype, it, eo, eg, err, flush=True)
        assert err < tol
        assert np.allclose(eg, eo, rtol=1e-3 if dtype == 0 else 1e-8)
    fo = S.f[S.slot[S.kin]]
    assert f_error(case.get_vdf().cpu().numpy(), fo, O.w) < (1e-10 if dtype == g.F64 else 1e-5)


def test_poly_refusals(g):
    """Calls outside the polyatomic gas's support fail with a clear error and
    leave the case usable; settings made after binding are refused."""
    m, grid, Kn, W, flags = workload("couette")
    case = g.Case(g.Mesh(m), grid, Kn, dtype=g.F64, dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    case.set_state(W)
    with pytest.raises(g.GsisError):
        case.step(g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=10, cfl=0.5))
    with pytest.raises(g.GsisError):
        g._check(g.lib().gsis_update_regions(case.handle, C.c_double(0.01), 0, None, g._stream()))
    A = np.array(N2["A"])
    with pytest.raises(g.GsisError):
        g._check(g.lib().gsis_set_internal_dof(case.handle, C.c_double(2.0), C.c_double(2.0),
                                              C.c_void_p(A.ctypes.data)))
    case.sweep(1)                      # still usable
    mono = g.Case(g.Mesh(m), grid, Kn, dtype=g.F64)
    mono.set_state(W)
    with pytest.raises(g.GsisError):
        mono.internal_moments()
    with pytest.raises(g.GsisError):   # point sets are not supported with d_r > 0
        g.Case(g.Mesh(m), gi.ball_grid(8, 4.0), Kn, dtype=g.F64, dr=2.0, Zr=2.0, A=N2["A"])
    with pytest.raises(g.GsisError):   # nor a reduced 2D grid
        g.Case(g.Mesh(m), gi.velocity_grid(2, 8, 4.0), Kn, dtype=g.F64, dr=2.0, Zr=2.0, A=N2["A"])
