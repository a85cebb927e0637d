"""GPU parity of the polyatomic gas (the two-VDF model of Sec. 2, nitrogen
parameters of Sec. 4) against the FP64 oracle: one sweep of both VDFs on the
Couette slab (walls), on a grid whose rows span two velocity tiles with a
ragged tail, and on the Mach-5 sphere's partial region (NS neighbours,
Grad-13 ghosts, far field, walls); the state filled from W; DVM, GSIS and
aGSIS outer iterations (synthetic solve with the internal-energy equation,
correction of both VDFs, region updates); the NS start; a converged GSIS
solution; the surface quantities with the internal energy; the correction
and the synthetic solve as calls of their own; and the calls the polyatomic
gas refuses.
Tolerances: FP32 1e-5 per sweep, FP64 1e-11; outer iterations FP64 1e-9,
FP32 1e-4 (the synthetic solve's 100-400 pseudo-time steps amplify the
sweep's rounding).
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


@pytest.mark.parametrize("name", ["couette", "couette_ragged", "sphere_small", "hexbox"])
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
    # T_r as the library holds it: T_t on NS cells, that of f1 on kinetic ones
    W = np.concatenate([W, W[:, 4:5]], 1)
    W[kin, 5] = mo[:, 14]
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
    case.set_state(S.W[:, :5], vdf=f0)
    p = g.SolveParams(mode=g.MODE_DVM)
    tol = 1e-10 if dtype == g.F64 else 1e-5
    for it in range(3):
        eo = S.step()
        eg = case.step(p)
        Wg = case.get_state()[0].cpu().numpy()
        err = np.abs(Wg - S.W[:, :5]).max() / np.abs(S.W[:, :5]).max()
        eTr = _rel(case.internal_temperature().cpu().numpy(), S.W[:, 5])
        print("poly dvm", dtype, it, eo, eg, err, eTr, flush=True)
        assert err < tol and eTr < tol
        assert np.allclose(eg, eo, rtol=1e-3 if dtype == 0 else 1e-8)
    fo = S.f[S.slot[S.kin]]
    assert f_error(case.get_vdf().cpu().numpy(), fo, O.w) < (1e-10 if dtype == g.F64 else 1e-5)


def _rel(a, b, scale=None):
    return float(np.abs(a - b).max() / (scale if scale is not None else np.abs(b).max()))


def _state_err(case, S):
    """W (rho, u, T_t) and T_r of every cell against the oracle's state."""
    Wg, fl = case.get_state()
    Wg = Wg.cpu().numpy()
    Trg = case.internal_temperature().cpu().numpy()
    e = {"rho": _rel(Wg[:, 0], S.W[:, 0]), "u": _rel(Wg[:, 1:4], S.W[:, 1:4], max(np.abs(S.W[:, 1:4]).max(), 1.0)),
         "T_t": _rel(Wg[:, 4], S.W[:, 4]), "T_r": _rel(Trg, S.W[:, 5])}
    return e, fl.cpu().numpy()


@pytest.mark.parametrize("dtype", [1, 0])
def test_poly_gsis_steps(g, oracle_mod, dtype):
    """Three GSIS outer iterations (every cell kinetic) on the Couette slab:
    the synthetic solve of the two-VDF gas, the correction of f0 and f1, T_r
    of every cell, residuals and rows against the oracle."""
    m, grid, Kn, W, flags = workload("couette")
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, dtype)
    S = oracle_mod.SteadySolver(O, mode="gsis", n_inner=100, cfl=0.5)
    f0 = _rows(grid, W, 11, dtype)
    S.set_state(W, f=f0)
    case.set_state(S.W[:, :5], vdf=f0)
    p = g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=100, cfl=0.5)
    tol = 1e-9 if dtype == g.F64 else 1e-4
    last = case.limiter_stats()
    for it in range(3):
        eo = S.step()
        eg = case.step(p)
        err, _ = _state_err(case, S)
        now = case.limiter_stats()
        cut = now["corrections_limited"] - last["corrections_limited"]
        last = now
        print("poly gsis", dtype, it, eo, eg, err, "cut", cut, S.stats["corrections_limited"], flush=True)
        assert max(err.values()) < tol, err
        assert np.allclose(eg, eo, rtol=1e-3 if dtype == 0 else 1e-7)
        assert cut == S.stats["corrections_limited"]
    fo = S.f[S.slot[S.kin]]
    assert f_error(case.get_vdf().cpu().numpy(), fo, O.w) < tol


def _agsis_params(g, n_inner=100):
    return g.SolveParams(mode=g.MODE_AGSIS, Kn_ref=0.01, n_macro_inner=n_inner, cfl=0.5, region_update_every=1,
                         force_wall_layers=2, ns_init_max_chunks=2)


def _agsis_compare(g, case, S, p, n_steps, tol, dtype):
    last = case.limiter_stats()
    for it in range(n_steps):
        eo = S.step()
        eg = case.step(p)
        err, fl = _state_err(case, S)
        now = case.limiter_stats()
        d = {k: now[k] - last[k] for k in now}
        last = now
        print("poly agsis", dtype, it, "eps", eo, eg, "n_kin", len(S.kin), case.n_kin, "err", err, "limiters", d,
              S.stats, flush=True)
        assert np.array_equal(fl, S.flags)
        assert max(err.values()) < tol, err
        assert np.allclose(eg, eo, rtol=1e-3 if dtype == 0 else 1e-7)
        assert d["g13_ghosts"] == S.stats["g13_ghosts"] and d["g13_ghost_limited"] == S.stats["g13_ghost_limited"]
        assert d["g13_new"] == S.stats["g13_new"] and d["g13_new_limited"] == S.stats["g13_new_limited"]
        assert d["corrections_limited"] == S.stats["corrections_limited"]


@pytest.mark.parametrize("dtype", [1, 0])
def test_poly_agsis_after_ns_start(g, oracle_mod, dtype):
    """The procedure of Sec. 3.4 for nitrogen on the Mach-5 sphere
    (tetrahedra, 16^3 grid): the NS start (every cell NS, the synthetic solve
    alone with the internal-energy equation, two chunks of 200 pseudo-time
    steps), the first flagging with the two-VDF Grad-13 rows of the new
    kinetic cells, then three aGSIS outer iterations with region updates:
    flags, W, T_r of every cell, rows, residuals and limiter activity against
    the oracle."""
    m, grid, Kn, W, _ = workload("sphere_fast")
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, dtype)
    S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=0.01, n_inner=200, cfl=0.5, region_every=1,
                                force_wall_layers=2)
    none = np.zeros(m["n_cells"], np.uint8)
    S.set_state(W, flags=none)
    k, eo = S.ns_init(tol=1e-6, chunk=200, max_chunks=2)
    case.set_state(W, flags=none)
    chunks = g.ns_init([case], _agsis_params(g, 200))
    err, fl = _state_err(case, S)
    print("poly ns start", dtype, k, chunks, eo, err, len(S.kin), case.n_kin, flush=True)
    assert chunks[0] == k
    assert np.array_equal(fl, S.flags)
    assert max(err.values()) < 1e-10, err     # the synthetic side is FP64 in both dtypes
    fo = S.f[S.slot[S.kin]]
    assert f_error(case.get_vdf().cpu().numpy(), fo, O.w) < (1e-10 if dtype == g.F64 else 1e-6)
    S.n_inner = 100
    _agsis_compare(g, case, S, _agsis_params(g), 3, 1e-9 if dtype == g.F64 else 1e-4, dtype)


def test_poly_agsis_rough_start(g, oracle_mod):
    """Two aGSIS outer iterations on the Mach-5 sphere from a seeded region of
    the synthetic shock-layer field (FP64): kinetic cells start far from the
    synthetic solution, so the correction limiter acts in about half of them
    and the Grad-13 rows of many new cells are built at once.  The limiters'
    decisions are discontinuous in the state, so this start is compared in
    FP64 only (a 1e-7 relative change of the oracle's own input moves its
    state by 5e-5 after one iteration)."""
    m, grid, Kn, W, flags = workload("sphere_fast")
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, g.F64)
    S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=0.01, n_inner=100, cfl=0.5, region_every=1,
                                force_wall_layers=2)
    S.set_state(W, flags=flags)
    case.set_state(W, flags=flags)
    _agsis_compare(g, case, S, _agsis_params(g), 2, 1e-9, 1)


def test_poly_gsis_converged(g, oracle_mod):
    """A converged GSIS solution of the two-VDF gas (slab between a moving
    heated wall and the far field, Kn 0.05, 12^3 grid) to eps < 1e-10: the
    GPU's fixed point against the oracle's (FP64)."""
    m = gi.slab_1d(16, gi._patch("wall", u=(0.0, 0.1, 0.0), T=1.1), gi._patch("far", rho=1.0, u=(0.0, 0.0, 0.0), T=1.0))
    grid = gi.velocity_grid(3, 12, 5.0)
    W0 = gi.couette_initial_W(16, seed=1)
    O, case = _pair(oracle_mod.Oracle, g, m, grid, 0.05, g.F64)
    S = oracle_mod.SteadySolver(O, mode="gsis", n_inner=400, cfl=0.5)
    S.set_state(W0)
    it_o, eo = S.solve(tol=1e-10, max_iter=2000)
    case.set_state(W0)
    it_g, eg, _ = case.solve(g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=400, cfl=0.5, tol=1e-10, max_iter=2000))
    err, _ = _state_err(case, S)
    print("poly converged", it_o, eo, it_g, eg, err, flush=True)
    assert abs(it_g - it_o) <= 2
    assert max(err.values()) < 1e-8, err
    # the internal modes are out of equilibrium with the translational ones
    assert np.abs(S.W[:, 5] - S.W[:, 4]).max() > 1e-4


def test_poly_refusals(g):
    """Calls outside the polyatomic gas's support fail with a clear error and
    leave the case usable; settings made after binding are refused."""
    m, grid, Kn, W, flags = workload("couette")
    case = g.Case(g.Mesh(m), grid, Kn, dtype=g.F64, dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    case.set_state(W)
    with pytest.raises(g.GsisError):
        case.correct(W)
    with pytest.raises(g.GsisError):
        case.macro_solve(W, np.zeros((m["n_cells"], 9)), n_inner=10)
    A = np.array(N2["A"])
    with pytest.raises(g.GsisError):
        g._check(g.lib().gsis_set_internal_dof(case.handle, C.c_double(2.0), C.c_double(2.0),
                                              C.c_void_p(A.ctypes.data)))
    with pytest.raises(g.GsisError):   # the half-step source is for the monatomic gas
        case.step(g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=10, source_half=1))
    case.sweep(1)                      # still usable
    mono = g.Case(g.Mesh(m), grid, Kn, dtype=g.F64)
    mono.set_state(W)
    with pytest.raises(g.GsisError):
        mono.internal_moments()
    with pytest.raises(g.GsisError):   # the two-VDF entry points refuse a monatomic case
        mono.correct_internal(W, W[:, 4])
    with pytest.raises(g.GsisError):
        mono.macro_solve_internal(W, W[:, 4], np.zeros((m["n_cells"], 9)), n_inner=10)
    with pytest.raises(g.GsisError):   # point sets are not supported with d_r > 0
        g.Case(g.Mesh(m), gi.ball_grid(8, 4.0), Kn, dtype=g.F64, dr=2.0, Zr=2.0, A=N2["A"])
    with pytest.raises(g.GsisError):   # nor a reduced 2D grid
        g.Case(g.Mesh(m), gi.velocity_grid(2, 8, 4.0), Kn, dtype=g.F64, dr=2.0, Zr=2.0, A=N2["A"])


def _wall_cells(m):
    fc = m["face_cells"]
    wall = [p for p, pt in enumerate(m["patches"]) if pt["kind"] == "wall"]
    b = fc[:, 1] < 0
    return np.unique(fc[b & np.isin(-1 - fc[:, 1], wall), 0])


@pytest.mark.parametrize("name", ["couette", "sphere_small", "couette_after_step"])
@pytest.mark.parametrize("dtype", [0, 1])
def test_poly_surface_matches_oracle(g, oracle_mod, name, dtype):
    """Surface quantities of the two-VDF gas (Sec. 4.2/4.3 with the internal
    energy of Sec. 2): kinetic wall cells whose f1 is out of equilibrium
    (T_r = 0.8 T, q_r != 0) and, on the sphere, NS wall cells beside them
    (every other wall cell switched to NS, T_r from the library's state); the
    Couette slab also after one GSIS outer iteration (the rows then sit in the
    other buffer).  The oracle takes the device's rows, W and T_r, so both
    sides sum the same numbers in FP64: 1e-10 of each column group's scale."""
    base = "couette" if name.startswith("couette") else name
    m, grid, Kn, W, flags = workload(base)
    flags = flags.copy()
    wc = _wall_cells(m)
    if base != "couette":
        flags[wc[::2]] = 0
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, dtype)
    kin = np.nonzero(flags)[0]
    case.set_state(W, vdf=_rows(grid, W[kin], 5, dtype), flags=flags)
    if name == "couette_after_step":
        case.step(g.SolveParams(mode=g.MODE_GSIS, n_macro_inner=20, cfl=0.5))
    Wg, fl = case.get_state()
    Wg, fl = Wg.cpu().numpy(), fl.cpu().numpy()
    Wo = np.concatenate([Wg, case.internal_temperature().cpu().numpy()[:, None]], 1)
    k = np.nonzero(fl)[0]
    slot = -np.ones(m["n_cells"], np.int64)
    slot[k] = np.arange(len(k))
    rows = case.get_vdf().cpu().numpy().astype(np.float64)
    faces_o, out_o = O.surface(rows, slot, Wo)
    faces, out, tot = case.surface()
    faces, out, tot = faces.cpu().numpy(), out.cpu().numpy(), tot.cpu().numpy()
    assert np.array_equal(faces, faces_o)
    scale_p = np.abs(out_o[:, 3]).max()
    scale_q = max(np.abs(out_o[:, 7]).max(), 1e-300)
    e_tau = np.abs(out[:, 0:7] - out_o[:, 0:7]).max() / scale_p
    e_q = np.abs(out[:, 7] - out_o[:, 7]).max() / scale_q
    e_m = np.abs(out[:, 8] - out_o[:, 8]).max() / scale_p
    S = m["face_area"][faces_o]
    tot_o = np.concatenate([(out_o[:, 0:3] * S[:, None]).sum(0), [(out_o[:, 7] * S).sum()]])
    e_tot = np.abs(tot - tot_o).max() / max(np.abs(tot_o).max(), 1e-300)
    n_kw = np.isin(wc, k).sum()
    print("poly surface", name, dtype, "wall cells", len(wc), "kinetic", n_kw, "tau", e_tau, "q", e_q, "mass", e_m,
          "totals", e_tot, flush=True)
    assert n_kw > 0 and (base == "couette" or n_kw < len(wc))
    assert e_tau < 1e-10 and e_q < 1e-10 and e_m < 1e-10 and e_tot < 1e-10


def test_poly_correction_alone(g, oracle_mod):
    """gsis_correct_internal (Sec. 3.1 eq. updatef with rho e_r in W) on the
    Couette slab, every cell kinetic, FP64: f0 += f_eq(W_new) - f_eq(W_half)
    and f1 += (d_r/4)(T_r,new f_eq(W_new) - T_r,half f_eq(W_half)), with the
    half state the rows' own moments and changes of a few percent (inside the
    correction limiter's range); rows, W and T_r against the oracle."""
    m, grid, Kn, W, _ = workload("couette")
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, g.F64)
    f0 = _rows(grid, W, 21, g.F64)
    mo = O.moments(f0)
    Wh = np.concatenate([mo[:, :5], mo[:, 14:15]], 1)
    case.set_state(Wh[:, :5], vdf=f0)
    Wn = Wh.copy()
    pert = gi.perturbation((len(Wn), 6), seed=22, amp=0.02)
    Wn[:, 0] *= pert[:, 0]
    Wn[:, 1:3] += 0.01 * (pert[:, 1:3] - 1)
    Wn[:, 4] *= pert[:, 4]
    Wn[:, 5] *= pert[:, 5]
    case.correct_internal(Wn[:, :5], Wn[:, 5])
    fo = np.stack([f0[i] + O.feq(Wn[i]) - O.feq(Wh[i]) for i in range(len(Wn))])
    ef = f_error(case.get_vdf().cpu().numpy(), fo, O.w)
    Wg = case.get_state()[0].cpu().numpy()
    Trg = case.internal_temperature().cpu().numpy()
    print("poly correction", ef, np.abs(Wg - Wn[:, :5]).max(), np.abs(Trg - Wn[:, 5]).max(), flush=True)
    assert ef < 1e-11
    # W and T_r become the new state (W_half + theta (W_new - W_half) with theta = 1:
    # equal up to the rounding of that form)
    assert np.abs(Wg - Wn[:, :5]).max() < 1e-13 and np.abs(Trg - Wn[:, 5]).max() < 1e-13
    ig = case.internal_moments().cpu().numpy()
    assert np.abs(ig[:, 0] - O.moments(fo)[:, 14]).max() < 1e-11


@pytest.mark.parametrize("name,cfl", [("sphere_small", 0.5), ("couette", -0.5)])
def test_poly_macro_solve_alone(g, oracle_mod, name, cfl):
    """gsis_macro_solve_internal (Sec. 2 eq. macroscopic_equation_2 with the
    internal-energy line, eq. macro): 60 pseudo-time steps from a field whose
    internal temperature is out of equilibrium, with seeded high-order terms
    (sigma, q_t, q_r) and sources, local steps on the sphere (walls, far
    field) and the global step on the Couette slab; W and T_r against the
    oracle's solve (FP64, 1e-10)."""
    m, grid, Kn, W, _ = workload(name)
    O, case = _pair(oracle_mod.Oracle, g, m, grid, Kn, g.F64)
    case.set_state(W)
    n = m["n_cells"]
    W6 = np.concatenate([W, (W[:, 4] * gi.perturbation((n,), seed=31, amp=0.1))[:, None]], 1)
    hot = 0.01 * (gi.perturbation((n, 12), seed=32, amp=1.0) - 1.0)
    src = 0.001 * (gi.perturbation((n, 6), seed=33, amp=1.0) - 1.0)
    Wo = O.macro(W6, hot, 60, cfl, src)
    Wg, Trg = case.macro_solve_internal(W6[:, :5], W6[:, 5], hot[:, :9], hot[:, 9:], src[:, :5], src[:, 5],
                                        n_inner=60, cfl=cfl)
    Wg, Trg = Wg.cpu().numpy(), Trg.cpu().numpy()
    err = {"rho": _rel(Wg[:, 0], Wo[:, 0]), "u": _rel(Wg[:, 1:4], Wo[:, 1:4], max(np.abs(Wo[:, 1:4]).max(), 1.0)),
           "T_t": _rel(Wg[:, 4], Wo[:, 4]), "T_r": _rel(Trg, Wo[:, 5])}
    moved = np.abs(Wo[:, 5] - W6[:, 5]).max()
    print("poly macro alone", name, cfl, err, "T_r moved", moved, flush=True)
    assert moved > 1e-4
    assert max(err.values()) < 1e-10, err
