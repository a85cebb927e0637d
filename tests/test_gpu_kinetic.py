"""GPU parity of the kinetic hot path against the FP64 oracle (via the C ABI).

One sweep from identical inputs (the FP32 runs start from FP32-rounded rows on
both sides); VDF compared per cell in the quadrature-weighted L2 norm, moments
per field (relative to the field's maximum).  Tolerances: FP32 1e-5, FP64 1e-11.
"""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import f_error, make_case, moment_errors, workload

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 1e-11}


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


def _setup(g, oracle_mod, name, dtype, seed=1):
    m, grid, Kn, W, flags = workload(name)
    O = oracle_mod.Oracle(m, grid, Kn)
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    f0 = gi.gaussian_rows(grid, W[kin], seed=seed, dtype=np.float32 if dtype == g.F32 else np.float64)
    f0 = f0.astype(np.float64)
    # W on kinetic cells is the moments of the VDF (both sides do this at set_state)
    W = W.copy()
    W[kin] = O.moments(f0)[:, :5]
    case = make_case(g, name, m, grid, Kn, dtype)
    case.set_state(W, vdf=f0, flags=flags)
    return m, grid, O, W, flags, kin, slot, f0, case


@pytest.mark.parametrize("name,dtype", [("couette", 1), ("couette", 0), ("couette:generic", 0),
                                        ("couette_ragged", 0), ("cavity", 0), ("cavity", 1),
                                        ("cavity:generic", 0), ("cylinder_small", 0), ("cylinder_fast", 0),
                                        ("cylinder_fast", 1), ("sphere_small", 0), ("sphere_small", 1),
                                        ("sphere_fast", 0), ("sphere_fast", 1), ("hexbox", 0), ("hexbox", 1)])
def test_one_sweep(g, oracle_mod, name, dtype):
    print("case", name, "dtype", dtype, flush=True)
    m, grid, O, W, flags, kin, slot, f0, case = _setup(g, oracle_mod, name, dtype)
    assert case.n_kin == len(kin)
    # inputs round-trip through the workspace unchanged
    assert np.array_equal(case.get_vdf().cpu().numpy().astype(np.float64), f0)
    ghost = O.ghost_params(W) if len(kin) < m["n_cells"] else None
    fo = O.sweep(f0, kin, slot, ghost)
    mo = O.moments(fo)
    case.sweep(1)
    fg = case.get_vdf().cpu().numpy()
    mg, kc = case.moments()
    assert np.array_equal(kc.cpu().numpy(), kin)
    ef = f_error(fg, fo, O.w)
    em = moment_errors(mg.cpu().numpy(), mo, u_scale=0.1)
    print(name, dtype, "f", ef, "moments", em, flush=True)
    assert ef < TOL[dtype]
    for k, v in em.items():
        assert v < TOL[dtype], (k, v)


def test_moments_of_filled_state(g, oracle_mod):
    """set_state without a VDF fills the conservation-fixed Maxwellian of W:
    its moments equal W exactly (FP64)."""
    m, grid, Kn, W, flags = workload("cylinder_small")
    case = g.Case(g.Mesh(m), grid, Kn, dtype=g.F64)
    case.set_state(W, flags=flags)
    mg, kc = case.moments()
    mg = mg.cpu().numpy()
    kc = kc.cpu().numpy()
    assert np.abs(mg[:, 0] / W[kc, 0] - 1).max() < 1e-12
    assert np.abs(mg[:, 1:3] - W[kc, 1:3]).max() < 1e-12
    assert np.abs(mg[:, 4] / W[kc, 4] - 1).max() < 1e-12
    O = oracle_mod.Oracle(m, grid, Kn)
    fo = np.stack([O.feq(W[c]) for c in kc[:50]])
    assert f_error(case.get_vdf().cpu().numpy()[:50], fo, O.w) < 1e-12


@pytest.mark.parametrize("specs", [[("couette_ragged:generic", 0), ("couette:generic", 0)],
                                   [("sphere_fast", 0), ("couette", 0)]])
def test_batched_equals_alone(g, oracle_mod, specs):
    """Cases swept in one batched launch give bitwise the results of separate launches
    (generic kernel: different grids; plane kernel: different meshes and regions)."""
    alone, mixed = [], []
    for _ in range(2):
        cs = []
        for name, dt in specs:
            m, grid, Kn, W, flags = workload(name)
            c = make_case(g, name, m, grid, Kn, dt)
            c.set_state(W, flags=flags)
            cs.append(c)
        if not alone:
            for c in cs:
                c.sweep(3)
            alone = [c.get_vdf().cpu().numpy() for c in cs]
        else:
            # specs list the case with the largest velocity axes first, as a batch requires
            g.kinetic_sweep(cs, 3)
            mixed = [c.get_vdf().cpu().numpy() for c in cs]
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)


def test_sweep_timing_and_errors(g):
    m, grid, Kn, W, flags = workload("couette")
    c = g.Case(g.Mesh(m), grid, Kn, dtype=g.F32)
    with pytest.raises(g.GsisError) as e:
        c.sweep(1)
    assert e.value.code == g.E_STATE
    Wbad = W.copy()
    Wbad[3, 4] = -1.0
    with pytest.raises(g.GsisError) as e:
        c.set_state(Wbad)
    assert e.value.code == g.E_NONFINITE
    c.set_state(W)
    c.sweep(2)
    assert c.last_sweep_ms() > 0
