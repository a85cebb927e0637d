"""GPU parity of the surface quantities (Sec. 4.2/4.3: wall stress, pressure,
heat flux, integrated force and heat) against the FP64 oracle, via the C ABI.

The oracle takes exactly the device's VDF rows (FP32 rows widened to FP64) and
macroscopic state, so both sides sum the same numbers in FP64: tolerance
1e-10 of the column group's scale.  Workloads mix kinetic and NS wall cells
(every other wall cell of the region is switched to NS), and the last test
takes the state left by a full outer iteration (the VDF then sits in the
other buffer).
"""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import make_case, workload

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


def _wall_cells(m):
    fc = m["face_cells"]
    wall = [p for p, pt in enumerate(m["patches"]) if pt["kind"] == "wall"]
    b = fc[:, 1] < 0
    return np.unique(fc[b & np.isin(-1 - fc[:, 1], wall), 0])


def _compare(O, case, m):
    kin, slot, _ = None, None, None
    W, fl = case.get_state()
    W, fl = W.cpu().numpy(), fl.cpu().numpy()
    kin = np.nonzero(fl)[0]
    slot = -np.ones(m["n_cells"], np.int64)
    slot[kin] = np.arange(len(kin))
    rows = case.get_vdf().cpu().numpy().astype(np.float64) if len(kin) else np.zeros((0, O.nfun, O.nv))
    faces_o, out_o = O.surface(rows, slot, W)
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
    print("surface errors: tau/p/shear", e_tau, "q", e_q, "mass", e_m, "totals", e_tot, flush=True)
    assert e_tau < TOL and e_q < TOL and e_m < TOL and e_tot < TOL
    return kin, slot


@pytest.mark.parametrize("name,dtype", [("couette", 1), ("couette", 0), ("cylinder_small", 0), ("cylinder_fast", 1),
                                        ("sphere_fast", 0)])
def test_surface_matches_oracle(g, oracle_mod, name, dtype):
    m, grid, Kn, W, flags = workload(name)
    flags = flags.copy()
    wc = _wall_cells(m)
    if name != "couette":
        flags[wc[::2]] = 0     # NS wall cells beside kinetic ones
    O = oracle_mod.Oracle(m, grid, Kn)
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    f0 = gi.gaussian_rows(grid, W[kin], seed=4, dtype=np.float32 if dtype == g.F32 else np.float64)
    case = make_case(g, name, m, grid, Kn, dtype)
    case.set_state(W, vdf=f0.astype(np.float64), flags=flags)
    k, _ = _compare(O, case, m)
    n_kw = np.isin(wc, k).sum()
    print(name, "wall cells", len(wc), "kinetic", n_kw, flush=True)
    assert n_kw > 0 and (name == "couette" or n_kw < len(wc))


def test_surface_after_step(g, oracle_mod):
    m, grid, Kn, W, flags = workload("cylinder_fast")
    O = oracle_mod.Oracle(m, grid, Kn)
    case = make_case(g, "cylinder_fast", m, grid, Kn, g.F32)
    case.set_state(W, flags=flags)
    case.step(g.SolveParams(mode=g.MODE_AGSIS, n_macro_inner=20, cfl=0.5, force_wall_layers=2))
    _compare(O, case, m)


def test_force_coefficients_hand_computed(g):
    """gsis_force_coefficients on totals with known answers: free stream along
    (3, 4, 0)/5 at rho 2, area 0.5, so rho |u|^2 A = 25 and C_h divides by 125:
    F = (3, 4, 0) gives C_d = 5/25 and C_l = 0; F = (-4, 3, 7) gives C_d = 0,
    C_l = 5/25 (F_z plays no part); Q = 10 gives C_h = 10/125; bad inputs are
    refused."""
    u = (3.0, 4.0, 0.0)
    c = g.force_coefficients([3.0, 4.0, 0.0, 10.0], 2.0, u, 0.5)
    assert abs(c["C_d"] - 0.2) < 1e-15 and abs(c["C_l"]) < 1e-15 and abs(c["C_h"] - 0.08) < 1e-15
    c = g.force_coefficients([-4.0, 3.0, 7.0, 0.0], 2.0, u, 0.5)
    assert abs(c["C_d"]) < 1e-15 and abs(c["C_l"] - 0.2) < 1e-15 and c["C_h"] == 0.0
    for bad in ((2.0, (0.0, 0.0, 0.0), 0.5), (0.0, u, 0.5), (2.0, u, 0.0)):
        with pytest.raises(g.GsisError):
            g.force_coefficients([1.0, 0.0, 0.0, 0.0], *bad)
