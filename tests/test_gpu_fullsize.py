"""Parity at the benchmark size and in the launch configuration the benchmark
times: Mach-5 sphere, 192,445 tetrahedra, 32^3 stretched velocities, FP32,
capacity 0.7 n_cells (one whole-row tile per kinetic cell, plane kernel,
4-face template).  About 45% of the cells are kinetic (87k rows, 11 GB).
The second-order and polyatomic legs are checked the same way in their own
launch configuration (capacity n_kin + 64).

The oracle cannot sweep 2.8e9 points in a test, so one sweep is compared on
48 sampled kinetic cells (random ones, wall cells, cells next to the NS
region and to the far field), each recomputed from exactly the same FP32
input rows; the GSIS correction is checked by a property that holds at any
size (the conserved moments of the corrected VDF are the new W) and on
sampled cells against the oracle.
"""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import f_error, moment_errors

pytestmark = pytest.mark.gpu

KN = 0.005
CAP_FRACTION = 0.7     # the benchmark's capacity rule
SEED_ROWS = 21


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


@pytest.fixture(scope="module")
def big(g):
    import torch
    mesh, grid, W = gi.sphere_workload(32)
    flags = gi.synthetic_region(mesh, 0.45, seed=11)
    kin = np.nonzero(flags)[0]
    print("sphere", mesh["n_cells"], "cells,", len(kin), "kinetic", flush=True)
    ax, ay, az = gi.separable_row_factors(grid, W, kin, seed=SEED_ROWS)
    case = g.Case(g.Mesh(mesh), grid, KN, dtype=g.F32, capacity=int(CAP_FRACTION * mesh["n_cells"]))
    assert case.sweep_layout() == (1, 32768, 1)
    # assemble the rows on the device with the same FP32 products, in the same
    # association order, as gi.assemble_separable_rows
    tx, ty, tz = (torch.from_numpy(a).cuda() for a in (ax, ay, az))
    rows = ((tx[:, :, None, None] * ty[:, None, :, None]) * tz[:, None, None, :]).reshape(len(kin), 1, -1)
    case.set_state(W, vdf=rows, flags=flags)
    del rows, tx, ty, tz
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"mesh": mesh, "grid": grid, "W": W, "flags": flags, "kin": kin, "case": case}


def _sample(mesh, flags, kin, seed=5):
    """16 random kinetic cells, 16 with a wall face, 16 next to an NS cell or the far field."""
    fc = mesh["face_cells"]
    rng = np.random.Generator(np.random.PCG64(seed))
    wall_p = {p for p, pt in enumerate(mesh["patches"]) if pt["kind"] == "wall"}
    bnd = fc[:, 1] < 0
    wall_cells = set(fc[bnd & np.isin(-1 - fc[:, 1], list(wall_p)), 0].tolist())
    far_cells = set(fc[bnd & ~np.isin(-1 - fc[:, 1], list(wall_p)), 0].tolist())
    inner = ~bnd
    a, b = fc[inner, 0], fc[inner, 1]
    edge = set(a[(flags[a] == 1) & (flags[b] == 0)].tolist()) | set(b[(flags[b] == 1) & (flags[a] == 0)].tolist())
    kset = set(kin.tolist())
    picks = set(rng.choice(kin, 16, replace=False).tolist())
    for pool in (sorted(wall_cells & kset), sorted((edge | far_cells) & kset)):
        pool = [c for c in pool if c not in picks]
        picks |= set(rng.choice(pool, min(16, len(pool)), replace=False).tolist())
    return np.array(sorted(picks), dtype=np.int64)


def _neighbours(mesh, cells):
    fc = mesh["face_cells"]
    inner = fc[:, 1] >= 0
    a, b = fc[inner, 0], fc[inner, 1]
    m = np.zeros(mesh["n_cells"], bool)
    m[cells] = True
    return np.union1d(b[m[a]], a[m[b]])


def test_fullsize_sweep_sampled(g, oracle_mod, big):
    import torch
    mesh, grid, W, flags, kin, case = (big[k] for k in ("mesh", "grid", "W", "flags", "kin", "case"))
    sample = _sample(mesh, flags, kin)
    pos = np.searchsorted(kin, sample)
    print("sampled", len(sample), "cells", flush=True)
    # rows the oracle needs: the sample, its kinetic neighbours, and the kinetic
    # neighbours of its NS neighbours (their moments enter the ghosts' gradients)
    nb = _neighbours(mesh, sample)
    ns_nb = nb[flags[nb] == 0]
    need = np.union1d(np.union1d(sample, nb[flags[nb] == 1]), _neighbours(mesh, ns_nb))
    need = need[flags[need] == 1]
    axs = gi.separable_row_factors(grid, W, need, seed=SEED_ROWS)
    rows32 = gi.assemble_separable_rows(*axs)
    # the device holds exactly these inputs
    fg0 = case.get_vdf()
    idx = torch.from_numpy(np.searchsorted(kin, need)).cuda()
    assert np.array_equal(fg0[idx].cpu().numpy(), rows32)
    del fg0
    torch.cuda.empty_cache()

    O = oracle_mod.Oracle(mesh, grid, KN)
    rows = rows32.astype(np.float64)
    Wo = W.copy()
    Wo[need] = O.moments(rows)[:, :5]
    ghost = O.ghost_params(Wo)
    slot = -np.ones(mesh["n_cells"], np.int32)
    slot[need] = np.arange(len(need), dtype=np.int32)
    fo = O.sweep(rows, sample, slot, ghost)[slot[sample]]
    mo = O.moments(fo)

    case.sweep(1)
    fg = case.get_vdf()
    fs = fg[torch.from_numpy(pos).cuda()].cpu().numpy()
    del fg
    torch.cuda.empty_cache()
    mg, kc = case.moments()
    assert np.array_equal(kc.cpu().numpy(), kin)
    ms = mg.cpu().numpy()[pos]
    ef = f_error(fs, fo, O.w)
    em = moment_errors(ms, mo, u_scale=1.0)
    print("full size: f", ef, "moments", em, flush=True)
    assert ef < 1e-5
    for k, v in em.items():
        assert v < 1e-5, (k, v)


def test_fullsize_correction_sampled(g, oracle_mod, big):
    """GSIS correction at the benchmark size, in the benchmark's launch
    configuration: f += f_eq(W_new) - f_eq(W_half) with fixed-up Maxwellians
    and the correction limiter, from the generator's rows.  The sampled cells
    are recomputed by the oracle from the same FP32 rows and the same W_new;
    on every kinetic cell the conserved moments of the result are W_new (FP32
    storage)."""
    import torch
    mesh, grid, W, flags, kin, case = (big[k] for k in ("mesh", "grid", "W", "flags", "kin", "case"))
    # reset to the generator's rows (earlier tests swept them)
    ax, ay, az = gi.separable_row_factors(grid, W, kin, seed=SEED_ROWS)
    tx, ty, tz = (torch.from_numpy(a).cuda() for a in (ax, ay, az))
    rows = ((tx[:, :, None, None] * ty[:, None, :, None]) * tz[:, None, None, :]).reshape(len(kin), 1, -1)
    case.set_state(W, vdf=rows, flags=flags)
    del rows, tx, ty, tz
    torch.cuda.empty_cache()
    n = mesh["n_cells"]
    ph = np.arange(n, dtype=np.float64)
    Wn = W.copy()
    Wn[:, 0] *= 1.0 + 0.01 * np.sin(ph)
    Wn[:, 1:4] += 0.01 * np.cos(ph)[:, None]
    Wn[:, 4] *= 1.0 + 0.01 * np.cos(0.7 * ph)
    case.correct(Wn)
    mg, kc = case.moments()
    mg = mg.cpu().numpy()
    sample = _sample(mesh, flags, kin, seed=8)
    pos = np.searchsorted(kin, sample)
    fg = case.get_vdf()
    fs = fg[torch.from_numpy(pos).cuda()].cpu().numpy()
    del fg
    torch.cuda.empty_cache()
    # oracle: the same rows, its own W_half, the same W_new through its limiter
    O = oracle_mod.Oracle(mesh, grid, KN)
    f = gi.assemble_separable_rows(*gi.separable_row_factors(grid, W, sample, seed=SEED_ROWS)).astype(np.float64)
    Wh = O.moments(f)[:, :5]
    fo = np.empty_like(f)
    Wk = np.empty((len(sample), 5))
    cut = 0
    for j, c in enumerate(sample):
        Wk[j], th = oracle_mod.limit_correction(Wh[j], Wn[c], with_theta=True)
        cut += th < 1.0
        fo[j] = f[j] + O.feq(Wk[j]) - O.feq(Wh[j])
    ef = f_error(fs, fo, O.w)
    em = moment_errors(mg[pos], O.moments(fo), u_scale=1.0)
    print("full size correction: f", ef, "moments", em, "limited", cut, flush=True)
    assert ef < 1e-5
    for k, v in em.items():
        assert v < 1e-5, (k, v)
    # every kinetic cell: the conserved moments are W_new (none is limited here)
    assert cut == 0
    Wk = Wn[kin]
    err_rho = np.abs(mg[:, 0] / Wk[:, 0] - 1).max()
    err_u = np.abs(mg[:, 1:4] - Wk[:, 1:4]).max()
    err_T = np.abs(mg[:, 4] / Wk[:, 4] - 1).max()
    print("correction property: rho", err_rho, "u", err_u, "T", err_T, flush=True)
    assert err_rho < 1e-5 and err_u < 1e-5 and err_T < 1e-5


def _need_for(mesh, flags, cells):
    """Kinetic cells whose rows the oracle needs to sweep `cells`: the cells,
    their kinetic neighbours, and the kinetic neighbours of their NS neighbours
    (whose moments enter the ghosts' gradients)."""
    nb = _neighbours(mesh, cells)
    ns_nb = nb[flags[nb] == 0]
    need = np.union1d(np.union1d(cells, nb[flags[nb] == 1]), _neighbours(mesh, ns_nb))
    return need[flags[need] == 1]


def test_fullsize_order2_sweep_sampled(g, oracle_mod, big):
    """Second-order face values at the benchmark size: one sweep (slope kernel
    and faces-as-rows sweep) on the sampled cells.  The oracle's slopes of the
    sample and of its kinetic neighbours come from their full stencils."""
    import torch
    mesh, grid, W, flags, kin = (big[k] for k in ("mesh", "grid", "W", "flags", "kin"))
    sample = _sample(mesh, flags, kin, seed=6)
    pos = np.searchsorted(kin, sample)
    nb = _neighbours(mesh, sample)
    slope_cells = np.union1d(sample, nb[flags[nb] == 1])
    need = np.union1d(_need_for(mesh, flags, sample), _need_for(mesh, flags, slope_cells))
    print("order 2: sampled", len(sample), "cells,", len(need), "rows", flush=True)
    case = g.Case(g.Mesh(mesh), grid, KN, dtype=g.F32, capacity=len(kin) + 64, order=2)
    ax, ay, az = gi.separable_row_factors(grid, W, kin, seed=SEED_ROWS)
    tx, ty, tz = (torch.from_numpy(a).cuda() for a in (ax, ay, az))
    rows = ((tx[:, :, None, None] * ty[:, None, :, None]) * tz[:, None, None, :]).reshape(len(kin), 1, -1)
    case.set_state(W, vdf=rows, flags=flags)
    del rows, tx, ty, tz
    torch.cuda.empty_cache()
    rows32 = gi.assemble_separable_rows(*gi.separable_row_factors(grid, W, need, seed=SEED_ROWS))
    O = oracle_mod.Oracle(mesh, grid, KN, order=2)
    f = rows32.astype(np.float64)
    Wo = W.copy()
    Wo[need] = O.moments(f)[:, :5]
    ghost = O.ghost_params(Wo)
    slot = -np.ones(mesh["n_cells"], np.int32)
    slot[need] = np.arange(len(need), dtype=np.int32)
    sl = O.slopes(f, slope_cells, slot)
    fo = O.sweep(f, sample, slot, ghost, slope=sl)[slot[sample]]
    case.sweep(1)
    fg = case.get_vdf()
    fs = fg[torch.from_numpy(pos).cuda()].cpu().numpy()
    del fg
    mg, _ = case.moments()
    ms = mg.cpu().numpy()[pos]
    case.close()
    del case
    torch.cuda.empty_cache()
    ef = f_error(fs, fo, O.w)
    em = moment_errors(ms, O.moments(fo), u_scale=1.0)
    print("full size order 2: f", ef, "moments", em, flush=True)
    assert ef < 1e-5
    for k, v in em.items():
        assert v < 1e-5, (k, v)


def test_fullsize_poly_sweep_sampled(g, oracle_mod, big):
    """The polyatomic gas (nitrogen) at the benchmark size: one sweep of
    (f0, f1) on the sampled cells, f1 = theta_i f0 with a per-cell factor
    (internal modes at 0.8 T), formed in FP32 on both sides."""
    import torch
    mesh, grid, W, flags, kin = (big[k] for k in ("mesh", "grid", "W", "flags", "kin"))
    sample = _sample(mesh, flags, kin, seed=7)
    pos = np.searchsorted(kin, sample)
    need = _need_for(mesh, flags, sample)
    print("poly: sampled", len(sample), "cells,", len(need), "rows", flush=True)
    A = (0.786, -0.201, -0.059, 0.842)
    case = g.Case(g.Mesh(mesh), grid, KN, omega=0.74, Pr=A[0], dtype=g.F32, capacity=len(kin) + 64,
                  dr=2.0, Zr=2.667, A=A)
    theta = (0.25 * 2.0 * 0.8 * W[:, 4]).astype(np.float32)
    ax, ay, az = gi.separable_row_factors(grid, W, kin, seed=SEED_ROWS)
    tx, ty, tz = (torch.from_numpy(a).cuda() for a in (ax, ay, az))
    r0 = ((tx[:, :, None, None] * ty[:, None, :, None]) * tz[:, None, None, :]).reshape(len(kin), 1, -1)
    th = torch.from_numpy(theta[kin]).cuda()
    rows = torch.cat([r0, r0 * th[:, None, None]], dim=1)
    del r0, tx, ty, tz
    case.set_state(W, vdf=rows, flags=flags)
    del rows
    torch.cuda.empty_cache()
    f0 = gi.assemble_separable_rows(*gi.separable_row_factors(grid, W, need, seed=SEED_ROWS))[:, 0]
    f1 = f0 * theta[need][:, None]
    f = np.stack([f0, f1], axis=1).astype(np.float64)
    O = oracle_mod.Oracle(mesh, grid, KN, omega=0.74, Pr=A[0], dr=2.0, Zr=2.667, A=A)
    # T_r of every cell as the library holds it: T_t on NS cells, that of f1
    # on kinetic ones (it enters the NS ghosts' T_r gradients)
    Wo = np.concatenate([W, W[:, 4:5]], 1)
    mf = O.moments(f)
    Wo[need, :5] = mf[:, :5]
    Wo[need, 5] = mf[:, 14]
    ghost = O.ghost_params(Wo)
    slot = -np.ones(mesh["n_cells"], np.int32)
    slot[need] = np.arange(len(need), dtype=np.int32)
    fo = O.sweep(f, sample, slot, ghost)[slot[sample]]
    case.sweep(1)
    fg = case.get_vdf()
    fs = fg[torch.from_numpy(pos).cuda()].cpu().numpy()
    del fg
    mg, _ = case.moments()
    ms = mg.cpu().numpy()[pos]
    ig = case.internal_moments().cpu().numpy()[pos]
    case.close()
    del case
    torch.cuda.empty_cache()
    mo = O.moments(fo)
    ef = f_error(fs, fo, O.w)
    em = moment_errors(ms, mo[:, :14], u_scale=1.0)
    eTr = np.abs(ig[:, 0] - mo[:, 14]).max() / np.abs(mo[:, 14]).max()
    print("full size poly: f", ef, "moments", em, "T_r", eTr, flush=True)
    assert ef < 1e-5 and eTr < 1e-5
    for k, v in em.items():
        assert v < 1e-5, (k, v)
