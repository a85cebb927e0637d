"""Edge cases of the second-order and polyatomic paths: batched launches give
each case exactly its unbatched result; an empty kinetic region is a no-op;
a lone kinetic cell has no slope (the second-order sweep reduces to the
damped first-order one); the largest velocity axis (128 nodes) at second
order on the reduced grid and for the polyatomic gas on a 3D grid."""
import numpy as np
import pytest

import gsis_inputs as gi
from _cases import f_error, workload

pytestmark = pytest.mark.gpu

N2 = dict(dr=2.0, Zr=2.667, A=(0.786, -0.201, -0.059, 0.842))


@pytest.fixture(scope="module")
def g():
    import paper_2501_02245_amd as g
    import torch
    assert torch.cuda.is_available()
    return g


def _case(g, m, grid, Kn, dtype, kind):
    if kind == "order2":
        return g.Case(g.Mesh(m), grid, Kn, dtype=dtype, order=2)
    return g.Case(g.Mesh(m), grid, Kn, omega=0.74, Pr=N2["A"][0], dtype=dtype, **N2)


def _rows(grid, W, seed, kind, dtype):
    f0 = gi.gaussian_rows(grid, W, seed=seed, amp=0.2, dtype=np.float64)
    if kind == "poly":
        f1 = 0.25 * N2["dr"] * 0.9 * W[:, 4][:, None] * f0[:, 0] * gi.perturbation(f0[:, 0].shape, seed=seed + 1)
        f0 = np.stack([f0[:, 0], f1], axis=1)
    return f0.astype(np.float32 if dtype == 0 else np.float64)


@pytest.mark.parametrize("kind", ["order2", "poly"])
def test_batched_equals_alone(g, kind):
    """Two cases (different slabs, states and walls) swept in one batched launch
    produce bit for bit the rows each produces alone."""
    grid = gi.velocity_grid(3, 12, 5.0)
    specs = [(gi.couette_1d(24, 0.2), gi.random_W(24, seed=1, u_scale=0.2)),
             (gi.fourier_1d(16, 1.0, 1.3), gi.random_W(16, seed=2, u_scale=0.1))]
    outs_alone, batch = [], []
    for m, W in specs:
        rows = _rows(grid, W, 5, kind, 0)
        for store in (outs_alone, batch):
            c = _case(g, m, grid, 0.05, 0, kind)
            c.set_state(W, vdf=rows)
            store.append(c)
    for c in outs_alone:
        c.sweep(2)
    g.kinetic_sweep(batch, 2)
    for a, b in zip(outs_alone, batch):
        fa, fb = a.get_vdf().cpu().numpy(), b.get_vdf().cpu().numpy()
        assert np.array_equal(fa, fb)


@pytest.mark.parametrize("kind", ["order2", "poly"])
def test_empty_region_is_a_no_op(g, kind):
    m, grid, Kn, W, _ = workload("sphere_small")
    flags = np.zeros(m["n_cells"], np.uint8)
    case = _case(g, m, grid, Kn, 1, kind)
    case.set_state(W, flags=flags)
    case.sweep(2)
    mg, kc = case.moments()
    assert case.n_kin == 0 and kc.numel() == 0
    Wg = case.get_state()[0].cpu().numpy()
    assert np.array_equal(Wg, W)
    if kind == "poly":
        assert case.internal_moments().numel() == 0


@pytest.mark.parametrize("dtype", [0, 1])
def test_order2_lone_cell_has_no_slope(g, oracle_mod, dtype):
    """One kinetic cell inside an NS region: no kinetic neighbour, no slope;
    the second-order sweep is the first-order one plus the pseudo-time term,
    checked against the oracle (whose own pins make the no-slope case exact)."""
    m, grid, Kn, W, _ = workload("cylinder_small")
    flags = np.zeros(m["n_cells"], np.uint8)
    flags[m["n_cells"] // 2] = 1
    kin, slot, _ = oracle_mod.regions_from_flags(flags)
    O = oracle_mod.Oracle(m, grid, Kn, order=2)
    f0 = _rows(grid, W[kin], 8, "order2", dtype).astype(np.float64)
    W = W.copy()
    W[kin] = O.moments(f0)[:, :5]
    case = _case(g, m, grid, Kn, dtype, "order2")
    case.set_state(W, vdf=f0, flags=flags)
    ghost = O.ghost_params(W)
    assert np.all(O.slopes(f0, kin, slot) == 0.0)
    fo = O.sweep(f0, kin, slot, ghost)
    case.sweep(1)
    ef = f_error(case.get_vdf().cpu().numpy(), fo, O.w)
    print("lone cell order 2", dtype, ef, flush=True)
    assert ef < (1e-5 if dtype == 0 else 1e-11)


@pytest.mark.parametrize("kind", ["order2", "poly"])
def test_largest_axis(g, oracle_mod, kind):
    """128 nodes per velocity axis: second order on the reduced 2D grid of a
    small cavity, and the polyatomic gas on a 128 x 16 x 16 3D grid of a slab
    (FP64)."""
    if kind == "order2":
        m = gi.quad_cavity_2d(6, 5, 0.2)
        grid = gi.velocity_grid(2, 128, 8.0, "stretched")
        O = oracle_mod.Oracle(m, grid, 0.05, order=2)
    else:
        m = gi.couette_1d(6, 0.2)
        grid = gi.velocity_grid(3, [128, 16, 16], [8.0, 5.0, 5.0])
        O = oracle_mod.Oracle(m, grid, 0.05, omega=0.74, Pr=N2["A"][0], **N2)
    n = m["n_cells"]
    W = gi.random_W(n, seed=4, u_scale=0.2)
    f0 = _rows(grid, W, 9, kind, 1).astype(np.float64)
    W[:, :5] = O.moments(f0)[:, :5]
    case = _case(g, m, grid, 0.05, 1, kind)
    case.set_state(W, vdf=f0)
    kin = np.arange(n)
    fo = O.sweep(f0, kin, kin)
    case.sweep(1)
    ef = f_error(case.get_vdf().cpu().numpy(), fo, O.w)
    print("largest axis", kind, ef, flush=True)
    assert ef < 1e-11
