"""Parity-test workloads and comparison metrics (shared by the GPU tests).

Every input comes from gsis_inputs (seeded); expected values come from the
oracle only.
"""
import contextlib
import os

import numpy as np

import gsis_inputs as gi

MACH5 = 5.0 * np.sqrt(5.0 / 6.0)


@contextlib.contextmanager
def sweep_layout(generic):
    """Force the generic sweep kernel for cases bound inside the block."""
    old = os.environ.get("GSIS_GENERIC_SWEEP")
    if generic:
        os.environ["GSIS_GENERIC_SWEEP"] = "1"
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("GSIS_GENERIC_SWEEP", None)
        else:
            os.environ["GSIS_GENERIC_SWEEP"] = old


def make_case(g, name, m, grid, Kn, dtype, **kw):
    """Bind a case for workload `name`; a ':generic' suffix forces the generic
    sweep kernel.  The layout chosen is checked against the grid shape."""
    generic = name.endswith(":generic")
    with sweep_layout(generic):
        case = g.Case(g.Mesh(m), grid, Kn, dtype=dtype, **kw)
    n = [len(x) for x in grid["nodes"]]
    if grid["vdim"] == 3:
        can_fast = 256 % n[2] == 0 and (n[1] * n[2]) % 256 == 0
    else:
        can_fast = 256 % n[1] == 0
    assert case.sweep_layout()[0] == int(can_fast and not generic)
    return case


def workload(name):
    """(mesh, grid, Kn, W, flags) for a named parity case (':generic' ignored)."""
    name = name.split(":")[0]
    if name == "couette":          # the plain FP64 Couette configuration (64 cells, 16^3 on [-5,5])
        m = gi.couette_1d(64, 0.1)
        g = gi.velocity_grid(3, 16, 5.0)
        W = gi.couette_initial_W(64, seed=0)
        return m, g, 0.1, W, np.ones(64, np.uint8)
    if name == "couette_ragged":   # 20^3 = 8000 nodes: two 4096-node tiles with a ragged tail
        m = gi.couette_1d(16, 0.1)
        g = gi.velocity_grid(3, 20, 5.0)
        W = gi.random_W(16, seed=3, u_scale=0.2)
        return m, g, 0.05, W, np.ones(16, np.uint8)
    if name == "cavity":           # lid-driven cavity, reduced 32^2 stretched grid on [-6,6]
        m = gi.quad_cavity_2d(64, 64, 0.1)
        g = gi.velocity_grid(2, 32, 6.0, "stretched")
        W = gi.random_W(m["n_cells"], seed=5, u_scale=0.1, dT=0.05, drho=0.05)
        W[:, 3] = 0.0
        return m, g, 0.1, W, np.ones(m["n_cells"], np.uint8)
    if name == "cylinder_small":   # Mach 5 cylinder, partial kinetic region with NS neighbours
        m = gi.cylinder_tri_2d(n_theta=48, n_rings=14, free=(1.0, (MACH5, 0.0, 0.0), 1.0))
        g = gi.velocity_grid(2, 24, 15.0, "stretched")
        W = gi.hypersonic_field(m)
        W[:, 3] = 0.0
        fl = gi.synthetic_region(m, 0.3, seed=11)
        return m, g, 0.01, W, fl
    if name == "cylinder_fast":    # as cylinder_small on a 32^2 grid (plane kernel)
        m = gi.cylinder_tri_2d(n_theta=48, n_rings=14, free=(1.0, (MACH5, 0.0, 0.0), 1.0))
        g = gi.velocity_grid(2, 32, 15.0, "stretched")
        W = gi.hypersonic_field(m)
        W[:, 3] = 0.0
        fl = gi.synthetic_region(m, 0.3, seed=11)
        return m, g, 0.01, W, fl
    if name == "sphere_fast":      # as sphere_small on a 16^3 grid (plane kernel)
        m = gi.sphere_tet_3d(h_wall=0.25, growth=0.6, h_max=1.5)
        g = gi.velocity_grid(3, 16, 15.0, "stretched")
        W = gi.hypersonic_field(m)
        fl = gi.synthetic_region(m, 0.2, seed=11)
        return m, g, 0.005, W, fl
    if name == "hexbox":           # hexahedra (six faces per cell), walls and far field, partial region, 16^3
        m = gi.hex_box_3d(5, 5, 5)
        g = gi.velocity_grid(3, 16, 6.0)
        W = gi.random_W(m["n_cells"], seed=13, u_scale=0.2, dT=0.1, drho=0.1)
        fl = gi.synthetic_region(m, 0.5, seed=11)
        return m, g, 0.05, W, fl
    if name == "sphere_small":     # Mach 5 sphere, tetrahedra, partial region
        m = gi.sphere_tet_3d(h_wall=0.25, growth=0.6, h_max=1.5)
        g = gi.velocity_grid(3, 12, 15.0, "stretched")
        W = gi.hypersonic_field(m)
        fl = gi.synthetic_region(m, 0.2, seed=11)
        return m, g, 0.005, W, fl
    raise KeyError(name)


def f_error(fg, fo, w):
    """Relative error of the rows, the larger of two measures, maxed over cells:
    the quadrature-weighted L2 error of the cell's rows over their L2 norm, and
    the element-wise max |g - o| over the cell's largest |o| (so that an error
    on low-weight tail nodes cannot hide in the L2 norm)."""
    fg = np.asarray(fg, dtype=np.float64).reshape(fo.shape)
    num = np.sqrt(np.einsum("k,ijk->i", w, (fg - fo) ** 2))
    den = np.sqrt(np.einsum("k,ijk->i", w, fo ** 2))
    cells = fo.reshape(fo.shape[0], -1)
    pw = np.abs(fg.reshape(cells.shape) - cells).max(axis=1) / np.abs(cells).max(axis=1)
    return float(max(np.max(num / den), np.max(pw)))


def moment_errors(mg, mo, u_scale=0.0):
    """Per-field error max_i |g - o| / max_i |o| (u divided by max(max|u|, u_scale)),
    and per cell ("*_cell"): rho and T relative to the cell's value, u to the
    cell's thermal speed sqrt(T), sigma to its pressure p = rho T and q to
    p sqrt(T), maxed over cells (a field that is small somewhere is still held
    to its physical scale there)."""
    mg = np.asarray(mg)
    out = {}
    for name, sl in (("rho", [0]), ("u", [1, 2, 3]), ("T", [4]), ("sigma", list(range(5, 11))),
                     ("q", [11, 12, 13])):
        d = np.abs(mg[:, sl] - mo[:, sl]).max()
        s = np.abs(mo[:, sl]).max()
        if name == "u":
            s = max(s, u_scale)
        out[name] = d / s if s > 0 else d
    rho, T = mo[:, 0], mo[:, 4]
    p = rho * T
    for name, sl, scale in (("rho_cell", [0], rho), ("u_cell", [1, 2, 3], np.sqrt(T)), ("T_cell", [4], T),
                            ("sigma_cell", list(range(5, 11)), p), ("q_cell", [11, 12, 13], p * np.sqrt(T))):
        out[name] = float((np.abs(mg[:, sl] - mo[:, sl]).max(axis=1) / scale).max())
    return out
