"""Pins of the oracle's relaxation time, convergence measure and limiters.

- tau = mu / p_t with the Kn definition of Sec. 2 and mu ~ T^omega: the
  converged kinetic solution of a sheared, heated slab at Kn = 0.01 must show
  the Newton and Fourier laws (Sec. 2 eq. NSF_constitutive) with the
  viscosity that the Kn definition fixes (the continuum limit; Chapman-Enskog).
- eps of Sec. 4 eq. convergence_critertion: hand-computed values on three cells.
- the correction limiter (reading R24): pass-through, halving in conserved
  variables, and the drop after ten halvings, with hand-computed results.
- the Grad-13 range limiter (reading R19b): an explicit parameter; inactive on
  smooth fields and on the parity workloads; exact scaling when active.
"""
import math

import numpy as np
import pytest

import gsis_inputs as gi
from _cases import workload


# ---------------------------------------------------------------------------
# tau: continuum limit (Sec. 2: tau = mu / p_t, mu = mu(T0) (T/T0)^omega,
# Kn = mu(T0) sqrt(pi R T0 / 2) / (p0 L))
# ---------------------------------------------------------------------------
def test_continuum_limit_fixes_tau_viscosity_law_and_prandtl(oracle_mod):
    """Slab between diffuse walls at T = 1 (moving -0.1) and T = 2 (moving
    +0.1), Kn = 0.01, omega = 0.74.  In scaled units (lengths / L, velocities
    / sqrt(2 R T0), stress / p0, heat flux / (p0 sqrt(2 R T0))) the Kn
    definition gives mu(T0) sqrt(2 R T0) / (p0 L) = 2 Kn / sqrt(pi), so away
    from the Knudsen layers the kinetic solution must satisfy

        sigma_xy = -(2 Kn / sqrt(pi)) T^omega du_y/dx,
        q_x      = -(5 Kn / (2 sqrt(pi) Pr)) T^omega dT/dx    (kappa = (mu R / 2) 5 / A_tt, Pr = A_tt = 2/3)

    to O(Kn).  The temperature doubles across the slab, so a wrong exponent
    of T in tau (or a tau off by any constant factor) fails pointwise.  The
    state is the GSIS fixed point, which equals the plain-DVM fixed point
    (pinned separately); sigma and q are the moments of the kinetic rows."""
    n, Kn, om = 30, 0.01, 0.74
    m = gi.slab_1d(n, gi._patch("wall", u=(0.0, -0.1, 0.0), T=1.0), gi._patch("wall", u=(0.0, 0.1, 0.0), T=2.0))
    g = gi.velocity_grid(3, 14, 6.0)
    O = oracle_mod.Oracle(m, g, Kn, omega=om)
    S = oracle_mod.SteadySolver(O, mode="gsis", n_inner=400, cfl=0.5)
    W0 = gi.uniform_W(n)
    W0[:, 4] = 1.0 + m["cell_center"][:, 0]
    S.set_state(W0)
    it, eps = S.solve(tol=1e-9, max_iter=600)
    assert eps.max() < 1e-9, (it, eps)
    mom = O.moments(S.f[S.slot[S.kin]])
    x = m["cell_center"][:, 0]
    uy, T, sxy, qx = mom[:, 2], mom[:, 4], mom[:, 8], mom[:, 11]
    i = np.arange(n)[(x > 0.2) & (x < 0.8)]
    dudx = (uy[i + 1] - uy[i - 1]) / (x[i + 1] - x[i - 1])
    dTdx = (T[i + 1] - T[i - 1]) / (x[i + 1] - x[i - 1])
    pred_s = -2.0 * Kn / math.sqrt(math.pi) * T[i] ** om * dudx
    pred_q = -5.0 * Kn / (2.0 * math.sqrt(math.pi) * (2.0 / 3.0)) * T[i] ** om * dTdx
    assert T.max() / T.min() > 1.8
    assert np.abs(sxy[i] / pred_s - 1.0).max() < 1e-2
    assert np.abs(qx[i] / pred_q - 1.0).max() < 1e-2
    # tau itself at one state: mu / p_t in scaled units
    assert abs(O.tau(1.3, 1.7) - 2.0 * Kn / math.sqrt(math.pi) * 1.7 ** om / (1.3 * 1.7)) < 1e-15


# ---------------------------------------------------------------------------
# eps (Sec. 4 eq. convergence_critertion)
# ---------------------------------------------------------------------------
def _three_cell_oracle(oracle_mod, volumes):
    m = gi.couette_1d(3, 0.0)
    m["cell_volume"] = np.asarray(volumes, dtype=np.float64)
    return oracle_mod.Oracle(m, gi.velocity_grid(3, 4, 4.0), Kn=0.1)


def test_residual_hand_computed(oracle_mod):
    """Volumes (1, 2, 1).
    rho: old (1, 1, 2), new (1.1, 0.9, 2): sum dr^2 V = 0.01 + 0.02 = 0.03,
         sum r^2 V = 1 + 2 + 4 = 7, eps = sqrt(3/700).
    u (as a vector): old (1,0,0), (0,2,0), (0,0,0); new (1,0,0.3), (0,2,0), (0.4,0,0):
         sum |du|^2 V = 0.09 + 0 + 0.16 = 0.25, sum |u|^2 V = 1 + 8 + 0 = 9, eps = 1/6.
         (Taken per component, z would have a zero denominator: the vector form
         is the reading.)
    T: old (1, 1, 1), new (1, 1.2, 1): 0.04 * 2 / 4 = 0.02, eps = sqrt(0.02)."""
    O = _three_cell_oracle(oracle_mod, (1.0, 2.0, 1.0))
    Wo = np.array([[1.0, 1.0, 0.0, 0.0, 1.0], [1.0, 0.0, 2.0, 0.0, 1.0], [2.0, 0.0, 0.0, 0.0, 1.0]])
    Wn = np.array([[1.1, 1.0, 0.0, 0.3, 1.0], [0.9, 0.0, 2.0, 0.0, 1.2], [2.0, 0.4, 0.0, 0.0, 1.0]])
    e = O.residual(Wn, Wo)
    assert abs(e[0] - math.sqrt(3.0 / 700.0)) < 1e-15
    assert abs(e[1] - 1.0 / 6.0) < 1e-15
    assert abs(e[2] - math.sqrt(0.02)) < 1e-15
    # from a gas at rest the velocity denominator vanishes and the absolute
    # change is used: sum |u_new|^2 V = 1.09 + 8 + 0.16 = 9.25
    Wo[:, 1:4] = 0.0
    e0 = O.residual(Wn, Wo)
    assert abs(e0[1] - math.sqrt(9.25)) < 1e-15
    assert O.residual(Wo, Wo).max() == 0.0


# ---------------------------------------------------------------------------
# correction limiter (reading R24)
# ---------------------------------------------------------------------------
def test_limit_correction_passes_changes_within_range(oracle_mod):
    Wh = np.array([1.0, 0.2, -0.1, 0.0, 1.0])
    for Wn in (np.array([1.9, 0.3, 0.0, 0.05, 0.6]), np.array([0.55, -0.4, 0.2, 0.0, 1.95])):
        W, th = oracle_mod.limit_correction(Wh, Wn, with_theta=True)
        assert th == 1.0
        assert np.allclose(W, Wn, rtol=1e-14, atol=1e-15)


def test_limit_correction_halves_in_conserved_variables(oracle_mod):
    """Wh = (1, 0, 0, 0, 1) [U = (1, 0, 0, 0, 1.5)], Wn = (5, 1, 0, 0, 1)
    [U = (5, 5, 0, 0, 12.5)]: theta 1 and 1/2 give rho 5 and 3 (> 2), theta
    1/4 gives U = (2, 1.25, 0, 0, 4.25), i.e. u = 0.625, T = (4.25 - 2 *
    0.625^2) / 3 = 1.15625: inside the range, kept."""
    Wh = np.array([1.0, 0.0, 0.0, 0.0, 1.0])
    Wn = np.array([5.0, 1.0, 0.0, 0.0, 1.0])
    W, th = oracle_mod.limit_correction(Wh, Wn, with_theta=True)
    assert th == 0.25
    assert np.array_equal(W, np.array([2.0, 0.625, 0.0, 0.0, 1.15625]))
    # a temperature-driven cut: T 1 -> 3 at rest needs one halving (T = 2)
    W, th = oracle_mod.limit_correction(Wh, np.array([1.0, 0.0, 0.0, 0.0, 3.0]), with_theta=True)
    assert th == 0.5 and np.array_equal(W, np.array([1.0, 0.0, 0.0, 0.0, 2.0]))


def test_limit_correction_drops_after_ten_halvings(oracle_mod):
    """rho 1 -> 1e4: even theta = 2^-10 gives rho = 1 + 9999/1024 > 2, so the
    change is dropped and W^{n+1/2} is kept."""
    Wh = np.array([1.0, 0.1, 0.0, 0.0, 1.0])
    W, th = oracle_mod.limit_correction(Wh, np.array([1e4, 0.1, 0.0, 0.0, 1.0]), with_theta=True)
    assert th == 0.0 and np.array_equal(W, Wh)


# ---------------------------------------------------------------------------
# Grad-13 range limiter (reading R19b)
# ---------------------------------------------------------------------------
def test_g13_limiter_parameter_and_exact_scaling(oracle_mod):
    """Unlimited (g13_rmax None) the parameters are the NSF values; with a
    limit rmax the limited rows have r = rmax exactly and the others are
    untouched; the flagged cells are exactly those with r_NSF > rmax."""
    m = gi.couette_1d(12, wall_speed=0.0)
    g = gi.velocity_grid(3, 12, 6.0)
    x = m["cell_center"][:, 0]
    W = np.zeros((12, 5))
    W[:, 0] = 1.0
    W[:, 2] = 0.3 * np.sin(2 * np.pi * x)
    W[:, 4] = 1.0 + 0.15 * x
    O = oracle_mod.Oracle(m, g, Kn=0.3, g13_rmax=None)
    raw = O.nsf_field(W)
    gh = O.ghost_params(W)
    assert not O.last_g13_limited.any()
    assert np.array_equal(gh[:, 5:11], raw[:, :6]) and np.array_equal(gh[:, 11:], raw[:, 6:])
    p = W[:, 0] * W[:, 4]
    r_raw = np.maximum(np.abs(raw[:, :6]).max(1) / p, np.linalg.norm(raw[:, 6:], axis=1) / (p * np.sqrt(W[:, 4])))
    for rmax in (0.3, 0.45):
        O.g13_rmax = rmax
        gl = O.ghost_params(W)
        lim = O.last_g13_limited
        assert np.array_equal(lim, r_raw > rmax) and lim.any() and not lim.all()
        r = np.maximum(np.abs(gl[:, 5:11]).max(1) / p, np.linalg.norm(gl[:, 11:], axis=1) / (p * np.sqrt(W[:, 4])))
        assert np.allclose(r[lim], rmax, rtol=1e-13)
        assert np.array_equal(gl[~lim], gh[~lim])


def test_g13_limiter_inactive_on_parity_workloads_and_smooth_runs(oracle_mod):
    """Where the Grad-13 rows are used by the parity tests the limiter does not
    fire: the ghost cells of the Mach-5 cylinder and sphere workloads with
    their seeded regions (the limiter does act on some shock cells of the
    cylinder that are not ghosts).  A near-continuum Couette slab run in aGSIS
    mode (NS start, 22 of 24 cells flagged, region update every iteration)
    scales no new-cell or ghost row and cuts no correction."""
    for name, any_limited in (("cylinder_small", True), ("sphere_small", False)):
        m, g, Kn, W, fl = workload(name)
        O = oracle_mod.Oracle(m, g, Kn)
        S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=0.01)
        S.set_state(W, flags=fl)
        O.ghost_params(S.W)
        gc = S.ghost_cells()
        assert len(gc) > 100
        assert O.last_g13_limited[gc].sum() == 0
        assert O.last_g13_limited.any() == any_limited
    m = gi.couette_1d(24, 0.1)
    O = oracle_mod.Oracle(m, gi.velocity_grid(3, 12, 5.0), 0.01)
    S = oracle_mod.SteadySolver(O, mode="agsis", Kn_ref=0.002, n_inner=200, region_every=1, force_wall_layers=1)
    S.set_state(gi.uniform_W(24), flags=np.zeros(24, np.uint8))
    S.ns_init(tol=1e-6, chunk=2000, max_chunks=50)
    assert S.stats["g13_new"] == 22 and S.stats["g13_new_limited"] == 0
    for _ in range(4):
        S.step()
        assert S.stats["g13_ghosts"] == 2
        for k in ("g13_ghost_limited", "g13_new_limited", "corrections_limited"):
            assert S.stats[k] == 0, (k, S.stats)
