"""Pins of the oracle's polyatomic gas (the two-VDF model of Sec. 2) against
closed forms: moments of known distributions, the relaxation identities of
the reference distributions (temperatures relax towards T at rate 1/Z_r, heat
fluxes by (I - A)), exact homogeneous-relaxation recurrences, the monatomic
limit, equilibrium between walls and upwind transport of both VDFs.
"""
import numpy as np
import pytest

import gsis_inputs as gi

# nitrogen as in Sec. 4: d_r = 2, Z_r = 2.667, omega = 0.74, A from the paper
N2 = dict(dr=2.0, Zr=2.667, omega=0.74, A=(0.786, -0.201, -0.059, 0.842))


def _rows(O, rho, u, Tt, Tr, qt, qr, sigma=(0, 0, 0, 0, 0, 0)):
    """f0 = Grad-13 form with (sigma, q_t) at (rho, u, T_t); f1 = (d_r T_r/4) M_t
    + (pi T_t)^-3/2 (q_r.c/T_t) e^{-c^2/T_t}, written out in numpy."""
    c = O.xi - np.asarray(u)[None, :]
    c2 = np.sum(c * c, axis=1)
    E = (np.pi * Tt) ** -1.5 * np.exp(-c2 / Tt)
    M = rho * E
    p = rho * Tt
    s = sigma
    scc = (s[0] * c[:, 0] ** 2 + s[1] * c[:, 1] ** 2 + s[2] * c[:, 2] ** 2
           + 2 * (s[3] * c[:, 0] * c[:, 1] + s[4] * c[:, 0] * c[:, 2] + s[5] * c[:, 1] * c[:, 2]))
    f0 = M * (1 + scc / (p * Tt) + 2 * (c @ np.asarray(qt)) / (p * Tt) * (0.4 * c2 / Tt - 1))
    f1 = 0.25 * O.dr * Tr * M + E * (c @ np.asarray(qr)) / Tt
    return np.stack([f0, f1])


def _oracle(oracle_mod, mesh, n=28, V=8.0, Kn=0.2, inv_dt=0.0, **kw):
    gas = dict(N2)
    gas.update(kw)
    g = gi.velocity_grid(3, n, V)
    return oracle_mod.Oracle(mesh, g, Kn=Kn, omega=gas["omega"], Pr=gas["A"][0], inv_dt=inv_dt,
                             dr=gas["dr"], Zr=gas["Zr"], A=gas["A"])


def test_poly_moments_of_known_rows(oracle_mod):
    O = _oracle(oracle_mod, oracle_mod.one_cell_mesh())
    rho, u, Tt, Tr = 1.2, (0.3, -0.1, 0.2), 1.3, 0.8
    qt, qr = (0.04, -0.02, 0.03), (0.02, 0.01, -0.015)
    m = O.moments(_rows(O, rho, u, Tt, Tr, qt, qr))
    assert m.shape == (18,)
    assert abs(m[0] - rho) < 1e-10 and np.allclose(m[1:4], u, atol=1e-10)
    assert abs(m[4] - Tt) < 1e-9 and abs(m[14] - Tr) < 1e-9
    assert np.allclose(m[11:14], qt, atol=1e-9) and np.allclose(m[15:18], qr, atol=1e-9)


def test_poly_relaxation_identities(oracle_mod):
    """Moments of the targets: rho, u and the total energy are those of f
    (the fix-up makes them exact); T_t(G0) = T_t + (T - T_t)/Z_r,
    T_r(G1) = T_r + (T - T_r)/Z_r, [q_t; q_r](G) = (I - A)[q_t; q_r], and G0
    carries no stress."""
    O = _oracle(oracle_mod, oracle_mod.one_cell_mesh())
    f = _rows(O, 0.9, (0.2, 0.1, -0.3), 1.25, 0.85, (0.05, -0.03, 0.02), (-0.02, 0.03, 0.01),
              sigma=(0.05, -0.03, -0.02, 0.04, -0.01, 0.02))
    m = O.moments(f)
    G = O.poly_target(m)
    mg = O.moments(G)
    dr, Zr = N2["dr"], N2["Zr"]
    A = np.array(N2["A"]).reshape(2, 2)
    Tt, Tr = m[4], m[14]
    T = (3 * Tt + dr * Tr) / (3 + dr)
    assert abs(mg[0] - m[0]) < 1e-13 and np.allclose(mg[1:4], m[1:4], atol=1e-13)
    E = lambda x: 1.5 * x[0] * x[4] + 0.5 * dr * x[0] * x[14]
    assert abs(E(mg) - E(m)) < 1e-12
    assert abs(mg[4] - (Tt + (T - Tt) / Zr)) < 1e-7
    assert abs(mg[14] - (Tr + (T - Tr) / Zr)) < 1e-7
    q = np.stack([m[11:14], m[15:18]])
    assert np.allclose(np.stack([mg[11:14], mg[15:18]]), (np.eye(2) - A) @ q, atol=1e-7)
    assert np.abs(mg[5:11]).max() < 1e-7


def test_poly_homogeneous_relaxation(oracle_mod):
    """One cell with no faces and a time step: every moment follows its exact
    recurrence x' = x + r (x(G) - x), r = dt/(dt + tau), tau = mu(T_t)/p_t."""
    dt = 0.05
    O = _oracle(oracle_mod, oracle_mod.one_cell_mesh(), inv_dt=1 / dt)
    f = _rows(O, 1.1, (0.2, 0.0, 0.1), 1.4, 0.7, (0.03, 0.02, -0.01), (0.01, -0.02, 0.02),
              sigma=(0.06, -0.02, -0.04, 0.05, 0.0, -0.02))[None]
    m = O.moments(f)[0]
    dr, Zr = N2["dr"], N2["Zr"]
    A = np.array(N2["A"]).reshape(2, 2)
    for _ in range(3):
        tau = O.tau(m[0], m[4])
        r = dt / (dt + tau)
        T = (3 * m[4] + dr * m[14]) / (3 + dr)
        f = O.sweep(f, [0], [0])
        m1 = O.moments(f)[0]
        assert np.allclose(m1[:4], m[:4], atol=1e-12)
        assert abs((3 * m1[4] + dr * m1[14]) / (3 + dr) - T) < 1e-12
        assert abs(m1[4] - (m[4] + r * (T - m[4]) / Zr)) < 1e-7
        assert abs(m1[14] - (m[14] + r * (T - m[14]) / Zr)) < 1e-7
        assert np.allclose(m1[5:11], (1 - r) * m[5:11], atol=1e-7)
        q = np.stack([m[11:14], m[15:18]])
        q1 = q - r * (A @ q)
        assert np.allclose(np.stack([m1[11:14], m1[15:18]]), q1, atol=1e-7)
        m = m1


def test_poly_monatomic_limit(oracle_mod):
    """With the internal modes in equilibrium at T_t and no q_r, G0 is the
    Shakhov target of the monatomic gas with Pr = A_tt as d_r -> 0."""
    mesh = oracle_mod.one_cell_mesh()
    O = _oracle(oracle_mod, mesh, n=20, V=6.0, dr=1e-10)
    Om = oracle_mod.Oracle(mesh, gi.velocity_grid(3, 20, 6.0), Kn=0.2, omega=0.74, Pr=N2["A"][0])
    f = _rows(O, 1.05, (0.1, -0.2, 0.05), 1.2, 1.2, (0.04, 0.01, -0.02), (0, 0, 0))
    m = O.moments(f)
    G = O.poly_target(m)
    Gm = Om.equilibrium(m[:14])
    assert np.abs(G[0] - Gm[0]).max() < 1e-8 * Gm.max()


def test_poly_rest_between_walls_is_fixed(oracle_mod):
    """A gas at rest at the walls' temperature, internal modes included, is a
    fixed point of the sweep (the walls return f1 = (d_r T_w/4) f0)."""
    m = gi.couette_1d(8, wall_speed=0.0, T_wall=1.1)
    O = _oracle(oracle_mod, m, n=16, V=5.0, Kn=0.1)
    f0 = O.feq(np.array([1.0, 0, 0, 0, 1.1]))
    assert np.allclose(O.moments(f0)[[0, 4, 14]], [1.0, 1.1, 1.1], atol=1e-12)
    f = np.stack([f0] * 8)
    kin = np.arange(8)
    f1 = O.sweep(f, kin, kin)
    assert np.abs(f1 - f).max() <= 1e-9 * f.max()


def test_poly_upwind_transport_free_molecular(oracle_mod):
    """Without collisions one sweep moves both VDFs one cell downstream."""
    m = gi.couette_1d(8, wall_speed=0.0)
    O = _oracle(oracle_mod, m, n=8, V=4.0, Kn=1e14)
    W = gi.random_W(8, seed=4)
    f = np.stack([O.feq(W[i]) for i in range(8)])
    f[:, 1] *= gi.perturbation(f[:, 1].shape, seed=6)
    kin = np.arange(8)
    f1 = O.sweep(f, kin, kin)
    pos, neg = O.xi[:, 0] > 0, O.xi[:, 0] < 0
    for q in (0, 1):
        assert np.abs(f1[1:, q, pos] - f[:-1, q, pos]).max() <= 1e-12 * f.max()
        assert np.abs(f1[:-1, q, neg] - f[1:, q, neg]).max() <= 1e-12 * f.max()
