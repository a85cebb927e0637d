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


# ---------------------------------------------------------------------------
# the synthetic side of the two-VDF gas (Sec. 2 eq. macroscopic_equation_2,
# last line; Sec. 3.1 eqs. full_constitutive, macro; Sec. 3.2 eq. G13_VDF)
# ---------------------------------------------------------------------------
def test_poly_g13_rows_reproduce_their_parameters(oracle_mod):
    """The two-VDF Grad-13 rows of an NS cell (eq. G13_VDF, f1 line with its
    q_r term) have the moments they are built from: rho, u, T_t, sigma, q_t,
    T_r and q_r, to quadrature accuracy; and they equal the rows written out
    independently in numpy."""
    O = _oracle(oracle_mod, oracle_mod.one_cell_mesh())
    rho, u, Tt, Tr = 1.1, (0.2, -0.3, 0.1), 1.2, 0.9
    sig, qt, qr = (0.04, -0.02, -0.02, 0.03, -0.01, 0.015), (0.03, -0.02, 0.01), (-0.015, 0.02, 0.01)
    # without stress and translational heat flux the bracket is 1: the rows
    # written out in numpy
    prm0 = np.array([rho, *u, Tt, *np.zeros(9), Tr, *qr])
    rows0 = O.g13(prm0)
    assert np.abs(rows0 - _rows(O, rho, u, Tt, Tr, (0, 0, 0), qr)).max() < 1e-13 * np.abs(rows0).max()
    prm = np.array([rho, *u, Tt, *sig, *qt, Tr, *qr])
    rows = O.g13(prm)
    m = O.moments(rows)
    assert abs(m[0] - rho) < 1e-9 and np.allclose(m[1:4], u, atol=1e-9)
    assert abs(m[4] - Tt) < 1e-8 and abs(m[14] - Tr) < 1e-8
    assert np.allclose(m[5:11], sig, atol=1e-8) and np.allclose(m[11:14], qt, atol=1e-8)
    assert np.allclose(m[15:18], qr, atol=1e-8)


def test_poly_synthetic_exchange_matches_kinetic_exchange(oracle_mod):
    """Uniform gas with T_t = 1.3, T_r = 0.7 in a slab: on interior cells the
    face fluxes cancel, so the kinetic balance of the internal energy is the
    collision term 2 sum w (G1 - f1)/tau of the model's targets, and the
    synthetic residual is the paper's exchange source (d_r/2) rho (T - T_r) /
    (Z_r tau) with T = (3 T_t + d_r T_r)/(3 + d_r).  The two agree to
    quadrature accuracy; mass, momentum and total energy do not change.
    Advanced in pseudo-time, the synthetic solve keeps rho, u and the total
    energy and relaxes T_t and T_r to the common T."""
    n = 13
    m = gi.slab_1d(n, gi._patch("far", rho=1.0, u=(0.1, 0.0, 0.0), T=1.0),
                   gi._patch("far", rho=1.0, u=(0.1, 0.0, 0.0), T=1.0))
    O = _oracle(oracle_mod, m, n=24, V=7.0, Kn=0.05)
    W = np.tile([1.0, 0.1, 0.0, 0.0, 1.3, 0.7], (n, 1))
    S = oracle_mod.SteadySolver(O, mode="gsis")
    S.set_state(W)
    Rk = O.kinetic_residual(S.f, S.kin, S.slot)
    Rm = O.macro_residual(S.W, np.zeros((n, 12)))
    inner = np.arange(2, n - 2)
    T = (3 * 1.3 + 2 * 0.7) / 5.0
    src = 0.5 * 2.0 * 1.0 * (T - 0.7) / (2.667 * O.tau(1.0, 1.3))
    assert np.allclose(Rm[inner, 5], src, rtol=1e-12)
    assert np.allclose(Rk[inner, 5], src, rtol=1e-8)
    assert np.abs(Rk[inner, :5]).max() < 1e-9 and np.abs(Rm[inner, :5]).max() < 1e-12
    # two pseudo-time steps (the far-field boundaries do not reach the middle
    # cell): rho, u, the total energy and T are kept, and T_t, T_r move
    # towards T by the same fraction
    Wm = O.macro(S.W, np.zeros((n, 12)), 2, cfl=-0.5)
    mid = n // 2
    E0 = 1.0 * 0.01 + 1.5 * 1.3 + 0.5 * 2.0 * 0.7
    E1 = Wm[mid, 0] * (Wm[mid, 1] ** 2) + 1.5 * Wm[mid, 0] * Wm[mid, 4] + Wm[mid, 0] * Wm[mid, 5]
    assert abs(E1 - E0) < 1e-13 and abs(Wm[mid, 0] - 1.0) < 1e-14 and abs(Wm[mid, 1] - 0.1) < 1e-14
    a_t, a_r = (Wm[mid, 4] - T) / (1.3 - T), (Wm[mid, 5] - T) / (0.7 - T)
    assert 0.0 < a_r < 1.0 and abs(a_t - a_r) < 1e-12


def test_poly_continuum_limit_fixes_the_conductivities(oracle_mod):
    """Nitrogen between diffuse walls at T = 1 (moving -0.1) and T = 2 (moving
    +0.1), Kn = 0.01, converged by GSIS: away from the Knudsen layers the
    kinetic stress and both heat fluxes obey the NSF laws of Sec. 2 with
    mu ~ T_t^omega and the conductivities of eq. mu_kappa,
    [kappa_t, kappa_r] = (mu R / 2) A^{-1} [5, d_r], i.e. in scaled units
    q_t = -(k_t Kn/sqrt(pi)) mu dT_t/dx and q_r = -(k_r Kn/sqrt(pi)) mu dT_r/dx
    with (k_t, k_r) = (3.548, 1.436) for the paper's A (Eucken factors 2.365,
    1.436).  The heat-flux mixing of the targets through A is what produces
    these conductivities; a wrong entry of A or of the mixing fails here."""
    n, Kn = 30, 0.01
    m = gi.slab_1d(n, gi._patch("wall", u=(0.0, -0.1, 0.0), T=1.0), gi._patch("wall", u=(0.0, 0.1, 0.0), T=2.0))
    g = gi.velocity_grid(3, 14, 6.0)
    O = oracle_mod.Oracle(m, g, Kn, omega=N2["omega"], Pr=N2["A"][0], dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    S = oracle_mod.SteadySolver(O, mode="gsis", n_inner=400, cfl=0.5)
    W0 = gi.uniform_W(n)
    W0[:, 4] = 1.0 + m["cell_center"][:, 0]
    S.set_state(W0)
    it, eps = S.solve(tol=1e-9, max_iter=600)
    assert eps.max() < 1e-9
    kt, kr = oracle_mod.conductivities(np.array(N2["A"]).reshape(2, 2), N2["dr"])
    assert abs(kt - 3.548) < 1e-3 and abs(kr - 1.436) < 1e-3
    mom = O.moments(S.f[S.slot[S.kin]])
    x = m["cell_center"][:, 0]
    uy, Tt, sxy, qt, Tr, qr = mom[:, 2], mom[:, 4], mom[:, 8], mom[:, 11], mom[:, 14], mom[:, 15]
    i = np.arange(n)[(x > 0.2) & (x < 0.8)]

    def d(v):
        return (v[i + 1] - v[i - 1]) / (x[i + 1] - x[i - 1])
    mu = Tt[i] ** N2["omega"]
    c = Kn / np.sqrt(np.pi)
    assert np.abs(sxy[i] / (-2 * c * mu * d(uy)) - 1).max() < 1e-2
    assert np.abs(qt[i] / (-kt * c * mu * d(Tt)) - 1).max() < 1e-2
    assert np.abs(qr[i] / (-kr * c * mu * d(Tr)) - 1).max() < 1e-2


def test_poly_gsis_fixed_point_is_dvm_fixed_point(oracle_mod):
    """Converged GSIS for nitrogen (the internal-energy equation in the
    synthetic solve, its exchange source, HoT of q_r, rho e_r in the
    correction) is converged plain DVM on the open slab of the monatomic pin,
    in far fewer iterations."""
    m = gi.slab_1d(16, gi._patch("wall", u=(0.0, 0.1, 0.0), T=1.1),
                   gi._patch("far", rho=1.0, u=(0.0, 0.0, 0.0), T=1.0))
    g = gi.velocity_grid(3, 12, 5.0)
    O = oracle_mod.Oracle(m, g, 0.05, omega=N2["omega"], Pr=N2["A"][0], dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    W0 = gi.couette_initial_W(16, seed=1)
    D = oracle_mod.SteadySolver(O, mode="dvm")
    D.set_state(W0)
    it_d, _ = D.solve(tol=1e-12, max_iter=20000)
    S = oracle_mod.SteadySolver(O, mode="gsis", n_inner=400, cfl=0.5)
    S.set_state(W0)
    it_s, _ = S.solve(tol=1e-12, max_iter=2000)
    assert it_s < it_d / 5
    assert np.abs(S.W - D.W).max() < 1e-9
    fd = D.f[D.slot[D.kin]]
    assert np.abs(S.f[S.slot[S.kin]] - fd).max() < 1e-9 * np.abs(fd).max()


# ---------------------------------------------------------------------------
# surface quantities of the two-VDF gas (Sec. 4.2/4.3 with the internal
# energy of Sec. 2): wall values of f1 are (d_r T_w/4) f0's
# ---------------------------------------------------------------------------
def _wall_side(m, faces):
    return np.sign(m["face_normal"][faces, 0])


def test_poly_surface_rest_at_wall_temperature(oracle_mod):
    """Nitrogen at rest at the walls' temperature with its internal modes in
    equilibrium (T_r = T_w; rows f0 = M, f1 = (d_r T_w/4) M): the wall stress
    is the pressure along the normal, no shear, no heat and no net mass flux,
    on kinetic and on NS wall cells."""
    m = gi.couette_1d(6, wall_speed=0.0, T_wall=1.2)
    O = _oracle(oracle_mod, m, n=16, V=5.0, Kn=0.1)
    M = O.maxwellian(0.9, [0, 0, 0], 1.2)[0]
    f = np.stack([np.stack([M, 0.25 * N2["dr"] * 1.2 * M])] * 6)
    W = np.tile([0.9, 0, 0, 0, 1.2, 1.2], (6, 1))
    kin = np.arange(6)
    for slot in (kin, -np.ones(6, np.int64)):
        faces, out = O.surface(f, slot, W)
        n = m["face_normal"][faces]
        p = out[:, 3]
        assert np.allclose(out[:, 0:3], p[:, None] * n, atol=1e-12)
        assert np.abs(out[:, 4:7]).max() < 1e-12
        assert np.abs(out[:, 7]).max() < 1e-12 and np.abs(out[:, 8]).max() < 1e-12
        assert np.allclose(p, 0.9 * 1.2, rtol=1e-6)


def test_poly_surface_free_molecular_fourier(oracle_mod):
    """Free-molecular nitrogen between stationary walls at T_L and T_R: in the
    discrete steady state the heat into each wall is the gas's total heat
    flux q_t + q_r (q_r = 2 sum w c f1 carries the internal energy), the two
    walls' heat sums to zero, and against the continuous closed form each
    molecule leaving a wall carries (d_r/2) T_w of internal energy besides its
    translational energy, so q = n_L sqrt(T_L)(T_L - T_R)(1 + d_r/4)/sqrt(pi)
    to the quadrature error.  A dropped factor 2 on f1 or a reflected f1 at
    the wrong temperature fails the last check."""
    TL, TR, n = 1.0, 1.5, 12
    m = gi.fourier_1d(n, TL, TR)
    g = gi.velocity_grid(3, (96, 16, 16), (8.0, 6.0, 6.0))
    O = oracle_mod.Oracle(m, g, Kn=1e14, omega=N2["omega"], Pr=N2["A"][0], dr=N2["dr"], Zr=N2["Zr"], A=N2["A"])
    f = np.stack([O.feq(np.array([1.0, 0, 0, 0, 1.0]))] * n)
    kin = np.arange(n)
    for _ in range(n + 2):
        f = O.sweep(f, kin, kin)
    mom = O.moments(f)
    W = np.concatenate([mom[:, :5], mom[:, 14:15]], 1)
    faces, out = O.surface(f, kin, W)
    side = _wall_side(m, faces)
    R, L = np.nonzero(side > 0)[0][0], np.nonzero(side < 0)[0][0]
    q = mom[0, 11] + mom[0, 15]
    assert mom[0, 15] < 0 and q < 0    # heat, internal part included, flows to the cold left wall
    assert abs(out[L, 7] / -q - 1) < 1e-10
    assert abs(out[R, 7] / q - 1) < 1e-10
    assert abs(out[L, 7] + out[R, 7]) < 1e-12 * abs(q)
    assert np.abs(out[:, 8]).max() < 1e-13
    xi, w = O.xi, O.w
    pos, neg = xi[:, 0] > 0, xi[:, 0] < 0
    wn = w * np.abs(xi[:, 0])

    def gauss(T):
        return (np.pi * T) ** -1.5 * np.exp(-np.sum(xi * xi, axis=1) / T)
    nL = np.sum(wn[neg] * gauss(1.0)[neg]) / np.sum(wn[pos] * gauss(TL)[pos])
    qcf = nL * np.sqrt(TL) * (TL - TR) * (1 + 0.25 * N2["dr"]) / np.sqrt(np.pi)
    assert abs(out[R, 7] / qcf - 1) < 5e-3


def test_poly_surface_ns_wall_linear_fields(oracle_mod):
    """NS wall cells of nitrogen: with u_y, T_t and T_r linear in x and the
    walls at the end values (T_r held at T_w as well), the one-sided gradients
    are exact, so the shear is -(2 Kn/sqrt(pi)) mu du_y/dx n_x and the heat
    into the wall is (k_t dT_t/dx + k_r dT_r/dx)(Kn/sqrt(pi)) mu (-n_x), with
    mu = T_w^omega and (k_t, k_r) = (1/2) A^{-1} (5, d_r) (eq. mu_kappa)."""
    n, a, b, Kn = 10, 0.3, 0.4, 0.05
    m = gi.couette_1d(n, wall_speed=0.5 * a)
    for p in m["patches"]:
        p["T"] = 1.0 + b * (0.0 if p["u"][1] < 0 else 1.0)
    x = m["cell_center"][:, 0]
    W = np.zeros((n, 6))
    W[:, 0] = 1.0
    W[:, 2] = a * (x - 0.5)
    W[:, 4] = 1.0 + b * x
    W[:, 5] = 1.0 + b * x
    O = _oracle(oracle_mod, m, n=8, V=5.0, Kn=Kn)
    faces, out = O.surface(np.zeros((n, 2, O.nv)), -np.ones(n, np.int64), W)
    side = _wall_side(m, faces)
    A = np.array(N2["A"]).reshape(2, 2)
    kt, kr = 0.5 * np.linalg.solve(A, [5.0, N2["dr"]])
    for j, fi in enumerate(faces):
        Tw = m["patches"][-1 - m["face_cells"][fi, 1]]["T"]
        mu = Tw ** N2["omega"]
        L = m["face_cells"][fi, 0]
        c = Kn / np.sqrt(np.pi) * mu
        assert abs(out[j, 1] - (-2 * c * a * side[j])) < 1e-12
        assert abs(out[j, 7] - (-(kt + kr) * c * b * side[j])) < 1e-12
        assert abs(out[j, 3] - W[L, 0] * W[L, 4]) < 1e-12
