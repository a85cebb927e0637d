/*
 * gsis_oracle.h -- plain FP64 CPU oracle for the adaptive GSIS kinetic sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library.
 *
 * Every function is the slow, obviously-correct form of one step of the
 * method of Zhang, Zeng & Wu, "Adaptive GSIS for rarefied gas flow
 * simulations" (arXiv 2501.02245), written in the dimensionless units
 *   x / L,  xi / v_m (v_m = sqrt(2 R T0)),  T / T0,  rho / rho0,
 *   p, sigma / (rho0 R T0),  q / (rho0 R T0 v_m),  f / (rho0 / v_m^3),
 * so that R T -> T/2 and the Maxwellian is rho (pi T)^(-3/2) exp(-c^2/T).
 *
 * Monatomic specialisation of the two-VDF kinetic model (d_r = 0): the
 * reference distribution reduces to the Shakhov form with Prandtl number
 * Pr = A_tt (Sec. 2, reference distributions and heat-flux mixing).
 *
 * Velocity grids are tensor products, or (vdim 3) arbitrary point sets with
 * their own weights (node k = point k).  vdim = 3 stores one function per
 * cell, index k = (ix*ny + iy)*nz + iz on a tensor grid.  vdim = 2 stores the reduced pair
 * (phi, psi) = (int f dxi_z, int xi_z^2 f dxi_z) per cell, index
 * k = ix*ny + iy, layout [fun][k].
 *
 * Moment vector (NMOM = 14): rho, ux, uy, uz, T, sxx, syy, szz, sxy, sxz,
 * syz, qx, qy, qz.
 */
#ifndef GSIS_ORACLE_H
#define GSIS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OC_NMOM 14
#define OC_WALL 0
#define OC_FAR 1

typedef struct {
    int32_t dim, n_cells, n_faces, n_patches;
    const int32_t *face_cells;   /* [n_faces][2] owner, other (<0: patch -1-p) */
    const double *face_normal;   /* [n_faces][3] unit, owner -> other */
    const double *face_area;     /* [n_faces] */
    const double *face_center;   /* [n_faces][3] */
    const double *cell_volume;   /* [n_cells] */
    const double *cell_center;   /* [n_cells][3] */
    const int32_t *patch_kind;   /* [n_patches] OC_WALL | OC_FAR */
    const double *patch_state;   /* [n_patches][5] rho, ux, uy, uz, T */
} oc_mesh;

typedef struct {
    int32_t vdim;                /* 2 (reduced) or 3 */
    int32_t n[3];                /* nodes per axis (n[2] ignored for vdim 2) */
    const double *x[3];
    const double *w[3];
    int32_t npts;                /* > 0: a point set instead of a tensor product (vdim 3) */
    const double *pts;           /* [npts][3] nodes */
    const double *pw;            /* [npts] weights */
} oc_grid;

typedef struct {
    double Kn;      /* reference Knudsen number (Sec. 2, definition of Kn) */
    double omega;   /* viscosity index, mu ~ T^omega */
    double Pr;      /* A_tt of the monatomic gas = Prandtl number */
    double inv_dt;  /* 1/dt of the kinetic update; 0 = steady iteration */
    double damp2;   /* second-order sweeps: pseudo-time 1/dt_i = damp2 max_k sum_{a_k>0} a_k */
    double dr;      /* polyatomic gas: internal degrees of freedom d_r (0: monatomic) */
    double Zr;      /* internal collision number */
    double A[4];    /* heat-flux relaxation matrix (A_tt, A_tr, A_rt, A_rr) */
} oc_gas;

int32_t oc_nv(const oc_grid *g);
int32_t oc_nfun(const oc_grid *g);
int32_t oc_threads(void);
void oc_set_threads(int32_t n);

/* Moments of one cell's distribution(s) f[nfun][nv] -> mom[OC_NMOM]. */
void oc_moments(const oc_grid *g, const double *f, double *mom);

/* Discrete Maxwellian M(rho, u, T) at the nodes -> out[nfun][nv]. */
void oc_maxwellian(const oc_grid *g, double rho, const double *u, double T, double *out);

/* Shakhov reference distribution built from moments (rho, u, T, q). */
void oc_shakhov(const oc_grid *g, double Pr, const double *mom, double *out);

/* Multiply g by (a0 + a.c + b c^2), c = xi - u, so that its discrete mass,
 * momentum and energy equal those of a gas at (rho, u, T).  Returns 0, or -1
 * if the linear system is singular. coef (nullable) receives a0, a[vdim], b. */
int32_t oc_fixup(const oc_grid *g, double rho, const double *u, double T, double *gv, double *coef);

/* Conservation-fixed Shakhov target of the relaxation term, from moments. */
int32_t oc_equilibrium(const oc_grid *g, const oc_gas *gas, const double *mom, double *out);

/* Conservation-fixed Maxwellian whose discrete (rho, rho u, E) equal W. */
int32_t oc_feq(const oc_grid *g, const double *W5, double *out);

/* Grad-13 type distribution from (rho, u, T, sigma[6], q[3]). */
void oc_g13(const oc_grid *g, const double *mom, double *out);

/* Mean collision time tau = mu / p in scaled units. */
double oc_tau(const oc_gas *gas, double rho, double T);

/* One point-Jacobi sweep of the implicit kinetic update over the kinetic
 * cells.  f_old/f_new: [n_slots][nfun][nv] addressed by slot_of_cell.
 * ghost: [n_cells][OC_NMOM] Grad-13 parameters used for NS neighbours.
 * Returns 0 or a negative error. */
int32_t oc_sweep(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                 int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                 const double *f_old, const double *ghost, double *f_new);

/* Limited least-squares slopes of every discrete-velocity value of the
 * kinetic cells (second-order face values; the readings are stated in the
 * source).  slope[n_slots][nfun * nv][3], addressed by slot_of_cell. */
int32_t oc_kinetic_slopes(const oc_mesh *m, const oc_grid *g, int32_t n_kin, const int32_t *kin_cell,
                          const int32_t *slot_of_cell, const double *f, double *slope);

/* oc_sweep with second-order face values on faces between kinetic cells,
 * as a deferred correction of the first-order implicit operator; slope from
 * oc_kinetic_slopes of f_old (NULL: first order, the same as oc_sweep). */
int32_t oc_sweep2(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                  int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                  const double *f_old, const double *ghost, const double *slope, double *f_new);

/* Moment balance of the kinetic scheme at f (per unit volume): R[n_cells][5]
 * = -sum_faces (S/V) sum_k w (xi.n) (1, xi, |xi|^2) f_upwind; zero rows for
 * non-kinetic cells. */
int32_t oc_kinetic_residual(const oc_mesh *m, const oc_grid *g,
                            int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                            const double *f_old, const double *ghost, double *R);

/* The same balance with the second-order face values of oc_sweep2. */
int32_t oc_kinetic_residual2(const oc_mesh *m, const oc_grid *g,
                             int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                             const double *f_old, const double *ghost, const double *slope, double *R);

/* Least-squares cell gradients of nvar fields phi[n_cells][nvar];
 * bnd[n_patches][nvar] holds boundary values (NaN = use the cell value).
 * grad[n_cells][nvar][3]. */
void oc_lsq_gradients(const oc_mesh *m, int32_t nvar, const double *phi, const double *bnd, double *grad);

/* NSF stress and heat flux from gradients of u (3x3, row = component) and T. */
void oc_nsf(const oc_gas *gas, double T, const double *grad_u, const double *grad_T,
            double *sigma6, double *q3);

/* Residual of the synthetic macroscopic equations at primitive W, per unit
 * volume: Rv[n_cells][5] = -(1/V) sum_f F.n S (no source term). */
int32_t oc_macro_residual(const oc_mesh *m, const oc_gas *gas, const double *hot,
                          const double *W, double *Rv);

/* N_inner explicit pseudo-time iterations of the synthetic macroscopic
 * equations (NSF + high-order terms) with an optional frozen source
 * src[n_cells][5] (per unit volume, nullable).  W[n_cells][5] primitive
 * (rho, u, T) in/out; hot[n_cells][9] (sigma 6, q 3, zero on NS cells).
 * cfl > 0: local steps; cfl < 0: one global step (conservative).
 * Returns 0, or -7 on a non-positive density/temperature. */
int32_t oc_macro(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *src,
                 int32_t n_inner, double cfl, double *W);

/* ------------------------------------------------------------------------
 * Polyatomic gas (Sec. 2, the two-VDF model with d_r > 0), 3D velocity grids.
 * Rows [2][nv] = (f0, f1); f1 is scaled so that sum w f1 = d_r rho T_r / 4 and
 * q_r = 2 sum w c f1.  Moment vector OC_NMOM_POLY = OC_NMOM (from f0: T is T_t,
 * q is q_t) followed by T_r, q_r[3].
 * ------------------------------------------------------------------------ */
#define OC_NMOM_POLY 18

void oc_moments_poly(const oc_grid *g, double d_r, const double *f, double *mom);

/* Relaxation targets G0 = g0t + (g0r - g0t)/Z_r and G1 = g1t + (g1r - g1t)/Z_r
 * from the moments, times the conservation fix-up (a0 + a.c + b c^2) that makes
 * their discrete mass, momentum and total energy those of the moments.
 * out [2][nv].  Returns 0 or -1 (singular fix-up). */
int32_t oc_poly_target(const oc_grid *g, const oc_gas *gas, const double *mom, double *out);

/* One point-Jacobi sweep of both VDFs (rows [n_slots][2][nv]).  Wall and
 * far-field values of f1 are (d_r T_b / 4) times those of f0 (internal modes
 * in equilibrium at the boundary temperature T_b); NS neighbours present the
 * Grad-13 rows of oc_g13_poly of ghost [n_cells][OC_NMOM_POLY]. */
int32_t oc_sweep_poly(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                      int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                      const double *f_old, const double *ghost, double *f_new);

/* Grad-13 rows of an NS cell for the two-VDF gas (Sec. 3.2 eq. G13_VDF):
 * f0 = the monatomic Grad-13 row of (rho, u, T_t, sigma, q_t) and
 * f1 = (d_r T_r / 4) f0 + (pi T_t)^(-3/2) (q_r.c / T_t) e^{-c^2/T_t}, so that
 * 2 sum w c f1 = q_r.  prm[OC_NMOM_POLY] = (rho, u, T_t, sigma, q_t, T_r, q_r). */
void oc_g13_poly(const oc_grid *g, double d_r, const double *prm, double *out);

/* NSF laws of the two-VDF gas (Sec. 2 eqs. NSF_constitutive, mu_kappa) in
 * scaled units: sigma = -(2 Kn/sqrt(pi)) mu (grad u + grad u^T - (2/3) div u I),
 * q_t = -(k_t Kn/sqrt(pi)) mu grad T_t, q_r = -(k_r Kn/sqrt(pi)) mu grad T_r,
 * mu = T_t^omega, [k_t, k_r] = (1/2) A^{-1} [5, d_r]. */
void oc_nsf_poly(const oc_gas *gas, double Tt, const double *grad_u, const double *grad_Tt, const double *grad_Tr,
                 double *sigma6, double *qt3, double *qr3);

/* Moment balance of the two-VDF kinetic scheme at f, per unit volume:
 * R[n_cells][6] = mass, momentum, total energy sum w (xi^2 f0 + 2 f1) of the
 * upwind face fluxes, and the internal energy 2 sum w f1: its face fluxes
 * plus the collision term 2 sum w (G1 - f1) / tau of the sweep's targets.
 * ghost [n_cells][OC_NMOM_POLY]. */
int32_t oc_kinetic_residual_poly(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                                 int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                                 const double *f_old, const double *ghost, double *R);

/* Synthetic equations of the two-VDF gas (Sec. 2 eq. macroscopic_equation_2
 * with the internal-energy equation, Sec. 3.1 eqs. full_constitutive, macro).
 * W[n_cells][6] = (rho, u, T_t, T_r); hot[n_cells][12] = HoT of sigma (6),
 * q_t (3), q_r (3).  The residual includes the internal relaxation source
 * (d_r/2) rho (T - T_r) / (Z_r tau), T = (3 T_t + d_r T_r)/(3 + d_r). */
int32_t oc_macro_residual_poly(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *W,
                               double *Rv);
int32_t oc_macro_poly(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *src,
                      int32_t n_inner, double cfl, double *W);

#ifdef __cplusplus
}
#endif
#endif
