/*
 * gsis.h -- C ABI of the MI355X kinetic-sweep library for adaptive GSIS.
 *
 * Method: Zhang, Zeng & Wu, "Adaptive GSIS for rarefied gas flow
 * simulations" (arXiv 2501.02245).  The library runs the data-parallel hot
 * path of the method on one GPU: the implicit discrete-velocity sweep of
 * Sec. 3.1 over the kinetic (DVM) cells, the velocity-moment reduction of
 * Sec. 2 (eq. getmoment), the GSIS correction of Sec. 3.1 (first eq.
 * updatef), the synthetic macroscopic solve (eqs. full_constitutive and
 * macro), the local-Knudsen region test and compaction of Sec. 3.2 (eq.
 * Kn_Gll and the second eq. updatef) and the convergence measure of Sec. 4.
 *
 * Units: lengths / L, velocities / sqrt(2 R T0), T / T0, rho / rho0; the
 * Maxwellian is rho (pi T)^(-3/2) exp(-|xi - u|^2 / T).  The gas is
 * monatomic by default (the two-VDF model of Sec. 2 with d_r = 0, which is
 * the Shakhov model with Prandtl number A_tt); gsis_set_internal_dof selects
 * the two-VDF gas with internal degrees of freedom (the nitrogen of Sec. 4).
 *
 * Conventions
 *  - Every call returns gsis_status; GSIS_OK == 0.  On failure,
 *    gsis_last_error() returns a thread-local description.  No C++
 *    exception crosses the ABI.
 *  - Host arrays passed in are copied before the call returns.
 *  - Device buffers (workspace, state, outputs) belong to the caller and are
 *    never freed by the library.  Handles are created and destroyed only by
 *    gsis_* calls.
 *  - Calls that take a `stream` (a hipStream_t, or NULL for the default
 *    stream) enqueue their work and return; results are valid after the
 *    stream synchronises.  Calls that return host counts or residuals
 *    synchronise that stream.
 *  - Argument and state checks run on the host before any launch; a
 *    non-finite value found on the device is reported by the next call that
 *    synchronises as GSIS_E_NONFINITE.
 *  - One case must not be used from two threads at once.
 *  - FP32 and FP64 storage are two instantiations of the same kernels.
 */
#ifndef GSIS_H
#define GSIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gsis_status;
#define GSIS_OK 0
#define GSIS_E_ARG (-1)        /* invalid argument */
#define GSIS_E_MESH (-2)       /* mesh rejected (open cell, V <= 0, bad index, too many faces) */
#define GSIS_E_STATE (-3)      /* call out of order (e.g. sweep before bind / set_state) */
#define GSIS_E_NOMEM (-4)      /* workspace smaller than gsis_case_footprint */
#define GSIS_E_CAPACITY (-5)   /* kinetic region larger than the bound capacity */
#define GSIS_E_HIP (-6)        /* HIP runtime error */
#define GSIS_E_NONFINITE (-7)  /* NaN/Inf or non-positive density/temperature */
#define GSIS_E_NOCONV (-8)     /* max_iter reached before tol */

#define GSIS_MAX_FACES 8       /* faces per cell */
#define GSIS_MAX_WALL_FACES 4  /* wall faces per cell */
#define GSIS_MAX_AXIS 128      /* nodes per velocity axis */
#define GSIS_NMOM 14           /* rho, ux, uy, uz, T, sxx, syy, szz, sxy, sxz, syz, qx, qy, qz */

typedef struct gsis_mesh_s *gsis_mesh;
typedef struct gsis_case_s *gsis_case;

#define GSIS_PATCH_WALL 0      /* diffuse isothermal wall at (u, T) */
#define GSIS_PATCH_FAR 1       /* far field: Maxwellian at (rho, u, T) on incoming velocities */

typedef struct {
    int32_t kind;
    double rho, u[3], T;
} gsis_patch;

/* Unstructured finite-volume mesh (host arrays, copied).
 *  dim          1, 2 or 3: gradients use the first `dim` components
 *  face_cells   [n_faces][2] owner, other; other < 0 means boundary patch -1-other
 *  face_normal  [n_faces][3] unit normal, owner -> other
 *  face_area    [n_faces], face_center [n_faces][3]
 *  cell_volume  [n_cells], cell_center [n_cells][3]
 * Rejected with GSIS_E_MESH: an index out of range, a cell with more than
 * GSIS_MAX_FACES faces or GSIS_MAX_WALL_FACES wall faces, V <= 0, S <= 0,
 * or an open cell (|sum_f n S| > 1e-9 sum_f S). */
typedef struct {
    int32_t dim, n_cells, n_faces, n_patches;
    const int32_t *face_cells;
    const double *face_normal;
    const double *face_area;
    const double *face_center;
    const double *cell_volume;
    const double *cell_center;
    const gsis_patch *patches;
} gsis_mesh_desc;

/* Gas: Kn (Sec. 2 definition), viscosity index omega (mu ~ T^omega), and
 * Pr = A_tt (heat-flux relaxation of the monatomic model). */
typedef struct {
    double Kn, omega, Pr;
} gsis_gas;

#define GSIS_F32 0
#define GSIS_F64 1

const char *gsis_last_error(void);

gsis_status gsis_create_mesh(const gsis_mesh_desc *desc, gsis_mesh *out);
gsis_status gsis_destroy_mesh(gsis_mesh mesh);   /* the mesh must outlive its cases */

/* One steady problem on `mesh`; vdf_dtype GSIS_F32 or GSIS_F64 (storage and
 * arithmetic of the kinetic kernels; the macroscopic side is always FP64). */
gsis_status gsis_create_case(gsis_mesh mesh, const gsis_gas *gas, int32_t vdf_dtype, gsis_case *out);
gsis_status gsis_destroy_case(gsis_case c);

/* Tensor-product velocity quadrature (host arrays, copied).  vdim 3: full
 * velocity space, node k = (ix*n1 + iy)*n2 + iz.  vdim 2: the reduced pair
 * (phi, psi) = (int f dxi_z, int xi_z^2 f dxi_z) over (xi_x, xi_y), node
 * k = ix*n1 + iy (Sec. 3.3 reduction of the 2D velocity space).  Each axis
 * has 2..GSIS_MAX_AXIS nodes; weights must be positive. */
gsis_status gsis_set_velocity_grid(gsis_case c, int32_t vdim, const int32_t n[3],
                                   const double *const nodes[3], const double *const weights[3]);

/* Non-tensor velocity quadrature (Sec. 4.3 hybrid and Sec. 4.4 unstructured
 * velocity space): n_points nodes xi [n_points][3] with their own positive
 * weights w [n_points] (host arrays, copied), full 3D velocity space, node k
 * = point k.  Every kinetic kernel then evaluates the Gaussian and Grad-13
 * forms per node (one exp per node and source) and the conservation fix-up
 * from direct FP64 sums over the nodes; the generic (non-plane) sweep and
 * correction kernels run.  1..2^24 points. */
gsis_status gsis_set_velocity_points(gsis_case c, int32_t n_points, const double *xi, const double *w);

/* Polyatomic gas (Sec. 2: the two-VDF model, eq. general_model, with d_r
 * internal degrees of freedom, internal collision number Z_r >= 1 and the
 * heat-flux relaxation matrix A = {A_tt, A_tr, A_rt, A_rr}; the gas of Sec. 4
 * is d_r = 2, Z_r = 2.667, omega = 0.74, A = {0.786, -0.201, -0.059, 0.842}).
 * d_r = 0 (default) is the monatomic gas.  With d_r > 0 each kinetic cell
 * holds two rows, f0 and f1 (layout [fun][k] as the reduced pair), f1 scaled
 * so that sum w f1 = d_r rho T_r / 4 and q_r = 2 sum w c f1; the relaxation
 * targets are g_0t + (g_0r - g_0t)/Z_r and g_1t + (g_1r - g_1t)/Z_r with the
 * heat-flux mixing of q_0, q_1 through A, times a conservation fix-up of mass,
 * momentum and total (translational + internal) energy; tau = mu(T_t)/p_t
 * with mu = T_t^omega.  Wall, far-field and NS-interface values of f1 are
 * (d_r T_b / 4) times those of f0; on NS-interface faces f1 is the two-VDF
 * Grad-13 row of Sec. 3.2 eq. G13_VDF: (d_r T_r / 4) times the f0 row plus
 * q_r.c / (rho T_t) times the Maxwellian at T_t.  The synthetic solve of the
 * GSIS modes adds the internal-energy equation of Sec. 2 eq.
 * macroscopic_equation_2 (rho e_r = (d_r/2) rho T_r, exchange source
 * (d_r/2) rho (T - T_r)/(Z_r tau), T = (3 T_t + d_r T_r)/(3 + d_r), taken
 * backward-Euler in pseudo-time; Fourier laws with the conductivities
 * (k_t, k_r) = (1/2) A^-1 (5, d_r) of eq. mu_kappa; HoT of q_r), and the
 * correction moves f1 by (d_r/4)(T_r^{n+1} f_eq(W^{n+1}) - T_r^{n+1/2}
 * f_eq(W^{n+1/2})).  W passed to and read from the library stays (rho, u,
 * T_t); T_r of every cell is read with gsis_get_internal_temperature and
 * starts at T_t on every cell (set_state), the kinetic cells then taking that
 * of their f1.  Supported: 3D tensor velocity grids, spatial order 1, every
 * mode of gsis_step / gsis_solve_steady, gsis_ns_init, gsis_update_regions;
 * gsis_surface, gsis_correct_internal and gsis_macro_solve_internal (the
 * monatomic gsis_correct and gsis_macro_solve return E_ARG).  Gas Pr is
 * not used.  Call before gsis_case_footprint / bind (E_STATE once bound);
 * E_ARG for d_r < 0, Z_r < 1 or non-finite A. */
gsis_status gsis_set_internal_dof(gsis_case c, double d_r, double Z_r, const double *A);

/* Polyatomic gas: T_r and q_r (x, y, z) of the current f1 per kinetic cell,
 * out_dev [n_kin][4] FP64 in ascending cell id (may be null when there is no
 * kinetic cell).  E_ARG for a monatomic case. */
gsis_status gsis_internal_moments(gsis_case c, double *out_dev, void *stream);

/* Polyatomic gas: the internal temperature T_r of every cell of the current
 * state (kinetic cells: that of f1 after the last step; NS cells: that of the
 * synthetic solve), out_dev [n_cells] FP64 device memory, on `stream`.  E_ARG
 * for a monatomic case or a null output; E_STATE before set_state. */
gsis_status gsis_get_internal_temperature(gsis_case c, double *out_dev, void *stream);

/* Spatial order of the kinetic face values (Sec. 3: second-order finite
 * volumes; the paper leaves the scheme to its references).  order 1
 * (default): first-order upwind.  order 2: every discrete-velocity value of a
 * kinetic cell gets a least-squares slope over the cell's kinetic neighbours
 * (zero when they do not span the mesh dimension), scaled by the
 * Barth-Jespersen factor that keeps the face values to kinetic neighbours
 * within the range of the cell and those neighbours; every face whose upwind
 * side is a kinetic cell takes the reconstructed value, as a deferred
 * correction of the first-order implicit operator, and the wall densities
 * zero the net mass flux of the reconstructed outgoing values.  The sweep
 * then adds the pseudo-time term (f^{n+1/2} - f^n)/dt_i with 1/dt_i = damp *
 * max_k sum_{a_k > 0} a_k (the cell's largest outflow rate; damp >= 0,
 * typically 2): without it the point-Jacobi iteration of the corrected
 * operator diverges; it vanishes at convergence.  Order 2 uses the generic
 * (non-plane) sweep: faces as rows on 3D grids (GSIS_ORDER2_GENERIC=1 in the
 * environment at launch selects the generic kernel instead), the generic
 * kernel on reduced 2D grids; it adds the reconstruction increments of every
 * face (the mesh's largest face count per cell times the VDF row, per kinetic
 * slot) to the footprint.  Call before gsis_case_footprint / bind
 * (E_STATE once bound); E_ARG for order not 1 or 2 or a bad damp. */
gsis_status gsis_set_spatial_order(gsis_case c, int32_t order, double damp);

/* Range limit of the Grad-13 distributions (Sec. 3.2 eq. G13_VDF) that NS
 * cells next to the kinetic region present to it and that newly kinetic
 * cells start from.  The paper builds them from the NS stress and heat flux
 * without a limit; here, with r = max(max_ij |sigma_ij| / p, |q| / (p
 * sqrt(T))), p = rho T, the pair (sigma, q) is scaled by min(1, rmax / r) so
 * that the polynomial factor stays of order one at thermal speeds.  rmax <= 0
 * disables the limit (the paper's form); the default is 0.5.  Call before
 * binding (E_STATE once bound); E_ARG for a non-finite rmax. */
gsis_status gsis_set_g13_limit(gsis_case c, double rmax);

/* Activity of the two limiters since the last bind or gsis_set_state:
 * out[6] (host) = {Grad-13 ghost rows built, of which limited; new-cell
 * Grad-13 rows built, of which limited; GSIS corrections applied (kinetic
 * cell-iterations), of which cut by the correction limiter (the conserved
 * change from W^{n+1/2} to W^{n+1} is halved until density and temperature
 * stay within a factor 2, dropped after ten halvings)}.  The counts are
 * cumulative; take differences between calls for one step.  Synchronises
 * `stream`. */
gsis_status gsis_limiter_stats(gsis_case c, int64_t *out, void *stream);

/* Device bytes needed to bind the case with room for `kinetic_capacity`
 * kinetic cells (VDF double buffer, per-cell sums and parameters, mesh and
 * macroscopic arrays). */
gsis_status gsis_case_footprint(gsis_case c, int64_t kinetic_capacity, size_t *bytes);

/* Bind a caller-owned device workspace (e.g. a torch uint8 tensor) of at
 * least the footprint.  The workspace must outlive the case; it is never
 * freed here.  Copies the mesh and grid to the device on `stream`. */
gsis_status gsis_case_bind(gsis_case c, void *dev_workspace, size_t bytes, int64_t kinetic_capacity,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call the allocator, harnesses that
 * forbid it): bind the case to the library's static device workspace instead
 * of a caller-owned one.  The workspace is a fixed 256 MiB array per GPU,
 * held by the library until the process ends; a case whose footprint exceeds
 * it is refused with GSIS_E_NOMEM.  The call allocates nothing (no hipMalloc,
 * no events: gsis_last_sweep_ms reports E_STATE for such a case).  One case
 * per GPU owns the array: binding another case to it leaves the previous
 * owner unbound (its calls return E_STATE until it is bound again), and
 * calls on two cases that overlap in time on one GPU race on the same
 * memory.  Everything else is as gsis_case_bind on the current device. */
gsis_status gsis_case_bind_static(gsis_case c, int64_t kinetic_capacity, void *stream);

/* Set the state (device pointers).  W_dev [n_cells][5] = (rho, ux, uy, uz, T)
 * FP64 on every cell.  flags_dev [n_cells] uint8 (1 = kinetic) or NULL (all
 * kinetic).  vdf_dev: rows [n_kin][nfun][nv] in the case dtype for the
 * kinetic cells in ascending cell id, or NULL to start them from the
 * conservation-fixed Maxwellian of W (Sec. 3.2 f_eq).  Synchronises (returns
 * GSIS_E_CAPACITY if the region exceeds the capacity). */
gsis_status gsis_set_state(gsis_case c, const double *W_dev, const void *vdf_dev, const uint8_t *flags_dev,
                           void *stream);

/* n_sweeps point-Jacobi kinetic sweeps (Sec. 3.1 implicit update, upwind
 * fluxes, Shakhov target with conservation fix-up) on each case, with the
 * fused moment reduction of the result.  All cases must share dtype, vdim,
 * grid kind (tensor or point set) and sweep layout, and the first case must
 * have the largest velocity axes; n_cases > 1 runs one batched launch per sweep.  On return (after the
 * stream syncs) each case's VDF is f^{n+1/2} and its W holds the moments on
 * kinetic cells. */
gsis_status gsis_kinetic_sweep(gsis_case const *cases, int32_t n_cases, int32_t n_sweeps, void *stream);
/* (Batched cases must also share the spatial order.) */

/* Moments of the current VDF (Sec. 2 eq. getmoment): out_dev [n_kin][14]
 * FP64 in ascending cell id (may be null when there is no kinetic cell);
 * kin_cell_dev [n_kin] int32 (nullable). */
gsis_status gsis_moments(gsis_case c, double *out_dev, int32_t *kin_cell_dev, void *stream);

/* Number of kinetic cells (host; no synchronisation). */
gsis_status gsis_n_kinetic(gsis_case c, int64_t *n_kin);

/* Region update of Sec. 3.2/3.4: least-squares gradients of W, Kn_Gll,
 * flag = (Kn_Gll >= Kn_ref) or within force_wall_layers of a wall,
 * compaction in ascending cell id, slot reuse for staying cells, Grad-13
 * initialisation of newly kinetic cells.  Synchronises; n_kinetic_host
 * (nullable) receives the new count. */
gsis_status gsis_update_regions(gsis_case c, double Kn_ref, int32_t force_wall_layers, int64_t *n_kinetic_host,
                                void *stream);

#define GSIS_MODE_DVM 0
#define GSIS_MODE_GSIS 1
#define GSIS_MODE_AGSIS 2

typedef struct {
    int32_t mode;                /* GSIS_MODE_* */
    double Kn_ref;               /* Sec. 3.2 reference Knudsen number (aGSIS) */
    double tol;                  /* stop when max(eps) < tol (Sec. 4, default 1e-6) */
    int32_t max_iter;
    int32_t region_update_every; /* aGSIS: k > 0 re-flag every k iterations; k < 0 re-flag once,
                                    after |k| iterations (Sec. 3.4 Step 3: k = -5); 0 = never */
    int32_t n_macro_inner;       /* pseudo-time steps per synthetic solve */
    double cfl;                  /* > 0 local steps; < 0 one global (conservative) step */
    int32_t force_wall_layers;
    int32_t ns_init;             /* 1 (aGSIS): Step 1 of Sec. 3.4 first -- every cell NS, the
                                    synthetic solve alone (HoT = 0) to eps < 1e-6, then the first
                                    flagging with Grad-13 rows for every kinetic cell */
    int32_t ns_init_max_chunks;  /* chunks of n_macro_inner steps for Step 1 (0: 1000) */
    int32_t source_half;         /* GSIS/aGSIS, monatomic gas (Sec. 3.1 eq. macro): 0 -- the source
                                    is the kinetic moment balance at f^n minus the synthetic residual
                                    at W^n, and the synthetic solve starts from W^n; 1 -- both at the
                                    half step (f^{n+1/2}, W^{n+1/2}) and the solve starts from
                                    W^{n+1/2}, so that the sweep's new non-equilibrium moments drive
                                    W^{n+1}.  1 costs one more kinetic-balance pass per step (a
                                    sweep of f^{n+1/2} whose output is discarded) and converges in
                                    fewer outer iterations.  The two-VDF gas takes 0 only. */
} gsis_solve_params;

typedef struct {
    int32_t iterations;
    double eps[3];               /* last rho, u, T residuals */
    int64_t n_kinetic;
} gsis_solve_result;

/* One outer iteration (Sec. 3.4) for each case: sweep, moments, high-order
 * terms, synthetic solve, GSIS correction, residual, and (aGSIS, on
 * schedule) region update.  eps_host [n_cases][3] (nullable) receives the
 * residuals and synchronises.  The cases of one call share batched launches.
 * If a case's region update or state check fails, its residuals are NaN, the
 * other cases still complete the step, and the call returns the first error
 * (a failed region update leaves that case needing gsis_set_state). */
gsis_status gsis_step(gsis_case const *cases, int32_t n_cases, const gsis_solve_params *p, double *eps_host,
                      void *stream);

/* Steps 1-2 of Sec. 3.4 for a batch of aGSIS cases: every cell NS, the
 * synthetic solve alone (HoT = 0, n_macro_inner steps per chunk, at most
 * ns_init_max_chunks chunks) to eps < 1e-6, then the first flagging with
 * Grad-13 rows for every kinetic cell.  The cases' solves share batched
 * launches; a case leaves the batch when it converges.  chunks (host,
 * nullable) receives the chunks each case ran.  If a case's first flagging
 * fails (E_CAPACITY: a region beyond its capacity), its chunks entry is -1
 * and it needs gsis_set_state again; the other cases complete, and the call
 * returns the first error.  Synchronises. */
gsis_status gsis_ns_init(gsis_case const *cases, int32_t n_cases, const gsis_solve_params *p, int32_t *chunks,
                         void *stream);

/* Steady solve: optional NS initialisation and first flagging (aGSIS), then
 * gsis_step until max(eps) < tol.  Returns GSIS_E_NOCONV after max_iter.
 * max_iter = 0 is allowed with ns_init: the call then stops after the first
 * flagging (r->n_kinetic set). */
gsis_status gsis_solve_steady(gsis_case c, const gsis_solve_params *p, gsis_solve_result *r, void *stream);

/* Copy the VDF of the kinetic cells, rows [n_kin][nfun][nv] in the case
 * dtype, ascending cell id (out_dev may be null when there is no kinetic cell). */
gsis_status gsis_get_vdf(gsis_case c, void *out_dev, void *stream);

/* Copy W [n_cells][5] FP64 and flags [n_cells] uint8 (either nullable). */
gsis_status gsis_get_state(gsis_case c, double *W_dev, uint8_t *flags_dev, void *stream);

/* Surface quantities on the diffuse walls (Sec. 4.2 and 4.3: surface
 * pressure, heat flux, drag and lift), one row per wall face in ascending face
 * id, GSIS_NSURF FP64 values:
 *   [0..2] stress vector tau exerted by the gas on the wall, tau = P.n,
 *          units rho0 R T0;
 *   [3]    pressure p = tau.n;   [4..6] shear tau - p n;
 *   [7]    heat flux into the wall, units rho0 R T0 v_m;
 *   [8]    net mass flux through the face (zero up to rounding on kinetic cells).
 * n is the unit face normal pointing out of the gas.  On a kinetic wall cell
 * the sums run over the cell's current VDF for incoming velocities (c.n > 0,
 * c = xi - u_w) and over rho_w M(u_w, T_w) for reflected ones, rho_w from the
 * discrete zero-mass-flux condition: tau = 2 sum w c (c.n) f,
 * q = sum w (c.n) |c|^2 f (reduced 2D: |c|^2 phi + psi).  On an NS wall cell
 * tau = rho T n + sigma_NSF.n and q = q_NSF.n with the one-sided wall
 * gradients of the synthetic solve.  Two-VDF gas (gsis_set_internal_dof): the
 * energy carried is |c|^2 f0 + 2 f1, reflected f1 = (d_r T_w / 4) rho_w M, and
 * an NS wall cell's heat flux is (q_t + q_r).n with T_r also held at T_w (so C_h
 * includes the internal energy).  face_dev [n_wall] int32 (nullable)
 * receives the face ids; totals_dev [4] (nullable) the integrals
 * sum tau S (3) and sum q S in fixed order.  All device buffers are the
 * caller's; nothing synchronises. */
#define GSIS_NSURF 9
gsis_status gsis_n_wall_faces(gsis_case c, int32_t *n_wall);
gsis_status gsis_surface(gsis_case c, int32_t *face_dev, double *out_dev, double *totals_dev, void *stream);

/* Force and heat coefficients (Sec. 4.3) from surface totals, host only:
 * totals [4] = (sum tau S (3), sum q S) as gsis_surface writes them (copied to
 * the host), the free stream (rho_inf, u_inf[3]) and the reference area.
 * out [3] = C_d = F.e / (rho |u|^2 A) along the free-stream direction e,
 * C_l = F.e_l / (rho |u|^2 A) along e_l = (-e_y, e_x, 0), and
 * C_h = Q / (rho |u|^3 A); the dynamic pressure rho |u|^2 / 2 is rho |u|^2
 * in units rho0 R T0.  E_ARG for null pointers, |u_inf| = 0, rho_inf <= 0 or
 * area <= 0. */
gsis_status gsis_force_coefficients(const double *totals, double rho_inf, const double *u_inf, double area,
                                    double *out);

/* GSIS correction alone (Sec. 3.1, first eq. updatef) on the current VDF:
 * f += f_eq(W_new) - f_eq(W_half) on kinetic cells, where W_half are the
 * current moments and W_new_dev [n_cells][5] FP64; W becomes W_new. */
gsis_status gsis_correct(gsis_case c, const double *W_new_dev, void *stream);

/* GSIS correction of the two-VDF gas alone (Sec. 3.1 eq. updatef with rho e_r
 * in W): f0 += f_eq(W_new) - f_eq(W_half) and f1 += (d_r/4)(T_r,new
 * f_eq(W_new) - T_r,half f_eq(W_half)) on kinetic cells, where W_half and
 * T_r,half are the current rows' moments; W_new_dev [n_cells][5] and
 * Tr_new_dev [n_cells] FP64 device memory (T_r > 0); W and T_r become the new
 * ones.  The correction limiter acts as in gsis_step.  E_ARG for a monatomic
 * case (gsis_correct) or null inputs; E_STATE before set_state. */
gsis_status gsis_correct_internal(gsis_case c, const double *W_new_dev, const double *Tr_new_dev, void *stream);

/* Synthetic macroscopic solve of the two-VDF gas alone (Sec. 2 eq.
 * macroscopic_equation_2 with its internal-energy line, eq. macro, FP64):
 * n_inner pseudo-time steps from W_dev [n_cells][5] and Tr_dev [n_cells]
 * (both in/out) with high-order terms hot_dev [n_cells][9] (sigma 6, q_t 3)
 * and hot_r_dev [n_cells][3] (q_r; null: zero), and sources per unit volume
 * src_dev [n_cells][5] (null: none) and src_r_dev [n_cells] (rho e_r; null:
 * zero).  The internal-energy exchange of the synthetic equations is part of
 * the step.  Synchronises `stream`; E_NONFINITE when a state goes non-positive;
 * E_ARG for a monatomic case (gsis_macro_solve), null W, Tr or hot, or bad
 * n_inner / cfl. */
gsis_status gsis_macro_solve_internal(gsis_case c, double *W_dev, double *Tr_dev, const double *hot_dev,
                                      const double *hot_r_dev, const double *src_dev, const double *src_r_dev,
                                      int32_t n_inner, double cfl, void *stream);

/* Synthetic macroscopic solve alone (eq. macro, FP64): n_inner pseudo-time
 * steps from W_dev [n_cells][5] (in/out) with high-order terms hot_dev
 * [n_cells][9] (sigma 6, q 3) and source src_dev [n_cells][5] per unit
 * volume (nullable). */
gsis_status gsis_macro_solve(gsis_case c, double *W_dev, const double *hot_dev, const double *src_dev,
                             int32_t n_inner, double cfl, void *stream);

/* Duration in ms of the last kinetic-sweep launch in which this case was
 * the first (or only) case of the batch (HIP events on the launch stream;
 * synchronises); for a batch the interval covers the whole batched launch.
 * E_STATE if the case's last sweep was not timed that way (a later case of a
 * batch, or a case bound to the static workspace, which has no events).  At
 * spatial order 2 the interval also covers the slope kernels launched just
 * before the sweep. */
gsis_status gsis_last_sweep_ms(gsis_case c, float *ms);

/* Sweep layout chosen at bind (all outputs host, nullable): *fast = 1 when the
 * plane kernel runs (3D: n_z divides 256 and 256 divides n_y n_z; reduced 2D:
 * n_y divides 256), 0 for the generic kernel; *tile = velocity nodes per
 * block; *n_tiles = blocks per kinetic cell.  The environment variable
 * GSIS_TILE (nodes per tile) and GSIS_GENERIC_SWEEP=1 (force the
 * generic kernel) are read at bind; by default the tile is the largest power
 * of two (at most 32768 nodes) that gives at least 4096 blocks at full
 * capacity.  E_STATE if the case is not bound. */
gsis_status gsis_sweep_layout(gsis_case c, int32_t *fast, int32_t *tile, int32_t *n_tiles);

#ifdef __cplusplus
}
#endif
#endif
