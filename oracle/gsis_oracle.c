/*
 * gsis_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * See gsis_oracle.h for units and layouts.  Each function follows one
 * passage of Zhang, Zeng & Wu, arXiv 2501.02245, cited by section and
 * equation label; readings of points the paper leaves open are stated where
 * they are used.  No blocking, fusion or reordering: loops run over cells,
 * faces and velocity nodes in the order the definitions are written.
 */
#include "gsis_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846;

int32_t oc_nv(const oc_grid *g)
{
    if (g->npts > 0) return g->npts;
    return g->vdim == 3 ? g->n[0] * g->n[1] * g->n[2] : g->n[0] * g->n[1];
}

int32_t oc_nfun(const oc_grid *g) { return g->vdim == 3 ? 1 : 2; }

/* threads an OpenMP loop of the oracle uses (reported beside its timings) */
int32_t oc_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the threads of the oracle's OpenMP loops (timing on one core); n <= 0
 * leaves the count unchanged */
void oc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}

/* velocity node k -> (xi, weight); xi_z = 0 for the reduced grid */
static void node(const oc_grid *g, int32_t k, double *xi, double *w)
{
    if (g->npts > 0) {
        for (int d = 0; d < 3; ++d) xi[d] = g->pts[3 * k + d];
        *w = g->pw[k];
    } else if (g->vdim == 3) {
        int32_t iz = k % g->n[2];
        int32_t iy = (k / g->n[2]) % g->n[1];
        int32_t ix = k / (g->n[2] * g->n[1]);
        xi[0] = g->x[0][ix]; xi[1] = g->x[1][iy]; xi[2] = g->x[2][iz];
        *w = g->w[0][ix] * g->w[1][iy] * g->w[2][iz];
    } else {
        int32_t iy = k % g->n[1];
        int32_t ix = k / g->n[1];
        xi[0] = g->x[0][ix]; xi[1] = g->x[1][iy]; xi[2] = 0.0;
        *w = g->w[0][ix] * g->w[1][iy];
    }
}

/* ------------------------------------------------------------------------
 * Moments, Sec. 2 eq. (getmoment), scaled:
 *   rho = sum w f, rho u = sum w xi f, c = xi - u,
 *   p = rho T = (2/3) sum w c^2 f, sigma = 2 sum w (cc - c^2 I/3) f,
 *   q = sum w c^2 c f.
 * Reduced pair (phi, psi): (3/2) p = sum w (c^2 phi + psi),
 *   sigma_xx = 2 sum w cx^2 phi - p, sigma_zz = 2 sum w psi - p,
 *   q = sum w c (c^2 phi + psi).
 * ------------------------------------------------------------------------ */
void oc_moments(const oc_grid *g, const double *f, double *mom)
{
    int32_t nv = oc_nv(g);
    double xi[3], w;
    double rho = 0, m[3] = {0, 0, 0};
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        rho += w * f[k];
        for (int d = 0; d < 3; ++d) m[d] += w * xi[d] * f[k];
    }
    double u[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
    double e = 0, cc[3][3] = {{0}}, q[3] = {0, 0, 0}, psum = 0;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c[3] = {xi[0] - u[0], xi[1] - u[1], xi[2] - u[2]};
        if (g->vdim == 2) c[2] = 0.0;
        double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        double fk = f[k];
        double psik = (g->vdim == 2) ? f[nv + k] : 0.0;
        e += w * (c2 * fk + psik);
        psum += w * psik;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) cc[i][j] += w * c[i] * c[j] * fk;
            q[i] += w * c[i] * (c2 * fk + psik);
        }
    }
    double p = (2.0 / 3.0) * e;
    mom[0] = rho;
    mom[1] = u[0]; mom[2] = u[1]; mom[3] = (g->vdim == 2) ? 0.0 : u[2];
    mom[4] = p / rho;
    if (g->vdim == 3) {
        mom[5] = 2.0 * cc[0][0] - p;
        mom[6] = 2.0 * cc[1][1] - p;
        mom[7] = 2.0 * cc[2][2] - p;
        mom[8] = 2.0 * cc[0][1];
        mom[9] = 2.0 * cc[0][2];
        mom[10] = 2.0 * cc[1][2];
        mom[11] = q[0]; mom[12] = q[1]; mom[13] = q[2];
    } else {
        mom[5] = 2.0 * cc[0][0] - p;
        mom[6] = 2.0 * cc[1][1] - p;
        mom[7] = 2.0 * psum - p;
        mom[8] = 2.0 * cc[0][1];
        mom[9] = 0.0; mom[10] = 0.0;
        mom[11] = q[0]; mom[12] = q[1]; mom[13] = 0.0;
    }
}

/* ------------------------------------------------------------------------
 * Equilibrium (Sec. 3.2, f_eq of the Grad-type construction), scaled:
 *   M = rho (pi T)^(-3/2) exp(-c^2/T);  reduced: phi = rho (pi T)^(-1)
 *   exp(-c^2/T), psi = (T/2) phi.
 * ------------------------------------------------------------------------ */
void oc_maxwellian(const oc_grid *g, double rho, const double *u, double T, double *out)
{
    int32_t nv = oc_nv(g);
    double xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c2 = 0;
        for (int d = 0; d < g->vdim; ++d) c2 += (xi[d] - u[d]) * (xi[d] - u[d]);
        if (g->vdim == 3) {
            out[k] = rho * pow(PI * T, -1.5) * exp(-c2 / T);
        } else {
            double phi = rho / (PI * T) * exp(-c2 / T);
            out[k] = phi;
            out[nv + k] = 0.5 * T * phi;
        }
    }
}

/* ------------------------------------------------------------------------
 * Reference distribution of the kinetic model (Sec. 2, reference
 * distributions g_0t, g_0r and the heat-flux mixing matrix).  For d_r = 0 the
 * combination g = (1 - 1/Z_r) g_0t + g_0r / Z_r has heat-flux coefficient
 * 3 (1 - A_tt) for every Z_r, i.e. the Shakhov form with Pr = A_tt:
 *   g = M [1 + (4/5)(1 - Pr) q.c / (p T) (c^2/T - 5/2)]   (scaled units).
 * Reduced (integrated over xi_z, u_z = q_z = 0):
 *   phi: M2 [1 + K q.c (c^2/T - 2)],  psi: (T/2) M2 [1 + K q.c (c^2/T - 1)].
 * ------------------------------------------------------------------------ */
void oc_shakhov(const oc_grid *g, double Pr, const double *mom, double *out)
{
    int32_t nv = oc_nv(g);
    double rho = mom[0], T = mom[4];
    const double *u = mom + 1, *q = mom + 11;
    double K = 0.8 * (1.0 - Pr) / (rho * T * T);
    double xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c[3] = {0, 0, 0}, c2 = 0, qc = 0;
        for (int d = 0; d < g->vdim; ++d) {
            c[d] = xi[d] - u[d];
            c2 += c[d] * c[d];
            qc += q[d] * c[d];
        }
        if (g->vdim == 3) {
            double M = rho * pow(PI * T, -1.5) * exp(-c2 / T);
            out[k] = M * (1.0 + K * qc * (c2 / T - 2.5));
        } else {
            double M = rho / (PI * T) * exp(-c2 / T);
            out[k] = M * (1.0 + K * qc * (c2 / T - 2.0));
            out[nv + k] = 0.5 * T * M * (1.0 + K * qc * (c2 / T - 1.0));
        }
    }
}

/* dense Gaussian elimination with partial pivoting, n <= 8 */
static int solve_small(int n, double *A, double *b)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0) return -1;
        if (piv != col) {
            for (int j = 0; j < n; ++j) {
                double t = A[col * n + j]; A[col * n + j] = A[piv * n + j]; A[piv * n + j] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double fac = A[r * n + col] / A[col * n + col];
            for (int j = col; j < n; ++j) A[r * n + j] -= fac * A[col * n + j];
            b[r] -= fac * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Conservation fix-up (reading: the paper states that the relaxation term
 * conserves mass, momentum and energy; on a truncated discrete grid it does
 * so only to quadrature error, so the target is multiplied by
 * P(c) = a0 + a.c + b c^2 chosen to make the discrete collision invariants
 * exact).  Basis and test functions {1, c_d, c^2}; for the reduced pair the
 * energy test function is c^2 on phi and 1 on psi, and P multiplies both.
 * ------------------------------------------------------------------------ */
int32_t oc_fixup(const oc_grid *g, double rho, const double *u, double T, double *gv, double *coef)
{
    int32_t nv = oc_nv(g);
    int nb = g->vdim + 2;
    double A[25] = {0}, b[5] = {0};
    double xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c[3] = {0, 0, 0}, c2 = 0;
        for (int d = 0; d < g->vdim; ++d) { c[d] = xi[d] - u[d]; c2 += c[d] * c[d]; }
        double p[5];
        p[0] = 1.0;
        for (int d = 0; d < g->vdim; ++d) p[1 + d] = c[d];
        p[nb - 1] = c2;
        double gf = gv[k];
        double gp = (g->vdim == 2) ? gv[nv + k] : 0.0;
        for (int a = 0; a < nb; ++a) {
            /* test function a applied to (g_phi, g_psi) */
            double t = p[a] * gf;
            if (a == nb - 1) t += gp;   /* energy: c^2 phi + psi */
            for (int bb = 0; bb < nb; ++bb) A[a * nb + bb] += w * t * p[bb];
        }
    }
    b[0] = rho;
    b[nb - 1] = 1.5 * rho * T;
    if (solve_small(nb, A, b) != 0) return -1;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c2 = 0, P = b[0];
        for (int d = 0; d < g->vdim; ++d) {
            double c = xi[d] - u[d];
            c2 += c * c;
            P += b[1 + d] * c;
        }
        P += b[nb - 1] * c2;
        gv[k] *= P;
        if (g->vdim == 2) gv[nv + k] *= P;
    }
    if (coef)
        for (int a = 0; a < nb; ++a) coef[a] = b[a];
    return 0;
}

int32_t oc_equilibrium(const oc_grid *g, const oc_gas *gas, const double *mom, double *out)
{
    oc_shakhov(g, gas->Pr, mom, out);
    return oc_fixup(g, mom[0], mom + 1, mom[4], out, NULL);
}

int32_t oc_feq(const oc_grid *g, const double *W5, double *out)
{
    oc_maxwellian(g, W5[0], W5 + 1, W5[4], out);
    return oc_fixup(g, W5[0], W5 + 1, W5[4], out, NULL);
}

/* ------------------------------------------------------------------------
 * Grad-type distribution (Sec. 3.2, eq. G13_VDF), scaled units:
 *   f = M [1 + sigma:cc / (p T) + (2 q.c / (p T)) (2 c^2 / (5 T) - 1)].
 * Reduced pair (sigma_xz = sigma_yz = q_z = u_z = 0):
 *   phi: M2 [1 + (s2:cc + sigma_zz T/2)/(pT) + (2q.c/(pT))(2c^2/(5T) - 4/5)]
 *   psi: (T/2) M2 [1 + (s2:cc + 3 T sigma_zz / 2)/(pT) + (2q.c/(pT))(2c^2/(5T) - 2/5)]
 * ------------------------------------------------------------------------ */
void oc_g13(const oc_grid *g, const double *mom, double *out)
{
    int32_t nv = oc_nv(g);
    double rho = mom[0], T = mom[4], p = rho * T;
    const double *u = mom + 1, *s = mom + 5, *q = mom + 11;
    double xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c[3] = {0, 0, 0}, c2 = 0, qc = 0;
        for (int d = 0; d < g->vdim; ++d) {
            c[d] = xi[d] - u[d];
            c2 += c[d] * c[d];
            qc += q[d] * c[d];
        }
        double scc = s[0] * c[0] * c[0] + s[1] * c[1] * c[1] + s[2] * c[2] * c[2]
                   + 2.0 * (s[3] * c[0] * c[1] + s[4] * c[0] * c[2] + s[5] * c[1] * c[2]);
        if (g->vdim == 3) {
            double M = rho * pow(PI * T, -1.5) * exp(-c2 / T);
            out[k] = M * (1.0 + scc / (p * T) + 2.0 * qc / (p * T) * (0.4 * c2 / T - 1.0));
        } else {
            double M = rho / (PI * T) * exp(-c2 / T);
            out[k] = M * (1.0 + (scc + 0.5 * T * s[2]) / (p * T)
                          + 2.0 * qc / (p * T) * (0.4 * c2 / T - 0.8));
            out[nv + k] = 0.5 * T * M * (1.0 + (scc + 1.5 * T * s[2]) / (p * T)
                                         + 2.0 * qc / (p * T) * (0.4 * c2 / T - 0.4));
        }
    }
}

/* tau = mu / p_t with mu = mu(T0) (T/T0)^omega and the Kn definition of
 * Sec. 2: tau = (2 Kn / sqrt(pi)) T^(omega - 1) / rho in scaled units. */
double oc_tau(const oc_gas *gas, double rho, double T)
{
    return 2.0 * gas->Kn / sqrt(PI) * pow(T, gas->omega - 1.0) / rho;
}

/* cell -> face adjacency (CSR) */
static void build_adjacency(const oc_mesh *m, int32_t **ptr_out, int32_t **idx_out)
{
    int32_t *cnt = (int32_t *)calloc((size_t)m->n_cells + 1, sizeof(int32_t));
    for (int32_t f = 0; f < m->n_faces; ++f) {
        cnt[m->face_cells[2 * f] + 1]++;
        if (m->face_cells[2 * f + 1] >= 0) cnt[m->face_cells[2 * f + 1] + 1]++;
    }
    for (int32_t i = 0; i < m->n_cells; ++i) cnt[i + 1] += cnt[i];
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt[m->n_cells] > 0 ? cnt[m->n_cells] : 1));
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->n_cells > 0 ? m->n_cells : 1));
    for (int32_t i = 0; i < m->n_cells; ++i) pos[i] = cnt[i];
    for (int32_t f = 0; f < m->n_faces; ++f) {
        idx[pos[m->face_cells[2 * f]]++] = f;
        if (m->face_cells[2 * f + 1] >= 0) idx[pos[m->face_cells[2 * f + 1]]++] = f;
    }
    free(pos);
    *ptr_out = cnt;
    *idx_out = idx;
}

/* ------------------------------------------------------------------------
 * Kinetic update of Sec. 3.1 (the discretised kinetic equation before
 * eq. updatef), first-order upwind face values, point-Jacobi lagging of the
 * neighbour values (readings: upwind by the sign of xi.n; neighbours and the
 * reference distribution at iterate n):
 *
 *   f_i^{n+1/2} = ( f_i^n/dt + g_i^n/tau_i^n + sum_{a<0} |a| f_j^n )
 *               / ( 1/dt + 1/tau_i^n + sum_{a>0} a ),   a = (xi.n) S / V.
 *
 * Upwind values: kinetic neighbour -> its f^n; NS neighbour -> Grad-13 of
 * its state (Sec. 3.2); diffuse wall -> rho_w M(u_w, T_w) with rho_w from a
 * zero discrete mass flux of f_i^n; far field -> M(rho, u, T) of the patch.
 * ------------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* scell (nullable): slopes of fcell; the outgoing values at the face are then
 * the second-order ones fcell + scell . r, r = x_face - x_cell */
static double wall_density(const oc_grid *g, const double *fcell, const double *scell, const double *r,
                           const double *n, const double *uw, double Tw, double *Mw)
{
    /* Mw receives M(1, uw, Tw) at the nodes */
    int32_t nv = oc_nv(g);
    oc_maxwellian(g, 1.0, uw, Tw, Mw);
    double out = 0, in = 0, xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double xn = xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2];
        if (xn > 0) out += w * xn * (fcell[k] + (scell ? dot3(scell + 3 * (size_t)k, r) : 0.0));
        else if (xn < 0) in += w * (-xn) * Mw[k];
    }
    return out / in;
}

/* Upwind source rows for the faces of kinetic cell i, all at iterate n:
 * srcp[l] points at the values on the far side of local face l; nrm[4l..]
 * holds the outward unit normal and S/V.  `scratch` has room for nf rows.
 * si (nullable): slopes of fi, for the second-order outgoing values that fix
 * the wall densities. */
static void face_sources(const oc_mesh *m, const oc_grid *g, const int32_t *cptr, const int32_t *cidx,
                         int32_t i, const int32_t *slot_of_cell, const double *f_old, const double *ghost,
                         const double *fi, const double *si, double *scratch, double *nrm, const double **srcp)
{
    size_t row = (size_t)oc_nfun(g) * oc_nv(g);
    int32_t nf = cptr[i + 1] - cptr[i];
    for (int32_t l = 0; l < nf; ++l) {
        int32_t f = cidx[cptr[i] + l];
        int32_t own = m->face_cells[2 * f], oth = m->face_cells[2 * f + 1];
        double sgn = (own == i) ? 1.0 : -1.0;
        int32_t nb = (own == i) ? oth : own;
        for (int d = 0; d < 3; ++d) nrm[4 * l + d] = sgn * m->face_normal[3 * f + d];
        nrm[4 * l + 3] = m->face_area[f] / m->cell_volume[i];
        double *s = scratch + (size_t)l * row;
        if (nb >= 0) {
            if (slot_of_cell[nb] >= 0) {
                srcp[l] = f_old + (size_t)slot_of_cell[nb] * row;
            } else {
                oc_g13(g, ghost + (size_t)nb * OC_NMOM, s);
                srcp[l] = s;
            }
        } else {
            int32_t p = -1 - nb;
            const double *ps = m->patch_state + 5 * p;
            if (m->patch_kind[p] == OC_WALL) {
                double r[3];
                for (int d = 0; d < 3; ++d) r[d] = m->face_center[3 * f + d] - m->cell_center[3 * i + d];
                double rw = wall_density(g, fi, si, r, nrm + 4 * l, ps + 1, ps[4], s);
                for (size_t k = 0; k < row; ++k) s[k] *= rw;
            } else {
                oc_maxwellian(g, ps[0], ps + 1, ps[4], s);
            }
            srcp[l] = s;
        }
    }
}

/* ------------------------------------------------------------------------
 * Second-order face values (Sec. 3: the kinetic equation is discretised by
 * a second-order finite-volume scheme whose details the paper leaves to its
 * references).  Readings:
 *  - each discrete-velocity value of a kinetic cell gets a least-squares
 *    gradient over the cell's kinetic neighbours (weights 1/|dx|^2, the first
 *    `dim` components; zero when those neighbours do not span `dim`
 *    dimensions: det(A) <= 1e-12 (tr A / dim)^dim);
 *  - the gradient is scaled by the Barth-Jespersen factor phi in [0, 1], the
 *    largest for which every face value f_i + phi g.(x_f - x_i) on a face to a
 *    kinetic neighbour lies between the smallest and largest of f_i and its
 *    kinetic neighbours' values;
 *  - a face value is reconstructed wherever its upwind side is a kinetic
 *    cell: the outgoing values of every face of a kinetic cell (walls, far
 *    field and NS interfaces included) and the incoming values from kinetic
 *    neighbours; incoming wall, far-field and Grad-13 ghost values are the
 *    face values themselves;
 *  - the wall density makes the net mass flux of the reconstructed outgoing
 *    and the wall's incoming values zero.
 * slope[n_slots][nfun * nv][3] = phi g, components beyond dim zero.
 * ------------------------------------------------------------------------ */
static int lsq_singular(int dim, const double *A)
{
    double tr = 0, det;
    for (int d = 0; d < dim; ++d) tr += A[d * dim + d];
    if (dim == 1) det = A[0];
    else if (dim == 2) det = A[0] * A[3] - A[1] * A[2];
    else
        det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
              A[2] * (A[3] * A[7] - A[4] * A[6]);
    return !(tr > 0) || det <= 1e-12 * pow(tr / dim, dim);
}

int32_t oc_kinetic_slopes(const oc_mesh *m, const oc_grid *g, int32_t n_kin, const int32_t *kin_cell,
                          const int32_t *slot_of_cell, const double *f, double *slope)
{
    int32_t nv = oc_nv(g), nfun = oc_nfun(g);
    size_t row = (size_t)nfun * nv;
    int dim = m->dim;
    int32_t *cptr, *cidx;
    build_adjacency(m, &cptr, &cidx);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < n_kin; ++t) {
        int32_t i = kin_cell[t];
        const double *fi = f + (size_t)slot_of_cell[i] * row;
        double *si = slope + (size_t)slot_of_cell[i] * row * 3;
        memset(si, 0, sizeof(double) * row * 3);
        /* kinetic neighbours: centre offsets and face-centre offsets */
        int32_t nk = 0;
        int32_t nbr[64];
        double dx[64][3], rf[64][3], A[9] = {0};
        for (int32_t l = cptr[i]; l < cptr[i + 1]; ++l) {
            int32_t fc = cidx[l];
            int32_t own = m->face_cells[2 * fc], oth = m->face_cells[2 * fc + 1];
            int32_t nb = (own == i) ? oth : own;
            if (nb < 0 || slot_of_cell[nb] < 0 || nk == 64) continue;
            nbr[nk] = nb;
            for (int d = 0; d < 3; ++d) {
                dx[nk][d] = m->cell_center[3 * nb + d] - m->cell_center[3 * i + d];
                rf[nk][d] = m->face_center[3 * fc + d] - m->cell_center[3 * i + d];
            }
            double r2 = 0;
            for (int d = 0; d < dim; ++d) r2 += dx[nk][d] * dx[nk][d];
            for (int a = 0; a < dim; ++a)
                for (int c = 0; c < dim; ++c) A[a * dim + c] += dx[nk][a] * dx[nk][c] / r2;
            ++nk;
        }
        if (nk == 0 || lsq_singular(dim, A)) continue;
        for (size_t k = 0; k < row; ++k) {
            double b[3] = {0, 0, 0}, Ak[9];
            double dmax = 0, dmin = 0;
            for (int32_t j = 0; j < nk; ++j) {
                double df = f[(size_t)slot_of_cell[nbr[j]] * row + k] - fi[k];
                double r2 = 0;
                for (int d = 0; d < dim; ++d) r2 += dx[j][d] * dx[j][d];
                for (int d = 0; d < dim; ++d) b[d] += dx[j][d] * df / r2;
                if (df > dmax) dmax = df;
                if (df < dmin) dmin = df;
            }
            memcpy(Ak, A, sizeof A);
            if (solve_small(dim, Ak, b) != 0) continue;
            /* Barth-Jespersen factor over the faces to kinetic neighbours */
            double phi = 1.0;
            for (int32_t j = 0; j < nk; ++j) {
                double ext = 0;
                for (int d = 0; d < dim; ++d) ext += b[d] * rf[j][d];
                if (ext > 0) phi = fmin(phi, dmax / ext);
                else if (ext < 0) phi = fmin(phi, dmin / ext);
            }
            for (int d = 0; d < dim; ++d) si[k * 3 + d] = phi * b[d];
        }
    }
    free(cptr);
    free(cidx);
    return 0;
}

/* face-centre offset r_own = x_face - x_i of local face l of cell i; for a
 * kinetic neighbour also r_nb = x_face - x_nb and its slot (else -1) */
static int32_t face_offsets(const oc_mesh *m, const int32_t *cptr, const int32_t *cidx, int32_t i, int32_t l,
                            const int32_t *slot_of_cell, double *r_own, double *r_nb)
{
    int32_t f = cidx[cptr[i] + l];
    int32_t own = m->face_cells[2 * f], oth = m->face_cells[2 * f + 1];
    int32_t nb = (own == i) ? oth : own;
    for (int d = 0; d < 3; ++d) r_own[d] = m->face_center[3 * f + d] - m->cell_center[3 * i + d];
    if (nb < 0 || slot_of_cell[nb] < 0) return -1;
    for (int d = 0; d < 3; ++d) r_nb[d] = m->face_center[3 * f + d] - m->cell_center[3 * nb + d];
    return slot_of_cell[nb];
}

/* The sweep below with second-order face values when slope is non-null:
 * the first-order implicit operator is kept, and the difference between the
 * reconstructed and first-order face fluxes, evaluated at iterate n, moves to
 * the right-hand side (deferred correction):
 *   outflow face (a > 0), any face:           num -= a (s_i . r_i)
 *   inflow face (a < 0) from a kinetic cell:  num += |a| (f_j + s_j . r_j)
 * with r = x_face - x_cell of the cell whose slope is used.  The point-Jacobi
 * iteration of this operator diverges without damping (its explicit
 * second-order terms couple downwind); a cell-wise pseudo-time term
 * (f_i^{n+1/2} - f_i^n)/dt_i, sized by the cell's largest outflow rate, makes
 * it converge and leaves its fixed point unchanged. */
static int32_t sweep_body(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                          int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                          const double *f_old, const double *ghost, const double *slope, double *f_new)
{
    int32_t nv = oc_nv(g), nfun = oc_nfun(g);
    size_t row = (size_t)nfun * nv;
    int32_t *cptr, *cidx;
    build_adjacency(m, &cptr, &cidx);
    int32_t err = 0;

#pragma omp parallel for schedule(dynamic, 1) reduction(min : err)
    for (int32_t t = 0; t < n_kin; ++t) {
        int32_t i = kin_cell[t];
        const double *fi = f_old + (size_t)slot_of_cell[i] * row;
        double *fo = f_new + (size_t)slot_of_cell[i] * row;
        int32_t nf = cptr[i + 1] - cptr[i];
        double mom[OC_NMOM];
        oc_moments(g, fi, mom);
        double tau = oc_tau(gas, mom[0], mom[4]);
        double *geq = (double *)malloc(sizeof(double) * row);
        double *src = (double *)malloc(sizeof(double) * row * (size_t)(nf > 0 ? nf : 1));
        double *nrm = (double *)malloc(sizeof(double) * 4 * (size_t)(nf > 0 ? nf : 1));
        const double **srcp = (const double **)malloc(sizeof(double *) * (size_t)(nf > 0 ? nf : 1));
        if (oc_equilibrium(g, gas, mom, geq) != 0) err = -7;
        const double *si = slope ? slope + (size_t)slot_of_cell[i] * row * 3 : NULL;
        face_sources(m, g, cptr, cidx, i, slot_of_cell, f_old, ghost, fi, si, src, nrm, srcp);
        /* pseudo-time step of the deferred-correction iteration (reading):
         * 1/dt_i = damp2 * max_k sum_{a_k > 0} a_k, the largest outflow rate
         * of the cell over the velocity grid; it vanishes at convergence */
        double inv_dt2 = 0.0;
        if (si) {
            double xk[3], wk;
            for (int32_t k = 0; k < nv; ++k) {
                node(g, k, xk, &wk);
                double out = 0.0;
                for (int32_t l = 0; l < nf; ++l) {
                    double a = (xk[0] * nrm[4 * l] + xk[1] * nrm[4 * l + 1] + xk[2] * nrm[4 * l + 2]) * nrm[4 * l + 3];
                    if (a > 0) out += a;
                }
                if (out > inv_dt2) inv_dt2 = out;
            }
            inv_dt2 *= gas->damp2;
        }
        int32_t *kslot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nf > 0 ? nf : 1));
        double *rown = (double *)malloc(sizeof(double) * 6 * (size_t)(nf > 0 ? nf : 1));
        for (int32_t l = 0; l < nf; ++l)
            kslot[l] = face_offsets(m, cptr, cidx, i, l, slot_of_cell, rown + 6 * l, rown + 6 * l + 3);
        double xi[3], w;
        for (int32_t k = 0; k < nv; ++k) {
            node(g, k, xi, &w);
            double den = gas->inv_dt + 1.0 / tau;
            double num[2];
            for (int32_t q = 0; q < nfun; ++q) num[q] = gas->inv_dt * fi[q * nv + k] + geq[q * nv + k] / tau;
            if (si) {
                den += inv_dt2;
                for (int32_t q = 0; q < nfun; ++q) num[q] += inv_dt2 * fi[q * nv + k];
            }
            for (int32_t l = 0; l < nf; ++l) {
                double a = (xi[0] * nrm[4 * l] + xi[1] * nrm[4 * l + 1] + xi[2] * nrm[4 * l + 2]) * nrm[4 * l + 3];
                if (a > 0) {
                    den += a;
                    if (si)
                        for (int32_t q = 0; q < nfun; ++q)
                            num[q] -= a * dot3(si + ((size_t)q * nv + k) * 3, rown + 6 * l);
                } else if (a < 0) {
                    for (int32_t q = 0; q < nfun; ++q) num[q] += -a * srcp[l][q * nv + k];
                    if (si && kslot[l] >= 0) {
                        const double *sj = slope + (size_t)kslot[l] * row * 3;
                        for (int32_t q = 0; q < nfun; ++q)
                            num[q] += -a * dot3(sj + ((size_t)q * nv + k) * 3, rown + 6 * l + 3);
                    }
                }
            }
            for (int32_t q = 0; q < nfun; ++q) fo[q * nv + k] = num[q] / den;
        }
        free(geq); free(src); free(nrm); free(srcp); free(kslot); free(rown);
    }
    free(cptr);
    free(cidx);
    return err;
}

int32_t oc_sweep(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                 int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                 const double *f_old, const double *ghost, double *f_new)
{
    return sweep_body(m, g, gas, n_kin, kin_cell, slot_of_cell, f_old, ghost, NULL, f_new);
}

int32_t oc_sweep2(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                  int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                  const double *f_old, const double *ghost, const double *slope, double *f_new)
{
    return sweep_body(m, g, gas, n_kin, kin_cell, slot_of_cell, f_old, ghost, slope, f_new);
}

/* ------------------------------------------------------------------------
 * Moment balance of the kinetic scheme at iterate n (the flux part of the
 * discretised kinetic equation of Sec. 3.1, summed against 1, xi, xi^2; the
 * relaxation term drops out because it conserves these moments):
 *   R_i = -sum_faces (S/V) sum_k w_k (xi_k.n) psi_k f_up,k
 * with the same upwind values as the sweep.  R[n_cells][5] = (mass,
 * momentum, energy) per unit volume; rows of non-kinetic cells are zero.
 * ------------------------------------------------------------------------ */
static int32_t residual_body(const oc_mesh *m, const oc_grid *g,
                             int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                             const double *f_old, const double *ghost, const double *slope, double *R)
{
    int32_t nv = oc_nv(g), nfun = oc_nfun(g);
    size_t row = (size_t)nfun * nv;
    int32_t *cptr, *cidx;
    build_adjacency(m, &cptr, &cidx);
    memset(R, 0, sizeof(double) * 5 * (size_t)m->n_cells);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t t = 0; t < n_kin; ++t) {
        int32_t i = kin_cell[t];
        const double *fi = f_old + (size_t)slot_of_cell[i] * row;
        int32_t nf = cptr[i + 1] - cptr[i];
        double *src = (double *)malloc(sizeof(double) * row * (size_t)(nf > 0 ? nf : 1));
        double *nrm = (double *)malloc(sizeof(double) * 4 * (size_t)(nf > 0 ? nf : 1));
        const double **srcp = (const double **)malloc(sizeof(double *) * (size_t)(nf > 0 ? nf : 1));
        const double *si = slope ? slope + (size_t)slot_of_cell[i] * row * 3 : NULL;
        face_sources(m, g, cptr, cidx, i, slot_of_cell, f_old, ghost, fi, si, src, nrm, srcp);
        double acc[5] = {0, 0, 0, 0, 0}, xi[3], w;
        for (int32_t l = 0; l < nf; ++l) {
            double rr[6];
            int32_t ks = face_offsets(m, cptr, cidx, i, l, slot_of_cell, rr, rr + 3);
            for (int32_t k = 0; k < nv; ++k) {
                node(g, k, xi, &w);
                double a = (xi[0] * nrm[4 * l] + xi[1] * nrm[4 * l + 1] + xi[2] * nrm[4 * l + 2]) * nrm[4 * l + 3];
                const double *up = (a > 0) ? fi : srcp[l];
                double fphi = up[k];
                double fpsi = (nfun == 2) ? up[nv + k] : 0.0;
                if (si && (a > 0 || ks >= 0)) {
                    /* reconstructed value of a kinetic upwind side */
                    const double *su = (a > 0) ? si : slope + (size_t)ks * row * 3;
                    const double *r = (a > 0) ? rr : rr + 3;
                    fphi += dot3(su + (size_t)k * 3, r);
                    if (nfun == 2) fpsi += dot3(su + ((size_t)nv + k) * 3, r);
                }
                double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
                acc[0] -= w * a * fphi;
                for (int d = 0; d < 3; ++d) acc[1 + d] -= w * a * xi[d] * fphi;
                acc[4] -= w * a * (x2 * fphi + fpsi);
            }
        }
        for (int c = 0; c < 5; ++c) R[5 * i + c] = acc[c];
        free(src); free(nrm); free(srcp);
    }
    free(cptr);
    free(cidx);
    return 0;
}

int32_t oc_kinetic_residual(const oc_mesh *m, const oc_grid *g,
                            int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                            const double *f_old, const double *ghost, double *R)
{
    return residual_body(m, g, n_kin, kin_cell, slot_of_cell, f_old, ghost, NULL, R);
}

int32_t oc_kinetic_residual2(const oc_mesh *m, const oc_grid *g,
                             int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                             const double *f_old, const double *ghost, const double *slope, double *R)
{
    return residual_body(m, g, n_kin, kin_cell, slot_of_cell, f_old, ghost, slope, R);
}

/* ------------------------------------------------------------------------
 * Least-squares gradients (Sec. 3.4 Step 2).  Reading: neighbours are the
 * cells across each face, weights 1/|dx|^2; a boundary face contributes the
 * patch value at the face centre (NaN entries: no contribution).  Only the
 * first `dim` components are solved; the rest are zero.
 * ------------------------------------------------------------------------ */
void oc_lsq_gradients(const oc_mesh *m, int32_t nvar, const double *phi, const double *bnd, double *grad)
{
    int32_t *cptr, *cidx;
    build_adjacency(m, &cptr, &cidx);
    int dim = m->dim;
    for (int32_t i = 0; i < m->n_cells; ++i) {
        for (int32_t v = 0; v < nvar; ++v) {
            double A[9] = {0}, b[3] = {0};
            for (int32_t l = cptr[i]; l < cptr[i + 1]; ++l) {
                int32_t f = cidx[l];
                int32_t own = m->face_cells[2 * f], oth = m->face_cells[2 * f + 1];
                int32_t nb = (own == i) ? oth : own;
                double dx[3], dphi;
                if (nb >= 0) {
                    for (int d = 0; d < 3; ++d) dx[d] = m->cell_center[3 * nb + d] - m->cell_center[3 * i + d];
                    dphi = phi[(size_t)nb * nvar + v] - phi[(size_t)i * nvar + v];
                } else {
                    double bv = bnd[(size_t)(-1 - nb) * nvar + v];
                    if (isnan(bv)) continue;
                    for (int d = 0; d < 3; ++d) dx[d] = m->face_center[3 * f + d] - m->cell_center[3 * i + d];
                    dphi = bv - phi[(size_t)i * nvar + v];
                }
                double r2 = 0;
                for (int d = 0; d < dim; ++d) r2 += dx[d] * dx[d];
                double wgt = 1.0 / r2;
                for (int a = 0; a < dim; ++a) {
                    for (int c = 0; c < dim; ++c) A[a * dim + c] += wgt * dx[a] * dx[c];
                    b[a] += wgt * dx[a] * dphi;
                }
            }
            double *gout = grad + ((size_t)i * nvar + v) * 3;
            gout[0] = gout[1] = gout[2] = 0.0;
            if (solve_small(dim, A, b) == 0)
                for (int d = 0; d < dim; ++d) gout[d] = b[d];
        }
    }
    free(cptr);
    free(cidx);
}

/* ------------------------------------------------------------------------
 * Newton and Fourier laws (Sec. 2, eq. NSF_constitutive) with the
 * conductivity of eq. mu_kappa for d_r = 0 (kappa = (mu R / 2) 5 / A_tt),
 * scaled: sigma = -(2 Kn/sqrt(pi)) mu (grad u + grad u^T - (2/3) div u I),
 *         q = -(5 Kn / (2 sqrt(pi) Pr)) mu grad T,   mu = T^omega.
 * grad_u[3*i + j] = d u_i / d x_j.
 * ------------------------------------------------------------------------ */
void oc_nsf(const oc_gas *gas, double T, const double *grad_u, const double *grad_T,
            double *sigma6, double *q3)
{
    double mu = pow(T, gas->omega);
    double cs = -2.0 * gas->Kn / sqrt(PI) * mu;
    double cq = -5.0 * gas->Kn / (2.0 * sqrt(PI) * gas->Pr) * mu;
    double div = grad_u[0] + grad_u[4] + grad_u[8];
    sigma6[0] = cs * (2.0 * grad_u[0] - 2.0 / 3.0 * div);
    sigma6[1] = cs * (2.0 * grad_u[4] - 2.0 / 3.0 * div);
    sigma6[2] = cs * (2.0 * grad_u[8] - 2.0 / 3.0 * div);
    sigma6[3] = cs * (grad_u[1] + grad_u[3]);
    sigma6[4] = cs * (grad_u[2] + grad_u[6]);
    sigma6[5] = cs * (grad_u[5] + grad_u[7]);
    for (int d = 0; d < 3; ++d) q3[d] = cq * grad_T[d];
}

/* ------------------------------------------------------------------------
 * Synthetic macroscopic equations (Sec. 2 eq. macroscopic_equation_2 with
 * the constitutive relations of eq. full_constitutive, discretised as in
 * eq. macro).  The paper defers F and Q to another work; this is the
 * reading used on both sides:
 *   conserved U = (rho, rho u, E = rho |u|^2 + 1.5 rho T), fluxes
 *   F.n = [rho u_n, rho u u_n + (p n + sigma.n)/2, (E + p) u_n + (sigma.n).u + q.n]
 *   convective part: kinetic flux-vector splitting, the xi.n > 0 half-range
 *   moments of the owner's Maxwellian plus the xi.n < 0 half of the other
 *   side's (the first-order upwinding of the kinetic sweep applied to the
 *   local equilibria, so both solvers carry the same numerical dissipation);
 *   viscous part: face gradients = mean of the two LSQ cell gradients plus a
 *   correction along the face normal that makes their projection on the
 *   centroid difference equal the jump (over-relaxed non-orthogonal form); sigma_f, q_f = NSF at T_f plus the mean
 *   of the two cells' high-order terms (zero on NS cells);
 *   far field: the same splitting against the patch state, no viscous flux;
 *   wall: isothermal no-slip (pressure plus the NSF viscous flux from
 *   one-sided gradients towards (u_w, T_w), no mass flux);
 *   source: an optional frozen per-cell term (the GSIS driver puts there the
 *   difference between the kinetic scheme's moment balance and this
 *   residual, both at iterate n, on kinetic cells);
 *   explicit update with local step dt_i = cfl V_i / sum_f S_f (|u_n| + a + 2 nu / d_f),
 *   d_f = normal distance between the centroids (twice the centroid-face
 *   normal distance on boundary faces),
 *   halved per cell (at most ten times) while the new rho or T would not be
 *   positive
 *   (cfl < 0: one global step, the minimum over cells of |cfl| V_i / sum ...),
 *   nu = max(4/3, 5/(3 Pr)) Kn T^omega / (sqrt(pi) rho).
 * ------------------------------------------------------------------------ */
static void prim_from_cons(const double *U, double *P)
{
    double rho = U[0];
    P[0] = rho;
    double u2 = 0;
    for (int d = 0; d < 3; ++d) { P[1 + d] = U[1 + d] / rho; u2 += P[1 + d] * P[1 + d]; }
    P[4] = (U[4] - rho * u2) / (1.5 * rho);
}

static void cons_from_prim(const double *P, double *U)
{
    double u2 = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    U[0] = P[0];
    for (int d = 0; d < 3; ++d) U[1 + d] = P[0] * P[1 + d];
    U[4] = P[0] * u2 + 1.5 * P[0] * P[4];
}

/* Half-range flux of a Maxwellian (kinetic flux-vector splitting): the
 * moments {1, xi, xi^2} x (xi.n) of M(rho, u, T) over xi.n > 0 (sgn = +1) or
 * xi.n < 0 (sgn = -1), in closed form with erf:
 *   <1> = (1 + sgn erf(s))/2 = A, B = sgn exp(-s^2)/(2 sqrt(pi)), s = u_n/sqrt(T)
 *   <xi_n>   = u_n A + sqrt(T) B
 *   <xi_n^2> = (u_n^2 + T/2) A + u_n sqrt(T) B
 *   <xi_n^3> = (u_n^3 + 3 u_n T/2) A + (u_n^2 + T) sqrt(T) B
 * mass = rho <xi_n>, momentum = rho (u_t <xi_n> + n <xi_n^2>),
 * energy = rho (<xi_n^3> + (|u_t|^2 + T) <xi_n>). */
static void half_flux(const double *P, const double *n, double sgn, double *F)
{
    double rho = P[0], T = P[4], sT = sqrt(T);
    double un = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
    double ut[3] = {P[1] - un * n[0], P[2] - un * n[1], P[3] - un * n[2]};
    double ut2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    double s = un / sT;
    double A = 0.5 * (1.0 + sgn * erf(s));
    double B = sgn * exp(-s * s) / (2.0 * sqrt(PI));
    double m1 = un * A + sT * B;
    double m2 = (un * un + 0.5 * T) * A + un * sT * B;
    double m3 = (un * un * un + 1.5 * un * T) * A + (un * un + T) * sT * B;
    F[0] = rho * m1;
    for (int d = 0; d < 3; ++d) F[1 + d] = rho * (ut[d] * m1 + n[d] * m2);
    F[4] = rho * (m3 + (ut2 + T) * m1);
}

/* Residual R_i = -sum_f F_f.n S_f (not divided by V_i) at primitive state W,
 * and the local-step denominators D_i = sum_f S_f (|u_n| + a + 2 nu / d_f).
 * Returns -7 if a density or temperature is not positive. */
static int32_t macro_residual(const oc_mesh *m, const oc_gas *gas,
                              const double *hot, const double *W,
                              double *R, double *D, double *pv, double *gr, const double *bv)
{
    int32_t nc = m->n_cells, nfc = m->n_faces;
    const double gam = 5.0 / 3.0;
    for (int32_t i = 0; i < nc; ++i) {
        if (!(W[5 * i] > 0) || !(W[5 * i + 4] > 0)) return -7;
        for (int c = 0; c < 4; ++c) pv[4 * i + c] = W[5 * i + 1 + c];
    }
    oc_lsq_gradients(m, 4, pv, bv, gr);
    memset(R, 0, sizeof(double) * 5 * (size_t)nc);
    memset(D, 0, sizeof(double) * (size_t)nc);
    for (int32_t f = 0; f < nfc; ++f) {
        int32_t L = m->face_cells[2 * f], Rc = m->face_cells[2 * f + 1];
        const double *n = m->face_normal + 3 * f;
        double S = m->face_area[f];
        const double *PL = W + 5 * L;
        double F[5] = {0, 0, 0, 0, 0};
        double aL = sqrt(gam * PL[4] / 2.0);
        double unL = PL[1] * n[0] + PL[2] * n[1] + PL[3] * n[2];
        double dL, dR = 0;
        int kindB = -1;
        const double *PR = NULL;
        double Pfar[5];
        if (Rc >= 0) {
            PR = W + 5 * Rc;
        } else {
            int32_t p = -1 - Rc;
            kindB = m->patch_kind[p];
            if (kindB == OC_FAR) {
                for (int c = 0; c < 5; ++c) Pfar[c] = m->patch_state[5 * p + c];
                PR = Pfar;
            }
        }
        if (PR) {
            /* convective flux: forward half of M(W_L) + backward half of M(W_R) */
            double FL[5], FR[5];
            half_flux(PL, n, 1.0, FL);
            half_flux(PR, n, -1.0, FR);
            for (int c = 0; c < 5; ++c) F[c] = FL[c] + FR[c];
        }
        if (Rc >= 0) {
            /* viscous flux on an interior face: mean gradient corrected along the
             * normal so that its projection on the centroid difference equals the
             * jump (exact for linear fields; compact normal coefficient 1/d_n) */
            double dx[3], dd = 0;
            for (int d = 0; d < 3; ++d) { dx[d] = m->cell_center[3 * Rc + d] - m->cell_center[3 * L + d]; dd += dx[d] * n[d]; }
            double G[4][3];
            for (int v = 0; v < 4; ++v) {
                double gx = 0;
                for (int d = 0; d < 3; ++d) { G[v][d] = 0.5 * (gr[12 * L + 3 * v + d] + gr[12 * Rc + 3 * v + d]); gx += G[v][d] * dx[d]; }
                double alpha = (pv[4 * Rc + v] - pv[4 * L + v] - gx) / dd;
                for (int d = 0; d < 3; ++d) G[v][d] += alpha * n[d];
            }
            double Tf = 0.5 * (PL[4] + PR[4]);
            double gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
            double sg[6], q[3];
            oc_nsf(gas, Tf, gu, G[3], sg, q);
            for (int c = 0; c < 6; ++c) sg[c] += 0.5 * (hot[9 * L + c] + hot[9 * Rc + c]);
            for (int c = 0; c < 3; ++c) q[c] += 0.5 * (hot[9 * L + 6 + c] + hot[9 * Rc + 6 + c]);
            double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2],
                            sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                            sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
            double uf[3] = {0.5 * (PL[1] + PR[1]), 0.5 * (PL[2] + PR[2]), 0.5 * (PL[3] + PR[3])};
            for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
            F[4] += sn[0] * uf[0] + sn[1] * uf[1] + sn[2] * uf[2] + q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
            dL = dd; dR = dd;      /* normal distance between the centroids */
        } else if (kindB == OC_WALL) {
            /* isothermal no-slip wall: pressure, plus the viscous flux from
             * one-sided gradients towards (u_w, T_w) */
            const double *ps = m->patch_state + 5 * (-1 - Rc);
            double dn = 0;
            for (int d = 0; d < 3; ++d) dn += (m->face_center[3 * f + d] - m->cell_center[3 * L + d]) * n[d];
            dL = 2.0 * dn;
            double pL = PL[0] * PL[4];
            for (int d = 0; d < 3; ++d) F[1 + d] = 0.5 * pL * n[d];
            double G[4][3], wv[4] = {ps[1], ps[2], ps[3], ps[4]};
            for (int v = 0; v < 4; ++v) {
                double gn = 0;
                for (int d = 0; d < 3; ++d) gn += gr[12 * L + 3 * v + d] * n[d];
                double jump = (wv[v] - pv[4 * L + v]) / dn;
                for (int d = 0; d < 3; ++d) G[v][d] = gr[12 * L + 3 * v + d] + (jump - gn) * n[d];
            }
            double gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
            double sg[6], q[3];
            oc_nsf(gas, ps[4], gu, G[3], sg, q);
            double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2],
                            sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                            sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
            for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
            F[4] += sn[0] * ps[1] + sn[1] * ps[2] + sn[2] * ps[3] + q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
        } else {
            double dn = 0;
            for (int d = 0; d < 3; ++d) dn += (m->face_center[3 * f + d] - m->cell_center[3 * L + d]) * n[d];
            dL = 2.0 * dn;
        }
        for (int c = 0; c < 5; ++c) R[5 * L + c] -= F[c] * S;
        if (Rc >= 0)
            for (int c = 0; c < 5; ++c) R[5 * Rc + c] += F[c] * S;
        /* spectral radii for the local step */
        double nuL = fmax(4.0 / 3.0, 5.0 / (3.0 * gas->Pr)) * gas->Kn * pow(PL[4], gas->omega) / (sqrt(PI) * PL[0]);
        D[L] += S * (fabs(unL) + aL + 2.0 * nuL / dL);
        if (Rc >= 0) {
            double aR = sqrt(gam * PR[4] / 2.0);
            double unR = PR[1] * n[0] + PR[2] * n[1] + PR[3] * n[2];
            double nuR = fmax(4.0 / 3.0, 5.0 / (3.0 * gas->Pr)) * gas->Kn * pow(PR[4], gas->omega) / (sqrt(PI) * PR[0]);
            D[Rc] += S * (fabs(unR) + aR + 2.0 * nuR / dR);
        }
    }
    return 0;
}

int32_t oc_macro_residual(const oc_mesh *m, const oc_gas *gas, const double *hot,
                          const double *W, double *Rv)
{
    int32_t nc = m->n_cells;
    double *D = (double *)malloc(sizeof(double) * (size_t)nc);
    double *pv = (double *)malloc(sizeof(double) * 4 * (size_t)nc);
    double *gr = (double *)malloc(sizeof(double) * 12 * (size_t)nc);
    double *bv = (double *)malloc(sizeof(double) * 4 * (size_t)(m->n_patches > 0 ? m->n_patches : 1));
    for (int32_t p = 0; p < m->n_patches; ++p)
        for (int c = 0; c < 4; ++c) bv[4 * p + c] = m->patch_state[5 * p + 1 + c];
    int32_t st = macro_residual(m, gas, hot, W, Rv, D, pv, gr, bv);
    if (st == 0)
        for (int32_t i = 0; i < nc; ++i)
            for (int c = 0; c < 5; ++c) Rv[5 * i + c] /= m->cell_volume[i];
    free(D); free(pv); free(gr); free(bv);
    return st;
}

int32_t oc_macro(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *src,
                 int32_t n_inner, double cfl, double *W)
{
    int32_t nc = m->n_cells;
    double *U = (double *)malloc(sizeof(double) * 5 * (size_t)nc);
    double *R = (double *)malloc(sizeof(double) * 5 * (size_t)nc);
    double *D = (double *)malloc(sizeof(double) * (size_t)nc);
    double *pv = (double *)malloc(sizeof(double) * 4 * (size_t)nc);
    double *gr = (double *)malloc(sizeof(double) * 12 * (size_t)nc);
    double *bv = (double *)malloc(sizeof(double) * 4 * (size_t)(m->n_patches > 0 ? m->n_patches : 1));
    for (int32_t p = 0; p < m->n_patches; ++p)
        for (int c = 0; c < 4; ++c) bv[4 * p + c] = m->patch_state[5 * p + 1 + c];
    for (int32_t i = 0; i < nc; ++i) cons_from_prim(W + 5 * i, U + 5 * i);
    int32_t status = 0;
    for (int32_t it = 0; it < n_inner && status == 0; ++it) {
        status = macro_residual(m, gas, hot, W, R, D, pv, gr, bv);
        if (status) break;
        if (src)
            for (int32_t i = 0; i < nc; ++i)
                for (int c = 0; c < 5; ++c) R[5 * i + c] += src[5 * i + c] * m->cell_volume[i];
        /* R_i is not yet divided by V_i.  Local step: dt_i / V_i = cfl / D_i.
         * cfl < 0 selects one global step dt = |cfl| min_i V_i / D_i, which
         * conserves sum_i V_i U_i exactly. */
        double gdt = INFINITY;
        if (cfl < 0)
            for (int32_t i = 0; i < nc; ++i) gdt = fmin(gdt, -cfl * m->cell_volume[i] / D[i]);
        for (int32_t i = 0; i < nc; ++i) {
            double k = (cfl < 0) ? gdt / m->cell_volume[i] : cfl / D[i];
            /* positivity safeguard (reading): halve this cell's increment until
             * the new density and temperature are positive; after ten halvings
             * the cell keeps its state for this pseudo-step */
            double Un[5], Pn[5];
            int ok = 0;
            for (int h = 0; h <= 10 && !ok; ++h) {
                for (int c = 0; c < 5; ++c) Un[c] = U[5 * i + c] + k * R[5 * i + c];
                prim_from_cons(Un, Pn);
                ok = (Pn[0] > 0) && (Pn[4] > 0);
                k *= 0.5;
            }
            if (ok)
                for (int c = 0; c < 5; ++c) U[5 * i + c] = Un[c];
        }
        for (int32_t i = 0; i < nc; ++i) prim_from_cons(U + 5 * i, W + 5 * i);
    }
    for (int32_t i = 0; i < nc && status == 0; ++i)
        if (!(W[5 * i] > 0) || !(W[5 * i + 4] > 0)) status = -7;
    free(U); free(R); free(D); free(pv); free(gr); free(bv);
    return status;
}

/* ------------------------------------------------------------------------
 * Polyatomic gas: the two-VDF kinetic model of Sec. 2 (eq. general_model,
 * reference distributions g_0t, g_0r, g_1t, g_1r, heat-flux mixing q_0, q_1
 * through A, tau = mu(T_t) / p_t), 3D velocity space, scaled units
 * (R T -> T/2).  f1 is measured in rho0 / v_m so that
 *   sum w f1 = d_r rho T_r / 4        ((d_r/2) rho R T_r)
 *   q_r = 2 sum w c f1               (q_r / (rho0 R T0 v_m)).
 * Scaled reference distributions:
 *   g0t = M_t [1 + (4/15) q_t.c / (T_t p_t) (c^2/T_t - 5/2)],  M_t = rho (pi T_t)^-3/2 e^{-c^2/T_t}
 *   g0r = M_r [1 + (4/15) q_0.c / (T p) (c^2/T - 5/2)],        M_r = rho (pi T)^-3/2 e^{-c^2/T}
 *   g1t = (d_r T_r / 4) g0t + (pi T_t)^-3/2 (q_r.c / T_t) e^{-c^2/T_t}
 *   g1r = (d_r T / 4) g0r + (pi T)^-3/2 (q_1.c / T) e^{-c^2/T}
 * with T = (3 T_t + d_r T_r)/(3 + d_r), p_t = rho T_t, p = rho T.
 * ------------------------------------------------------------------------ */
void oc_moments_poly(const oc_grid *g, double d_r, const double *f, double *mom)
{
    int32_t nv = oc_nv(g);
    oc_moments(g, f, mom);   /* f0: rho, u, T_t, sigma, q_t */
    double xi[3], w, e1 = 0, qr[3] = {0, 0, 0};
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        e1 += w * f[nv + k];
        for (int d = 0; d < 3; ++d) qr[d] += 2.0 * w * (xi[d] - mom[1 + d]) * f[nv + k];
    }
    mom[14] = (d_r > 0) ? 4.0 * e1 / (d_r * mom[0]) : mom[4];
    for (int d = 0; d < 3; ++d) mom[15 + d] = qr[d];
}

int32_t oc_poly_target(const oc_grid *g, const oc_gas *gas, const double *mom, double *out)
{
    int32_t nv = oc_nv(g);
    const double dr = gas->dr, Zr = gas->Zr;
    const double Att = gas->A[0], Atr = gas->A[1], Art = gas->A[2], Arr = gas->A[3];
    const double rho = mom[0], Tt = mom[4], Tr = mom[14];
    const double *u = mom + 1, *qt = mom + 11, *qr = mom + 15;
    const double T = (3.0 * Tt + dr * Tr) / (3.0 + dr), pt = rho * Tt, p = rho * T;
    double q0[3], q1[3];
    for (int d = 0; d < 3; ++d) {
        q0[d] = ((2.0 - 3.0 * Att) * Zr + 1.0) * qt[d] - 3.0 * Atr * Zr * qr[d];
        q1[d] = -Art * Zr * qt[d] + (1.0 - Arr * Zr) * qr[d];
    }
    double xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c[3], c2 = 0, qtc = 0, q0c = 0, qrc = 0, q1c = 0;
        for (int d = 0; d < 3; ++d) {
            c[d] = xi[d] - u[d];
            c2 += c[d] * c[d];
            qtc += qt[d] * c[d];
            q0c += q0[d] * c[d];
            qrc += qr[d] * c[d];
            q1c += q1[d] * c[d];
        }
        double Et = pow(PI * Tt, -1.5) * exp(-c2 / Tt), Er = pow(PI * T, -1.5) * exp(-c2 / T);
        double g0t = rho * Et * (1.0 + (4.0 / 15.0) * qtc / (Tt * pt) * (c2 / Tt - 2.5));
        double g0r = rho * Er * (1.0 + (4.0 / 15.0) * q0c / (T * p) * (c2 / T - 2.5));
        double g1t = 0.25 * dr * Tr * g0t + Et * qrc / Tt;
        double g1r = 0.25 * dr * T * g0r + Er * q1c / T;
        out[k] = g0t + (g0r - g0t) / Zr;
        out[nv + k] = g1t + (g1r - g1t) / Zr;
    }
    /* conservation fix-up: P(c) = a0 + a.c + b c^2 on both targets, with
     * sum w P G0 = rho, sum w c P G0 = 0, sum w (c^2 G0 + 2 G1) P =
     * (3/2) rho T_t + (d_r/2) rho T_r (the discrete moments of f) */
    double M[25] = {0}, b[5] = {0};
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c[3], c2 = 0;
        for (int d = 0; d < 3; ++d) { c[d] = xi[d] - u[d]; c2 += c[d] * c[d]; }
        double ph[5] = {1.0, c[0], c[1], c[2], c2};
        double G0 = out[k], G1 = out[nv + k];
        for (int a = 0; a < 5; ++a) {
            double t = (a < 4) ? ph[a] * G0 : c2 * G0 + 2.0 * G1;
            for (int bb = 0; bb < 5; ++bb) M[a * 5 + bb] += w * t * ph[bb];
        }
    }
    b[0] = rho;
    b[4] = 1.5 * rho * Tt + 0.5 * dr * rho * Tr;
    if (solve_small(5, M, b) != 0) return -1;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c2 = 0, P = b[0];
        for (int d = 0; d < 3; ++d) {
            double c = xi[d] - u[d];
            c2 += c * c;
            P += b[1 + d] * c;
        }
        P += b[4] * c2;
        out[k] *= P;
        out[nv + k] *= P;
    }
    return 0;
}

/* Upwind rows of the faces of kinetic cell i for the two-VDF gas (as
 * face_sources, rows of 2 nv; f1 on boundary and NS faces = (d_r T_b/4) f0). */
static void face_sources_poly(const oc_mesh *m, const oc_grid *g, const oc_gas *gas, const int32_t *cptr,
                              const int32_t *cidx, int32_t i, const int32_t *slot_of_cell, const double *f_old,
                              const double *ghost, const double *fi, double *scratch, double *nrm,
                              const double **srcp)
{
    int32_t nv = oc_nv(g);
    size_t row = 2 * (size_t)nv;
    int32_t nf = cptr[i + 1] - cptr[i];
    for (int32_t l = 0; l < nf; ++l) {
        int32_t f = cidx[cptr[i] + l];
        int32_t own = m->face_cells[2 * f], oth = m->face_cells[2 * f + 1];
        double sgn = (own == i) ? 1.0 : -1.0;
        int32_t nb = (own == i) ? oth : own;
        for (int d = 0; d < 3; ++d) nrm[4 * l + d] = sgn * m->face_normal[3 * f + d];
        nrm[4 * l + 3] = m->face_area[f] / m->cell_volume[i];
        double *s = scratch + (size_t)l * row;
        double Tb;
        if (nb >= 0 && slot_of_cell[nb] >= 0) {
            srcp[l] = f_old + (size_t)slot_of_cell[nb] * row;
            continue;
        }
        if (nb >= 0) {
            /* NS neighbour: the two-VDF Grad-13 rows (eq. G13_VDF) */
            oc_g13_poly(g, gas->dr, ghost + (size_t)nb * OC_NMOM_POLY, s);
            srcp[l] = s;
            continue;
        } else {
            int32_t p = -1 - nb;
            const double *ps = m->patch_state + 5 * p;
            Tb = ps[4];
            if (m->patch_kind[p] == OC_WALL) {
                double rw = wall_density(g, fi, NULL, NULL, nrm + 4 * l, ps + 1, ps[4], s);
                for (int32_t k = 0; k < nv; ++k) s[k] *= rw;
            } else {
                oc_maxwellian(g, ps[0], ps + 1, ps[4], s);
            }
        }
        for (int32_t k = 0; k < nv; ++k) s[nv + k] = 0.25 * gas->dr * Tb * s[k];
        srcp[l] = s;
    }
}

int32_t oc_sweep_poly(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                      int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                      const double *f_old, const double *ghost, double *f_new)
{
    if (g->vdim != 3) return -1;
    int32_t nv = oc_nv(g);
    size_t row = 2 * (size_t)nv;
    int32_t *cptr, *cidx;
    build_adjacency(m, &cptr, &cidx);
    int32_t err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : err)
    for (int32_t t = 0; t < n_kin; ++t) {
        int32_t i = kin_cell[t];
        const double *fi = f_old + (size_t)slot_of_cell[i] * row;
        double *fo = f_new + (size_t)slot_of_cell[i] * row;
        int32_t nf = cptr[i + 1] - cptr[i];
        double mom[OC_NMOM_POLY];
        oc_moments_poly(g, gas->dr, fi, mom);
        double tau = oc_tau(gas, mom[0], mom[4]);   /* tau = mu(T_t) / p_t */
        double *G = (double *)malloc(sizeof(double) * row);
        double *src = (double *)malloc(sizeof(double) * row * (size_t)(nf > 0 ? nf : 1));
        double *nrm = (double *)malloc(sizeof(double) * 4 * (size_t)(nf > 0 ? nf : 1));
        const double **srcp = (const double **)malloc(sizeof(double *) * (size_t)(nf > 0 ? nf : 1));
        if (oc_poly_target(g, gas, mom, G) != 0) err = -7;
        face_sources_poly(m, g, gas, cptr, cidx, i, slot_of_cell, f_old, ghost, fi, src, nrm, srcp);
        double xi[3], w;
        for (int32_t k = 0; k < nv; ++k) {
            node(g, k, xi, &w);
            double den = gas->inv_dt + 1.0 / tau;
            double num[2];
            for (int q = 0; q < 2; ++q) num[q] = gas->inv_dt * fi[q * nv + k] + G[q * nv + k] / tau;
            for (int32_t l = 0; l < nf; ++l) {
                double a = (xi[0] * nrm[4 * l] + xi[1] * nrm[4 * l + 1] + xi[2] * nrm[4 * l + 2]) * nrm[4 * l + 3];
                if (a > 0) den += a;
                else if (a < 0)
                    for (int q = 0; q < 2; ++q) num[q] += -a * srcp[l][q * nv + k];
            }
            for (int q = 0; q < 2; ++q) fo[q * nv + k] = num[q] / den;
        }
        free(G); free(src); free(nrm); free(srcp);
    }
    free(cptr);
    free(cidx);
    return err;
}

/* ------------------------------------------------------------------------
 * Grad-13 rows of the two-VDF gas (Sec. 3.2 eq. G13_VDF) in scaled units:
 * f0 is the monatomic Grad-13 row at T_t; f1 = (d_r T_r/4) f0 plus the
 * internal heat-flux term q_r.c/(rho T_t) times the Maxwellian at T_t (the
 * scaled form of the paper's q_r.c/(rho T_t) f_eq: with q_r = 2 sum w c f1
 * its first moment is q_r, and the Grad bracket of f0 has none).
 * ------------------------------------------------------------------------ */
void oc_g13_poly(const oc_grid *g, double d_r, const double *prm, double *out)
{
    int32_t nv = oc_nv(g);
    oc_g13(g, prm, out);
    const double rho = prm[0], Tt = prm[4], Tr = prm[14];
    const double *u = prm + 1, *qr = prm + 15;
    double xi[3], w;
    for (int32_t k = 0; k < nv; ++k) {
        node(g, k, xi, &w);
        double c2 = 0, qc = 0;
        for (int d = 0; d < 3; ++d) {
            double c = xi[d] - u[d];
            c2 += c * c;
            qc += qr[d] * c;
        }
        double M = rho * pow(PI * Tt, -1.5) * exp(-c2 / Tt);
        out[nv + k] = 0.25 * d_r * Tr * out[k] + qc / (rho * Tt) * M;
    }
}

/* thermal-conduction factors [k_t, k_r] = (1/2) A^{-1} [5, d_r] (eq. mu_kappa,
 * kappa = k mu R) */
static void conduction_factors(const oc_gas *gas, double *kt, double *kr)
{
    const double a = gas->A[0], b = gas->A[1], c = gas->A[2], d = gas->A[3];
    const double det = a * d - b * c;
    *kt = 0.5 * (d * 5.0 - b * gas->dr) / det;
    *kr = 0.5 * (-c * 5.0 + a * gas->dr) / det;
}

void oc_nsf_poly(const oc_gas *gas, double Tt, const double *grad_u, const double *grad_Tt, const double *grad_Tr,
                 double *sigma6, double *qt3, double *qr3)
{
    double mu = pow(Tt, gas->omega);
    double cs = -2.0 * gas->Kn / sqrt(PI) * mu;
    double kt, kr;
    conduction_factors(gas, &kt, &kr);
    double div = grad_u[0] + grad_u[4] + grad_u[8];
    sigma6[0] = cs * (2.0 * grad_u[0] - 2.0 / 3.0 * div);
    sigma6[1] = cs * (2.0 * grad_u[4] - 2.0 / 3.0 * div);
    sigma6[2] = cs * (2.0 * grad_u[8] - 2.0 / 3.0 * div);
    sigma6[3] = cs * (grad_u[1] + grad_u[3]);
    sigma6[4] = cs * (grad_u[2] + grad_u[6]);
    sigma6[5] = cs * (grad_u[5] + grad_u[7]);
    for (int d = 0; d < 3; ++d) {
        qt3[d] = -kt * gas->Kn / sqrt(PI) * mu * grad_Tt[d];
        qr3[d] = -kr * gas->Kn / sqrt(PI) * mu * grad_Tr[d];
    }
}

int32_t oc_kinetic_residual_poly(const oc_mesh *m, const oc_grid *g, const oc_gas *gas,
                                 int32_t n_kin, const int32_t *kin_cell, const int32_t *slot_of_cell,
                                 const double *f_old, const double *ghost, double *R)
{
    int32_t nv = oc_nv(g);
    size_t row = 2 * (size_t)nv;
    int32_t *cptr, *cidx;
    build_adjacency(m, &cptr, &cidx);
    memset(R, 0, sizeof(double) * 6 * (size_t)m->n_cells);
    int32_t err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : err)
    for (int32_t t = 0; t < n_kin; ++t) {
        int32_t i = kin_cell[t];
        const double *fi = f_old + (size_t)slot_of_cell[i] * row;
        int32_t nf = cptr[i + 1] - cptr[i];
        double *src = (double *)malloc(sizeof(double) * row * (size_t)(nf > 0 ? nf : 1));
        double *nrm = (double *)malloc(sizeof(double) * 4 * (size_t)(nf > 0 ? nf : 1));
        const double **srcp = (const double **)malloc(sizeof(double *) * (size_t)(nf > 0 ? nf : 1));
        double *G = (double *)malloc(sizeof(double) * row);
        face_sources_poly(m, g, gas, cptr, cidx, i, slot_of_cell, f_old, ghost, fi, src, nrm, srcp);
        double acc[6] = {0, 0, 0, 0, 0, 0}, xi[3], w;
        for (int32_t l = 0; l < nf; ++l) {
            for (int32_t k = 0; k < nv; ++k) {
                node(g, k, xi, &w);
                double a = (xi[0] * nrm[4 * l] + xi[1] * nrm[4 * l + 1] + xi[2] * nrm[4 * l + 2]) * nrm[4 * l + 3];
                const double *up = (a > 0) ? fi : srcp[l];
                double x2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
                acc[0] -= w * a * up[k];
                for (int d = 0; d < 3; ++d) acc[1 + d] -= w * a * xi[d] * up[k];
                acc[4] -= w * a * (x2 * up[k] + 2.0 * up[nv + k]);
                acc[5] -= w * a * 2.0 * up[nv + k];
            }
        }
        /* exchange with the translational modes: the collision term of f1 */
        double mom[OC_NMOM_POLY];
        oc_moments_poly(g, gas->dr, fi, mom);
        if (oc_poly_target(g, gas, mom, G) != 0) err = -7;
        double tau = oc_tau(gas, mom[0], mom[4]);
        for (int32_t k = 0; k < nv; ++k) {
            node(g, k, xi, &w);
            acc[5] += 2.0 * w * (G[nv + k] - fi[nv + k]) / tau;
        }
        for (int c = 0; c < 6; ++c) R[6 * i + c] = acc[c];
        free(src); free(nrm); free(srcp); free(G);
    }
    free(cptr);
    free(cidx);
    return err;
}

/* ------------------------------------------------------------------------
 * Synthetic equations of the two-VDF gas.  Readings (in addition to those
 * of the monatomic synthetic solve above, which carry over):
 *   conserved U = (rho, rho u, E, rho e_r), E = rho |u|^2 + (3/2) rho T_t +
 *   rho e_r, rho e_r = (d_r/2) rho T_r (scaled units, energy / (rho0 R T0));
 *   convective flux: the kinetic splitting at T_t, with the internal energy
 *   e_r = (d_r/2) T_r of each side carried by its half-range mass flux
 *   (internal modes in local equilibrium);
 *   viscous flux: NSF of oc_nsf_poly at the face T_t plus the mean HoT of
 *   sigma, q_t and q_r; energy flux sigma.u + (q_t + q_r).n, internal-energy
 *   flux q_r.n;
 *   walls: isothermal no-slip for T_t and T_r alike; far field: the patch
 *   state with T_r = T;
 *   internal relaxation source S_r = (d_r/2) rho (T - T_r)/(Z_r tau),
 *   tau = mu(T_t)/p_t, T = (3 T_t + d_r T_r)/(3 + d_r).  In the pseudo-time
 *   iteration it is taken implicitly (backward Euler in rho e_r with tau of
 *   the old state and T of the new total energy, which the exchange leaves
 *   unchanged), so that stiff exchange stays stable and the steady state is
 *   that of the explicit residual;
 *   local step: D_i = sum_f S_f (|u_n| + a + 2 nu / d_f), a = sqrt(gamma T/2),
 *   gamma = (5 + d_r)/(3 + d_r), nu = max(4/3, 2 k_t/3, 2 k_r/d_r) Kn
 *   T_t^omega / (sqrt(pi) rho);
 *   positivity: rho, T_t and T_r.
 * ------------------------------------------------------------------------ */
static void prim_from_cons_poly(const double *U, double dr, double *P)
{
    double rho = U[0], u2 = 0;
    P[0] = rho;
    for (int d = 0; d < 3; ++d) { P[1 + d] = U[1 + d] / rho; u2 += P[1 + d] * P[1 + d]; }
    P[5] = U[5] / (0.5 * dr * rho);
    P[4] = (U[4] - rho * u2 - U[5]) / (1.5 * rho);
}

static void cons_from_prim_poly(const double *P, double dr, double *U)
{
    double u2 = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    U[0] = P[0];
    for (int d = 0; d < 3; ++d) U[1 + d] = P[0] * P[1 + d];
    U[5] = 0.5 * dr * P[0] * P[5];
    U[4] = P[0] * u2 + 1.5 * P[0] * P[4] + U[5];
}

static void half_flux_poly(const double *P, const double *n, double sgn, double dr, double *F)
{
    half_flux(P, n, sgn, F);           /* translational part at T_t = P[4] */
    double er = 0.5 * dr * P[5];
    F[4] += er * F[0];
    F[5] = er * F[0];
}

static double relax_source(const oc_gas *gas, const double *P)
{
    double T = (3.0 * P[4] + gas->dr * P[5]) / (3.0 + gas->dr);
    return 0.5 * gas->dr * P[0] * (T - P[5]) / (gas->Zr * oc_tau(gas, P[0], P[4]));
}

/* R (not divided by V) of the flux balance, plus V S_r when with_src; D the
 * local-step denominators.  pv[n][5] = (u, T_t, T_r), gr[n][5][3]. */
static int32_t macro_residual_poly(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *W,
                                   int with_src, double *R, double *D, double *pv, double *gr, const double *bv)
{
    int32_t nc = m->n_cells, nfc = m->n_faces;
    const double dr = gas->dr, gam = (5.0 + dr) / (3.0 + dr);
    double kt, kr;
    conduction_factors(gas, &kt, &kr);
    const double nuf = fmax(4.0 / 3.0, fmax(2.0 * kt / 3.0, 2.0 * kr / dr));
    for (int32_t i = 0; i < nc; ++i) {
        const double *Pi = W + 6 * i;
        if (!(Pi[0] > 0) || !(Pi[4] > 0) || !(Pi[5] > 0)) return -7;
        for (int c = 0; c < 5; ++c) pv[5 * i + c] = Pi[1 + c];
    }
    oc_lsq_gradients(m, 5, pv, bv, gr);
    memset(R, 0, sizeof(double) * 6 * (size_t)nc);
    memset(D, 0, sizeof(double) * (size_t)nc);
    for (int32_t f = 0; f < nfc; ++f) {
        int32_t L = m->face_cells[2 * f], Rc = m->face_cells[2 * f + 1];
        const double *n = m->face_normal + 3 * f;
        double S = m->face_area[f];
        const double *PL = W + 6 * L;
        double F[6] = {0, 0, 0, 0, 0, 0};
        double dL, dR = 0;
        int kindB = -1;
        const double *PR = NULL;
        double Pfar[6];
        if (Rc >= 0) {
            PR = W + 6 * Rc;
        } else {
            int32_t p = -1 - Rc;
            kindB = m->patch_kind[p];
            if (kindB == OC_FAR) {
                for (int c = 0; c < 5; ++c) Pfar[c] = m->patch_state[5 * p + c];
                Pfar[5] = Pfar[4];
                PR = Pfar;
            }
        }
        if (PR) {
            double FL[6], FR[6];
            half_flux_poly(PL, n, 1.0, dr, FL);
            half_flux_poly(PR, n, -1.0, dr, FR);
            for (int c = 0; c < 6; ++c) F[c] = FL[c] + FR[c];
        }
        if (Rc >= 0) {
            double dx[3], dd = 0;
            for (int d = 0; d < 3; ++d) { dx[d] = m->cell_center[3 * Rc + d] - m->cell_center[3 * L + d]; dd += dx[d] * n[d]; }
            double G[5][3];
            for (int v = 0; v < 5; ++v) {
                double gx = 0;
                for (int d = 0; d < 3; ++d) { G[v][d] = 0.5 * (gr[15 * L + 3 * v + d] + gr[15 * Rc + 3 * v + d]); gx += G[v][d] * dx[d]; }
                double alpha = (pv[5 * Rc + v] - pv[5 * L + v] - gx) / dd;
                for (int d = 0; d < 3; ++d) G[v][d] += alpha * n[d];
            }
            double Tf = 0.5 * (PL[4] + PR[4]);
            double gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
            double sg[6], qt[3], qr[3];
            oc_nsf_poly(gas, Tf, gu, G[3], G[4], sg, qt, qr);
            for (int c = 0; c < 6; ++c) sg[c] += 0.5 * (hot[12 * L + c] + hot[12 * Rc + c]);
            for (int c = 0; c < 3; ++c) {
                qt[c] += 0.5 * (hot[12 * L + 6 + c] + hot[12 * Rc + 6 + c]);
                qr[c] += 0.5 * (hot[12 * L + 9 + c] + hot[12 * Rc + 9 + c]);
            }
            double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2],
                            sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                            sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
            double uf[3] = {0.5 * (PL[1] + PR[1]), 0.5 * (PL[2] + PR[2]), 0.5 * (PL[3] + PR[3])};
            double qtn = qt[0] * n[0] + qt[1] * n[1] + qt[2] * n[2], qrn = qr[0] * n[0] + qr[1] * n[1] + qr[2] * n[2];
            for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
            F[4] += sn[0] * uf[0] + sn[1] * uf[1] + sn[2] * uf[2] + qtn + qrn;
            F[5] += qrn;
            dL = dd; dR = dd;
        } else if (kindB == OC_WALL) {
            const double *ps = m->patch_state + 5 * (-1 - Rc);
            double dn = 0;
            for (int d = 0; d < 3; ++d) dn += (m->face_center[3 * f + d] - m->cell_center[3 * L + d]) * n[d];
            dL = 2.0 * dn;
            double pL = PL[0] * PL[4];
            for (int d = 0; d < 3; ++d) F[1 + d] = 0.5 * pL * n[d];
            double G[5][3], wv[5] = {ps[1], ps[2], ps[3], ps[4], ps[4]};
            for (int v = 0; v < 5; ++v) {
                double gn = 0;
                for (int d = 0; d < 3; ++d) gn += gr[15 * L + 3 * v + d] * n[d];
                double jump = (wv[v] - pv[5 * L + v]) / dn;
                for (int d = 0; d < 3; ++d) G[v][d] = gr[15 * L + 3 * v + d] + (jump - gn) * n[d];
            }
            double gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
            double sg[6], qt[3], qr[3];
            oc_nsf_poly(gas, ps[4], gu, G[3], G[4], sg, qt, qr);
            double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2],
                            sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                            sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
            double qtn = qt[0] * n[0] + qt[1] * n[1] + qt[2] * n[2], qrn = qr[0] * n[0] + qr[1] * n[1] + qr[2] * n[2];
            for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
            F[4] += sn[0] * ps[1] + sn[1] * ps[2] + sn[2] * ps[3] + qtn + qrn;
            F[5] += qrn;
        } else {
            double dn = 0;
            for (int d = 0; d < 3; ++d) dn += (m->face_center[3 * f + d] - m->cell_center[3 * L + d]) * n[d];
            dL = 2.0 * dn;
        }
        for (int c = 0; c < 6; ++c) R[6 * L + c] -= F[c] * S;
        if (Rc >= 0)
            for (int c = 0; c < 6; ++c) R[6 * Rc + c] += F[c] * S;
        double TL = (3.0 * PL[4] + dr * PL[5]) / (3.0 + dr);
        double unL = PL[1] * n[0] + PL[2] * n[1] + PL[3] * n[2];
        double nuL = nuf * gas->Kn * pow(PL[4], gas->omega) / (sqrt(PI) * PL[0]);
        D[L] += S * (fabs(unL) + sqrt(gam * TL / 2.0) + 2.0 * nuL / dL);
        if (Rc >= 0) {
            double TR = (3.0 * PR[4] + dr * PR[5]) / (3.0 + dr);
            double unR = PR[1] * n[0] + PR[2] * n[1] + PR[3] * n[2];
            double nuR = nuf * gas->Kn * pow(PR[4], gas->omega) / (sqrt(PI) * PR[0]);
            D[Rc] += S * (fabs(unR) + sqrt(gam * TR / 2.0) + 2.0 * nuR / dR);
        }
    }
    if (with_src)
        for (int32_t i = 0; i < nc; ++i) R[6 * i + 5] += m->cell_volume[i] * relax_source(gas, W + 6 * i);
    return 0;
}

static void patch_values_poly(const oc_mesh *m, double *bv)
{
    for (int32_t p = 0; p < m->n_patches; ++p) {
        for (int c = 0; c < 4; ++c) bv[5 * p + c] = m->patch_state[5 * p + 1 + c];
        bv[5 * p + 4] = m->patch_state[5 * p + 4];
    }
}

int32_t oc_macro_residual_poly(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *W,
                               double *Rv)
{
    int32_t nc = m->n_cells;
    double *D = (double *)malloc(sizeof(double) * (size_t)nc);
    double *pv = (double *)malloc(sizeof(double) * 5 * (size_t)nc);
    double *gr = (double *)malloc(sizeof(double) * 15 * (size_t)nc);
    double *bv = (double *)malloc(sizeof(double) * 5 * (size_t)(m->n_patches > 0 ? m->n_patches : 1));
    patch_values_poly(m, bv);
    int32_t st = macro_residual_poly(m, gas, hot, W, 1, Rv, D, pv, gr, bv);
    if (st == 0)
        for (int32_t i = 0; i < nc; ++i)
            for (int c = 0; c < 6; ++c) Rv[6 * i + c] /= m->cell_volume[i];
    free(D); free(pv); free(gr); free(bv);
    return st;
}

int32_t oc_macro_poly(const oc_mesh *m, const oc_gas *gas, const double *hot, const double *src,
                      int32_t n_inner, double cfl, double *W)
{
    int32_t nc = m->n_cells;
    const double dr = gas->dr;
    double *U = (double *)malloc(sizeof(double) * 6 * (size_t)nc);
    double *R = (double *)malloc(sizeof(double) * 6 * (size_t)nc);
    double *D = (double *)malloc(sizeof(double) * (size_t)nc);
    double *pv = (double *)malloc(sizeof(double) * 5 * (size_t)nc);
    double *gr = (double *)malloc(sizeof(double) * 15 * (size_t)nc);
    double *bv = (double *)malloc(sizeof(double) * 5 * (size_t)(m->n_patches > 0 ? m->n_patches : 1));
    patch_values_poly(m, bv);
    for (int32_t i = 0; i < nc; ++i) cons_from_prim_poly(W + 6 * i, dr, U + 6 * i);
    int32_t status = 0;
    for (int32_t it = 0; it < n_inner && status == 0; ++it) {
        status = macro_residual_poly(m, gas, hot, W, 0, R, D, pv, gr, bv);
        if (status) break;
        if (src)
            for (int32_t i = 0; i < nc; ++i)
                for (int c = 0; c < 6; ++c) R[6 * i + c] += src[6 * i + c] * m->cell_volume[i];
        double gdt = INFINITY;
        if (cfl < 0)
            for (int32_t i = 0; i < nc; ++i) gdt = fmin(gdt, -cfl * m->cell_volume[i] / D[i]);
        for (int32_t i = 0; i < nc; ++i) {
            double k = (cfl < 0) ? gdt / m->cell_volume[i] : cfl / D[i];
            const double *Po = W + 6 * i;
            double x0 = m->cell_volume[i] / (gas->Zr * oc_tau(gas, Po[0], Po[4]));   /* dt/(Z_r tau) = k x0 */
            double Un[6], Pn[6];
            int ok = 0;
            for (int h = 0; h <= 10 && !ok; ++h) {
                for (int c = 0; c < 6; ++c) Un[c] = U[6 * i + c] + k * R[6 * i + c];
                /* internal relaxation, backward Euler at the new total temperature */
                double u2 = (Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]) / (Un[0] * Un[0]);
                double T = (Un[4] - Un[0] * u2) / (0.5 * (3.0 + dr) * Un[0]);
                double x = k * x0;
                Un[5] = (Un[5] + x * 0.5 * dr * Un[0] * T) / (1.0 + x);
                prim_from_cons_poly(Un, dr, Pn);
                ok = (Pn[0] > 0) && (Pn[4] > 0) && (Pn[5] > 0);
                k *= 0.5;
            }
            if (ok)
                for (int c = 0; c < 6; ++c) U[6 * i + c] = Un[c];
        }
        for (int32_t i = 0; i < nc; ++i) prim_from_cons_poly(U + 6 * i, dr, W + 6 * i);
    }
    for (int32_t i = 0; i < nc && status == 0; ++i)
        if (!(W[6 * i] > 0) || !(W[6 * i + 4] > 0) || !(W[6 * i + 5] > 0)) status = -7;
    free(U); free(R); free(D); free(pv); free(gr); free(bv);
    return status;
}
