// gsis_poly.hip -- the synthetic side of the two-VDF (polyatomic) gas.
//
// Sec. 2 eq. macroscopic_equation_2 with its internal-energy equation
//   d(rho e_r)/dt + div(rho e_r u + q_r) = (d_r/2) rho (T - T_r)/(Z_r tau),
// the NSF laws with mu(T_t) and the conductivities of eq. mu_kappa, Sec. 3.1
// eq. full_constitutive with the HoT of q_r, and the Grad-13 rows of Sec. 3.2
// eq. G13_VDF (T_r and the q_r term of f1).  Scaled units: rho e_r =
// (d_r/2) rho T_r, E = rho |u|^2 + (3/2) rho T_t + rho e_r, tau = mu(T_t)/p_t,
// T = (3 T_t + d_r T_r)/(3 + d_r).
//
// The discretisation is that of the monatomic synthetic solve, extended:
// kinetic flux-vector splitting at T_t with the internal energy of each side
// carried by its half-range mass flux; viscous fluxes with the face T_t;
// isothermal no-slip walls for T_t and T_r; the exchange source taken
// backward-Euler in rho e_r within each pseudo-time step (tau of the old
// state, T of the new total energy), so its steady state is that of the
// explicit residual.  These kernels run one thread per cell or face: the
// internal-energy equation is the two-VDF gas's own path, not the bench's.
#include <math.h>

#include "gsis_impl.hpp"

namespace gsis {

namespace {

// [k_t, k_r] = (1/2) A^{-1} [5, d_r]  (kappa = k mu R)
__device__ __forceinline__ void cond_factors(const CaseView &C, double &kt, double &kr)
{
    const double a = C.A[0], b = C.A[1], c = C.A[2], d = C.A[3];
    const double det = a * d - b * c;
    kt = 0.5 * (d * 5.0 - b * C.dr) / det;
    kr = 0.5 * (-c * 5.0 + a * C.dr) / det;
}

// scaled NSF laws: sigma = -(2 Kn/sqrt(pi)) mu (G + G^T - 2/3 tr G I),
// q_t = -(k_t Kn/sqrt(pi)) mu grad T_t, q_r = -(k_r Kn/sqrt(pi)) mu grad T_r
__device__ void nsf_poly(const CaseView &C, double Tt, const double *Gu, const double *GTt, const double *GTr,
                         double *s, double *qt, double *qr)
{
    const double mu = pow(Tt, C.omega);
    const double cs = -2.0 * C.Kn / sqrt(M_PI) * mu;
    double kt, kr;
    cond_factors(C, kt, kr);
    const double div = Gu[0] + Gu[4] + Gu[8];
    s[0] = cs * (2.0 * Gu[0] - 2.0 / 3.0 * div);
    s[1] = cs * (2.0 * Gu[4] - 2.0 / 3.0 * div);
    s[2] = cs * (2.0 * Gu[8] - 2.0 / 3.0 * div);
    s[3] = cs * (Gu[1] + Gu[3]);
    s[4] = cs * (Gu[2] + Gu[6]);
    s[5] = cs * (Gu[5] + Gu[7]);
    for (int d = 0; d < 3; ++d) {
        qt[d] = -kt * C.Kn / sqrt(M_PI) * mu * GTt[d];
        qr[d] = -kr * C.Kn / sqrt(M_PI) * mu * GTr[d];
    }
}

__device__ __forceinline__ double tau_of(const CaseView &C, double rho, double Tt)
{
    return 2.0 * C.Kn / sqrt(M_PI) * pow(Tt, C.omega - 1.0) / rho;
}

__device__ __forceinline__ double exchange(const CaseView &C, double rho, double Tt, double Tr)
{
    const double T = (3.0 * Tt + C.dr * Tr) / (3.0 + C.dr);
    return 0.5 * C.dr * rho * (T - Tr) / (C.Zr * tau_of(C, rho, Tt));
}

// half-range flux of the translational Maxwellian at T_t, plus the internal
// energy e_r = (d_r/2) T_r carried by its mass flux; P = (rho, u, T_t), Tr
__device__ void half_flux_p(const CaseView &C, const double *P, double Tr, const double *n, double sgn, double *F)
{
    const double rho = P[0], T = P[4], sT = sqrt(T);
    const double un = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
    const double ut[3] = {P[1] - un * n[0], P[2] - un * n[1], P[3] - un * n[2]};
    const double ut2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    const double s = un / sT;
    const double A = 0.5 * (1.0 + sgn * erf(s));
    const double B = sgn * exp(-s * s) / (2.0 * sqrt(M_PI));
    const double m1 = un * A + sT * B;
    const double m2 = (un * un + 0.5 * T) * A + un * sT * B;
    const double m3 = (un * un * un + 1.5 * un * T) * A + (un * un + T) * sT * B;
    F[0] = rho * m1;
    for (int d = 0; d < 3; ++d) F[1 + d] = rho * (ut[d] * m1 + n[d] * m2);
    const double er = 0.5 * C.dr * Tr;
    F[4] = rho * (m3 + (ut2 + T) * m1) + er * F[0];
    F[5] = er * F[0];
}

// the (u, T_t) gradient rows of cell i (launch_lsq), as in the monatomic solve
__device__ __forceinline__ const double *grad_ut(const CaseView &C, int i) { return C.grad + 12 * (size_t)i; }

// local step denominator D_i = sum_f S_f (|u_n| + a + 2 nu / d_f), a = sqrt(gamma T/2),
// gamma = (5 + d_r)/(3 + d_r), nu = max(4/3, 2 k_t/3, 2 k_r/d_r) Kn T_t^omega/(sqrt(pi) rho)
__device__ double cell_D_poly(const CaseView &C, int i, const double *Wi, double Tr)
{
    double kt, kr;
    cond_factors(C, kt, kr);
    const double T = (3.0 * Wi[4] + C.dr * Tr) / (3.0 + C.dr);
    const double gam = (5.0 + C.dr) / (3.0 + C.dr);
    const double a = sqrt(gam * T / 2.0);
    const double nu = fmax(4.0 / 3.0, fmax(2.0 * kt / 3.0, 2.0 * kr / C.dr)) * C.Kn * pow(Wi[4], C.omega) /
                      (sqrt(M_PI) * Wi[0]);
    double un = 0.0;
    for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
        const double *n = C.cf_nsv + 3 * (size_t)e;
        un += fabs(Wi[1] * n[0] + Wi[2] * n[1] + Wi[3] * n[2]);
    }
    const double *sS = C.cell_sS + 2 * (size_t)i;
    return C.cell_volume[i] * un + a * sS[0] + 2.0 * nu * sS[1];
}

// least-squares gradient of T_r (the coefficients of the other fields; a
// boundary face contributes the patch temperature)
// one lane per face of a cell (G lanes per cell, MCELLS_Q cells per block);
// the lanes' terms are added in a fixed tree order
template <int G>
__global__ __launch_bounds__(MCELLS_Q * G) void k_lsq_tr(const CaseView *__restrict__ cvp, const double *__restrict__ Tr)
{
    const CaseView &C = *cvp;
    const int i = xcd_remap(blockIdx.x, gridDim.x) * MCELLS_Q + (int)threadIdx.x / G;
    const int l = (int)threadIdx.x % G;
    if (i >= C.n_cells) return;   // whole groups leave together
    const double ti = Tr[i];
    const int e0 = C.cf_ptr[i], nf = C.cf_ptr[i + 1] - e0;
    double g[3] = {0.0, 0.0, 0.0};
    if (l < nf) {
        const int e = e0 + l;
        const int o = C.cf_other[e];
        const double to = (o >= 0) ? Tr[o] : C.patch_state[5 * (-1 - o) + 4];
        const double *ca = C.lsq + 3 * (size_t)e;
        for (int d = 0; d < 3; ++d) g[d] = ca[d] * (to - ti);
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] += __shfl_xor(g[d], off, G);
    if (l == 0)
        for (int d = 0; d < 3; ++d) C.gTr[3 * (size_t)i + d] = g[d];
}

// Grad-13 parameters of the two-VDF gas: (rho, u, T_t, sigma, q_t) in ghost,
// (T_r, q_r) in ghr; the range limit also bounds the q_r term of f1 against
// its equilibrium part: r = max(|sigma|/p_t, |q_t|/(p_t sqrt T_t),
// 4 |q_r| / (d_r rho T_r sqrt T_t))
__global__ void k_ghost_p(const CaseView *__restrict__ cvp, const double *__restrict__ W, const double *__restrict__ Tr)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    const double *Wi = W + 5 * (size_t)i;
    double *g = C.ghost + (size_t)i * GSIS_NMOM;
    for (int c = 0; c < 5; ++c) g[c] = Wi[c];
    const double *gr = grad_ut(C, i);
    double s[6], qt[3], qr[3];
    nsf_poly(C, Wi[4], gr, gr + 9, C.gTr + 3 * (size_t)i, s, qt, qr);
    const double p = Wi[0] * Wi[4], sT = sqrt(Wi[4]);
    double smax = 0.0;
    for (int c = 0; c < 6; ++c) smax = fmax(smax, fabs(s[c]));
    double r = fmax(smax / p, sqrt(qt[0] * qt[0] + qt[1] * qt[1] + qt[2] * qt[2]) / (p * sT));
    r = fmax(r, 4.0 * sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2]) / (C.dr * Wi[0] * Tr[i] * sT));
    const double rmax = C.g13_rmax;
    const double th = (rmax > 0.0 && r > rmax) ? rmax / r : 1.0;
    C.g13_th[i] = th;
    for (int c = 0; c < 6; ++c) g[5 + c] = s[c] * th;
    for (int c = 0; c < 3; ++c) g[11 + c] = qt[c] * th;
    double *h = C.ghr + 4 * (size_t)i;
    h[0] = Tr[i];
    for (int c = 0; c < 3; ++c) h[1 + c] = qr[c] * th;
}

// HoT on kinetic cells: sigma, q_t (hot) and q_r (hotr) of f^{n+1/2} minus the
// NSF values at W^{n+1/2} (gradients of Wh in grad, of Trh in gTr)
__global__ void k_hot_p(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    double *h = C.hot + 9 * (size_t)i, *hr = C.hotr + 3 * (size_t)i;
    const int slot = C.slot_of_cell[i];
    if (slot < 0) {
        for (int c = 0; c < 9; ++c) h[c] = 0.0;
        for (int c = 0; c < 3; ++c) hr[c] = 0.0;
        return;
    }
    const double *mom = C.mom + (size_t)slot * MOMS;
    const double *gr = grad_ut(C, i);
    double s[6], qt[3], qr[3];
    nsf_poly(C, C.Wh[5 * (size_t)i + 4], gr, gr + 9, C.gTr + 3 * (size_t)i, s, qt, qr);
    for (int c = 0; c < 6; ++c) h[c] = mom[5 + c] - s[c];
    for (int c = 0; c < 3; ++c) h[6 + c] = mom[11 + c] - qt[c];
    for (int c = 0; c < 3; ++c) hr[c] = mom[MOM_INT + 1 + c] - qr[c];
}

// T_r of the moments on kinetic cells, of Tr elsewhere (out may be Tr itself)
__global__ void k_tr_mom(const CaseView *__restrict__ cvp, double *out)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    const int slot = C.slot_of_cell[i];
    out[i] = (slot >= 0) ? C.mom[(size_t)slot * MOMS + MOM_INT] : C.Tr[i];
}

// face means of the frozen HoT projected on the normal: sigma.n (3), q_t.n,
// and q_r.n (hfr), once per solve; zero on boundary faces and without HoT
// (hot null; with hot, the q_r part is read from hotr)
__global__ void k_hot_face_p(const CaseView *__restrict__ cvp, const double *__restrict__ hot)
{
    const CaseView &C = *cvp;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= C.n_faces) return;
    const int L = C.face_cells[2 * f], Rc = C.face_cells[2 * f + 1];
    double o[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (Rc >= 0 && hot) {
        const double *n = C.face_normal + 3 * (size_t)f;
        const double *hL = hot + 9 * (size_t)L, *hR = hot + 9 * (size_t)Rc;
        double sg[6], q[3], qr[3];
        for (int c = 0; c < 6; ++c) sg[c] = 0.5 * (hL[c] + hR[c]);
        for (int c = 0; c < 3; ++c) {
            q[c] = 0.5 * (hL[6 + c] + hR[6 + c]);
            qr[c] = 0.5 * (C.hotr[3 * (size_t)L + c] + C.hotr[3 * (size_t)Rc + c]);
        }
        o[0] = sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2];
        o[1] = sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2];
        o[2] = sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2];
        o[3] = q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
        o[4] = qr[0] * n[0] + qr[1] * n[1] + qr[2] * n[2];
    }
    double *hf = C.hface + 4 * (size_t)f;
    for (int c = 0; c < 4; ++c) hf[c] = o[c];
    C.hfr[f] = o[4];
}

// face fluxes: fflux [f][5] (mass, momentum, total energy) and fr [f] (rho e_r)
__global__ void k_face_flux_p(const CaseView *__restrict__ cvp, const double *__restrict__ W,
                              const double *__restrict__ Tr)
{
    const CaseView &C = *cvp;
    const int f = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= C.n_faces) return;
    const int L = C.face_cells[2 * f], Rc = C.face_cells[2 * f + 1];
    const double *n = C.face_normal + 3 * (size_t)f;
    const double *PL = W + 5 * (size_t)L;
    const double TrL = Tr[L];
    double F[6] = {0, 0, 0, 0, 0, 0};
    if (Rc >= 0 || C.patch_kind[-1 - Rc] == GSIS_PATCH_FAR) {
        const double *PR = (Rc >= 0) ? W + 5 * (size_t)Rc : C.patch_state + 5 * (-1 - Rc);
        const double TrR = (Rc >= 0) ? Tr[Rc] : PR[4];
        double FL[6], FR[6];
        half_flux_p(C, PL, TrL, n, 1.0, FL);
        half_flux_p(C, PR, TrR, n, -1.0, FR);
        for (int c = 0; c < 6; ++c) F[c] = FL[c] + FR[c];
        if (Rc >= 0) {
            // mean gradients corrected along n to match the jumps (u, T_t, T_r)
            const double *dx = C.face_dx + 3 * (size_t)f;
            const double dn = C.face_dist[f];
            double G[5][3];
            const double *gL = grad_ut(C, L), *gR = grad_ut(C, Rc);
            const double *tL = C.gTr + 3 * (size_t)L, *tR = C.gTr + 3 * (size_t)Rc;
            for (int v = 0; v < 5; ++v) {
                double gx = 0.0;
                for (int d = 0; d < 3; ++d) {
                    G[v][d] = (v < 4) ? 0.5 * (gL[3 * v + d] + gR[3 * v + d]) : 0.5 * (tL[d] + tR[d]);
                    gx += G[v][d] * dx[d];
                }
                const double fl = (v < 3) ? PL[1 + v] : ((v == 3) ? PL[4] : TrL);
                const double fr = (v < 3) ? PR[1 + v] : ((v == 3) ? PR[4] : TrR);
                const double alpha = (fr - fl - gx) / dn;
                for (int d = 0; d < 3; ++d) G[v][d] += alpha * n[d];
            }
            const double Tf = 0.5 * (PL[4] + PR[4]);
            double Gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
            double sg[6], qt[3], qr[3];
            nsf_poly(C, Tf, Gu, G[3], G[4], sg, qt, qr);
            const double *hf = C.hface + 4 * (size_t)f;
            const double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2] + hf[0],
                                  sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2] + hf[1],
                                  sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2] + hf[2]};
            const double uf[3] = {0.5 * (PL[1] + PR[1]), 0.5 * (PL[2] + PR[2]), 0.5 * (PL[3] + PR[3])};
            const double qtn = qt[0] * n[0] + qt[1] * n[1] + qt[2] * n[2] + hf[3];
            const double qrn = qr[0] * n[0] + qr[1] * n[1] + qr[2] * n[2] + C.hfr[f];
            for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
            F[4] += sn[0] * uf[0] + sn[1] * uf[1] + sn[2] * uf[2] + qtn + qrn;
            F[5] += qrn;
        }
    } else {
        // isothermal no-slip wall for T_t and T_r: pressure plus the NSF
        // fluxes from one-sided gradients towards (u_w, T_w, T_w)
        const double *ps = C.patch_state + 5 * (-1 - Rc);
        const double dn = 0.5 * C.face_dist[f];
        const double *gL = grad_ut(C, L), *tL = C.gTr + 3 * (size_t)L;
        const double pL = PL[0] * PL[4];
        for (int d = 0; d < 3; ++d) F[1 + d] = 0.5 * pL * n[d];
        double G[5][3];
        for (int v = 0; v < 5; ++v) {
            const double *gv = (v < 4) ? gL + 3 * v : tL;
            const double gn = gv[0] * n[0] + gv[1] * n[1] + gv[2] * n[2];
            const double fl = (v < 3) ? PL[1 + v] : ((v == 3) ? PL[4] : TrL);
            const double wv = (v < 3) ? ps[1 + v] : ps[4];
            const double jump = (wv - fl) / dn;
            for (int d = 0; d < 3; ++d) G[v][d] = gv[d] + (jump - gn) * n[d];
        }
        double Gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
        double sg[6], qt[3], qr[3];
        nsf_poly(C, ps[4], Gu, G[3], G[4], sg, qt, qr);
        const double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2], sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                              sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
        const double qtn = qt[0] * n[0] + qt[1] * n[1] + qt[2] * n[2];
        const double qrn = qr[0] * n[0] + qr[1] * n[1] + qr[2] * n[2];
        for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
        F[4] += sn[0] * ps[1] + sn[1] * ps[2] + sn[2] * ps[3] + qtn + qrn;
        F[5] = qrn;
    }
    for (int c = 0; c < 5; ++c) C.fflux[5 * (size_t)f + c] = F[c];
    C.fr[f] = F[5];
}

// flux balance of cell i (not divided by V), fixed order over its faces
__device__ __forceinline__ void balance_p(const CaseView &C, int i, double *R)
{
    for (int c = 0; c < 6; ++c) R[c] = 0.0;
    for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
        const int f = C.cf_face[e];
        const double fs = C.cf_fs[e];
        for (int c = 0; c < 5; ++c) R[c] += C.fflux[5 * (size_t)f + c] * fs;
        R[5] += C.fr[f] * fs;
    }
}

__global__ void k_residual_p(const CaseView *__restrict__ cvp, const double *__restrict__ W,
                             const double *__restrict__ Tr, double *__restrict__ Rout, double *__restrict__ Rrout)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    double R[6];
    balance_p(C, i, R);
    const double iv = 1.0 / C.cell_volume[i];
    for (int c = 0; c < 5; ++c) Rout[5 * (size_t)i + c] = R[c] * iv;
    const double *Wi = W + 5 * (size_t)i;
    Rrout[i] = R[5] * iv + exchange(C, Wi[0], Wi[4], Tr[i]);
}

// source of eq. macro on kinetic cells: kinetic balance at f^n minus the
// synthetic residual at W^n, for the five conserved moments and rho e_r
__global__ void k_src_p(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    const bool kin = C.slot_of_cell[i] >= 0;
    for (int c = 0; c < 5; ++c) C.src[5 * (size_t)i + c] = kin ? C.Rk[5 * (size_t)i + c] - C.Rm[5 * (size_t)i + c] : 0.0;
    C.srcr[i] = kin ? C.Rkr[i] - C.Rmr[i] : 0.0;
}

__global__ void k_cons_p(const CaseView *__restrict__ cvp, const double *__restrict__ W, const double *__restrict__ Tr)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    const double *P = W + 5 * (size_t)i;
    double *U = C.U + 5 * (size_t)i;
    const double u2 = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    const double er = 0.5 * C.dr * P[0] * Tr[i];
    U[0] = P[0];
    for (int d = 0; d < 3; ++d) U[1 + d] = P[0] * P[1 + d];
    U[4] = P[0] * u2 + 1.5 * P[0] * P[4] + er;
    C.Ur[i] = er;
}

// dloc[block] = min over the block's cells of V_i / D_i (global steps)
__global__ __launch_bounds__(MBLOCK) void k_dloc_p(const CaseView *__restrict__ cvp, const double *__restrict__ W,
                                                   const double *__restrict__ Tr)
{
    const CaseView &C = *cvp;
    const int blk = blockIdx.x;
    const int i = blk * MBLOCK + (int)threadIdx.x;
    __shared__ double sm[MBLOCK];
    double v = INFINITY;
    if (i < C.n_cells) v = C.cell_volume[i] / cell_D_poly(C, i, W + 5 * (size_t)i, Tr[i]);
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int st = MBLOCK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) C.dloc[blk] = sm[0];
}

__global__ __launch_bounds__(256) void k_min_p(const CaseView *__restrict__ cvp, int nb)
{
    const CaseView &C = *cvp;
    __shared__ double sm[256];
    double v = INFINITY;
    for (int i = threadIdx.x; i < nb; i += 256) v = fmin(v, C.dloc[i]);
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) C.red[0] = sm[0];
}

// one pseudo-time step of a cell: U += k (R + V src) for the five conserved
// moments and rho e_r (src: the case's src and srcr, or none), then the
// exchange backward-Euler at the new total energy; halved (at most ten times)
// while rho, T_t or T_r would not be positive
// one lane per face of a cell (G lanes, MCELLS_Q cells per block): the flux
// balance and sum_f |u.n| S/V in a fixed tree order, then lane 0 steps the cell
template <int G>
__global__ __launch_bounds__(MCELLS_Q * G) void k_update_p(const CaseView *__restrict__ cvp, double *__restrict__ W,
                                                           double *__restrict__ Tr, const double *__restrict__ src,
                                                           double cfl)
{
    const CaseView &C = *cvp;
    const int i = xcd_remap(blockIdx.x, gridDim.x) * MCELLS_Q + (int)threadIdx.x / G;
    const int l = (int)threadIdx.x % G;
    if (i >= C.n_cells) return;   // whole groups leave together
    double *Wi = W + 5 * (size_t)i;
    double Wc[5];
    for (int c = 0; c < 5; ++c) Wc[c] = Wi[c];
    const double tri = Tr[i];
    const int e0 = C.cf_ptr[i], nf = C.cf_ptr[i + 1] - e0;
    double R[6] = {0, 0, 0, 0, 0, 0}, un = 0.0;
    if (l < nf) {
        const int e = e0 + l;
        const int f = C.cf_face[e];
        const double fs = C.cf_fs[e];   // -S if i owns the face, +S otherwise
        for (int c = 0; c < 5; ++c) R[c] = C.fflux[5 * (size_t)f + c] * fs;
        R[5] = C.fr[f] * fs;
        const double *n = C.cf_nsv + 3 * (size_t)e;
        un = fabs(Wc[1] * n[0] + Wc[2] * n[1] + Wc[3] * n[2]);
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 6; ++c) R[c] += __shfl_xor(R[c], off, G);
        un += __shfl_xor(un, off, G);
    }
    if (l != 0) return;
    const double V = C.cell_volume[i];
    if (src) {
        for (int c = 0; c < 5; ++c) R[c] += src[5 * (size_t)i + c] * V;
        R[5] += C.srcr[i] * V;
    }
    double k;
    if (cfl < 0) {
        k = (-cfl * C.red[0]) / V;
    } else {
        // D_i = sum_f S_f (|u_n| + a + 2 nu / d_f), a = sqrt(gamma T/2), gamma = (5 + d_r)/(3 + d_r),
        // nu = max(4/3, 2 k_t/3, 2 k_r/d_r) Kn T_t^omega/(sqrt(pi) rho)
        double kt, kr;
        cond_factors(C, kt, kr);
        const double T = (3.0 * Wc[4] + C.dr * tri) / (3.0 + C.dr);
        const double gam = (5.0 + C.dr) / (3.0 + C.dr);
        const double a = sqrt(gam * T / 2.0);
        const double nu = fmax(4.0 / 3.0, fmax(2.0 * kt / 3.0, 2.0 * kr / C.dr)) * C.Kn * pow(Wc[4], C.omega) /
                          (sqrt(M_PI) * Wc[0]);
        const double *sS = C.cell_sS + 2 * (size_t)i;
        k = cfl / (V * un + a * sS[0] + 2.0 * nu * sS[1]);
    }
    const double x0 = V / (C.Zr * tau_of(C, Wc[0], Wc[4]));   // dt/(Z_r tau) = k x0
    double *U = C.U + 5 * (size_t)i;
    const double dr = C.dr;
    double Un[6], Pn[5], Trn = 0.0;
    bool ok = false;
    for (int h = 0; h <= 10 && !ok; ++h) {
        for (int c = 0; c < 5; ++c) Un[c] = U[c] + k * R[c];
        Un[5] = C.Ur[i] + k * R[5];
        const double u2 = (Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]) / (Un[0] * Un[0]);
        const double T = (Un[4] - Un[0] * u2) / (0.5 * (3.0 + dr) * Un[0]);
        const double x = k * x0;
        Un[5] = (Un[5] + x * 0.5 * dr * Un[0] * T) / (1.0 + x);
        Pn[0] = Un[0];
        for (int d = 0; d < 3; ++d) Pn[1 + d] = Un[1 + d] / Un[0];
        Trn = Un[5] / (0.5 * dr * Un[0]);
        Pn[4] = (Un[4] - Un[0] * u2 - Un[5]) / (1.5 * Un[0]);
        ok = (Pn[0] > 0.0) && (Pn[4] > 0.0) && (Trn > 0.0);
        k *= 0.5;
    }
    if (ok) {
        for (int c = 0; c < 5; ++c) {
            U[c] = Un[c];
            Wi[c] = Pn[c];
        }
        C.Ur[i] = Un[5];
        Tr[i] = Trn;
    }
    const double *Wf = ok ? Pn : Wc;
    const double tf = ok ? Trn : tri;
    if (!isfinite(Wf[0] + Wf[1] + Wf[2] + Wf[3] + Wf[4] + tf)) atomicOr(C.status, 1);
}

__global__ void k_tt(const CaseView *__restrict__ cvp, double *__restrict__ out)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C.n_cells) out[i] = C.W[5 * (size_t)i + 4];
}

__global__ void k_copy_dd(double *d, const double *s, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// surface quantities on the NS wall cells of the two-VDF gas (Sec. 4.2/4.3):
// the wall flux of its synthetic equations -- pressure rho T_t plus the NSF
// stress, and the heat flux (q_t + q_r).n, from the LSQ gradients of u, T_t
// and T_r whose normal parts are replaced by one-sided differences to the
// wall values (T_r held at T_w like T_t).  One thread per wall face; faces of
// kinetic cells are left to k_surface.
__global__ __launch_bounds__(256) void k_surface_ns_p(const CaseView *__restrict__ cvp, double *__restrict__ out)
{
    const CaseView &C = *cvp;
    const int j = blockIdx.x * 256 + (int)threadIdx.x;
    if (j >= C.n_wall) return;
    const int f = C.wall_face[j];
    const int L = C.face_cells[2 * f], p = -1 - C.face_cells[2 * f + 1];
    if (C.slot_of_cell[L] >= 0) return;
    const double *ps = C.patch_state + 5 * p;
    const double *n = C.face_normal + 3 * (size_t)f;
    const double *PL = C.W + 5 * (size_t)L;
    const double TrL = C.Tr[L];
    const double dn = 0.5 * C.face_dist[f];
    const double *gL = grad_ut(C, L), *tL = C.gTr + 3 * (size_t)L;
    double G[5][3];
    for (int v = 0; v < 5; ++v) {
        const double *gv = (v < 4) ? gL + 3 * v : tL;
        const double gn = gv[0] * n[0] + gv[1] * n[1] + gv[2] * n[2];
        const double fl = (v < 3) ? PL[1 + v] : ((v == 3) ? PL[4] : TrL);
        const double wv = (v < 3) ? ps[1 + v] : ps[4];
        const double jump = (wv - fl) / dn;
        for (int d = 0; d < 3; ++d) G[v][d] = gv[d] + (jump - gn) * n[d];
    }
    double Gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
    double sg[6], qt[3], qr[3];
    nsf_poly(C, ps[4], Gu, G[3], G[4], sg, qt, qr);
    const double pL = PL[0] * PL[4];
    const double tau[3] = {pL * n[0] + sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2],
                           pL * n[1] + sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                           pL * n[2] + sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
    const double pn = tau[0] * n[0] + tau[1] * n[1] + tau[2] * n[2];
    double *o = out + (size_t)j * GSIS_NSURF;
    for (int d = 0; d < 3; ++d) {
        o[d] = tau[d];
        o[4 + d] = tau[d] - pn * n[d];
    }
    o[3] = pn;
    o[7] = (qt[0] + qr[0]) * n[0] + (qt[1] + qr[1]) * n[1] + (qt[2] + qr[2]) * n[2];
    o[8] = 0.0;
}

// the lane-per-face cell kernels: blocks of MCELLS_Q cells covering n_cells,
// G = 4 lanes per cell on tetrahedral meshes, else GSIS_MAX_FACES
void lsq_tr(const CaseView *cv, int n_cells, int nfmax, const double *Tr, hipStream_t s)
{
    const dim3 g((n_cells + MCELLS_Q - 1) / MCELLS_Q);
    if (nfmax <= 4) hipLaunchKernelGGL((k_lsq_tr<4>), g, dim3(MCELLS_Q * 4), 0, s, cv, Tr);
    else hipLaunchKernelGGL((k_lsq_tr<MAXF>), g, dim3(MCELLS_Q * MAXF), 0, s, cv, Tr);
}

void update_p(const CaseView *cv, int n_cells, int nfmax, double *W, double *Tr, const double *src, double cfl,
              hipStream_t s)
{
    const dim3 g((n_cells + MCELLS_Q - 1) / MCELLS_Q);
    if (nfmax <= 4) hipLaunchKernelGGL((k_update_p<4>), g, dim3(MCELLS_Q * 4), 0, s, cv, W, Tr, src, cfl);
    else hipLaunchKernelGGL((k_update_p<MAXF>), g, dim3(MCELLS_Q * MAXF), 0, s, cv, W, Tr, src, cfl);
}

}  // namespace

hipError_t launch_copy_d(double *dst, const double *src, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_dd, dim3((n + 255) / 256), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_tt_copy(const CaseView *cv, const CaseView &h, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_tt, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv, out);
    return hipGetLastError();
}

hipError_t launch_ghost_poly(const CaseView *cv, const CaseView &h, const double *W, const double *Tr, hipStream_t s)
{
    const dim3 g((h.n_cells + 127) / 128);
    lsq_tr(cv, h.n_cells, h.nfmax, Tr, s);
    hipLaunchKernelGGL(k_ghost_p, g, dim3(128), 0, s, cv, W, Tr);
    return hipGetLastError();
}

hipError_t launch_hot_poly(const CaseView *cv, const CaseView &h, hipStream_t s)
{
    const dim3 g((h.n_cells + 127) / 128);
    lsq_tr(cv, h.n_cells, h.nfmax, (const double *)h.Trh, s);
    hipLaunchKernelGGL(k_hot_p, g, dim3(128), 0, s, cv);
    return hipGetLastError();
}

hipError_t launch_surface_ns_poly(const CaseView *cv, const CaseView &h, double *out, hipStream_t s)
{
    if (h.n_wall <= 0) return hipSuccess;
    // T_r gradients of the current state (the u, T_t rows come with the
    // surface launch's own LSQ pass)
    lsq_tr(cv, h.n_cells, h.nfmax, (const double *)h.Tr, s);
    hipLaunchKernelGGL(k_surface_ns_p, dim3((h.n_wall + 255) / 256), dim3(256), 0, s, cv, out);
    return hipGetLastError();
}

hipError_t launch_tr_half(const CaseView *cv, const CaseView &h, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_tr_mom, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv, out);
    return hipGetLastError();
}

hipError_t launch_macro_residual_poly(const CaseView *cv, const CaseView &h, const double *W, const double *Tr,
                                      const double *hot, double *Rout, double *Rrout, hipStream_t s)
{
    hipError_t e = launch_lsq(cv, h, W, 4, s);
    if (e != hipSuccess) return e;
    const dim3 gc((h.n_cells + 127) / 128), gf((h.n_faces + 127) / 128);
    lsq_tr(cv, h.n_cells, h.nfmax, Tr, s);
    if (h.n_faces > 0) {
        hipLaunchKernelGGL(k_hot_face_p, gf, dim3(128), 0, s, cv, hot);
        hipLaunchKernelGGL(k_face_flux_p, gf, dim3(128), 0, s, cv, W, Tr);
    }
    hipLaunchKernelGGL(k_residual_p, gc, dim3(128), 0, s, cv, W, Tr, Rout, Rrout);
    return hipGetLastError();
}

hipError_t launch_src_poly(const CaseView *cv, const CaseView &h, hipStream_t s)
{
    hipLaunchKernelGGL(k_src_p, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv);
    return hipGetLastError();
}

// n_inner pseudo-time steps of each case of the batch, one case after the
// other (every launch covers one case; the two-VDF gas is not the bench's
// batched path).  The batch carries the device views; the cell and face
// counts come from its block prefixes.
hipError_t launch_macro_steps_poly(const MBatch &b, int n_inner, double cfl, hipStream_t s)
{
    for (int j = 0; j < b.n; ++j) {
        const CaseView *cv = b.cv[j];
        const int ncb = b.bc[j + 1] - b.bc[j];   // blocks of MBLOCK cells
        const int nfb = b.bf[j + 1] - b.bf[j];   // blocks of MBLOCK_F faces
        const dim3 gc(ncb * (MBLOCK / 128)), gf(nfb * (MBLOCK_F / 128));
        double *W = b.W[j], *Tr = b.Tr[j];
        const double *hot = b.hot[j], *src = b.src[j];
        // the same case alone, for the gradient launches
        MBatch one{};
        one.cv[0] = cv;
        one.W[0] = W;
        one.bc[1] = ncb;
        one.bf[1] = nfb;
        one.bq[1] = b.bq[j + 1] - b.bq[j];
        one.n = 1;
        one.nfmax = b.nfmax;
        hipLaunchKernelGGL(k_cons_p, gc, dim3(128), 0, s, cv, (const double *)W, (const double *)Tr);
        if (nfb > 0) hipLaunchKernelGGL(k_hot_face_p, gf, dim3(128), 0, s, cv, hot);
        for (int it = 0; it < n_inner; ++it) {
            hipError_t e = launch_lsq_batch(one, 4, s);
            if (e != hipSuccess) return e;
            lsq_tr(cv, ncb * MBLOCK, b.nfmax, (const double *)Tr, s);
            if (nfb > 0)
                hipLaunchKernelGGL(k_face_flux_p, gf, dim3(128), 0, s, cv, (const double *)W, (const double *)Tr);
            if (cfl < 0) {
                hipLaunchKernelGGL(k_dloc_p, dim3(ncb), dim3(MBLOCK), 0, s, cv, (const double *)W, (const double *)Tr);
                hipLaunchKernelGGL(k_min_p, dim3(1), dim3(256), 0, s, cv, ncb);
            }
            update_p(cv, ncb * MBLOCK, b.nfmax, W, Tr, src, cfl, s);
        }
    }
    return hipGetLastError();
}

}  // namespace gsis
