// gsis_macro.hip -- FP64 macroscopic side and region management for gfx950.
//
// Synthetic macroscopic equations of Sec. 3.1 (eqs. full_constitutive and
// macro, monatomic form of eq. macroscopic_equation_2), least-squares
// gradients (Sec. 3.4 Step 2), Grad-13 interface distributions (Sec. 3.2),
// the gradient-length local Knudsen number and DVM-region flags (Sec. 3.2),
// compaction of the kinetic list, and the convergence measure of Sec. 4.
//
// The paper leaves the macroscopic fluxes F and sources Q to another work;
// the discretisation here is: kinetic flux-vector splitting of the local
// Maxwellians for the convective part (the kinetic sweep's own upwinding
// applied to the equilibria), NSF plus high-order terms with corrected face
// gradients for the viscous part, an isothermal no-slip wall, and a frozen
// per-cell source.  All reductions are deterministic (fixed
// order, no floating-point atomics).
#include <math.h>
#include <stdlib.h>

#include "gsis_impl.hpp"

namespace gsis {

// fields for gradients: 0..2 u, 3 T, 4 rho, 5 |u|
__device__ __forceinline__ double field(const double *W, int v)
{
    if (v < 3) return W[1 + v];
    if (v == 3) return W[4];
    if (v == 4) return W[0];
    return sqrt(W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

// boundary value of field v on patch p; NaN = no contribution
__device__ __forceinline__ double bfield(const CaseView &C, int p, int v)
{
    const double *ps = C.patch_state + 5 * p;
    if (v < 3) return ps[1 + v];
    if (v == 3) return ps[4];
    if (v == 4) return (C.patch_kind[p] == GSIS_PATCH_FAR) ? ps[0] : NAN;
    return sqrt(ps[1] * ps[1] + ps[2] * ps[2] + ps[3] * ps[3]);
}

// logical block index of the cell and face kernels (XCD-contiguous ranges)
__device__ __forceinline__ int mblk() { return xcd_remap(blockIdx.x, gridDim.x); }

// case of a block in a batched launch (block-uniform)
__device__ __forceinline__ int mb_case(const int32_t *start, int n)
{
    const int b = mblk();
    int j = 0;
    while (j + 1 < n && b >= start[j + 1]) ++j;
    return j;
}

// a single case: the same kernels without the batch lookup (all pointers are
// direct kernel arguments)
struct MOne {
    const CaseView *cv;
    double *W;
    const double *hot;
    const double *src;
};

struct MLoc {
    const CaseView *cv;
    double *W;
    const double *hot;
    const double *src;
    int base;   // first block of the case
};

// block prefix kinds: cells (MBLOCK per block), faces (MBLOCK_F), cell groups (MCELLS_Q)
enum { PK_CELL = 0, PK_FACE = 1, PK_GROUP = 2 };

__device__ __forceinline__ MLoc mb_loc(const MBatch &B, int kind)
{
    const int32_t *pre = (kind == PK_FACE) ? B.bf : ((kind == PK_GROUP) ? B.bq : B.bc);
    const int j = mb_case(pre, B.n);
    return {B.cv[j], B.W[j], B.hot[j], B.src[j], pre[j]};
}

__device__ __forceinline__ MLoc mb_loc(const MOne &B, int) { return {B.cv, B.W, B.hot, B.src, 0}; }

static MOne mone_of(const MBatch &b) { return {b.cv[0], b.W[0], b.hot[0], b.src[0]}; }

void mbatch_add(MBatch &b, const CaseView *cv, const CaseView &h, double *W, const double *hot, const double *src,
                double *Tr)
{
    const int j = b.n;
    if (j == 0) b.bc[0] = b.bf[0] = b.bq[0] = 0, b.nfmax = 0, b.poly = h.poly;
    b.cv[j] = cv;
    b.W[j] = W;
    b.Tr[j] = Tr;
    b.hot[j] = hot;
    b.src[j] = src;
    b.bc[j + 1] = b.bc[j] + (h.n_cells + MBLOCK - 1) / MBLOCK;
    b.bf[j + 1] = b.bf[j] + (h.n_faces + MBLOCK_F - 1) / MBLOCK_F;
    b.bq[j + 1] = b.bq[j] + (h.n_cells + MCELLS_Q - 1) / MCELLS_Q;
    b.nfmax = (h.nfmax > b.nfmax) ? h.nfmax : b.nfmax;
    b.n = j + 1;
}

// Gradient storage: the (u, T) rows of every cell, [n_cells][4][3], then the
// (rho, |u|) rows, [n_cells][2][3].  The synthetic iteration reads only the
// first block, which stays dense (96 B per cell).
__device__ __forceinline__ double *grad_row(const CaseView &C, int i, int v)
{
    return (v < 4) ? C.grad + 12 * (size_t)i + 3 * v : C.grad + 12 * (size_t)C.n_cells + 6 * (size_t)i + 3 * (v - 4);
}

// least-squares gradients (Sec. 3.4 Step 2) from the per-face coefficients
// built with the mesh: grad_v = sum_e c_e (phi_e - phi_i); the density uses
// the coefficients without wall faces.  Variables: 0..2 u, 3 T [, 4 rho, 5 |u|].
// NF bounds the faces per cell: all loads of a cell are issued first.
template <int NV, int NF>
__device__ __forceinline__ void lsq_cell(const CaseView &C, const double *__restrict__ W, int i)
{
    const size_t nnz = (size_t)C.nnz;
    const int e0 = C.cf_ptr[i], nf = C.cf_ptr[i + 1] - e0;
    int oth[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) oth[l] = (l < nf) ? C.cf_other[e0 + l] : 0;
    double c[NF][3], cr[NF][3], fo[NF][NV];
    bool wall[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        wall[l] = false;
        for (int d = 0; d < 3; ++d) c[l][d] = cr[l][d] = 0.0;
        for (int v = 0; v < NV; ++v) fo[l][v] = 0.0;
        if (l < nf) {
            const double *ca = C.lsq + 3 * (size_t)(e0 + l);
            for (int d = 0; d < 3; ++d) c[l][d] = ca[d];
            if (NV > 4)
                for (int d = 0; d < 3; ++d) cr[l][d] = ca[3 * nnz + d];
            if (oth[l] >= 0) {
                const double *Wo = W + 5 * (size_t)oth[l];
                for (int v = 0; v < NV; ++v) fo[l][v] = field(Wo, v);
            } else {
                const int p = -1 - oth[l];
                wall[l] = C.patch_kind[p] == GSIS_PATCH_WALL;
                for (int v = 0; v < NV; ++v) fo[l][v] = (v == 4 && wall[l]) ? 0.0 : bfield(C, p, v);
            }
        }
    }
    const double *Wi = W + 5 * (size_t)i;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double *go = grad_row(C, i, v);
        const double fi = field(Wi, v);
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
        for (int l = 0; l < NF; ++l) {
            if (l >= nf || (v == 4 && wall[l])) continue;
            const double d = fo[l][v] - fi;
            const double *cc = (v == 4) ? cr[l] : c[l];
            g0 += cc[0] * d;
            g1 += cc[1] * d;
            g2 += cc[2] * d;
        }
        go[0] = g0;
        go[1] = g1;
        go[2] = g2;
    }
}

template <int NV, int NF, class BT>
__global__ __launch_bounds__(MBLOCK) void k_lsq(BT B)
{
    const MLoc ML = mb_loc(B, PK_CELL);
    const int i = (mblk() - ML.base) * MBLOCK + (int)threadIdx.x;
    if (i >= ML.cv->n_cells) return;
    lsq_cell<NV, NF>(*ML.cv, ML.W, i);
}

// The same gradients with one lane per face: G lanes (G >= the cell's faces)
// per cell each gather one neighbour and form its contribution, then the G
// lanes add theirs in a fixed butterfly order.  Four (eight) times the
// memory-level parallelism of one thread per cell.
template <int NV, int G, class BT>
__global__ __launch_bounds__(MCELLS_Q * G) void k_lsq_q(BT B)
{
    const MLoc ML = mb_loc(B, PK_GROUP);
    const CaseView &C = *ML.cv;
    const double *__restrict__ W = ML.W;
    const int i = (mblk() - ML.base) * MCELLS_Q + (int)threadIdx.x / G;
    const int l = (int)threadIdx.x % G;
    if (i >= C.n_cells) return;   // whole groups leave together
    const size_t nnz = (size_t)C.nnz;
    // the cell's own values are loaded with its face range (independent loads)
    const double *Wi = W + 5 * (size_t)i;
    double fi[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) fi[v] = field(Wi, v);
    const int e0 = C.cf_ptr[i], nf = C.cf_ptr[i + 1] - e0;
    double g[NV][3];
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v][0] = g[v][1] = g[v][2] = 0.0;
    if (l < nf) {
        const int e = e0 + l;
        const int oth = C.cf_other[e];
        const double *ca = C.lsq + 3 * (size_t)e;
        double c[3] = {ca[0], ca[1], ca[2]}, cr[3] = {0.0, 0.0, 0.0};
        if (NV > 4)
            for (int d = 0; d < 3; ++d) cr[d] = ca[3 * nnz + d];
        bool wall = false;
        double fo[NV];
        if (oth >= 0) {
            const double *Wo = W + 5 * (size_t)oth;
#pragma unroll
            for (int v = 0; v < NV; ++v) fo[v] = field(Wo, v);
        } else {
            const int p = -1 - oth;
            wall = C.patch_kind[p] == GSIS_PATCH_WALL;
#pragma unroll
            for (int v = 0; v < NV; ++v) fo[v] = (v == 4 && wall) ? 0.0 : bfield(C, p, v);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (v == 4 && wall) continue;
            const double d = fo[v] - fi[v];
            const double *cc = (v == 4) ? cr : c;
            g[v][0] = cc[0] * d;
            g[v][1] = cc[1] * d;
            g[v][2] = cc[2] * d;
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[v][d] += __shfl_xor(g[v][d], off, G);
    // every lane holds the sums: lane l writes the variables v = l (mod G)
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (v % G == l) {
            double *go = grad_row(C, i, v);
#pragma unroll
            for (int d = 0; d < 3; ++d) go[d] = g[v][d];
        }
}

template <class BT>
static void launch_lsq_t(const BT &b, dim3 g, int nfmax, int nvar, hipStream_t s)
{
    if (nfmax <= 4) {
        if (nvar == 6) hipLaunchKernelGGL((k_lsq<6, 4, BT>), g, dim3(MBLOCK), 0, s, b);
        else hipLaunchKernelGGL((k_lsq<4, 4, BT>), g, dim3(MBLOCK), 0, s, b);
    } else {
        if (nvar == 6) hipLaunchKernelGGL((k_lsq<6, MAXF, BT>), g, dim3(MBLOCK), 0, s, b);
        else hipLaunchKernelGGL((k_lsq<4, MAXF, BT>), g, dim3(MBLOCK), 0, s, b);
    }
}

template <class BT>
static void launch_lsq_q(const BT &b, dim3 g, int nfmax, int nvar, hipStream_t s)
{
    if (nfmax <= 4) {
        if (nvar == 6) hipLaunchKernelGGL((k_lsq_q<6, 4, BT>), g, dim3(MCELLS_Q * 4), 0, s, b);
        else hipLaunchKernelGGL((k_lsq_q<4, 4, BT>), g, dim3(MCELLS_Q * 4), 0, s, b);
    } else {
        if (nvar == 6) hipLaunchKernelGGL((k_lsq_q<6, MAXF, BT>), g, dim3(MCELLS_Q * MAXF), 0, s, b);
        else hipLaunchKernelGGL((k_lsq_q<4, MAXF, BT>), g, dim3(MCELLS_Q * MAXF), 0, s, b);
    }
}

// GSIS_MACRO_LANES=0 selects the one-thread-per-cell gradient and update kernels
bool macro_lanes()
{
    static const bool on = [] {
        const char *e = std::getenv("GSIS_MACRO_LANES");
        return !(e && e[0] == '0');
    }();
    return on;
}

static void launch_lsq_b(const MBatch &b, int nvar, hipStream_t s)
{
    if (macro_lanes()) {
        const dim3 g(b.bq[b.n]);
        if (b.n == 1) launch_lsq_q(mone_of(b), g, b.nfmax, nvar, s);
        else launch_lsq_q(b, g, b.nfmax, nvar, s);
        return;
    }
    const dim3 g(b.bc[b.n]);
    if (b.n == 1) launch_lsq_t(mone_of(b), g, b.nfmax, nvar, s);
    else launch_lsq_t(b, g, b.nfmax, nvar, s);
}


hipError_t launch_lsq_batch(const MBatch &b, int nvar, hipStream_t s)
{
    launch_lsq_b(b, nvar, s);
    return hipGetLastError();
}

hipError_t launch_lsq(const CaseView *cv, const CaseView &h, const double *W, int nvar, hipStream_t s)
{
    MBatch b{};
    mbatch_add(b, cv, h, const_cast<double *>(W), nullptr, nullptr);
    launch_lsq_b(b, nvar, s);
    return hipGetLastError();
}

// T^omega of the viscosity law: the square root, correctly rounded, for hard
// spheres (omega = 1/2), else pow
__device__ __forceinline__ double t_pow_omega(const CaseView &C, double T)
{
    return (C.omega == 0.5) ? sqrt(T) : pow(T, C.omega);
}

// Newton and Fourier laws (Sec. 2 eq. NSF_constitutive, kappa of eq.
// mu_kappa with d_r = 0), scaled: sigma = -(2Kn/sqrt(pi)) T^w (G + G^T -
// 2/3 tr G I), q = -(5 Kn / (2 sqrt(pi) Pr)) T^w grad T; G[i][j] = du_i/dx_j
__device__ void nsf(const CaseView &C, double T, const double *Gu, const double *GT, double *s, double *q)
{
    double mu = t_pow_omega(C, T);
    double cs = (-2.0 / sqrt(M_PI)) * C.Kn * mu;
    double cq = (-2.5 / sqrt(M_PI)) * C.Kn / C.Pr * mu;
    double div = Gu[0] + Gu[4] + Gu[8];
    s[0] = cs * (2.0 * Gu[0] - 2.0 / 3.0 * div);
    s[1] = cs * (2.0 * Gu[4] - 2.0 / 3.0 * div);
    s[2] = cs * (2.0 * Gu[8] - 2.0 / 3.0 * div);
    s[3] = cs * (Gu[1] + Gu[3]);
    s[4] = cs * (Gu[2] + Gu[6]);
    s[5] = cs * (Gu[5] + Gu[7]);
    for (int d = 0; d < 3; ++d) q[d] = cq * GT[d];
}

__device__ __forceinline__ void cell_nsf(const CaseView &C, int i, double T, double *s, double *q)
{
    const double *g = grad_row(C, i, 0);   // rows u_x, u_y, u_z, T (each d/dx_j)
    double Gu[9];
    for (int a = 0; a < 9; ++a) Gu[a] = g[a];
    nsf(C, T, Gu, g + 9, s, q);
}

// Grad-13 parameters of every cell from W and the gradients of W

__global__ void k_ghost(const CaseView *__restrict__ cvp, const double *__restrict__ W)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    double *g = C.ghost + (size_t)i * GSIS_NMOM;
    const double *Wi = W + 5 * (size_t)i;
    for (int c = 0; c < 5; ++c) g[c] = Wi[c];
    double s[6], q[3];
    cell_nsf(C, i, Wi[4], s, q);
    // Grad expansion inside its range: (sigma, q) scaled by min(1, rmax / r),
    // r = max(max |sigma_ij| / p, |q| / (p sqrt T)), p = rho T (rmax <= 0: no limit)
    const double p = Wi[0] * Wi[4];
    double smax = 0.0;
    for (int c = 0; c < 6; ++c) smax = fmax(smax, fabs(s[c]));
    const double r = fmax(smax / p, sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) / (p * sqrt(Wi[4])));
    const double rmax = C.g13_rmax;
    const double th = (rmax > 0.0 && r > rmax) ? rmax / r : 1.0;
    C.g13_th[i] = th;
    for (int c = 0; c < 6; ++c) g[5 + c] = s[c] * th;
    for (int c = 0; c < 3; ++c) g[11 + c] = q[c] * th;
    if (C.vdim == 2) {
        g[3] = 0.0;
        g[9] = g[10] = 0.0;
        g[13] = 0.0;
    }
}

hipError_t launch_ghost(const CaseView *cv, const CaseView &h, const double *W, hipStream_t s)
{
    hipLaunchKernelGGL(k_ghost, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv, W);
    return hipGetLastError();
}

// limiter counters: cells of a list, and those whose Grad-13 pair was scaled
// (one atomic per wave; the integer sums do not depend on the order)
__global__ void k_count_g13(const CaseView *__restrict__ cvp, const int32_t *__restrict__ list, int n, int which)
{
    const CaseView &C = *cvp;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool lim = (t < n) && C.g13_th[list[t]] < 1.0;
    const unsigned long long m = __ballot(lim);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&C.lim[2 * which + 1], (unsigned long long)__popcll(m));
    if (t == 0) atomicAdd(&C.lim[2 * which], (unsigned long long)n);
}

hipError_t launch_count_g13(const CaseView *cv, const int32_t *list, int n, int which, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_g13, dim3((n + 255) / 256), dim3(256), 0, s, cv, list, n, which);
    return hipGetLastError();
}

// high-order terms (eq. full_constitutive) on kinetic cells, zero elsewhere;
// gradients of W^{n+1/2} must be in C.grad
__global__ void k_hot(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    double *h = C.hot + 9 * (size_t)i;
    int slot = C.slot_of_cell[i];
    if (slot < 0) {
        for (int c = 0; c < 9; ++c) h[c] = 0.0;
        return;
    }
    const double *mom = C.mom + (size_t)slot * MOMS;
    double s[6], q[3];
    cell_nsf(C, i, C.Wh[5 * (size_t)i + 4], s, q);
    for (int c = 0; c < 6; ++c) h[c] = mom[5 + c] - s[c];
    for (int c = 0; c < 3; ++c) h[6 + c] = mom[11 + c] - q[c];
}

hipError_t launch_hot(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    hipLaunchKernelGGL(k_hot, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv);
    return hipGetLastError();
}

// W^{n+1/2}: moments of f^{n+1/2} on kinetic cells, W^n on NS cells
__global__ void k_whalf(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    int slot = C.slot_of_cell[i];
    const double *src = (slot >= 0) ? C.mom + (size_t)slot * MOMS : C.W + 5 * (size_t)i;
    for (int c = 0; c < 5; ++c) C.Wh[5 * (size_t)i + c] = src[c];
}

hipError_t launch_whalf(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    hipLaunchKernelGGL(k_whalf, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// face fluxes
// ---------------------------------------------------------------------------
// half-range moments {1, xi, |xi|^2} x (xi.n) of M(rho, u, T) over sgn (xi.n) > 0
__device__ void half_flux(const double *P, const double *n, double sgn, double *F)
{
    double rho = P[0], T = P[4], sT = sqrt(T);
    double un = P[1] * n[0] + P[2] * n[1] + P[3] * n[2];
    double ut[3] = {P[1] - un * n[0], P[2] - un * n[1], P[3] - un * n[2]};
    double ut2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    double s = un / sT;
    double A = 0.5 * (1.0 + sgn * erf(s));
    double B = sgn * exp(-s * s) * (0.5 / sqrt(M_PI));   // 1/(2 sqrt(pi)), folded at compile time
    double m1 = un * A + sT * B;
    double m2 = (un * un + 0.5 * T) * A + un * sT * B;
    double m3 = (un * un * un + 1.5 * un * T) * A + (un * un + T) * sT * B;
    F[0] = rho * m1;
    for (int d = 0; d < 3; ++d) F[1 + d] = rho * (ut[d] * m1 + n[d] * m2);
    F[4] = rho * (m3 + (ut2 + T) * m1);
}

// The high-order terms are frozen during a macroscopic solve, and enter the
// interior face flux only through their face means projected on the normal:
// hface = (0.5 (sigma_L + sigma_R).n, 0.5 (q_L + q_R).n), formed once per solve
// (zero on boundary faces and without high-order terms).
__device__ __forceinline__ void hot_face_one(const CaseView &C, const double *__restrict__ hot, int f)
{
    const int L = C.face_cells[2 * f], Rc = C.face_cells[2 * f + 1];
    double o[4] = {0.0, 0.0, 0.0, 0.0};
    if (Rc >= 0 && hot) {
        const double *n = C.face_normal + 3 * (size_t)f;
        const double *hL = hot + 9 * (size_t)L, *hR = hot + 9 * (size_t)Rc;
        double sg[6], q[3];
        for (int c = 0; c < 6; ++c) sg[c] = 0.5 * (hL[c] + hR[c]);
        for (int c = 0; c < 3; ++c) q[c] = 0.5 * (hL[6 + c] + hR[6 + c]);
        o[0] = sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2];
        o[1] = sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2];
        o[2] = sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2];
        o[3] = q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
    }
    double *hf = C.hface + 4 * (size_t)f;
    for (int c = 0; c < 4; ++c) hf[c] = o[c];
}

template <class BT>
__global__ __launch_bounds__(MBLOCK_F) void k_hot_face(BT B)
{
    const MLoc ML = mb_loc(B, PK_FACE);
    const int f = (mblk() - ML.base) * MBLOCK_F + (int)threadIdx.x;
    if (f >= ML.cv->n_faces) return;
    hot_face_one(*ML.cv, ML.hot, f);
}

__device__ __forceinline__ void face_flux_one(const CaseView &C, const double *__restrict__ W, int f)
{
    int L = C.face_cells[2 * f], Rc = C.face_cells[2 * f + 1];
    const double *n = C.face_normal + 3 * (size_t)f;
    const double *PL = W + 5 * (size_t)L;
    double F[5] = {0, 0, 0, 0, 0};
    if (Rc >= 0 || C.patch_kind[-1 - Rc] == GSIS_PATCH_FAR) {
        const double *PR = (Rc >= 0) ? W + 5 * (size_t)Rc : C.patch_state + 5 * (-1 - Rc);
        double FL[5], FR[5];
        half_flux(PL, n, 1.0, FL);
        half_flux(PR, n, -1.0, FR);
        for (int c = 0; c < 5; ++c) F[c] = FL[c] + FR[c];
        if (Rc >= 0) {
            // mean gradient corrected along n so that its projection on the
            // centroid difference equals the jump (exact for linear fields)
            const double *dx = C.face_dx + 3 * (size_t)f;
            const double idn = 1.0 / C.face_dist[f];
            double G[4][3];
            const double *gL = grad_row(C, L, 0), *gR = grad_row(C, Rc, 0);
            for (int v = 0; v < 4; ++v) {
                double gx = 0.0;
                for (int d = 0; d < 3; ++d) {
                    G[v][d] = 0.5 * (gL[3 * v + d] + gR[3 * v + d]);
                    gx += G[v][d] * dx[d];
                }
                double fl = (v < 3) ? PL[1 + v] : PL[4];
                double fr = (v < 3) ? PR[1 + v] : PR[4];
                double alpha = (fr - fl - gx) * idn;
                for (int d = 0; d < 3; ++d) G[v][d] += alpha * n[d];
            }
            double Tf = 0.5 * (PL[4] + PR[4]);
            double Gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
            double sg[6], q[3];
            nsf(C, Tf, Gu, G[3], sg, q);
            // plus the face means of the frozen high-order terms (projected once per solve)
            const double *hf = C.hface + 4 * (size_t)f;
            double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2] + hf[0],
                            sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2] + hf[1],
                            sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2] + hf[2]};
            double uf[3] = {0.5 * (PL[1] + PR[1]), 0.5 * (PL[2] + PR[2]), 0.5 * (PL[3] + PR[3])};
            for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
            F[4] += sn[0] * uf[0] + sn[1] * uf[1] + sn[2] * uf[2] + q[0] * n[0] + q[1] * n[1] + q[2] * n[2] + hf[3];
        }
    } else {
        // isothermal no-slip wall: pressure plus the NSF viscous flux from
        // one-sided gradients towards (u_w, T_w)
        const double *ps = C.patch_state + 5 * (-1 - Rc);
        const double dn = 0.5 * C.face_dist[f];
        const double *gL = grad_row(C, L, 0);
        double pL = PL[0] * PL[4];
        for (int d = 0; d < 3; ++d) F[1 + d] = 0.5 * pL * n[d];
        double G[4][3];
        for (int v = 0; v < 4; ++v) {
            double gn = gL[3 * v] * n[0] + gL[3 * v + 1] * n[1] + gL[3 * v + 2] * n[2];
            double fl = (v < 3) ? PL[1 + v] : PL[4];
            double jump = (ps[1 + v] - fl) / dn;
            for (int d = 0; d < 3; ++d) G[v][d] = gL[3 * v + d] + (jump - gn) * n[d];
        }
        double Gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
        double sg[6], q[3];
        nsf(C, ps[4], Gu, G[3], sg, q);
        double sn[3] = {sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2], sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                        sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
        for (int d = 0; d < 3; ++d) F[1 + d] += 0.5 * sn[d];
        F[4] += sn[0] * ps[1] + sn[1] * ps[2] + sn[2] * ps[3] + q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
    }
    for (int c = 0; c < 5; ++c) C.fflux[5 * (size_t)f + c] = F[c];
}

template <class BT>
__global__ __launch_bounds__(MBLOCK_F) void k_face_flux(BT B)
{
    const MLoc ML = mb_loc(B, PK_FACE);
    const int f = (mblk() - ML.base) * MBLOCK_F + (int)threadIdx.x;
    if (f >= ML.cv->n_faces) return;
    face_flux_one(*ML.cv, ML.W, f);
}

// per-cell flux balance R_i = -sum_f (+-F_f) S_f (deterministic order over the cell's faces)
__device__ __forceinline__ void cell_balance(const CaseView &C, int i, double *R)
{
    for (int c = 0; c < 5; ++c) R[c] = 0.0;
    for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
        const int f = C.cf_face[e];
        const double fs = C.cf_fs[e];   // -S if i owns the face, +S otherwise
        for (int c = 0; c < 5; ++c) R[c] += C.fflux[5 * (size_t)f + c] * fs;
    }
}

__global__ void k_residual_cells(const CaseView *__restrict__ cvp, double *__restrict__ Rout)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    double R[5];
    cell_balance(C, i, R);
    double iv = 1.0 / C.cell_volume[i];
    for (int c = 0; c < 5; ++c) Rout[5 * (size_t)i + c] = R[c] * iv;
}

hipError_t launch_macro_residual(const CaseView *cv, const CaseView &h, const double *W, const double *hot,
                                 double *Rout, hipStream_t s)
{
    hipError_t e = launch_lsq(cv, h, W, 4, s);
    if (e != hipSuccess) return e;
    MBatch b{};
    mbatch_add(b, cv, h, const_cast<double *>(W), hot, nullptr);
    if (b.bf[1] > 0) {
        hipLaunchKernelGGL(k_hot_face<MOne>, dim3(b.bf[1]), dim3(MBLOCK_F), 0, s, mone_of(b));
        hipLaunchKernelGGL(k_face_flux<MOne>, dim3(b.bf[1]), dim3(MBLOCK_F), 0, s, mone_of(b));
    }
    hipLaunchKernelGGL(k_residual_cells, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv, Rout);
    return hipGetLastError();
}

// source of eq. macro on kinetic cells: kinetic moment balance at f^n minus
// the synthetic residual at W^n (both per unit volume); zero on NS cells
__global__ void k_src(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    bool kin = C.slot_of_cell[i] >= 0;
    for (int c = 0; c < 5; ++c)
        C.src[5 * (size_t)i + c] = kin ? C.Rk[5 * (size_t)i + c] - C.Rm[5 * (size_t)i + c] : 0.0;
}

hipError_t launch_src(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    hipLaunchKernelGGL(k_src, dim3((h.n_cells + 127) / 128), dim3(128), 0, s, cv);
    return hipGetLastError();
}

// local step denominator D_i = sum_f S_f (|u_n| + a + 2 nu / d_f)
__device__ double cell_D(const CaseView &C, int i, const double *Wi)
{
    const double gam = 5.0 / 3.0;
    double a = sqrt(gam * Wi[4] / 2.0);
    double nu = fmax(4.0 / 3.0, 5.0 / (3.0 * C.Pr)) * C.Kn * t_pow_omega(C, Wi[4]) / (sqrt(M_PI) * Wi[0]);
    // sum_f S_f |u.n_f| = V sum_e |u . (n S / V)_e|; the rest from the per-cell sums
    double un = 0.0;
    for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
        const double *n = C.cf_nsv + 3 * (size_t)e;
        un += fabs(Wi[1] * n[0] + Wi[2] * n[1] + Wi[3] * n[2]);
    }
    const double *sS = C.cell_sS + 2 * (size_t)i;
    return C.cell_volume[i] * un + a * sS[0] + 2.0 * nu * sS[1];
}

__device__ __forceinline__ void cons_cell(const CaseView &C, const double *__restrict__ W, int i)
{
    const double *P = W + 5 * (size_t)i;
    double *U = C.U + 5 * (size_t)i;
    double u2 = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    U[0] = P[0];
    for (int d = 0; d < 3; ++d) U[1 + d] = P[0] * P[1 + d];
    U[4] = P[0] * u2 + 1.5 * P[0] * P[4];
}

template <class BT>
__global__ __launch_bounds__(MBLOCK) void k_cons(BT B)
{
    const MLoc ML = mb_loc(B, PK_CELL);
    const int i = (mblk() - ML.base) * MBLOCK + (int)threadIdx.x;
    if (i >= ML.cv->n_cells) return;
    cons_cell(*ML.cv, ML.W, i);
}

// dloc_i = V_i / D_i, then a two-level min reduction into red[0]
// dloc[block] = min over the block's cells of V_i / D_i (blocks of each case)
template <class BT>
__global__ __launch_bounds__(MBLOCK) void k_dloc(BT B)
{
    const MLoc ML = mb_loc(B, PK_CELL);
    const CaseView &C = *ML.cv;
    const double *__restrict__ W = ML.W;
    const int blk = mblk() - ML.base;
    const int i = blk * MBLOCK + (int)threadIdx.x;
    __shared__ double sm[MBLOCK];
    double v = INFINITY;
    if (i < C.n_cells) v = C.cell_volume[i] / cell_D(C, i, W + 5 * (size_t)i);
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int st = MBLOCK / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) C.dloc[blk] = sm[0];
}

// one block per case: red[0] = the case's global pseudo-time step factor
__global__ __launch_bounds__(256) void k_min_final(MBatch B)
{
    const int j = blockIdx.x;
    const CaseView &C = *B.cv[j];
    const int nb = B.bc[j + 1] - B.bc[j];
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

// U_i += k_i (R_i + V_i src_i), k_i = cfl / D_i (local) or |cfl| min V/D / V_i
// (global), halved while the new state is not positive; W = prim(U).  NF
// bounds the faces per cell: the face data of a cell is loaded first.
template <int NF>
__device__ __forceinline__ void update_cell(const CaseView &C, double *__restrict__ W, const double *__restrict__ src,
                                            int i, double cfl)
{
    double *Wi = W + 5 * (size_t)i;
    const int e0 = C.cf_ptr[i], nf = C.cf_ptr[i + 1] - e0;
    int fc[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) fc[l] = (l < nf) ? C.cf_face[e0 + l] : 0;
    double fs[NF], F[NF][5], ns[NF][3];
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fs[l] = 0.0;
        for (int c = 0; c < 5; ++c) F[l][c] = 0.0;
        for (int d = 0; d < 3; ++d) ns[l][d] = 0.0;
        if (l < nf) {
            fs[l] = C.cf_fs[e0 + l];
            for (int c = 0; c < 5; ++c) F[l][c] = C.fflux[5 * (size_t)fc[l] + c];
            for (int d = 0; d < 3; ++d) ns[l][d] = C.cf_nsv[3 * (size_t)(e0 + l) + d];
        }
    }
    // per-cell flux balance R_i = -sum_f (+-F_f) S_f, fixed order over the faces
    double R[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int l = 0; l < NF; ++l)
        for (int c = 0; c < 5; ++c) R[c] += F[l][c] * fs[l];
    const double V = C.cell_volume[i];
    if (src)
        for (int c = 0; c < 5; ++c) R[c] += src[5 * (size_t)i + c] * V;
    double k;
    if (cfl < 0) {
        k = (-cfl * C.red[0]) / V;
    } else {
        // D_i = sum_f S_f (|u.n| + a + 2 nu / d_f)
        double un = 0.0;
#pragma unroll
        for (int l = 0; l < NF; ++l) un += fabs(Wi[1] * ns[l][0] + Wi[2] * ns[l][1] + Wi[3] * ns[l][2]);
        const double a = sqrt(5.0 / 3.0 * Wi[4] / 2.0);
        const double nu = fmax(4.0 / 3.0, 5.0 / (3.0 * C.Pr)) * C.Kn * t_pow_omega(C, Wi[4]) / (sqrt(M_PI) * Wi[0]);
        const double *sS = C.cell_sS + 2 * (size_t)i;
        k = cfl / (V * un + a * sS[0] + 2.0 * nu * sS[1]);
    }
    double *U = C.U + 5 * (size_t)i;
    // positivity safeguard: halve this cell's increment (at most ten times)
    // while the new density or temperature would not be positive
    double Un[5], Pn[5];
    bool ok = false;
    for (int h = 0; h <= 10 && !ok; ++h) {
        for (int c = 0; c < 5; ++c) Un[c] = U[c] + k * R[c];
        Pn[0] = Un[0];
        double u2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            Pn[1 + d] = Un[1 + d] / Un[0];
            u2 += Pn[1 + d] * Pn[1 + d];
        }
        Pn[4] = (Un[4] - Un[0] * u2) / (1.5 * Un[0]);
        ok = (Pn[0] > 0.0) && (Pn[4] > 0.0);
        k *= 0.5;
    }
    if (ok) {
        for (int c = 0; c < 5; ++c) {
            U[c] = Un[c];
            Wi[c] = Pn[c];
        }
    }
    if (!isfinite(Wi[0] + Wi[1] + Wi[2] + Wi[3] + Wi[4])) atomicOr(C.status, 1);
}

template <int NF, class BT>
__global__ __launch_bounds__(MBLOCK) void k_update(BT B, double cfl)
{
    const MLoc ML = mb_loc(B, PK_CELL);
    const int i = (mblk() - ML.base) * MBLOCK + (int)threadIdx.x;
    if (i >= ML.cv->n_cells) return;
    update_cell<NF>(*ML.cv, ML.W, ML.src, i, cfl);
}

// The update with one lane per face: each of the G lanes of a cell loads one
// face's flux and geometry; the flux balance and sum |u.n S/V| are added over
// the lanes in a fixed butterfly order, then lane 0 updates the cell exactly
// as k_update does.
template <int G, class BT>
__global__ __launch_bounds__(MCELLS_Q * G) void k_update_q(BT B, double cfl)
{
    const MLoc ML = mb_loc(B, PK_GROUP);
    const CaseView &C = *ML.cv;
    double *__restrict__ W = ML.W;
    const double *__restrict__ src = ML.src;
    const int i = (mblk() - ML.base) * MCELLS_Q + (int)threadIdx.x / G;
    const int l = (int)threadIdx.x % G;
    if (i >= C.n_cells) return;   // whole groups leave together
    double *Wi = W + 5 * (size_t)i;
    double *U = C.U + 5 * (size_t)i;
    // the cell's own data first: these loads do not wait for its face range
    double Wc[5], Uc[5], Sc[5] = {0, 0, 0, 0, 0};
    for (int c = 0; c < 5; ++c) {
        Wc[c] = Wi[c];
        Uc[c] = U[c];
        if (src) Sc[c] = src[5 * (size_t)i + c];
    }
    const double V = C.cell_volume[i];
    const double sS0 = C.cell_sS[2 * (size_t)i], sS1 = C.cell_sS[2 * (size_t)i + 1];
    const int e0 = C.cf_ptr[i], nf = C.cf_ptr[i + 1] - e0;
    double R[5] = {0, 0, 0, 0, 0}, un = 0.0;
    if (l < nf) {
        const int e = e0 + l;
        const double fs = C.cf_fs[e];
        const double *F = C.fflux + 5 * (size_t)C.cf_face[e];
        for (int c = 0; c < 5; ++c) R[c] = F[c] * fs;
        if (cfl >= 0) {
            const double *n = C.cf_nsv + 3 * (size_t)e;
            un = fabs(Wc[1] * n[0] + Wc[2] * n[1] + Wc[3] * n[2]);
        }
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int c = 0; c < 5; ++c) R[c] += __shfl_xor(R[c], off, G);
        un += __shfl_xor(un, off, G);
    }
    if (l != 0) return;
    if (src)
        for (int c = 0; c < 5; ++c) R[c] += Sc[c] * V;
    double k;
    if (cfl < 0) {
        k = (-cfl * C.red[0]) / V;
    } else {
        const double a = sqrt(5.0 / 3.0 * Wc[4] / 2.0);
        const double nu = fmax(4.0 / 3.0, 5.0 / (3.0 * C.Pr)) * C.Kn * t_pow_omega(C, Wc[4]) / (sqrt(M_PI) * Wc[0]);
        k = cfl / (V * un + a * sS0 + 2.0 * nu * sS1);
    }
    // positivity safeguard: halve this cell's increment (at most ten times)
    // while the new density or temperature would not be positive
    double Un[5], Pn[5];
    bool ok = false;
    for (int h = 0; h <= 10 && !ok; ++h) {
        for (int c = 0; c < 5; ++c) Un[c] = Uc[c] + k * R[c];
        Pn[0] = Un[0];
        const double ir = 1.0 / Un[0];
        double u2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            Pn[1 + d] = Un[1 + d] * ir;
            u2 += Pn[1 + d] * Pn[1 + d];
        }
        Pn[4] = (Un[4] - Un[0] * u2) * ((1.0 / 1.5) * ir);
        ok = (Pn[0] > 0.0) && (Pn[4] > 0.0);
        k *= 0.5;
    }
    if (ok) {
        for (int c = 0; c < 5; ++c) {
            U[c] = Un[c];
            Wi[c] = Pn[c];
        }
    }
    const double *Wf = ok ? Pn : Wc;
    if (!isfinite(Wf[0] + Wf[1] + Wf[2] + Wf[3] + Wf[4])) atomicOr(C.status, 1);
}

template <class BT>
static void macro_steps_t(const BT &bt, const MBatch &b, int n_inner, double cfl, hipStream_t s)
{
    const dim3 gc(b.bc[b.n]), gf(b.bf[b.n]);
    hipLaunchKernelGGL(k_cons<BT>, gc, dim3(MBLOCK), 0, s, bt);
    if (b.bf[b.n] > 0) hipLaunchKernelGGL(k_hot_face<BT>, gf, dim3(MBLOCK_F), 0, s, bt);
    const bool lanes = macro_lanes();
    const dim3 gq(b.bq[b.n]);
    for (int it = 0; it < n_inner; ++it) {
        if (lanes) launch_lsq_q(bt, gq, b.nfmax, 4, s);
        else launch_lsq_t(bt, gc, b.nfmax, 4, s);
        if (b.bf[b.n] > 0) hipLaunchKernelGGL(k_face_flux<BT>, gf, dim3(MBLOCK_F), 0, s, bt);
        if (cfl < 0) {
            // one global (conservative) step per case
            hipLaunchKernelGGL(k_dloc<BT>, gc, dim3(MBLOCK), 0, s, bt);
            hipLaunchKernelGGL(k_min_final, dim3(b.n), dim3(256), 0, s, b);
        }
        if (lanes) {
            if (b.nfmax <= 4) hipLaunchKernelGGL((k_update_q<4, BT>), gq, dim3(MCELLS_Q * 4), 0, s, bt, cfl);
            else hipLaunchKernelGGL((k_update_q<MAXF, BT>), gq, dim3(MCELLS_Q * MAXF), 0, s, bt, cfl);
        } else {
            if (b.nfmax <= 4) hipLaunchKernelGGL((k_update<4, BT>), gc, dim3(MBLOCK), 0, s, bt, cfl);
            else hipLaunchKernelGGL((k_update<MAXF, BT>), gc, dim3(MBLOCK), 0, s, bt, cfl);
        }
    }
}

// Small cases (at most SMALL_CELLS cells) run all their pseudo-time steps in
// one workgroup each: the cell and face loops of a step are strided over the
// block's lanes with a barrier between the phases, so a 64-cell box pays one
// launch per solve instead of three per step.  The per-cell and per-face
// arithmetic is that of the one-thread-per-cell kernels (lsq_cell,
// face_flux_one, update_cell); a case takes this path by its size alone, so
// its results do not depend on the batch it runs in.
constexpr int SMALL_T = 512;
constexpr int SMALL_CELLS = 1024;

template <int NF>
__global__ __launch_bounds__(SMALL_T) void k_macro_small(MBatch B, int n_inner, double cfl)
{
    const int j = blockIdx.x;
    const CaseView &C = *B.cv[j];
    double *__restrict__ W = B.W[j];
    const double *__restrict__ hot = B.hot[j];
    const double *__restrict__ src = B.src[j];
    const int nc = C.n_cells, nfc = C.n_faces;
    const int t = threadIdx.x;
    __shared__ double sm[SMALL_T];
    for (int i = t; i < nc; i += SMALL_T) cons_cell(C, W, i);
    for (int f = t; f < nfc; f += SMALL_T) hot_face_one(C, hot, f);
    __syncthreads();
    for (int it = 0; it < n_inner; ++it) {
        for (int i = t; i < nc; i += SMALL_T) lsq_cell<4, NF>(C, W, i);
        __syncthreads();
        for (int f = t; f < nfc; f += SMALL_T) face_flux_one(C, W, f);
        if (cfl < 0) {
            // one global step: min over the cells of V / D (exact in any order)
            double v = INFINITY;
            for (int i = t; i < nc; i += SMALL_T) v = fmin(v, C.cell_volume[i] / cell_D(C, i, W + 5 * (size_t)i));
            sm[t] = v;
            __syncthreads();
            for (int st = SMALL_T / 2; st > 0; st >>= 1) {
                if (t < st) sm[t] = fmin(sm[t], sm[t + st]);
                __syncthreads();
            }
            if (t == 0) C.red[0] = sm[0];
        }
        __syncthreads();
        for (int i = t; i < nc; i += SMALL_T) update_cell<NF>(C, W, src, i, cfl);
        __syncthreads();
    }
}

bool macro_small_on()
{
    static const bool on = [] {
        const char *e = std::getenv("GSIS_MACRO_SMALL");
        return !(e && e[0] == '0');
    }();
    return on;
}

// case j of batch b appended to batch o (prefixes rebuilt from j's block counts)
static void mbatch_take(MBatch &o, const MBatch &b, int j)
{
    const int k = o.n;
    if (k == 0) o.bc[0] = o.bf[0] = o.bq[0] = 0, o.nfmax = b.nfmax, o.poly = b.poly;
    o.cv[k] = b.cv[j];
    o.W[k] = b.W[j];
    o.Tr[k] = b.Tr[j];
    o.hot[k] = b.hot[j];
    o.src[k] = b.src[j];
    o.bc[k + 1] = o.bc[k] + (b.bc[j + 1] - b.bc[j]);
    o.bf[k + 1] = o.bf[k] + (b.bf[j + 1] - b.bf[j]);
    o.bq[k + 1] = o.bq[k] + (b.bq[j + 1] - b.bq[j]);
    o.n = k + 1;
}

hipError_t launch_macro_steps_batch(const MBatch &b, int n_inner, double cfl, hipStream_t s)
{
    if (b.n <= 0) return hipSuccess;
    if (b.poly) return launch_macro_steps_poly(b, n_inner, cfl, s);
    MBatch small{}, large{};
    for (int j = 0; j < b.n; ++j) {
        const bool sm = macro_small_on() && (b.bc[j + 1] - b.bc[j]) * MBLOCK <= SMALL_CELLS;
        mbatch_take(sm ? small : large, b, j);
    }
    if (small.n > 0 && n_inner > 0) {
        if (small.nfmax <= 4) hipLaunchKernelGGL(k_macro_small<4>, dim3(small.n), dim3(SMALL_T), 0, s, small, n_inner, cfl);
        else hipLaunchKernelGGL(k_macro_small<MAXF>, dim3(small.n), dim3(SMALL_T), 0, s, small, n_inner, cfl);
    }
    if (large.n == 1) macro_steps_t(mone_of(large), large, n_inner, cfl, s);
    else if (large.n > 1) macro_steps_t(large, large, n_inner, cfl, s);
    return hipGetLastError();
}

hipError_t launch_macro_steps(const CaseView *cv, const CaseView &h, double *W, const double *hot, const double *src,
                              int n_inner, double cfl, hipStream_t s)
{
    MBatch b{};
    mbatch_add(b, cv, h, W, hot, src);
    return launch_macro_steps_batch(b, n_inner, cfl, s);
}

// ---------------------------------------------------------------------------
// surface quantities on the diffuse walls (Sec. 4.2/4.3): one block per wall
// face.  Kinetic wall cell: incoming velocities (c.n > 0, c = xi - u_w) from
// the cell's VDF, reflected ones from rho_w M(1, u_w, T_w) with rho_w from
// zero net mass flux; FP64 sums per thread, then a fixed-order block tree.
// NS wall cell: pressure plus the NSF stress and heat flux of the one-sided
// wall gradients (the wall flux of the synthetic solve).
// ---------------------------------------------------------------------------
constexpr int NSS = 10;   // incoming: a f, c (c.n) f (3), (c.n) e f; reflected: |a| M, c (c.n) M (3), (c.n) e M

template <class T>
__global__ __launch_bounds__(256) void k_surface(const CaseView *__restrict__ cvp, int cur, double *__restrict__ out)
{
    const CaseView &C = *cvp;
    const int j = blockIdx.x;   // grid = n_wall
    const int f = C.wall_face[j];
    const int L = C.face_cells[2 * f], p = -1 - C.face_cells[2 * f + 1];
    const double *ps = C.patch_state + 5 * p;
    const double *n = C.face_normal + 3 * (size_t)f;
    const int slot = C.slot_of_cell[L];
    double *o = out + (size_t)j * GSIS_NSURF;
    if (slot < 0) {
        // the two-VDF gas's NS wall cells take the two-temperature NSF laws
        // (k_surface_ns_p)
        if (C.poly || threadIdx.x != 0) return;
        const double *PL = C.W + 5 * (size_t)L;
        const double dn = 0.5 * C.face_dist[f];
        const double *gL = grad_row(C, L, 0);
        double G[4][3];
        for (int v = 0; v < 4; ++v) {
            double gn = gL[3 * v] * n[0] + gL[3 * v + 1] * n[1] + gL[3 * v + 2] * n[2];
            double fl = (v < 3) ? PL[1 + v] : PL[4];
            double jump = (ps[1 + v] - fl) / dn;
            for (int d = 0; d < 3; ++d) G[v][d] = gL[3 * v + d] + (jump - gn) * n[d];
        }
        double Gu[9] = {G[0][0], G[0][1], G[0][2], G[1][0], G[1][1], G[1][2], G[2][0], G[2][1], G[2][2]};
        double sg[6], q[3];
        nsf(C, ps[4], Gu, G[3], sg, q);
        const double pL = PL[0] * PL[4];
        double tau[3] = {pL * n[0] + sg[0] * n[0] + sg[3] * n[1] + sg[4] * n[2],
                         pL * n[1] + sg[3] * n[0] + sg[1] * n[1] + sg[5] * n[2],
                         pL * n[2] + sg[4] * n[0] + sg[5] * n[1] + sg[2] * n[2]};
        const double pn = tau[0] * n[0] + tau[1] * n[1] + tau[2] * n[2];
        for (int d = 0; d < 3; ++d) {
            o[d] = tau[d];
            o[4 + d] = tau[d] - pn * n[d];
        }
        o[3] = pn;
        o[7] = q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
        o[8] = 0.0;
        return;
    }
    const int vd = C.vdim;
    const int nvp = C.row / C.nfun;
    const T *row = (const T *)C.f[cur] + (size_t)slot * C.row;
    const double Tw = ps[4], it = 1.0 / Tw;
    const double amp = (vd == 3) ? pow(M_PI * Tw, -1.5) : 1.0 / (M_PI * Tw);
    double acc[NSS];
    for (int a = 0; a < NSS; ++a) acc[a] = 0.0;
    for (int k = threadIdx.x; k < C.nv; k += 256) {
        double xi[3], w;
        vnode(C, k, xi, w);
        double c[3] = {xi[0] - ps[1], xi[1] - ps[2], (vd == 3) ? xi[2] - ps[3] : 0.0};
        const double a = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
        const double c2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        if (a > 0.0) {
            // energy carried: |c|^2 f (3D), |c|^2 phi + psi (reduced 2D),
            // |c|^2 f0 + 2 f1 (two-VDF gas: translational plus internal)
            const double f0 = (double)row[k];
            const double e = C.poly ? c2 * f0 + 2.0 * (double)row[nvp + k]
                                    : ((vd == 3) ? c2 * f0 : c2 * f0 + (double)row[nvp + k]);
            acc[0] += w * a * f0;
            for (int d = 0; d < 3; ++d) acc[1 + d] += w * a * c[d] * f0;
            acc[4] += w * a * e;
        } else if (a < 0.0) {
            // reflected: the wall Maxwellian, with f1 = (d_r T_w / 4) M for the two-VDF gas
            const double m = amp * exp(-c2 * it);
            const double e = C.poly ? (c2 + 0.5 * C.dr * Tw) * m : ((vd == 3) ? c2 * m : (c2 + 0.5 * Tw) * m);
            acc[5] -= w * a * m;
            for (int d = 0; d < 3; ++d) acc[6 + d] += w * a * c[d] * m;
            acc[9] += w * a * e;
        }
    }
    __shared__ double lds[4][NSS];
    for (int a = 0; a < NSS; ++a) {
        double v = acc[a];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6][a] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double S[NSS];
    for (int a = 0; a < NSS; ++a) S[a] = ((lds[0][a] + lds[1][a]) + lds[2][a]) + lds[3][a];
    const double rw = S[0] / S[5];
    double tau[3];
    for (int d = 0; d < 3; ++d) tau[d] = 2.0 * (S[1 + d] + rw * S[6 + d]);
    const double pn = tau[0] * n[0] + tau[1] * n[1] + tau[2] * n[2];
    for (int d = 0; d < 3; ++d) {
        o[d] = tau[d];
        o[4 + d] = tau[d] - pn * n[d];
    }
    o[3] = pn;
    o[7] = S[4] + rw * S[9];
    o[8] = S[0] - rw * S[5];
}

// integrals sum tau S (3) and sum q S over the wall faces, fixed order
__global__ __launch_bounds__(256) void k_surface_totals(const CaseView *__restrict__ cvp, const double *__restrict__ out,
                                                        double *__restrict__ tot)
{
    const CaseView &C = *cvp;
    __shared__ double sm[4][256];
    double a[4] = {0, 0, 0, 0};
    for (int j = threadIdx.x; j < C.n_wall; j += 256) {
        const double S = C.face_area[C.wall_face[j]];
        const double *o = out + (size_t)j * GSIS_NSURF;
        a[0] += o[0] * S;
        a[1] += o[1] * S;
        a[2] += o[2] * S;
        a[3] += o[7] * S;
    }
    for (int c = 0; c < 4; ++c) sm[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int c = 0; c < 4; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) tot[threadIdx.x] = sm[threadIdx.x][0];
}

hipError_t launch_surface(const CaseView *cv, const CaseView &h, int cur, double *out, double *totals, hipStream_t s)
{
    if (h.n_wall <= 0) {
        if (totals) return hipMemsetAsync(totals, 0, 4 * sizeof(double), s);
        return hipSuccess;
    }
    // one-sided wall gradients of the NS wall cells come from the current W
    hipError_t e = launch_lsq(cv, h, h.W, 4, s);
    if (e != hipSuccess) return e;
    if (h.dtype == GSIS_F32) hipLaunchKernelGGL(k_surface<float>, dim3(h.n_wall), dim3(256), 0, s, cv, cur, out);
    else hipLaunchKernelGGL(k_surface<double>, dim3(h.n_wall), dim3(256), 0, s, cv, cur, out);
    if (h.poly) {
        e = launch_surface_ns_poly(cv, h, out, s);
        if (e != hipSuccess) return e;
    }
    if (totals) hipLaunchKernelGGL(k_surface_totals, dim3(1), dim3(256), 0, s, cv, (const double *)out, totals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// convergence measure (Sec. 4): eps_W = sqrt(sum (W^n - W^{n-1})^2 V / sum (W^{n-1})^2 V)
// for W in {rho, u (vector), T}; block partials then one fixed-order pass
// ---------------------------------------------------------------------------
__global__ void k_eps_part(const CaseView *__restrict__ cvp, const double *__restrict__ Wn,
                           const double *__restrict__ Wo)
{
    const CaseView &C = *cvp;
    __shared__ double sm[6][256];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (i < C.n_cells) {
        double V = C.cell_volume[i];
        const double *a = Wn + 5 * (size_t)i, *b = Wo + 5 * (size_t)i;
        v[0] = (a[0] - b[0]) * (a[0] - b[0]) * V;
        v[1] = b[0] * b[0] * V;
        for (int d = 1; d < 4; ++d) {
            v[2] += (a[d] - b[d]) * (a[d] - b[d]) * V;
            v[3] += b[d] * b[d] * V;
        }
        v[4] = (a[4] - b[4]) * (a[4] - b[4]) * V;
        v[5] = b[4] * b[4] * V;
    }
    for (int c = 0; c < 6; ++c) sm[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int c = 0; c < 6; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) C.red[8 + 6 * (size_t)blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

// one block: thread t sums block partials t, t + 256, ... (fixed order), then
// a fixed-order tree
__global__ __launch_bounds__(256) void k_eps_final(const CaseView *__restrict__ cvp, int nb)
{
    const CaseView &C = *cvp;
    __shared__ double sm[6][256];
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += 256)
        for (int c = 0; c < 6; ++c) s[c] += C.red[8 + 6 * (size_t)b + c];
    for (int c = 0; c < 6; ++c) sm[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int c = 0; c < 6; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        double num = sm[2 * k][0], den = sm[2 * k + 1][0];
        C.eps[k] = (den > 1e-30) ? sqrt(num / den) : sqrt(num);
    }
}

hipError_t launch_eps(const CaseView *cv, const CaseView &h, const double *Wnew, const double *Wold, hipStream_t s)
{
    int nb = (h.n_cells + 255) / 256;
    hipLaunchKernelGGL(k_eps_part, dim3(nb), dim3(256), 0, s, cv, Wnew, Wold);
    hipLaunchKernelGGL(k_eps_final, dim3(1), dim3(256), 0, s, cv, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// region test (Sec. 3.2): Kn_Gll = lambda max(|grad rho|/rho, |grad U|/max(U, a),
// |grad T|/T), lambda = Kn T^(omega - 1/2) / rho; flag = Kn_Gll >= Kn_ref, plus
// cells within `layers` face hops of a wall.  Gradients of (u, T, rho, |u|) of
// W must be in C.grad.  Result in scan_tmp[0..n_cells).
// ---------------------------------------------------------------------------
__global__ void k_kn_flags(const CaseView *__restrict__ cvp, double Kn_ref, int layers, int32_t *out)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    const double *W = C.W + 5 * (size_t)i;
    const double *g = grad_row(C, i, 0);
    double rho = W[0], T = W[4];
    double U = sqrt(W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
    double a = sqrt(5.0 * T / 6.0);
    double lam = C.Kn * pow(T, C.omega - 0.5) / rho;
    auto nrm = [](const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); };
    double kn = lam * fmax(fmax(nrm(grad_row(C, i, 4)) / rho, nrm(grad_row(C, i, 5)) / fmax(U, a)), nrm(g + 9) / T);
    int flag = kn >= Kn_ref;
    if (layers > 0)
        for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
            int oth = C.cf_other[e];
            if (oth < 0 && C.patch_kind[-1 - oth] == GSIS_PATCH_WALL) flag |= 2;
        }
    out[i] = flag;
}

// grow the wall band by one face hop: bit 1 marks the band
__global__ void k_grow(const CaseView *__restrict__ cvp, const int32_t *in, int32_t *out)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    int v = in[i];
    if (!(v & 2))
        for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
            int oth = C.cf_other[e];
            if (oth >= 0 && (in[oth] & 2)) {
                v |= 2;
                break;
            }
        }
    out[i] = v;
}

__global__ void k_copy_i(int32_t *d, const int32_t *s, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

hipError_t launch_flags(const CaseView *cv, const CaseView &h, double Kn_ref, int layers, hipStream_t s)
{
    const int gc = (h.n_cells + 127) / 128;
    hipError_t e = launch_lsq(cv, h, h.W, 6, s);
    if (e != hipSuccess) return e;
    int32_t *a = h.scan_tmp, *b = h.scan_tmp + h.n_cells;
    hipLaunchKernelGGL(k_kn_flags, dim3(gc), dim3(128), 0, s, cv, Kn_ref, layers, a);
    for (int l = 1; l < layers; ++l) {
        hipLaunchKernelGGL(k_grow, dim3(gc), dim3(128), 0, s, cv, a, b);
        int32_t *t = a;
        a = b;
        b = t;
    }
    if (a != h.scan_tmp) hipLaunchKernelGGL(k_copy_i, dim3(gc), dim3(128), 0, s, h.scan_tmp, a, h.n_cells);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// compaction (deterministic, multi-block): new flags in scan_tmp[0..n); the
// kinetic list in ascending cell id; staying cells keep their slot; freed
// slots are reused lowest-first by new cells in ascending cell id.  Every list
// is a prefix sum: per-block counts, one block scans the block totals, then
// each block writes its items at its offset (block-local order by a scan).
// scan_tmp layout: flags [n] | used [cap] | free list [cap] | block sums.
// ---------------------------------------------------------------------------
constexpr int CB = 256;   // items per block of the compaction kernels

// 1024-thread exclusive scan of one int per thread; returns the prefix, sm[1024] = total
__device__ int block_excl_scan(int v, int *sm)
{
    const int tid = threadIdx.x;
    sm[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int x = (tid >= off) ? sm[tid - off] : 0;
        __syncthreads();
        sm[tid] += x;
        __syncthreads();
    }
    const int incl = sm[tid];
    const int total = sm[1023];
    __syncthreads();
    if (tid == 0) sm[1024] = total;
    __syncthreads();
    return incl - v;
}

// exclusive scan of one int per thread over a 256-thread block; *total = sum
__device__ int block_excl_scan256(int v, int *sm, int *total)
{
    const int tid = threadIdx.x;
    sm[tid] = v;
    __syncthreads();
    for (int off = 1; off < CB; off <<= 1) {
        const int x = (tid >= off) ? sm[tid - off] : 0;
        __syncthreads();
        sm[tid] += x;
        __syncthreads();
    }
    const int incl = sm[tid];
    *total = sm[CB - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_used_clear(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < C.capacity) C.scan_tmp[C.n_cells + s] = 0;
}

// slots of staying cells; per-block counts of kinetic and new cells
__global__ __launch_bounds__(CB) void k_compact_count(const CaseView *__restrict__ cvp, int nbc)
{
    const CaseView &C = *cvp;
    __shared__ int sm[CB];
    const int n = C.n_cells, cap = C.capacity;
    int32_t *used = C.scan_tmp + n;
    int32_t *bsum = C.scan_tmp + n + 2 * cap;     // [2 nbc] kinetic, new; then [nbs] free slots
    const int i = blockIdx.x * CB + threadIdx.x;
    int kin = 0, nw = 0;
    if (i < n) {
        kin = C.scan_tmp[i] != 0;
        const int old = C.slot_of_cell[i];
        if (kin && old >= 0) used[old] = 1;
        nw = kin && old < 0;
    }
    int tk, tn;
    block_excl_scan256(kin, sm, &tk);
    block_excl_scan256(nw, sm, &tn);
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = tk;
        bsum[nbc + blockIdx.x] = tn;
    }
}

// per-block counts of free slots (after every staying cell has marked its slot)
__global__ __launch_bounds__(CB) void k_free_count(const CaseView *__restrict__ cvp, int nbc)
{
    const CaseView &C = *cvp;
    __shared__ int sm[CB];
    const int n = C.n_cells, cap = C.capacity;
    const int s = blockIdx.x * CB + threadIdx.x;
    const int f = (s < cap) ? !C.scan_tmp[n + s] : 0;
    int tf;
    block_excl_scan256(f, sm, &tf);
    if (threadIdx.x == 0) C.scan_tmp[n + 2 * cap + 2 * nbc + blockIdx.x] = tf;
}

// exclusive scans of the block totals (one block; three lists), totals to the device counters
__global__ __launch_bounds__(1024) void k_block_offsets(const CaseView *__restrict__ cvp, int nbc, int nbs)
{
    const CaseView &C = *cvp;
    __shared__ int sm[1025];
    const int n = C.n_cells, cap = C.capacity;
    int32_t *bsum = C.scan_tmp + n + 2 * cap;
    for (int list = 0; list < 3; ++list) {
        int32_t *b = bsum + list * nbc;
        const int m = (list < 2) ? nbc : nbs;
        int carry = 0;
        for (int base = 0; base < m; base += 1024) {
            const int j = base + threadIdx.x;
            const int v = (j < m) ? b[j] : 0;
            const int ex = block_excl_scan(v, sm);
            const int tot = sm[1024];
            if (j < m) b[j] = carry + ex;
            carry += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (list == 0) {
                *C.n_kin_dev = carry;
                if (carry > cap) C.status[1] = 1;
            } else if (list == 1) {
                *C.n_new_dev = carry;
            }
        }
    }
}

__global__ __launch_bounds__(CB) void k_free_scatter(const CaseView *__restrict__ cvp, int nbc)
{
    const CaseView &C = *cvp;
    __shared__ int sm[CB];
    const int n = C.n_cells, cap = C.capacity;
    const int s = blockIdx.x * CB + threadIdx.x;
    const int f = (s < cap) ? !C.scan_tmp[n + s] : 0;
    int tf;
    const int ex = block_excl_scan256(f, sm, &tf);
    if (f) C.scan_tmp[n + cap + C.scan_tmp[n + 2 * cap + 2 * nbc + blockIdx.x] + ex] = s;
}

__global__ __launch_bounds__(CB) void k_compact_scatter(const CaseView *__restrict__ cvp, int nbc)
{
    const CaseView &C = *cvp;
    __shared__ int sm[CB];
    const int n = C.n_cells, cap = C.capacity;
    const int32_t *freelist = C.scan_tmp + n + cap;
    const int32_t *bsum = C.scan_tmp + n + 2 * cap;
    if (*C.n_kin_dev > cap) return;   // capacity exceeded: the lists stay as they were (block-uniform)
    const int i = blockIdx.x * CB + threadIdx.x;
    int kin = 0, old = -1;
    if (i < n) {
        kin = C.scan_tmp[i] != 0;
        old = C.slot_of_cell[i];
    }
    const int nw = kin && old < 0;
    int tk, tn;
    const int ek = block_excl_scan256(kin, sm, &tk);
    const int en = block_excl_scan256(nw, sm, &tn);
    if (i < n) {
        if (kin) {
            C.kin_cell[bsum[blockIdx.x] + ek] = i;
            if (nw) {
                const int q = bsum[nbc + blockIdx.x] + en;
                C.new_cell[q] = i;
                C.slot_of_cell[i] = freelist[q];
            }
        } else {
            C.slot_of_cell[i] = -1;
        }
        C.flags[i] = kin;
    }
}

// NS cells with a kinetic face neighbour -> mark in scan_tmp (after compaction)
__global__ void k_ghost_mark(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    int g = 0;
    if (C.slot_of_cell[i] < 0)
        for (int e = C.cf_ptr[i]; e < C.cf_ptr[i + 1]; ++e) {
            const int o = C.cf_other[e];
            if (o >= 0 && C.slot_of_cell[o] >= 0) g = 1;
        }
    C.scan_tmp[i] = g;
}

// marked cells in ascending id -> rows of grow: per-block counts, one block
// scans them, each block writes its rows
__global__ __launch_bounds__(CB) void k_ghost_count(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    __shared__ int sm[CB];
    const int i = blockIdx.x * CB + threadIdx.x;
    const int g = (i < C.n_cells) ? C.scan_tmp[i] : 0;
    int t;
    block_excl_scan256(g, sm, &t);
    if (threadIdx.x == 0) C.scan_tmp[C.n_cells + blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void k_ghost_offsets(const CaseView *__restrict__ cvp, int nb)
{
    const CaseView &C = *cvp;
    __shared__ int sm[1025];
    int32_t *b = C.scan_tmp + C.n_cells;
    int carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int j = base + threadIdx.x;
        const int v = (j < nb) ? b[j] : 0;
        const int ex = block_excl_scan(v, sm);
        const int tot = sm[1024];
        if (j < nb) b[j] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *C.n_ghost_dev = carry;
        if (carry > C.gcap) C.status[1] = 1;
    }
}

__global__ __launch_bounds__(CB) void k_ghost_scatter(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    __shared__ int sm[CB];
    if (*C.n_ghost_dev > C.gcap) return;
    const int i = blockIdx.x * CB + threadIdx.x;
    const int g = (i < C.n_cells) ? C.scan_tmp[i] : 0;
    int t;
    const int ex = block_excl_scan256(g, sm, &t);
    if (i < C.n_cells) {
        if (g) {
            const int r = C.scan_tmp[C.n_cells + blockIdx.x] + ex;
            C.ghost_cell[r] = i;
            C.ghost_slot[i] = r;
        } else {
            C.ghost_slot[i] = -1;
        }
    }
}

hipError_t launch_compact(const CaseView *cv, const CaseView &h, hipStream_t s)
{
    const int nbc = (h.n_cells + CB - 1) / CB, nbs = (h.capacity + CB - 1) / CB;
    hipLaunchKernelGGL(k_used_clear, dim3(nbs), dim3(CB), 0, s, cv);
    hipLaunchKernelGGL(k_compact_count, dim3(nbc), dim3(CB), 0, s, cv, nbc);
    hipLaunchKernelGGL(k_free_count, dim3(nbs), dim3(CB), 0, s, cv, nbc);
    hipLaunchKernelGGL(k_block_offsets, dim3(1), dim3(1024), 0, s, cv, nbc, nbs);
    hipLaunchKernelGGL(k_free_scatter, dim3(nbs), dim3(CB), 0, s, cv, nbc);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nbc), dim3(CB), 0, s, cv, nbc);
    hipLaunchKernelGGL(k_ghost_mark, dim3(nbc), dim3(CB), 0, s, cv);
    hipLaunchKernelGGL(k_ghost_count, dim3(nbc), dim3(CB), 0, s, cv);
    hipLaunchKernelGGL(k_ghost_offsets, dim3(1), dim3(1024), 0, s, cv, nbc);
    hipLaunchKernelGGL(k_ghost_scatter, dim3(nbc), dim3(CB), 0, s, cv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__global__ void k_copy(double *d, const double *s, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

hipError_t launch_copy_W(double *dst, const double *src, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3((5 * n + 255) / 256), dim3(256), 0, s, dst, src, 5 * n);
    return hipGetLastError();
}

__global__ void k_set_flags(const CaseView *__restrict__ cvp, const uint8_t *fl, int fill)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C.n_cells) C.scan_tmp[i] = fl ? (fl[i] != 0) : fill;
}

hipError_t launch_set_flags(const CaseView *cv, const CaseView &h, const uint8_t *flags, int fill, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_flags, dim3((h.n_cells + 255) / 256), dim3(256), 0, s, cv, flags, fill);
    return hipGetLastError();
}

__global__ void k_get_flags(const CaseView *__restrict__ cvp, uint8_t *fl)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C.n_cells) fl[i] = (uint8_t)(C.flags[i] != 0);
}

hipError_t launch_get_flags(const CaseView *cv, const CaseView &h, uint8_t *flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_get_flags, dim3((h.n_cells + 255) / 256), dim3(256), 0, s, cv, flags);
    return hipGetLastError();
}

__global__ void k_moments_out(const CaseView *__restrict__ cvp, int n_kin, double *out, int32_t *kc)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_kin) return;
    int cell = C.kin_cell[t];
    const double *m = C.mom + (size_t)C.slot_of_cell[cell] * MOMS;
    for (int c = 0; c < GSIS_NMOM; ++c) out[(size_t)t * GSIS_NMOM + c] = m[c];
    if (kc) kc[t] = cell;
}

hipError_t launch_moments_out(const CaseView *cv, const CaseView &h, int n_kin, double *out, int32_t *kc,
                              hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_moments_out, dim3((n_kin + 127) / 128), dim3(128), 0, s, cv, n_kin, out, kc);
    return hipGetLastError();
}

__global__ void k_internal_out(const CaseView *__restrict__ cvp, int n_kin, double *out)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_kin) return;
    const double *m = C.mom + (size_t)C.slot_of_cell[C.kin_cell[t]] * MOMS + MOM_INT;
    for (int c = 0; c < 4; ++c) out[4 * (size_t)t + c] = m[c];
}

hipError_t launch_internal_out(const CaseView *cv, const CaseView &h, int n_kin, double *out, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_internal_out, dim3((n_kin + 127) / 128), dim3(128), 0, s, cv, n_kin, out);
    return hipGetLastError();
}

__global__ void k_W_from_mom(const CaseView *__restrict__ cvp, int n_kin, double *W)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_kin) return;
    int cell = C.kin_cell[t];
    const double *m = C.mom + (size_t)C.slot_of_cell[cell] * MOMS;
    for (int c = 0; c < 5; ++c) W[5 * (size_t)cell + c] = m[c];
}

hipError_t launch_W_from_mom(const CaseView *cv, const CaseView &h, int n_kin, double *W, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_W_from_mom, dim3((n_kin + 127) / 128), dim3(128), 0, s, cv, n_kin, W);
    return hipGetLastError();
}

__global__ void k_check_W(const CaseView *__restrict__ cvp, const double *W)
{
    const CaseView &C = *cvp;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C.n_cells) return;
    const double *w = W + 5 * (size_t)i;
    if (!(w[0] > 0.0) || !(w[4] > 0.0) || !isfinite(w[1] + w[2] + w[3])) atomicOr(C.status, 1);
}

hipError_t launch_check_W(const CaseView *cv, const CaseView &h, const double *W, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_W, dim3((h.n_cells + 255) / 256), dim3(256), 0, s, cv, W);
    return hipGetLastError();
}

}  // namespace gsis
