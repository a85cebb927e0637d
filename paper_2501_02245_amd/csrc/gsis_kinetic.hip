// gsis_kinetic.hip -- kinetic-side kernels for gfx950.
//
// Hot path of Sec. 3.1 (Zhang, Zeng & Wu, arXiv 2501.02245): the implicit
// discrete-velocity update over the kinetic cells with first-order upwind
// face values and point-Jacobi lagging, the velocity-moment reduction of
// Sec. 2 (eq. getmoment) fused into its epilogue, the per-cell relaxation
// parameters with the conservation fix-up, and the GSIS correction (first
// eq. updatef).
//
// Layout: VDF rows are velocity-innermost, one row of nfun * nv_pad values
// per kinetic slot ([slot][fun][k]); consecutive lanes touch consecutive k,
// so every global access of the streaming kernels is coalesced.  One block of
// 256 threads handles one (kinetic cell, velocity tile); blocks are numbered
// tile-major and remapped so that each of the eight XCDs walks a contiguous
// run of cells (neighbour rows then meet in that XCD's L2).  Face data,
// node/weight tables and the separable Gaussian factor tables
// exp(-(x_j - u_d)^2 / T) of every Maxwellian the block needs live in LDS, so
// a point's equilibrium costs three LDS reads and two multiplies, no exp.
#include <math.h>

#include <cstdlib>

#include "gsis_impl.hpp"

namespace gsis {

enum { K_KIN = 0, K_WALL = 1, K_FAR = 2, K_GHOST = 3 };

template <int NS>
__device__ __forceinline__ void block_reduce_store(double (&v)[NS], double *out, double *lds)
{
    // fixed-order butterfly inside each wave, then the four waves in order
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        v[i] = x;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) lds[wave * NS + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double s = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) s += lds[w * NS + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// velocity-node index of point k and the per-256 increment
struct VIdx {
    int ix, iy, iz;
    int dx, dy, dz;
};

template <int VD>
__device__ __forceinline__ VIdx vidx_init(int k, int n1, int n2)
{
    VIdx v;
    if (VD == 3) {
        v.iz = k % n2;
        int r = k / n2;
        v.iy = r % n1;
        v.ix = r / n1;
        v.dz = BLOCK % n2;
        int q = BLOCK / n2;
        v.dy = q % n1;
        v.dx = q / n1;
    } else {
        v.iz = 0;
        v.iy = k % n1;
        v.ix = k / n1;
        v.dz = 0;
        v.dy = BLOCK % n1;
        v.dx = BLOCK / n1;
    }
    return v;
}

template <int VD>
__device__ __forceinline__ void vidx_step(VIdx &v, int n1, int n2)
{
    if (VD == 3) {
        v.iz += v.dz;
        int c = v.iz >= n2;
        v.iz -= c ? n2 : 0;
        v.iy += v.dy + c;
        int c2 = v.iy >= n1;
        v.iy -= c2 ? n1 : 0;
        v.ix += v.dx + c2;
    } else {
        v.iy += v.dy;
        int c = v.iy >= n1;
        v.iy -= c ? n1 : 0;
        v.ix += v.dx + c;
    }
}

// ---------------------------------------------------------------------------
// Per-cell FP64 algebra: separable Gaussian moments and the fix-up solve
// ---------------------------------------------------------------------------
struct GMom {
    double g[3][8];   // g[d][p] = sum_j w_j c^p exp(-c^2/T), c = x_j - u_d
};

__device__ void gauss_moments(const CaseView &C, const double *u, double it, GMom &G)
{
    for (int d = 0; d < C.vdim; ++d) {
        for (int p = 0; p < 8; ++p) G.g[d][p] = 0.0;
        for (int j = 0; j < C.n[d]; ++j) {
            double c = C.xv[d * MAXA + j] - u[d];
            double e = C.wv[d * MAXA + j] * exp(-c * c * it);
            double cp = 1.0;
            for (int p = 0; p < 8; ++p) {
                G.g[d][p] += e * cp;
                cp *= c;
            }
        }
    }
    if (C.vdim == 2)
        for (int p = 0; p < 8; ++p) G.g[2][p] = (p == 0) ? 1.0 : 0.0;
}

__device__ __forceinline__ double gs(const GMom &G, int i, int j, int k) { return G.g[0][i] * G.g[1][j] * G.g[2][k]; }

// sum_k w c^(i,j,k) E (1 + kq.c (c^2/T - 5/2))   (3D Shakhov weight)
__device__ double sh3(const GMom &G, const double *kq, double it, int i, int j, int k)
{
    double v = gs(G, i, j, k);
    if (kq) {
        v += kq[0] * ((gs(G, i + 3, j, k) + gs(G, i + 1, j + 2, k) + gs(G, i + 1, j, k + 2)) * it - 2.5 * gs(G, i + 1, j, k));
        v += kq[1] * ((gs(G, i + 2, j + 1, k) + gs(G, i, j + 3, k) + gs(G, i, j + 1, k + 2)) * it - 2.5 * gs(G, i, j + 1, k));
        v += kq[2] * ((gs(G, i + 2, j, k + 1) + gs(G, i, j + 2, k + 1) + gs(G, i, j, k + 3)) * it - 2.5 * gs(G, i, j, k + 1));
    }
    return v;
}

// reduced pair: phi weight (1 + kq.c (c^2/T - 2)), psi weight (T/2)(1 + kq.c (c^2/T - 1))
__device__ double sh2(const GMom &G, const double *kq, double it, double shift, int i, int j)
{
    double v = gs(G, i, j, 0);
    if (kq) {
        v += kq[0] * ((gs(G, i + 3, j, 0) + gs(G, i + 1, j + 2, 0)) * it - shift * gs(G, i + 1, j, 0));
        v += kq[1] * ((gs(G, i + 2, j + 1, 0) + gs(G, i, j + 3, 0)) * it - shift * gs(G, i, j + 1, 0));
    }
    return v;
}

__device__ int solve_dense(int n, double *A, double *b)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (!(fabs(A[piv * n + col]) > 0.0)) return -1;
        if (piv != col) {
            for (int j = 0; j < n; ++j) {
                double t = A[col * n + j];
                A[col * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
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

// ---------------------------------------------------------------------------
// point-set grids: the conservation fix-up from direct FP64 sums over the
// nodes, one block per item.  The target is E S(c) (a0 + a.c + b c^2) with
// E = exp(-c^2 / T) and S the Shakhov factor (or 1); its discrete moments
// {1, c, c^2} must equal (rho, 0, 3 rho T / 2) in the frame u.
//   mode 0: the relaxation target of ParamRec (rho from the moments)
//   mode 1: the Maxwellians of W_new and W_half (FeqRec 0 and 1)
//   mode 2: the Maxwellian of W (FeqRec 0, initial fill)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_fix_pts(const CaseView *__restrict__ cvp, const int32_t *list, int mode)
{
    const CaseView &C = *cvp;
    const int cell = list[blockIdx.x];
    const int slot = C.slot_of_cell[cell];
    __shared__ double red[(BLOCK / 64) * 15];
    const int nrun = (mode == 1) ? 2 : 1;
    for (int which = 0; which < nrun; ++which) {
        double u[3], it, rho, kq[3] = {0.0, 0.0, 0.0};
        double *fx;
        if (mode == 0) {
            ParamRec &P = C.param[slot];
            for (int d = 0; d < 3; ++d) u[d] = P.u[d], kq[d] = P.kq[d];
            it = P.it;
            rho = C.mom[(size_t)slot * MOMS];
            fx = P.fx;
        } else {
            FeqRec &F = C.feq[2 * (size_t)slot + which];
            for (int d = 0; d < 3; ++d) u[d] = F.u[d];
            it = F.it;
            const double *W = (mode == 2) ? C.W + 5 * (size_t)cell
                                          : ((which == 0 ? C.Wn : C.Wh) + 5 * (size_t)cell);
            rho = W[0];
            fx = F.fx;
        }
        double acc[15];
#pragma unroll
        for (int a = 0; a < 15; ++a) acc[a] = 0.0;
        for (int k = threadIdx.x; k < C.nv; k += BLOCK) {
            double xi[3], w;
            vnode(C, k, xi, w);
            const double c0 = xi[0] - u[0], c1 = xi[1] - u[1], c2 = xi[2] - u[2];
            const double cc = c0 * c0 + c1 * c1 + c2 * c2;
            double g = w * exp(-cc * it);
            if (mode == 0) g *= 1.0 + (kq[0] * c0 + kq[1] * c1 + kq[2] * c2) * (cc * it - 2.5);
            const double b[5] = {1.0, c0, c1, c2, cc};
#pragma unroll
            for (int a = 0; a < 5; ++a)
#pragma unroll
                for (int c = a; c < 5; ++c) acc[a * 5 - a * (a - 1) / 2 + (c - a)] += g * b[a] * b[c];
        }
        // fixed-order block reduction
#pragma unroll
        for (int m = 0; m < 15; ++m) {
            double v = acc[m];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * 15 + m] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double S[15];
            for (int m = 0; m < 15; ++m) {
                S[m] = 0.0;
                for (int wv = 0; wv < BLOCK / 64; ++wv) S[m] += red[wv * 15 + m];
            }
            double A[25], bb[5];
            int m = 0;
            for (int a = 0; a < 5; ++a)
                for (int c = a; c < 5; ++c) {
                    A[a * 5 + c] = S[m];
                    A[c * 5 + a] = S[m];
                    ++m;
                }
            const double T = 1.0 / it;
            bb[0] = rho;
            bb[1] = bb[2] = bb[3] = 0.0;
            bb[4] = 1.5 * rho * T;
            if (solve_dense(5, A, bb)) atomicOr(C.status, 1);
            for (int a = 0; a < 5; ++a) fx[a] = bb[a];
        }
        __syncthreads();
    }
}

hipError_t launch_fix_pts(const CaseView *cv, const CaseView &h, int n_items, const int32_t *list, int mode,
                          hipStream_t s)
{
    if (!h.points || n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fix_pts, dim3(n_items), dim3(BLOCK), 0, s, cv, list, mode);
    return hipGetLastError();
}

// Multiplier (a0, a, b) of the unit-amplitude target E * S(c) (S = Shakhov
// factor, or 1 when kq == nullptr) so that its discrete mass, momentum and
// energy in the frame u equal (rho, 0, 3 rho T / 2).
__device__ int fixup_coefs(const CaseView &C, const double *u, double T, double rho, const double *kq, double *fx)
{
    GMom G;
    double it = 1.0 / T;
    gauss_moments(C, u, it, G);
    if (C.vdim == 3) {
        const int nb = 5;
        // basis monomials: 1, cx, cy, cz, c^2 (three terms)
        const int bm[5][3][3] = {{{0, 0, 0}, {-1, 0, 0}, {-1, 0, 0}},
                                 {{1, 0, 0}, {-1, 0, 0}, {-1, 0, 0}},
                                 {{0, 1, 0}, {-1, 0, 0}, {-1, 0, 0}},
                                 {{0, 0, 1}, {-1, 0, 0}, {-1, 0, 0}},
                                 {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}}};
        double A[25], b[5];
        for (int a = 0; a < nb; ++a)
            for (int c = 0; c < nb; ++c) {
                double s = 0.0;
                for (int ta = 0; ta < 3 && bm[a][ta][0] >= 0; ++ta)
                    for (int tb = 0; tb < 3 && bm[c][tb][0] >= 0; ++tb)
                        s += sh3(G, kq, it, bm[a][ta][0] + bm[c][tb][0], bm[a][ta][1] + bm[c][tb][1],
                                 bm[a][ta][2] + bm[c][tb][2]);
                A[a * nb + c] = s;
            }
        b[0] = rho; b[1] = b[2] = b[3] = 0.0; b[4] = 1.5 * rho * T;
        if (solve_dense(nb, A, b)) return -1;
        for (int a = 0; a < 5; ++a) fx[a] = b[a];
    } else {
        const int nb = 4;
        const int bm[4][2][2] = {{{0, 0}, {-1, 0}}, {{1, 0}, {-1, 0}}, {{0, 1}, {-1, 0}}, {{2, 0}, {0, 2}}};
        double A[16], b[4];
        for (int a = 0; a < nb; ++a)
            for (int c = 0; c < nb; ++c) {
                double s = 0.0;
                for (int ta = 0; ta < 2 && bm[a][ta][0] >= 0; ++ta)
                    for (int tb = 0; tb < 2 && bm[c][tb][0] >= 0; ++tb)
                        s += sh2(G, kq, it, 2.0, bm[a][ta][0] + bm[c][tb][0], bm[a][ta][1] + bm[c][tb][1]);
                if (a == 3)   // energy row adds the psi function, test function 1
                    for (int tb = 0; tb < 2 && bm[c][tb][0] >= 0; ++tb)
                        s += 0.5 * T * sh2(G, kq, it, 1.0, bm[c][tb][0], bm[c][tb][1]);
                A[a * nb + c] = s;
            }
        b[0] = rho; b[1] = b[2] = 0.0; b[3] = 1.5 * rho * T;
        if (solve_dense(nb, A, b)) return -1;
        for (int a = 0; a < 4; ++a) fx[a] = b[a];
        fx[4] = 0.0;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// bind-time: wall-flux denominators sum_{a<0} w |a| M(1, u_w, T_w)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_wall_den(const CaseView *__restrict__ cvp, int nnz)
{
    const CaseView &C = *cvp;
    __shared__ double lds[BLOCK / 64];
    for (int e = blockIdx.x; e < nnz; e += gridDim.x) {
        int oth = C.cf_other[e];
        if (oth >= 0 || C.patch_kind[-1 - oth] != GSIS_PATCH_WALL) continue;   // block-uniform
        const double *ps = C.patch_state + 5 * (-1 - oth);
        const double *n = C.cf_nsv + 3 * e;
        double T = ps[4], it = 1.0 / T;
        double amp = (C.vdim == 3) ? pow(M_PI * T, -1.5) : 1.0 / (M_PI * T);
        double acc = 0.0;
        for (int k = threadIdx.x; k < C.nv; k += BLOCK) {
            double xi[3], w;
            vnode(C, k, xi, w);
            double a = xi[0] * n[0] + xi[1] * n[1] + xi[2] * n[2];
            if (a < 0) {
                double c2 = 0.0;
                for (int d = 0; d < C.vdim; ++d) c2 += (xi[d] - ps[1 + d]) * (xi[d] - ps[1 + d]);
                acc += w * (-a) * amp * exp(-c2 * it);
            }
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) s += lds[w];
            const_cast<double *>(C.wall_den)[e] = s;
        }
        __syncthreads();
    }
}

hipError_t launch_wall_den(const CaseView *cv, const CaseView &h, hipStream_t s)
{
    const int nnz = h.nnz;
    int grid = nnz < 4096 ? (nnz > 0 ? nnz : 1) : 4096;
    hipLaunchKernelGGL(k_wall_den, dim3(grid), dim3(BLOCK), 0, s, cv, nnz);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tile sums -> moments (FP64), kinetic moment balance, wall numerators
// ---------------------------------------------------------------------------
// with_res: 0 the moments, 1 the moments and the kinetic balance Rk, 2 the
// balance alone (a pass whose output rows are discarded: moments, wall sums
// and the state checks stay those of the last real sweep)
__global__ void k_reduce(const CaseView *__restrict__ cvp, int n_kin, int with_res)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_kin) return;
    int cell = C.kin_cell[t];
    int slot = C.slot_of_cell[cell];
    double S[NSUM];
    for (int i = 0; i < NSUM; ++i) S[i] = 0.0;
    const double *P = C.partial + (size_t)slot * C.ntile * NSUM;
    for (int tl = 0; tl < C.ntile; ++tl)
        for (int i = 0; i < NSUM; ++i) S[i] += P[tl * NSUM + i];
    const double *ur = C.param[slot].u;
    if (with_res == 2) {
        double *R = C.Rk + 5 * (size_t)cell;
        const double r0 = S[S_RES];
        const double rc[3] = {S[S_RES + 1], S[S_RES + 2], S[S_RES + 3]};
        R[0] = r0;
        for (int d = 0; d < 3; ++d) R[1 + d] = rc[d] + ur[d] * r0;
        const double u2 = ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2];
        R[4] = S[S_RES + 4] + 2.0 * (ur[0] * rc[0] + ur[1] * rc[1] + ur[2] * rc[2]) + u2 * r0;
        return;
    }
    double *mom = C.mom + (size_t)slot * MOMS;
    double rho = S[0];
    double dl[3] = {S[1] / rho, S[2] / rho, (C.vdim == 3) ? S[3] / rho : 0.0};
    double c2[3][3];
    double q[3] = {0, 0, 0};
    double P0 = 0.0, P1[3] = {0, 0, 0};
    if (C.vdim == 3) {
        double S2[3][3] = {{S[4], S[7], S[8]}, {S[7], S[5], S[9]}, {S[8], S[9], S[6]}};
        double tr = S[4] + S[5] + S[6];
        double d2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) c2[a][b] = S2[a][b] - rho * dl[a] * dl[b];
        for (int d = 0; d < 3; ++d) {
            double s2d = S2[d][0] * dl[0] + S2[d][1] * dl[1] + S2[d][2] * dl[2];
            q[d] = S[10 + d] - dl[d] * tr - 2.0 * s2d + 2.0 * rho * d2 * dl[d];
        }
    } else {
        double S2[3][3] = {{S[3], S[5], 0}, {S[5], S[4], 0}, {0, 0, 0}};
        double tr = S[3] + S[4];
        double d2 = dl[0] * dl[0] + dl[1] * dl[1];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) c2[a][b] = S2[a][b] - rho * dl[a] * dl[b];
        P0 = S[8];
        P1[0] = S[9] - dl[0] * P0;
        P1[1] = S[10] - dl[1] * P0;
        for (int d = 0; d < 2; ++d) {
            double s2d = S2[d][0] * dl[0] + S2[d][1] * dl[1];
            q[d] = S[6 + d] - dl[d] * tr - 2.0 * s2d + 2.0 * rho * d2 * dl[d] + P1[d];
        }
    }
    double e = c2[0][0] + c2[1][1] + c2[2][2] + P0;   // sum w (c^2 phi + psi)
    double p = (2.0 / 3.0) * e;
    mom[0] = rho;
    for (int d = 0; d < 3; ++d) mom[1 + d] = ur[d] + dl[d];
    if (C.vdim == 2) mom[3] = 0.0;
    mom[4] = p / rho;
    mom[5] = 2.0 * c2[0][0] - p;
    mom[6] = 2.0 * c2[1][1] - p;
    mom[7] = (C.vdim == 3) ? 2.0 * c2[2][2] - p : 2.0 * P0 - p;
    mom[8] = 2.0 * c2[0][1];
    mom[9] = 2.0 * c2[0][2];
    mom[10] = 2.0 * c2[1][2];
    for (int d = 0; d < 3; ++d) mom[11 + d] = q[d];
    for (int w = 0; w < MAXW; ++w) mom[GSIS_NMOM + w] = S[S_WALL + w];
    if (C.poly) {
        // second function: T_r = 4 sum w f1 / (d_r rho), q_r = 2 sum w c f1
        double Q[PSUM] = {0, 0, 0, 0, 0};
        const double *ps = C.psum + (size_t)slot * C.ntile * PSUM;
        for (int tl = 0; tl < C.ntile; ++tl)
            for (int i = 0; i < PSUM; ++i) Q[i] += ps[tl * PSUM + i];
        mom[MOM_INT] = 4.0 * Q[0] / (C.dr * rho);
        for (int d = 0; d < 3; ++d) mom[MOM_INT + 1 + d] = 2.0 * (Q[1 + d] - dl[d] * Q[0]);
        if (!(mom[MOM_INT] > 0.0)) atomicOr(C.status, 1);
        // kinetic balance of rho e_r = 2 sum w f1 (flux and exchange)
        if (with_res) C.Rkr[cell] = 2.0 * Q[4];
    }
    int bad = !(rho > 0.0) || !(p > 0.0) || !isfinite(q[0] + q[1] + q[2] + mom[5] + mom[8]);
    if (bad) atomicOr(C.status, 1);
    if (with_res) {
        double *R = C.Rk + 5 * (size_t)cell;
        double r0 = S[S_RES];
        double rc[3] = {S[S_RES + 1], S[S_RES + 2], S[S_RES + 3]};
        double re = S[S_RES + 4];
        R[0] = r0;
        for (int d = 0; d < 3; ++d) R[1 + d] = rc[d] + ur[d] * r0;
        double u2 = ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2];
        R[4] = re + 2.0 * (ur[0] * rc[0] + ur[1] * rc[1] + ur[2] * rc[2]) + u2 * r0;
    }
}

hipError_t launch_reduce(const CaseView *cv, const CaseView &h, int n_kin, int with_res, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3((n_kin + 127) / 128), dim3(128), 0, s, cv, n_kin, with_res);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// relaxation parameters of the next sweep (Sec. 2: tau = mu/p, Shakhov
// target of the d_r = 0 model, conservation fix-up), wall densities
// ---------------------------------------------------------------------------
__global__ void k_param(const CaseView *__restrict__ cvp, int n_kin)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_kin) return;
    int cell = C.kin_cell[t];
    int slot = C.slot_of_cell[cell];
    const double *mom = C.mom + (size_t)slot * MOMS;
    ParamRec P;
    double rho = mom[0], T = mom[4];
    for (int d = 0; d < 3; ++d) P.u[d] = mom[1 + d];
    P.it = 1.0 / T;
    P.Th = 0.5 * T;
    P.itau = rho * pow(T, 1.0 - C.omega) * sqrt(M_PI) / (2.0 * C.Kn);
    double K = 0.8 * (1.0 - C.Pr) / (rho * T * T);
    for (int d = 0; d < 3; ++d) P.kq[d] = K * mom[11 + d];
    if (C.vdim == 2) P.kq[2] = 0.0;
    // point-set grids: k_fix_pts forms the multiplier from direct sums
    if (!C.points && fixup_coefs(C, P.u, T, rho, P.kq, P.fx)) atomicOr(C.status, 1);
    // wall densities from the outgoing half-range mass flux of f^n
    int e0 = C.cf_ptr[cell], e1 = C.cf_ptr[cell + 1];
    for (int w = 0; w < MAXW; ++w) P.rw[w] = 0.0;
    for (int e = e0; e < e1; ++e) {
        int wi = C.cf_wall[e];
        if (wi >= 0) P.rw[wi] = mom[GSIS_NMOM + wi] / C.wall_den[e];
    }
    P.pad[0] = P.pad[1] = P.pad[2] = 0.0;
    C.param[slot] = P;
}

// GSIS_POLY_VEC=0 keeps one node per lane in the two-VDF sweep
static bool poly_vec_on()
{
    static const bool on = [] {
        const char *e = std::getenv("GSIS_POLY_VEC");
        return !(e && e[0] == '0');
    }();
    return on;
}

hipError_t launch_param_poly(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);

hipError_t launch_param(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    if (h.poly) return launch_param_poly(cv, h, n_kin, s);
    hipLaunchKernelGGL(k_param, dim3((n_kin + 63) / 64), dim3(64), 0, s, cv, n_kin);
    return launch_fix_pts(cv, h, n_kin, h.kin_cell, 0, s);
}

// conservation-fixed Maxwellians of W_new (Wn) and W_half (Wh) per kinetic
// slot (mode 0, GSIS correction), or of W (mode 1, initial fill); Th is the
// factor of the second function (T/2 of the reduced pair, d_r T_r/4 of the
// two-VDF gas)
__global__ void k_feqpar(const CaseView *__restrict__ cvp, int n_items, const int32_t *list, int mode)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t < n_items;
    const int cell = live ? list[t] : 0;
    bool cut = false;
    if (mode == 0 && live) {
        // limiter of the correction: halve the conserved-variable change from
        // W_half to W_new (at most ten times, then drop it) until density and
        // temperature stay within a factor 2 of W_half; W_new takes the result
        // (two-VDF gas: the conserved variables include rho e_r = (d_r/2) rho T_r,
        // and T_r is held to the same range)
        double *wn = C.Wn + 5 * (size_t)cell;
        const double *wh = C.Wh + 5 * (size_t)cell;
        const bool poly = C.poly != 0;
        const double trh = poly ? C.Trh[cell] : 0.0, trn = poly ? C.Trn[cell] : 0.0;
        double Uh[6], Ud[6];
        for (int s = 0; s < 2; ++s) {
            const double *w = s ? wn : wh;
            double *U = s ? Ud : Uh;
            const double er = poly ? 0.5 * C.dr * w[0] * (s ? trn : trh) : 0.0;
            U[0] = w[0];
            for (int d = 0; d < 3; ++d) U[1 + d] = w[0] * w[1 + d];
            U[4] = w[0] * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) + 1.5 * w[0] * w[4] + er;
            U[5] = er;
        }
        for (int c = 0; c < 6; ++c) Ud[c] -= Uh[c];
        double th = 1.0, Wl[5], Trl = 0.0;
        bool ok = false;
        int h = 0;
        for (; h <= 10 && !ok; ++h) {
            double U0 = Uh[0] + th * Ud[0];
            double u2 = 0.0;
            Wl[0] = U0;
            for (int d = 0; d < 3; ++d) {
                Wl[1 + d] = (Uh[1 + d] + th * Ud[1 + d]) / U0;
                u2 += Wl[1 + d] * Wl[1 + d];
            }
            const double er = Uh[5] + th * Ud[5];
            Wl[4] = (Uh[4] + th * Ud[4] - U0 * u2 - er) / (1.5 * U0);
            ok = (wh[0] / 2.0 <= Wl[0]) && (Wl[0] <= 2.0 * wh[0]) && (wh[4] / 2.0 <= Wl[4]) && (Wl[4] <= 2.0 * wh[4]);
            if (poly) {
                Trl = er / (0.5 * C.dr * U0);
                ok = ok && (trh / 2.0 <= Trl) && (Trl <= 2.0 * trh);
            }
            th *= 0.5;
        }
        cut = !ok || h > 1;
        for (int c = 0; c < 5; ++c) wn[c] = ok ? Wl[c] : wh[c];
        if (poly) C.Trn[cell] = ok ? Trl : trh;
    }
    if (mode == 0) {
        // limiter counters (one atomic per wave)
        const unsigned long long m = __ballot(cut);
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(&C.lim[5], (unsigned long long)__popcll(m));
        if (t == 0) atomicAdd(&C.lim[4], (unsigned long long)n_items);
    }
    if (!live) return;
    int slot = C.slot_of_cell[cell];
    for (int which = 0; which < (mode == 0 ? 2 : 1); ++which) {
        const double *W = (mode == 0) ? ((which == 0 ? C.Wn : C.Wh) + 5 * (size_t)cell) : (C.W + 5 * (size_t)cell);
        FeqRec F;
        for (int d = 0; d < 3; ++d) F.u[d] = W[1 + d];
        if (C.vdim == 2) F.u[2] = 0.0;
        F.it = 1.0 / W[4];
        F.Th = 0.5 * W[4];
        if (C.poly) {
            // f_eq,1 = (d_r T_r / 4) f_eq,0
            const double *Trs = (mode == 0) ? (which == 0 ? C.Trn : C.Trh) : C.Tr;
            F.Th = 0.25 * C.dr * Trs[cell];
        }
        if (!C.points && fixup_coefs(C, F.u, W[4], W[0], nullptr, F.fx)) atomicOr(C.status, 1);
        C.feq[2 * (size_t)slot + which] = F;
    }
}

hipError_t launch_feqpar(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_feqpar, dim3((n_kin + 63) / 64), dim3(64), 0, s, cv, n_kin, h.kin_cell, 0);
    return launch_fix_pts(cv, h, n_kin, h.kin_cell, 1, s);
}

// ---------------------------------------------------------------------------
// second-order face values (Sec. 3 second-order finite volumes; the scheme is
// left to the paper's references).  Slope of every discrete-velocity value of
// a kinetic cell: least squares over the kinetic neighbours (weights
// 1/|dx|^2, the mesh's `dim` components; zero when the neighbours do not span
// them: det A <= 1e-12 (tr A / dim)^dim), times the Barth-Jespersen factor
// that keeps every face value to a kinetic neighbour inside the range of the
// cell and those neighbours.  What is stored is the reconstruction increment
// delta_l = phi g . (x_face_l - x_cell) of every face l of the cell: a sweep then
// reads one value per face, its own for outgoing values and the neighbour's on
// the shared face for incoming ones.  One block per (kinetic cell, velocity
// tile), blocks remapped so that each XCD walks a contiguous run of cells,
// the stencil's geometry formed once in FP64 by one thread (the inverse
// normal matrix folded into per-neighbour coefficient vectors), then one lane
// per velocity node with the loads of SLOPE_U nodes issued before use.  The
// block also sums, per wall face, sum_{a>0} w a delta of the first function:
// the reconstruction part of the outgoing mass flux that fixes the next wall
// density.
// ---------------------------------------------------------------------------
// a wave-uniform pointer held in SGPRs (the value is the same in every lane)
template <typename P>
__device__ __forceinline__ P wave_uniform(P p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T ratio_lim(T num, T den);
template <>
__device__ __forceinline__ float ratio_lim(float num, float den)
{
    return num * __builtin_amdgcn_rcpf(den);
}
template <>
__device__ __forceinline__ double ratio_lim(double num, double den)
{
    return num / den;
}

#ifndef SLOPE_U
#define SLOPE_U 2
#endif

// LDS of the slope kernels' set-up (thread 0): the least-squares stencil of a
// kinetic cell over its kinetic neighbours (coefficients c_j, face offsets r_j,
// neighbour slots), the offsets of every face (ra_l) and the wall faces (FP64
// normals, offsets, wall index); work arrays of the 3x3 solve
template <typename T>
struct SlopeSh {
    T s_c[MAXF][3], s_r[MAXF][3], s_ra[MAXF][3];
    int s_nb[MAXF];
    double s_wn[MAXW][3];
    T s_wr[MAXW][3];
    int s_ww[MAXW];
    int s_nk, s_nw, s_nf;
    double red[(BLOCK / 64) * MAXW];
    double dx[MAXF][3], iw[MAXF], A[9], I[9];
};

// thread 0: the stencil of `cell` (a neighbour set that does not span dim
// gives no stencil: nk = 0, zero slopes)
template <typename T>
__device__ void slope_setup(const CaseView &C, int cell, int D, SlopeSh<T> &sh)
{
    T(&s_c)[MAXF][3] = sh.s_c;
    T(&s_r)[MAXF][3] = sh.s_r;
    T(&s_ra)[MAXF][3] = sh.s_ra;
    int(&s_nb)[MAXF] = sh.s_nb;
    double(&s_wn)[MAXW][3] = sh.s_wn;
    T(&s_wr)[MAXW][3] = sh.s_wr;
    int(&s_ww)[MAXW] = sh.s_ww;
    double(&dx)[MAXF][3] = sh.dx;
    double(&iw)[MAXF] = sh.iw;
    double(&A)[9] = sh.A;
    double(&I)[9] = sh.I;
    const int e0 = C.cf_ptr[cell], e1 = C.cf_ptr[cell + 1];
    const double *xc = C.cell_center + 3 * (size_t)cell;
    for (int i = 0; i < 9; ++i) A[i] = I[i] = 0.0;
    int nk = 0, nw = 0;
    sh.s_nf = e1 - e0;
    for (int e = e0; e < e1; ++e) {
        const int oth = C.cf_other[e];
        const double *fc = C.face_center + 3 * (size_t)C.cf_face[e];
        for (int d = 0; d < 3; ++d) s_ra[e - e0][d] = (T)(d < D ? fc[d] - xc[d] : 0.0);
        if (C.cf_wall[e] >= 0 && nw < MAXW) {
            s_ww[nw] = C.cf_wall[e];
            for (int d = 0; d < 3; ++d) {
                s_wn[nw][d] = C.cf_nsv[3 * (size_t)e + d];
                s_wr[nw][d] = (T)(d < D ? fc[d] - xc[d] : 0.0);
            }
            ++nw;
        }
        if (oth < 0 || C.slot_of_cell[oth] < 0) continue;
        const double *xo = C.cell_center + 3 * (size_t)oth;
        double r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            dx[nk][d] = (d < D) ? xo[d] - xc[d] : 0.0;
            r2 += dx[nk][d] * dx[nk][d];
        }
        iw[nk] = 1.0 / r2;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) A[a * D + b] += dx[nk][a] * dx[nk][b] * iw[nk];
        s_nb[nk] = C.slot_of_cell[oth];
        for (int d = 0; d < 3; ++d) s_r[nk][d] = (T)(d < D ? fc[d] - xc[d] : 0.0);
        ++nk;
    }
    double tr = 0.0, det;
    for (int d = 0; d < D; ++d) tr += A[d * D + d];
    if (D == 1) {
        det = A[0];
        I[0] = 1.0 / A[0];
    } else if (D == 2) {
        det = A[0] * A[3] - A[1] * A[2];
        I[0] = A[3] / det;
        I[1] = -A[1] / det;
        I[2] = -A[2] / det;
        I[3] = A[0] / det;
    } else {
        const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
        det = A[0] * c00 + A[1] * c01 + A[2] * c02;
        I[0] = c00 / det;
        I[1] = (A[2] * A[7] - A[1] * A[8]) / det;
        I[2] = (A[1] * A[5] - A[2] * A[4]) / det;
        I[3] = c01 / det;
        I[4] = (A[0] * A[8] - A[2] * A[6]) / det;
        I[5] = (A[2] * A[3] - A[0] * A[5]) / det;
        I[6] = c02 / det;
        I[7] = (A[1] * A[6] - A[0] * A[7]) / det;
        I[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    }
    const bool singular = nk == 0 || !(tr > 0.0) || det <= 1e-12 * pow(tr / D, (double)D);
    if (singular) nk = 0;
    for (int j = 0; j < nk; ++j)
        for (int d = 0; d < 3; ++d) {
            double c = 0.0;
            if (d < D)
                for (int b = 0; b < D; ++b) c += I[d * D + b] * dx[j][b] * iw[j];
            s_c[j][d] = (T)c;
        }
    sh.s_nk = nk;
    sh.s_nw = nw;
}

template <typename T, int NK>
__global__ __launch_bounds__(BLOCK) void k_slope(const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    const CaseView &C = *cvp;
    __shared__ SlopeSh<T> sh;
    T(&s_c)[MAXF][3] = sh.s_c;
    T(&s_r)[MAXF][3] = sh.s_r;
    T(&s_ra)[MAXF][3] = sh.s_ra;
    int(&s_nb)[MAXF] = sh.s_nb;
    double(&s_wn)[MAXW][3] = sh.s_wn;
    T(&s_wr)[MAXW][3] = sh.s_wr;
    int(&s_ww)[MAXW] = sh.s_ww;
    double *red = sh.red;
    // XCD-contiguous runs of cells: neighbour rows meet in the XCD's L2
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin;
    const int t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const int D = C.dim;
    if (threadIdx.x == 0) slope_setup<T>(C, cell, D, sh);
    __syncthreads();
    const int nk = sh.s_nk, nw = sh.s_nw, nfa = sh.s_nf;
    const T *fo = (const T *)C.f[cur];
    const size_t row = (size_t)C.row;
    const int nvp = C.row / C.nfun;
    const T *fi_row = wave_uniform(fo + (size_t)slot * row);
    // increments of the cell's faces: delta_l at (slot nfmax + l) row
    T *so[NK];
    T a0[NK], a1[NK], a2[NK];
#pragma unroll
    for (int l = 0; l < NK; ++l) {
        const bool on = l < nfa;
        so[l] = wave_uniform((T *)C.slope + ((size_t)slot * C.nfmax + (on ? l : 0)) * row);
        a0[l] = on ? s_ra[l][0] : (T)0;
        a1[l] = on ? s_ra[l][1] : (T)0;
        a2[l] = on ? s_ra[l][2] : (T)0;
    }
    // the stencil in registers: absent neighbours read the cell's own row
    // with zero coefficients and offsets (they change nothing)
    const T *nbr[NK];
    T c0[NK], c1[NK], c2[NK], r0[NK], r1[NK], r2[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const bool on = j < nk;
        nbr[j] = wave_uniform(on ? fo + (size_t)s_nb[j] * row : fi_row);
        c0[j] = on ? s_c[j][0] : (T)0;
        c1[j] = on ? s_c[j][1] : (T)0;
        c2[j] = on ? s_c[j][2] : (T)0;
        r0[j] = on ? s_r[j][0] : (T)0;
        r1[j] = on ? s_r[j][1] : (T)0;
        r2[j] = on ? s_r[j][2] : (T)0;
    }
    const int k0 = vt * C.tile;
    const int kend = min(k0 + C.tile, C.nv);
    double wacc[MAXW];
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wacc[j] = 0.0;
    // SLOPE_U nodes per lane per pass: all their loads are issued before any
    // is used (the kernel is bound by load latency, not by bandwidth)
    for (int kb = k0 + threadIdx.x; kb < kend; kb += SLOPE_U * BLOCK) {
        T w0[SLOPE_U], w1[SLOPE_U], w2[SLOPE_U];   // slopes of the first function
        for (int q = 0; q < C.nfun; ++q) {
            T v[SLOPE_U][NK], fi[SLOPE_U];
#pragma unroll
            for (int u = 0; u < SLOPE_U; ++u) {
                const int k = kb + u * BLOCK;
                const size_t kk = (size_t)q * nvp + (k < kend ? k : kb);   // in-range address for idle nodes
#pragma unroll
                for (int j = 0; j < NK; ++j) v[u][j] = nbr[j][kk];
                fi[u] = fi_row[kk];
            }
#pragma unroll
            for (int u = 0; u < SLOPE_U; ++u) {
                const int k = kb + u * BLOCK;
                T g0 = (T)0, g1 = (T)0, g2 = (T)0, dmax = (T)0, dmin = (T)0;
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    const T d = v[u][j] - fi[u];
                    g0 += c0[j] * d;
                    g1 += c1[j] * d;
                    g2 += c2[j] * d;
                    dmax = fmax(dmax, d);
                    dmin = fmin(dmin, d);
                }
                // Barth-Jespersen: phi = min over faces of min(1, bound / ext)
                T phi = (T)1;
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    const T ext = g0 * r0[j] + g1 * r1[j] + g2 * r2[j];
                    if (ext > dmax) phi = fmin(phi, ratio_lim(dmax, ext));
                    else if (ext < dmin) phi = fmin(phi, ratio_lim(dmin, ext));
                }
                g0 *= phi;
                g1 *= phi;
                g2 *= phi;
                if (k < kend) {
                    const size_t kk = (size_t)q * nvp + k;
#pragma unroll
                    for (int l = 0; l < NK; ++l)
                        if (l < nfa) __builtin_nontemporal_store(g0 * a0[l] + g1 * a1[l] + g2 * a2[l], &so[l][kk]);
                }
                if (q == 0) {
                    w0[u] = g0;
                    w1[u] = g1;
                    w2[u] = g2;
                }
            }
        }
        if (nw > 0) {
#pragma unroll
            for (int u = 0; u < SLOPE_U; ++u) {
                const int k = kb + u * BLOCK;
                if (k >= kend) break;
                double xi[3], wd;
                vnode(C, k, xi, wd);
#pragma unroll
                for (int j = 0; j < MAXW; ++j)
                    if (j < nw) {
                        const double a = xi[0] * s_wn[j][0] + xi[1] * s_wn[j][1] + xi[2] * s_wn[j][2];
                        if (a > 0.0)
                            wacc[j] += wd * a * (double)(w0[u] * s_wr[j][0] + w1[u] * s_wr[j][1] + w2[u] * s_wr[j][2]);
                    }
            }
        }
    }
    // per wall index (static selects keep the sums in registers)
    double wsum[MAXW];
#pragma unroll
    for (int w = 0; w < MAXW; ++w) {
        wsum[w] = 0.0;
#pragma unroll
        for (int j = 0; j < MAXW; ++j) wsum[w] += (j < nw && s_ww[j] == w) ? wacc[j] : 0.0;
    }
    block_reduce_store<MAXW>(wsum, C.wsl + ((size_t)slot * C.ntile + vt) * MAXW, red);
}

// The slope kernel on 3D tensor grids in the 16-byte-row plane layout: a lane
// keeps one y node and four consecutive z nodes and loops over the tile's
// x-planes, reading its own row and the kinetic neighbours' rows as 16-byte
// vectors and writing each face's increments the same way.  The per-node
// arithmetic is that of k_slope; tiles must cover whole x-planes.
#ifndef SLOPE_V4_U
#define SLOPE_V4_U 2
#endif
template <typename T, int NK>
__global__ __launch_bounds__(BLOCK) void k_slope_v4(const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    typedef T V4 __attribute__((ext_vector_type(4)));
    const CaseView &C = *cvp;
    __shared__ SlopeSh<T> sh;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin;
    const int t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    if (threadIdx.x == 0) slope_setup<T>(C, cell, C.dim, sh);
    __syncthreads();
    const int nk = sh.s_nk, nw = sh.s_nw, nfa = sh.s_nf;
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    const size_t row = (size_t)C.row;
    const T *fo = (const T *)C.f[cur];
    const T *fi_row = wave_uniform(fo + (size_t)slot * row);
    T *so[NK];
    T a0[NK], a1[NK], a2[NK];
#pragma unroll
    for (int l = 0; l < NK; ++l) {
        const bool on = l < nfa;
        so[l] = wave_uniform((T *)C.slope + ((size_t)slot * C.nfmax + (on ? l : 0)) * row);
        a0[l] = on ? sh.s_ra[l][0] : (T)0;
        a1[l] = on ? sh.s_ra[l][1] : (T)0;
        a2[l] = on ? sh.s_ra[l][2] : (T)0;
    }
    const T *nbr[NK];
    T c0[NK], c1[NK], c2[NK], r0[NK], r1[NK], r2[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
        const bool on = j < nk;
        nbr[j] = wave_uniform(on ? fo + (size_t)sh.s_nb[j] * row : fi_row);
        c0[j] = on ? sh.s_c[j][0] : (T)0;
        c1[j] = on ? sh.s_c[j][1] : (T)0;
        c2[j] = on ? sh.s_c[j][2] : (T)0;
        r0[j] = on ? sh.s_r[j][0] : (T)0;
        r1[j] = on ? sh.s_r[j][1] : (T)0;
        r2[j] = on ? sh.s_r[j][2] : (T)0;
    }
    // lane -> (x group, y, first of four z nodes)
    const int Q = nz >> 2, PL = ny * Q, G = BLOCK / PL;
    const int xg = threadIdx.x / PL, pr = threadIdx.x - xg * PL;
    const int iy = pr / Q, iz0 = 4 * (pr - iy * Q);
    const int P2 = ny * nz;
    const int ix0 = (vt * C.tile) / P2, ix1 = min(nx, ((vt + 1) * C.tile) / P2);
    double wacc[MAXW];
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wacc[j] = 0.0;
    for (int ixr = ix0 + xg; ixr < ix1; ixr += SLOPE_V4_U * G) {
        V4 v[SLOPE_V4_U][NK], fi[SLOPE_V4_U];
#pragma unroll
        for (int u = 0; u < SLOPE_V4_U; ++u) {
            const size_t k = (size_t)min(ixr + u * G, ix1 - 1) * P2 + 4 * pr;   // in-range address for idle planes
#pragma unroll
            for (int j = 0; j < NK; ++j) v[u][j] = *(const V4 *)(nbr[j] + k);
            fi[u] = *(const V4 *)(fi_row + k);
        }
#pragma unroll
        for (int u = 0; u < SLOPE_V4_U; ++u) {
            const int ix = ixr + u * G;
            if (ix >= ix1) break;
            const size_t k = (size_t)ix * P2 + 4 * pr;
            V4 out[NK];
            T w0[4], w1[4], w2[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                T g0 = (T)0, g1 = (T)0, g2 = (T)0, dmax = (T)0, dmin = (T)0;
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    const T d = v[u][j][q] - fi[u][q];
                    g0 += c0[j] * d;
                    g1 += c1[j] * d;
                    g2 += c2[j] * d;
                    dmax = fmax(dmax, d);
                    dmin = fmin(dmin, d);
                }
                // Barth-Jespersen: phi = min over faces of min(1, bound / ext)
                T phi = (T)1;
#pragma unroll
                for (int j = 0; j < NK; ++j) {
                    const T ext = g0 * r0[j] + g1 * r1[j] + g2 * r2[j];
                    if (ext > dmax) phi = fmin(phi, ratio_lim(dmax, ext));
                    else if (ext < dmin) phi = fmin(phi, ratio_lim(dmin, ext));
                }
                g0 *= phi;
                g1 *= phi;
                g2 *= phi;
#pragma unroll
                for (int l = 0; l < NK; ++l) out[l][q] = g0 * a0[l] + g1 * a1[l] + g2 * a2[l];
                w0[q] = g0;
                w1[q] = g1;
                w2[q] = g2;
            }
#pragma unroll
            for (int l = 0; l < NK; ++l)
                if (l < nfa) __builtin_nontemporal_store(out[l], (V4 *)(so[l] + k));
            if (nw > 0) {
                // the slope part of the outgoing wall fluxes (FP64, rare cells)
                const double xx = C.xv[ix], yy = C.xv[MAXA + iy];
                const double wxy = C.wv[ix] * C.wv[MAXA + iy];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double zz = C.xv[2 * MAXA + iz0 + q];
                    const double wd = wxy * C.wv[2 * MAXA + iz0 + q];
#pragma unroll
                    for (int j = 0; j < MAXW; ++j)
                        if (j < nw) {
                            const double a = xx * sh.s_wn[j][0] + yy * sh.s_wn[j][1] + zz * sh.s_wn[j][2];
                            if (a > 0.0)
                                wacc[j] += wd * a *
                                           (double)(w0[q] * sh.s_wr[j][0] + w1[q] * sh.s_wr[j][1] +
                                                    w2[q] * sh.s_wr[j][2]);
                        }
                }
            }
        }
    }
    double wsum[MAXW];
#pragma unroll
    for (int w = 0; w < MAXW; ++w) {
        wsum[w] = 0.0;
#pragma unroll
        for (int j = 0; j < MAXW; ++j) wsum[w] += (j < nw && sh.s_ww[j] == w) ? wacc[j] : 0.0;
    }
    block_reduce_store<MAXW>(wsum, C.wsl + ((size_t)slot * C.ntile + vt) * MAXW, sh.red);
}

hipError_t launch_slope(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    const int blocks = n_kin * h.ntile;
    const bool f4 = h.nfmax <= 4;
    // 16-byte rows on 3D tensor grids whose (y, z) plane splits into 64-256
    // lanes of four z nodes and whose tiles cover whole planes (GSIS_SLOPE_V4=0
    // keeps the node-per-thread kernel)
    static const bool v4_on = [] {
        const char *e = std::getenv("GSIS_SLOPE_V4");
        return !(e && e[0] == '0');
    }();
    const int P2 = h.n[1] * h.n[2];
    if (v4_on && h.vdim == 3 && !h.points && h.nfun == 1 && h.n[2] % 4 == 0 && P2 / 4 >= 64 && P2 / 4 <= BLOCK &&
        BLOCK % (P2 / 4) == 0 && h.tile % P2 == 0) {
        if (h.dtype == GSIS_F32) {
            if (f4) hipLaunchKernelGGL((k_slope_v4<float, 4>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
            else hipLaunchKernelGGL((k_slope_v4<float, MAXF>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
        } else {
            if (f4) hipLaunchKernelGGL((k_slope_v4<double, 4>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
            else hipLaunchKernelGGL((k_slope_v4<double, MAXF>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
        }
        return hipGetLastError();
    }
    if (h.dtype == GSIS_F32) {
        if (f4) hipLaunchKernelGGL((k_slope<float, 4>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_slope<float, MAXF>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
    } else {
        if (f4) hipLaunchKernelGGL((k_slope<double, 4>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_slope<double, MAXF>), dim3(blocks), dim3(BLOCK), 0, s, cv, n_kin, cur);
    }
    return hipGetLastError();
}

// each cell's largest outflow rate over the velocity grid,
// amax = max_k sum_{a_k > 0} a_k (a = xi.n S/V): the pseudo-time scale of the
// second-order iteration (one block per cell, FP64)
__global__ __launch_bounds__(BLOCK) void k_amax(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    __shared__ double nsv[MAXF][3];
    __shared__ double red[BLOCK / 64];
    const int cell = blockIdx.x;
    const int e0 = C.cf_ptr[cell], nf = C.cf_ptr[cell + 1] - e0;
    if (threadIdx.x < nf)
        for (int d = 0; d < 3; ++d) nsv[threadIdx.x][d] = C.cf_nsv[3 * (size_t)(e0 + threadIdx.x) + d];
    __syncthreads();
    double mx = 0.0;
    for (int k = threadIdx.x; k < C.nv; k += BLOCK) {
        double xi[3], wd;
        vnode(C, k, xi, wd);
        double out = 0.0;
        for (int l = 0; l < nf; ++l) {
            const double a = xi[0] * nsv[l][0] + xi[1] * nsv[l][1] + xi[2] * nsv[l][2];
            if (a > 0.0) out += a;
        }
        mx = fmax(mx, out);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < BLOCK / 64; ++w) m = fmax(m, red[w]);
        C.amax[cell] = m;
    }
}

hipError_t launch_amax(const CaseView *cv, const CaseView &h, hipStream_t s)
{
    if (h.n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_amax, dim3(h.n_cells), dim3(BLOCK), 0, s, cv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// shared epilogue: moment sums of the produced f relative to u_ref
// ---------------------------------------------------------------------------
template <typename A, int VD>
__device__ __forceinline__ void acc_moments(A (&s)[NSUM], A w, A f0, A f1, A c0, A c1, A c2, A cc)
{
    A h = w * f0;
    A hc0 = h * c0, hc1 = h * c1;
    s[0] += h;
    s[1] += hc0;
    s[2] += hc1;
    if (VD == 3) {
        A hc2 = h * c2;
        s[3] += hc2;
        s[4] += hc0 * c0;
        s[5] += hc1 * c1;
        s[6] += hc2 * c2;
        s[7] += hc0 * c1;
        s[8] += hc0 * c2;
        s[9] += hc1 * c2;
        A hcc = h * cc;
        s[10] += hcc * c0;
        s[11] += hcc * c1;
        s[12] += hcc * c2;
    } else {
        s[3] += hc0 * c0;
        s[4] += hc1 * c1;
        s[5] += hc0 * c1;
        A hcc = h * cc;
        s[6] += hcc * c0;
        s[7] += hcc * c1;
        A hp = w * f1;
        s[8] += hp;
        s[9] += hp * c0;
        s[10] += hp * c1;
    }
}

// ---------------------------------------------------------------------------
// the kinetic sweep (Sec. 3.1): one block per (kinetic cell, velocity tile)
// ---------------------------------------------------------------------------
template <typename T>
struct FaceS {
    const T *nb;      // upwind row of a kinetic neighbour
    const T *od;      // order 2: the cell's reconstruction increments on this face
    const T *nd;      // order 2: the kinetic neighbour's increments on this face (or null)
    T n[3];           // outward n S / V
    T A, Th, it;      // Gaussian source: amplitude, psi factor, 1/T
    T u[3];
    T s[6], q[3];     // Grad-13 coefficients (ghost)
    int kind, wall, tab;
};

template <typename T, int VD, bool PTS, bool O2>
__global__ __launch_bounds__(BLOCK) void k_sweep(Batch B)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ FaceS<T> fs[MAXF];
    __shared__ double red[(BLOCK / 64) * NSUM];
    __shared__ int s_nf, s_nw, s_wl[MAXW];

    const int nb = gridDim.x;
    const int b = xcd_remap(blockIdx.x, nb);
    int ci = 0;
    while (ci + 1 < B.n && b >= B.start[ci + 1]) ++ci;
    const CaseView &C = *B.cv[ci];
    const int cur = B.cur[ci];
    const int item = b - B.start[ci];
    const int n_kin = (B.start[ci + 1] - B.start[ci]) / C.ntile;
    const int vt = item / n_kin;
    const int t = item - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const T *__restrict__ fold = (const T *)C.f[cur];
    T *__restrict__ fnew = (T *)C.f[cur ^ 1];
    const int n0 = C.n[0], n1 = C.n[1], n2 = (VD == 3) ? C.n[2] : 0;
    const int NA3 = n0 + n1 + n2;
    // FP64 offsets and weights for the moment sums (the sums are accumulated
    // in FP64 from the stored values: this kernel serves any grid shape, so
    // there is no plane structure to compensate the FP32 products with)
    double *csd = (double *)smem_raw;
    double *wsd = csd + NA3;
    T *xs = (T *)(wsd + NA3);
    T *ws = xs + NA3;
    T *cs = ws + NA3;      // c_d = x_j - u_d of the own target, formed in FP64 and rounded once
    T *tabs = cs + NA3;
    const ParamRec &P = C.param[slot];
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;

    if (threadIdx.x == 0) {
        s_nf = nf;
        int nw = 0;
        for (int l = 0; l < nf; ++l)
            if (C.cf_wall[e0 + l] >= 0) s_wl[nw++] = l;
        s_nw = nw;
    }
    if (threadIdx.x < nf) {
        const int l = threadIdx.x;
        FaceS<T> F;
        const int e = e0 + l;
        const int oth = C.cf_other[e];
        for (int d = 0; d < 3; ++d) F.n[d] = (T)C.cf_nsv[3 * e + d];
        F.wall = C.cf_wall[e];
        F.tab = 1 + l;
        F.nb = nullptr;
        F.od = O2 ? (const T *)C.slope + ((size_t)slot * C.nfmax + l) * C.row : nullptr;
        F.nd = nullptr;
        F.A = F.Th = F.it = (T)0;
        for (int d = 0; d < 3; ++d) F.u[d] = (T)0, F.q[d] = (T)0;
        for (int d = 0; d < 6; ++d) F.s[d] = (T)0;
        if (oth >= 0) {
            const int so = C.slot_of_cell[oth];
            if (so >= 0) {
                F.kind = K_KIN;
                F.nb = fold + (size_t)so * C.row;
                if (O2) F.nd = (const T *)C.slope + ((size_t)so * C.nfmax + C.cf_back[e]) * C.row;
            } else {
                // Grad-13 ghost of the NS neighbour (Sec. 3.2)
                F.kind = K_GHOST;
                const double *g = C.ghost + (size_t)oth * GSIS_NMOM;
                double rho = g[0], Tg = g[4], p = rho * Tg;
                F.A = (T)((VD == 3) ? rho * pow(M_PI * Tg, -1.5) : rho / (M_PI * Tg));
                for (int d = 0; d < 3; ++d) F.u[d] = (T)g[1 + d];
                F.it = (T)(1.0 / Tg);
                F.Th = (T)(0.5 * Tg);
                for (int d = 0; d < 6; ++d) F.s[d] = (T)(g[5 + d] / (p * Tg));
                for (int d = 0; d < 3; ++d) F.q[d] = (T)(2.0 * g[11 + d] / (p * Tg));
            }
        } else {
            const int pi = -1 - oth;
            const double *ps = C.patch_state + 5 * pi;
            double Tp = ps[4];
            double amp = (VD == 3) ? pow(M_PI * Tp, -1.5) : 1.0 / (M_PI * Tp);
            if (C.patch_kind[pi] == GSIS_PATCH_WALL) {
                F.kind = K_WALL;
                double rw = P.rw[F.wall];
                if (O2) {
                    // slope part of the outgoing mass flux of f^n (from the slope kernel)
                    double ws = 0.0;
                    for (int tl = 0; tl < C.ntile; ++tl) ws += C.wsl[((size_t)slot * C.ntile + tl) * MAXW + F.wall];
                    rw += ws / C.wall_den[e];
                }
                amp *= rw;
            } else {
                F.kind = K_FAR;
                amp *= ps[0];
            }
            F.A = (T)amp;
            for (int d = 0; d < 3; ++d) F.u[d] = (T)ps[1 + d];
            F.it = (T)(1.0 / Tp);
            F.Th = (T)(0.5 * Tp);
        }
        fs[l] = F;
    }
    // node / weight tables (tensor grids; a point set reads its nodes per point)
    for (int j = threadIdx.x; j < (PTS ? 0 : NA3); j += BLOCK) {
        int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        xs[j] = (T)C.xv[d * MAXA + jj];
        ws[j] = (T)C.wv[d * MAXA + jj];
        cs[j] = (T)(C.xv[d * MAXA + jj] - P.u[d]);
        csd[j] = C.xv[d * MAXA + jj] - P.u[d];
        wsd[j] = C.wv[d * MAXA + jj];
    }
    __syncthreads();
    // separable Gaussian factors exp(-(x_j - u_d)^2 / T), evaluated in FP64:
    // table 0 = own target, 1 + l = face l
    for (int idx = threadIdx.x; idx < (PTS ? 0 : (1 + nf) * NA3); idx += BLOCK) {
        int src = idx / NA3, j = idx - src * NA3;
        int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        double c, it;
        if (src == 0) {
            c = C.xv[d * MAXA + jj] - P.u[d];
            it = P.it;
        } else {
            const FaceS<T> &F = fs[src - 1];
            if (F.kind == K_KIN) continue;
            c = C.xv[d * MAXA + jj] - (double)F.u[d];
            it = (double)F.it;
        }
        tabs[src * NA3 + j] = (T)exp(-c * c * it);
    }
    __syncthreads();

    // own target coefficients
    const T it = (T)P.it, Th = (T)P.Th, itau = (T)P.itau;
    const T kq0 = (T)P.kq[0], kq1 = (T)P.kq[1], kq2 = (T)P.kq[2];
    const T fx0 = (T)P.fx[0], fx1 = (T)P.fx[1], fx2 = (T)P.fx[2], fx3 = (T)P.fx[3], fx4 = (T)P.fx[4];
    // order 2: the pseudo-time term damp * amax joins the diagonal
    const T inv_dt = (T)(C.inv_dt + (O2 ? C.damp2 * C.amax[cell] : 0.0));
    const int nw = s_nw;
    const T *fo = fold + (size_t)slot * C.row;
    T *fn = fnew + (size_t)slot * C.row;
    const int nvp = C.row / ((VD == 3) ? 1 : 2);   // padded length of one function

    double acc[NSUM], wj[MAXW];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = 0.0;
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wj[j] = 0.0;

    const int k0 = vt * C.tile;
    const int kend = min(k0 + C.tile, C.nv);
    int k = k0 + threadIdx.x;
    VIdx vi = vidx_init<VD>(PTS ? 0 : k, n1, (VD == 3) ? n2 : 1);
    const T *tx = tabs, *ty = tabs + n0, *tz = tabs + n0 + n1;
    for (; k < kend; k += BLOCK) {
        T x0, x1, x2, w, c0, c1, c2, E;
        double wd, d0, d1, d2;
        if constexpr (PTS) {
            // point set: the node and its Gaussian factor (one exp per node)
            const double *q = C.vpt + 4 * (size_t)k;
            d0 = q[0] - P.u[0];
            d1 = q[1] - P.u[1];
            d2 = q[2] - P.u[2];
            wd = q[3];
            x0 = (T)q[0];
            x1 = (T)q[1];
            x2 = (T)q[2];
            w = (T)wd;
            c0 = (T)d0;
            c1 = (T)d1;
            c2 = (T)d2;
        } else {
            x0 = xs[vi.ix];
            x1 = xs[n0 + vi.iy];
            x2 = (VD == 3) ? xs[n0 + n1 + vi.iz] : (T)0;
            w = ws[vi.ix] * ws[n0 + vi.iy] * ((VD == 3) ? ws[n0 + n1 + vi.iz] : (T)1);
            c0 = cs[vi.ix];
            c1 = cs[n0 + vi.iy];
            c2 = (VD == 3) ? cs[n0 + n1 + vi.iz] : (T)0;
            wd = wsd[vi.ix] * wsd[n0 + vi.iy] * ((VD == 3) ? wsd[n0 + n1 + vi.iz] : 1.0);
            d0 = csd[vi.ix];
            d1 = csd[n0 + vi.iy];
            d2 = (VD == 3) ? csd[n0 + n1 + vi.iz] : 0.0;
        }
        const T cc = c0 * c0 + c1 * c1 + c2 * c2;
        if constexpr (PTS) E = exp(-cc * it);
        else E = tx[vi.ix] * ty[vi.iy] * ((VD == 3) ? tz[vi.iz] : (T)1);
        const T kqc = kq0 * c0 + kq1 * c1 + kq2 * c2;
        T Pf, g0, g1 = (T)0;
        if (VD == 3) {
            Pf = fx0 + fx1 * c0 + fx2 * c1 + fx3 * c2 + fx4 * cc;
            g0 = E * Pf * ((T)1 + kqc * (cc * it - (T)2.5));
        } else {
            Pf = fx0 + fx1 * c0 + fx2 * c1 + fx3 * cc;
            const T EP = E * Pf;
            g0 = EP * ((T)1 + kqc * (cc * it - (T)2));
            g1 = Th * EP * ((T)1 + kqc * (cc * it - (T)1));
        }
        const T o0 = fo[k];
        const T o1 = (VD == 2) ? fo[nvp + k] : (T)0;
        T den = inv_dt + itau;
        T num0 = itau * g0 + inv_dt * o0;
        T num1 = (VD == 2) ? itau * g1 + inv_dt * o1 : (T)0;
        for (int l = 0; l < s_nf; ++l) {
            const FaceS<T> &F = fs[l];
            const T a = x0 * F.n[0] + x1 * F.n[1] + x2 * F.n[2];
            if (a > (T)0) {
                den += a;
                if constexpr (O2) {
                    // deferred correction of the outgoing value: f_i + delta_i
                    num0 -= a * F.od[k];
                    if (VD == 2) num1 -= a * F.od[nvp + k];
                }
            } else if (a < (T)0) {
                T v0, v1 = (T)0;
                if (F.kind == K_KIN) {
                    v0 = F.nb[k];
                    if (VD == 2) v1 = F.nb[nvp + k];
                    if constexpr (O2) {
                        // reconstructed incoming value f_j + delta_j on this face
                        v0 += F.nd[k];
                        if (VD == 2) v1 += F.nd[nvp + k];
                    }
                } else {
                    T Es;
                    if constexpr (PTS) {
                        const T e0 = x0 - F.u[0], e1 = x1 - F.u[1], e2 = x2 - F.u[2];
                        Es = F.A * exp(-(e0 * e0 + e1 * e1 + e2 * e2) * F.it);
                    } else {
                        const T *tb = tabs + F.tab * NA3;
                        Es = F.A * tb[vi.ix] * tb[n0 + vi.iy] * ((VD == 3) ? tb[n0 + n1 + vi.iz] : (T)1);
                    }
                    if (F.kind == K_GHOST) {
                        const T d0 = x0 - F.u[0], d1 = x1 - F.u[1], d2 = (VD == 3) ? x2 - F.u[2] : (T)0;
                        const T dd = d0 * d0 + d1 * d1 + d2 * d2;
                        const T Q2 = F.s[0] * d0 * d0 + F.s[1] * d1 * d1 + F.s[2] * d2 * d2 +
                                     (T)2 * (F.s[3] * d0 * d1 + F.s[4] * d0 * d2 + F.s[5] * d1 * d2);
                        const T qd = F.q[0] * d0 + F.q[1] * d1 + F.q[2] * d2;
                        if (VD == 3) {
                            v0 = Es * ((T)1 + Q2 + qd * ((T)0.4 * dd * F.it - (T)1));
                        } else {
                            const T Tg = (T)2 * F.Th;
                            v0 = Es * ((T)1 + Q2 + F.Th * F.s[2] + qd * ((T)0.4 * dd * F.it - (T)0.8));
                            v1 = F.Th * Es * ((T)1 + Q2 + (T)1.5 * Tg * F.s[2] + qd * ((T)0.4 * dd * F.it - (T)0.4));
                        }
                    } else {
                        v0 = Es;
                        if (VD == 2) v1 = F.Th * Es;
                    }
                }
                num0 -= a * v0;
                if (VD == 2) num1 -= a * v1;
            }
        }
        const T rden = (T)1 / den;
        const T n0v = num0 * rden;
        fn[k] = n0v;
        T n1v = (T)0;
        if (VD == 2) {
            n1v = num1 * rden;
            fn[nvp + k] = n1v;
        }
        const double dcc = d0 * d0 + d1 * d1 + d2 * d2;
        acc_moments<double, VD>(acc, wd, (double)n0v, (double)n1v, d0, d1, d2, dcc);
        // moment balance at the old iterate: w (num - den f_old) (1, c, c^2 [+psi])
        const double r0 = wd * (double)(num0 - den * o0);
        acc[S_RES] += r0;
        acc[S_RES + 1] += r0 * d0;
        acc[S_RES + 2] += r0 * d1;
        if (VD == 3) acc[S_RES + 3] += r0 * d2;
        double re = r0 * dcc;
        if (VD == 2) re += wd * (double)(num1 - den * o1);
        acc[S_RES + 4] += re;
        // outgoing mass flux through wall faces (numerator of the next rho_w),
        // per wall face in registers (a runtime index would put acc in scratch)
#pragma unroll
        for (int j = 0; j < MAXW; ++j)
            if (j < nw) {
                const FaceS<T> &F = fs[s_wl[j]];
                const T a = x0 * F.n[0] + x1 * F.n[1] + x2 * F.n[2];
                if (a > (T)0) wj[j] += wd * (double)(a * n0v);
            }
        if constexpr (!PTS) vidx_step<VD>(vi, n1, (VD == 3) ? n2 : 1);
    }
#pragma unroll
    for (int j = 0; j < MAXW; ++j)
#pragma unroll
        for (int w = 0; w < MAXW; ++w) acc[S_WALL + w] += (j < nw && fs[s_wl[j]].wall == w) ? wj[j] : 0.0;
    block_reduce_store<NSUM>(acc, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
}

// ---------------------------------------------------------------------------
// the kinetic sweep on point-set grids, faces as rows: every face reads one
// row -- a kinetic neighbour's VDF, the Grad-13 ghost row of an NS neighbour
// (built once per sweep) or the patch row of a wall (times rho_w) or the far
// field -- so the per-node work is the own target (one exp), NF loads and the
// upwind sums.  Faces are wave-uniform (row bases in SGPRs); the NF loads of a
// node are issued before they are used; the moment sums are FP64 per thread
// and block-reduced in a fixed order into the per-(slot, tile) partials.
// ---------------------------------------------------------------------------

template <typename T, int NF, bool O2>
__global__ __launch_bounds__(BLOCK) void k_sweep_prow(Batch B)
{
    __shared__ double red[(BLOCK / 64) * NSUM];
    const int nb = gridDim.x;
    const int b = xcd_remap(blockIdx.x, nb);
    int ci = 0;
    while (ci + 1 < B.n && b >= B.start[ci + 1]) ++ci;
    const CaseView &C = *B.cv[ci];
    const int cur = B.cur[ci];
    const int item = b - B.start[ci];
    const int n_kin = (B.start[ci + 1] - B.start[ci]) / C.ntile;
    const int vt = item / n_kin;
    const int t = item - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const size_t row = (size_t)C.row;
    const T *fold = (const T *)C.f[cur];
    const T *fo = wave_uniform(fold + (size_t)slot * row);
    T *fn = wave_uniform((T *)C.f[cur ^ 1] + (size_t)slot * row);
    // faces: row base, scale (rho_w on walls), n S / V, wall-sum index
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    const T *fnb[NF];
    T fsc[NF], fnx[NF], fny[NF], fnz[NF];
    int fwall[NF];
    // order 2: the cell's reconstruction increments per face (dio) and each
    // kinetic neighbour's increments on the shared face (dnb, weighted by qk =
    // 1; other faces read the cell's first row with weight 0)
    const T *dl0 = O2 ? (const T *)C.slope : nullptr;
    const T *dio[NF];
    const T *dnb[NF];
    T qk[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fnb[l] = fo;
        dio[l] = O2 ? dl0 + ((size_t)slot * C.nfmax + (l < nf ? l : 0)) * row : nullptr;
        dnb[l] = dio[l];
        qk[l] = (T)0;
        fsc[l] = fnx[l] = fny[l] = fnz[l] = (T)0;
        fwall[l] = -1;
        if (l < nf) {
            const int e = e0 + l;
            const int oth = C.cf_other[e];
            fnx[l] = (T)C.cf_nsv[3 * e];
            fny[l] = (T)C.cf_nsv[3 * e + 1];
            fnz[l] = (T)C.cf_nsv[3 * e + 2];
            fsc[l] = (T)1;
            if (oth >= 0) {
                const int so = C.slot_of_cell[oth];
                fnb[l] = (so >= 0) ? fold + (size_t)so * row : (const T *)C.grow + (size_t)C.ghost_slot[oth] * row;
                if (O2 && so >= 0) {
                    dnb[l] = dl0 + ((size_t)so * C.nfmax + C.cf_back[e]) * row;
                    qk[l] = (T)1;
                }
            } else {
                fnb[l] = (const T *)C.prow + (size_t)(-1 - oth) * row;
                fwall[l] = C.cf_wall[e];
                if (fwall[l] >= 0) {
                    double rw = P.rw[fwall[l]];
                    if (O2) {
                        // slope part of the outgoing mass flux of f^n (slope kernel)
                        double ws = 0.0;
                        for (int tl = 0; tl < C.ntile; ++tl)
                            ws += C.wsl[((size_t)slot * C.ntile + tl) * MAXW + fwall[l]];
                        rw += ws / C.wall_den[e];
                    }
                    fsc[l] = (T)rw;
                }
            }
        }
        fnb[l] = wave_uniform(fnb[l]);
        if (O2) {
            dio[l] = wave_uniform(dio[l]);
            dnb[l] = wave_uniform(dnb[l]);
        }
    }
    const double u0 = P.u[0], u1 = P.u[1], u2 = P.u[2];
    // order 2: the pseudo-time term damp * amax joins the diagonal
    const T it = (T)P.it, itau = (T)P.itau, idt = (T)(C.inv_dt + (O2 ? C.damp2 * C.amax[cell] : 0.0));
    const T kq0 = (T)P.kq[0], kq1 = (T)P.kq[1], kq2 = (T)P.kq[2];
    const T fx0 = (T)P.fx[0], fx1 = (T)P.fx[1], fx2 = (T)P.fx[2], fx3 = (T)P.fx[3], fx4 = (T)P.fx[4];
    const T tu0 = (T)u0, tu1 = (T)u1, tu2 = (T)u2;
    double acc[NSUM], wacc[NF];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = 0.0;
#pragma unroll
    for (int l = 0; l < NF; ++l) wacc[l] = 0.0;
    const int k0 = vt * C.tile;
    const int kend = min(k0 + C.tile, C.nv);
    for (int k = k0 + (int)threadIdx.x; k < kend; k += BLOCK) {
        T v[NF];
#pragma unroll
        for (int l = 0; l < NF; ++l) v[l] = fnb[l][k];
        const T o = fo[k];
        // order 2: the cell's increments per face, and each face's incoming
        // value reconstructed by its kinetic neighbour
        T di[NF];
        if constexpr (O2) {
#pragma unroll
            for (int l = 0; l < NF; ++l) {
                di[l] = dio[l][k];
                v[l] += qk[l] * dnb[l][k];
            }
        }
        T x0, x1, x2, w;
        if constexpr (sizeof(T) == 4) {
            const float4 q = reinterpret_cast<const float4 *>(C.vptf)[k];
            x0 = q.x, x1 = q.y, x2 = q.z, w = q.w;
        } else {
            const double *q = C.vpt + 4 * (size_t)k;
            x0 = q[0], x1 = q[1], x2 = q[2], w = q[3];
        }
        const T c0 = x0 - tu0, c1 = x1 - tu1, c2 = x2 - tu2;
        const T cc = c0 * c0 + c1 * c1 + c2 * c2;
        const T g = exp(-cc * it) * (fx0 + fx1 * c0 + fx2 * c1 + fx3 * c2 + fx4 * cc) *
                    ((T)1 + (kq0 * c0 + kq1 * c1 + kq2 * c2) * (cc * it - (T)2.5));
        T num = itau * g + idt * o;
        T den = itau + idt;
        T ap[NF];
#pragma unroll
        for (int l = 0; l < NF; ++l) {
            const T a = x0 * fnx[l] + x1 * fny[l] + x2 * fnz[l];
            ap[l] = fmax(a, (T)0);
            den += ap[l];
            num -= fmin(a, (T)0) * fsc[l] * v[l];
            // deferred correction of the outgoing value f_i + delta_i
            if constexpr (O2) num -= ap[l] * di[l];
        }
        const T fnv = num / den;
        __builtin_nontemporal_store(fnv, &fn[k]);
        // moment sums relative to u_ref, FP64
        const double wd = (double)w;
        const double d0 = (double)x0 - u0, d1 = (double)x1 - u1, d2 = (double)x2 - u2;
        const double dcc = d0 * d0 + d1 * d1 + d2 * d2;
        acc_moments<double, 3>(acc, wd, (double)fnv, 0.0, d0, d1, d2, dcc);
        const double r0 = wd * (double)(num - den * o);
        acc[S_RES] += r0;
        acc[S_RES + 1] += r0 * d0;
        acc[S_RES + 2] += r0 * d1;
        acc[S_RES + 3] += r0 * d2;
        acc[S_RES + 4] += r0 * dcc;
#pragma unroll
        for (int l = 0; l < NF; ++l) wacc[l] += wd * (double)(ap[l] * fnv);
    }
    // outgoing wall sums into their wall slots (static indices: the sums stay in registers)
#pragma unroll
    for (int l = 0; l < NF; ++l)
#pragma unroll
        for (int w = 0; w < MAXW; ++w) acc[S_WALL + w] += (fwall[l] == w) ? wacc[l] : 0.0;
    block_reduce_store<NSUM>(acc, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
}


// ---------------------------------------------------------------------------
// polyatomic gas: the two-VDF model of Sec. 2 (eq. general_model; reference
// distributions g_0t, g_0r, g_1t, g_1r; heat-flux mixing q_0, q_1 through A;
// tau = mu(T_t)/p_t), 3D tensor grids.  Rows hold (f0, f1), f1 scaled so that
// sum w f1 = d_r rho T_r / 4 and q_r = 2 sum w c f1.  Boundary and NS-interface
// values of f1 are (d_r T_b / 4) times those of f0.
// ---------------------------------------------------------------------------
__global__ void k_param_poly(const CaseView *__restrict__ cvp, int n_kin)
{
    const CaseView &C = *cvp;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_kin) return;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const double *mom = C.mom + (size_t)slot * MOMS;
    const double rho = mom[0], Tt = mom[4], Tr = mom[MOM_INT];
    const double *qt = mom + 11, *qr = mom + MOM_INT + 1;
    const double dr = C.dr, Zr = C.Zr;
    const double T = (3.0 * Tt + dr * Tr) / (3.0 + dr), pt = rho * Tt, p = rho * T;
    const double wt = 1.0 - 1.0 / Zr, wr = 1.0 / Zr;
    const double ct = pow(M_PI * Tt, -1.5), cr = pow(M_PI * T, -1.5);
    PolyRec R;
    for (int d = 0; d < 3; ++d) R.u[d] = mom[1 + d];
    R.itt = 1.0 / Tt;
    R.it = 1.0 / T;
    R.itau = rho * pow(Tt, 1.0 - C.omega) * sqrt(M_PI) / (2.0 * C.Kn);
    R.at = rho * ct * wt;
    R.ar = rho * cr * wr;
    for (int d = 0; d < 3; ++d) {
        const double q0 = ((2.0 - 3.0 * C.A[0]) * Zr + 1.0) * qt[d] - 3.0 * C.A[1] * Zr * qr[d];
        const double q1 = -C.A[2] * Zr * qt[d] + (1.0 - C.A[3] * Zr) * qr[d];
        R.kt[d] = (4.0 / 15.0) * qt[d] / (Tt * pt);
        R.k0[d] = (4.0 / 15.0) * q0 / (T * p);
        R.bt[d] = ct * wt * qr[d] / Tt;
        R.br[d] = cr * wr * q1 / T;
    }
    R.tht = 0.25 * dr * Tr;
    R.thr = 0.25 * dr * T;
    R.fx[0] = 1.0;
    for (int d = 1; d < 5; ++d) R.fx[d] = 0.0;
    for (int w = 0; w < MAXW; ++w) R.rw[w] = 0.0;
    for (int e = C.cf_ptr[cell]; e < C.cf_ptr[cell + 1]; ++e) {
        const int wi = C.cf_wall[e];
        if (wi >= 0) R.rw[wi] = mom[GSIS_NMOM + wi] / C.wall_den[e];
    }
    if (!(rho > 0.0) || !(Tt > 0.0) || !(Tr > 0.0)) atomicOr(C.status, 1);
    C.prec[slot] = R;
    // the sums of the next sweep are taken relative to u
    for (int d = 0; d < 3; ++d) C.param[slot].u[d] = R.u[d];
}

// conservation fix-up of the polyatomic targets: P(c) = a0 + a.c + b c^2 on
// both, with sum w P G0 = rho, sum w c P G0 = 0 and
// sum w (c^2 G0 + 2 G1) P = (3/2) rho T_t + (d_r/2) rho T_r.  On a tensor grid
// every sum needed is a combination of sums of w E c^alpha over the nodes,
// E one of the two Gaussians exp(-c^2/T_t), exp(-c^2/T), and each of those
// factorises into three 1D sums: S[g][d][m] = sum_j w_dj e_g(c_dj) c_dj^m,
// m <= 7.  So the block forms 2 x 3 x 8 one-dimensional FP64 sums (O(n) work
// instead of O(n^3)), their 2 x 8^3 products, and one thread per matrix entry
// assembles it from those.
// One block of 64 threads per kinetic cell.
constexpr int FIXP_THREADS = 64;

// sum_nodes w E_g c^alpha (c.c)^n, n <= 3, from the products of 1D sums
// P[(p0 8 + p1) 8 + p2] = S[g][0][p0] S[g][1][p1] S[g][2][p2]: (c.c)^n expanded
// by the multinomial theorem, sum over i + j + k = n of n!/(i! j! k!)
// c0^2i c1^2j c2^2k
__device__ __forceinline__ int fact3(int x)
{
    return x < 2 ? 1 : (x == 2 ? 2 : 6);
}

__device__ __forceinline__ double gmom(const double *P, int a0, int a1, int a2, int n)
{
    double s = 0.0;
    for (int i = 0; i <= n; ++i)
        for (int j = 0; i + j <= n; ++j) {
            const int k = n - i - j;
            const int coef = fact3(n) / (fact3(i) * fact3(j) * fact3(k));
            s += (double)coef * P[((a0 + 2 * i) * 8 + a1 + 2 * j) * 8 + a2 + 2 * k];
        }
    return s;
}

// sum w E_g (1 + (kap.c)(c^2 iT - 5/2)) c^alpha (c.c)^n
__device__ __forceinline__ double gshak(const double *P, const double *kap, double iT, int a0, int a1, int a2,
                                        int n)
{
    double s = gmom(P, a0, a1, a2, n);
    for (int i = 0; i < 3; ++i) {
        const int b0 = a0 + (i == 0), b1 = a1 + (i == 1), b2 = a2 + (i == 2);
        s += kap[i] * (iT * gmom(P, b0, b1, b2, n + 1) - 2.5 * gmom(P, b0, b1, b2, n));
    }
    return s;
}

// sum w E_g (bet.c) c^alpha (c.c)^n
__device__ __forceinline__ double glin(const double *P, const double *bet, int a0, int a1, int a2, int n)
{
    return bet[0] * gmom(P, a0 + 1, a1, a2, n) + bet[1] * gmom(P, a0, a1 + 1, a2, n) +
           bet[2] * gmom(P, a0, a1, a2 + 1, n);
}

__global__ __launch_bounds__(FIXP_THREADS) void k_fix_poly(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    __shared__ double M[25], Bv[5];
    __shared__ double S[2][3][8];
    __shared__ double P[2][512];
    const int cell = C.kin_cell[blockIdx.x];
    const int slot = C.slot_of_cell[cell];
    const PolyRec &R = C.prec[slot];
    if (threadIdx.x < 48) {
        // one 1D sum per lane, straight from the axis nodes and weights (no
        // LDS tables: the block's small LDS footprint keeps more cells in flight)
        const int g = threadIdx.x / 24, d = (threadIdx.x / 8) % 3, m = threadIdx.x % 8;
        const double u = R.u[d], iT = g ? R.it : R.itt;
        double s = 0.0;
        for (int j = 0; j < C.n[d]; ++j) {
            const double c = C.xv[d * MAXA + j] - u;
            double pw = C.wv[d * MAXA + j] * exp(-c * c * iT);
            for (int r = 0; r < m; ++r) pw *= c;
            s += pw;
        }
        S[g][d][m] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 1024; i += FIXP_THREADS) {
        const int g = i >> 9, r = i & 511;
        P[g][r] = S[g][0][r >> 6] * S[g][1][(r >> 3) & 7] * S[g][2][r & 7];
    }
    __syncthreads();
    if (threadIdx.x < 25) {
        // entry (a, b): sum w ph_a ph_b G0 for a < 4, sum w ph_b (c^2 G0 + 2 G1)
        // for a = 4, with ph = (1, c0, c1, c2, c^2): ph_a ph_b = c^alpha (c.c)^n
        const int a = threadIdx.x / 5, b = threadIdx.x % 5;
        const int al0 = (a == 1) + (b == 1), al1 = (a == 2) + (b == 2), al2 = (a == 3) + (b == 3);
        const int n = (a == 4) + (b == 4);
        double v = R.at * gshak(P[0], R.kt, R.itt, al0, al1, al2, n) + R.ar * gshak(P[1], R.k0, R.it, al0, al1, al2, n);
        if (a == 4) {
            const int m0 = (b == 1), m1 = (b == 2), m2 = (b == 3), nb = (b == 4);
            const double g1 = R.tht * R.at * gshak(P[0], R.kt, R.itt, m0, m1, m2, nb) + glin(P[0], R.bt, m0, m1, m2, nb) +
                              R.thr * R.ar * gshak(P[1], R.k0, R.it, m0, m1, m2, nb) + glin(P[1], R.br, m0, m1, m2, nb);
            v += 2.0 * g1;
        }
        M[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double *mom = C.mom + (size_t)slot * MOMS;
        const double rho = mom[0], Tt = mom[4], Tr = mom[MOM_INT];
        // elimination in place in LDS (row swaps index at run time: private
        // arrays would live in scratch memory)
        double *A = M, *b = Bv;
        b[0] = rho;
        b[1] = b[2] = b[3] = 0.0;
        b[4] = 1.5 * rho * Tt + 0.5 * C.dr * rho * Tr;
        bool ok = true;
        for (int col = 0; col < 5 && ok; ++col) {
            int piv = col;
            for (int r = col + 1; r < 5; ++r)
                if (fabs(A[r * 5 + col]) > fabs(A[piv * 5 + col])) piv = r;
            if (!(fabs(A[piv * 5 + col]) > 0.0)) {
                ok = false;
                break;
            }
            if (piv != col) {
                for (int j = 0; j < 5; ++j) {
                    const double tmp = A[col * 5 + j];
                    A[col * 5 + j] = A[piv * 5 + j];
                    A[piv * 5 + j] = tmp;
                }
                const double tmp = b[col];
                b[col] = b[piv];
                b[piv] = tmp;
            }
            for (int r = col + 1; r < 5; ++r) {
                const double fac = A[r * 5 + col] / A[col * 5 + col];
                for (int j = col; j < 5; ++j) A[r * 5 + j] -= fac * A[col * 5 + j];
                b[r] -= fac * b[col];
            }
        }
        if (ok) {
            for (int r = 4; r >= 0; --r) {
                double sum = b[r];
                for (int j = r + 1; j < 5; ++j) sum -= A[r * 5 + j] * b[j];
                b[r] = sum / A[r * 5 + r];
            }
            for (int d = 0; d < 5; ++d) C.prec[slot].fx[d] = b[d];
        } else {
            atomicOr(C.status, 1);
        }
    }
}

// rows of the polyatomic gas and their sums: mode 0 fills f0 with the
// conservation-fixed Maxwellian of W (FeqRec) and f1 = Th f0 (Th = d_r T_r/4);
// mode 1 (new kinetic cells) and mode 3 (Grad-13 ghost rows of NS cells, no
// sums) the two-VDF Grad-13 rows of the cell's parameters (ghost, ghr):
// f0 = the monatomic row at T_t, f1 = (d_r T_r/4) f0 + (q_r.c/(rho T_t)) M_t
// (Sec. 3.2 eq. G13_VDF, scaled); mode 2 keeps the rows.  Modes 0-2 write the
// partial sums of f0 and f1.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill_poly(const CaseView *__restrict__ cvp, const int32_t *list,
                                                     int n_items, int mode, int cur)
{
    const CaseView &C = *cvp;
    __shared__ double red[(BLOCK / 64) * NSUM];
    __shared__ double wn[MAXW][3];
    __shared__ int s_wi[MAXW], s_nw;
    __shared__ double t_c[3 * MAXA], t_e[3 * MAXA], t_x[3 * MAXA], t_w[3 * MAXA];
    const int vt = blockIdx.x / n_items, t = blockIdx.x - vt * n_items;
    const int cell = list[t];
    const int slot = (mode == 3) ? C.ghost_slot[cell] : C.slot_of_cell[cell];
    double u[3], it = 1.0, th = 0.0, fx[5] = {0, 0, 0, 0, 0};
    double A = 0.0, sg[6] = {0, 0, 0, 0, 0, 0}, qg[3] = {0, 0, 0}, qr[3] = {0, 0, 0};
    if (mode == 0) {
        const FeqRec &F = C.feq[2 * (size_t)slot];
        for (int d = 0; d < 3; ++d) u[d] = F.u[d];
        it = F.it;
        th = F.Th;
        for (int d = 0; d < 5; ++d) fx[d] = F.fx[d];
    } else if (mode == 2) {
        for (int d = 0; d < 3; ++d) u[d] = C.W[5 * (size_t)cell + 1 + d];
    } else {
        const double *g = C.ghost + (size_t)cell * GSIS_NMOM;
        const double *gr = C.ghr + 4 * (size_t)cell;
        const double rho = g[0], Tg = g[4], p = rho * Tg;
        for (int d = 0; d < 3; ++d) u[d] = g[1 + d];
        it = 1.0 / Tg;
        th = 0.25 * C.dr * gr[0];
        A = rho * pow(M_PI * Tg, -1.5);
        for (int d = 0; d < 6; ++d) sg[d] = g[5 + d] / (p * Tg);
        for (int d = 0; d < 3; ++d) {
            qg[d] = 2.0 * g[11 + d] / (p * Tg);
            qr[d] = gr[1 + d] / p;   // q_r / (rho T_t)
        }
    }
    if (threadIdx.x == 0) {
        if (vt == 0 && mode != 3)
            for (int d = 0; d < 3; ++d) C.param[slot].u[d] = u[d];
        int nw = 0;
        if (mode != 3)
            for (int e = C.cf_ptr[cell]; e < C.cf_ptr[cell + 1]; ++e)
                if (C.cf_wall[e] >= 0) {
                    for (int d = 0; d < 3; ++d) wn[nw][d] = C.cf_nsv[3 * (size_t)e + d];
                    s_wi[nw++] = C.cf_wall[e];
                }
        s_nw = nw;
    }
    // per axis node j (axes concatenated): the offset c = x - u, the 1D
    // Gaussian factor exp(-c^2/T), the node and its weight (a node's Gaussian
    // is the product of its three factors)
    const int n0 = C.n[0], n1 = C.n[1], n2 = C.n[2], NA3 = n0 + n1 + n2;
    for (int j = threadIdx.x; j < NA3; j += BLOCK) {
        const int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        const int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        const double x = C.xv[d * MAXA + jj], c = x - u[d];
        t_c[j] = c;
        t_e[j] = exp(-c * c * it);
        t_x[j] = x;
        t_w[j] = C.wv[d * MAXA + jj];
    }
    __syncthreads();
    const int nw = s_nw;
    const int nvp = C.row / 2;
    T *fr = (T *)((mode == 3) ? C.grow : C.f[cur]) + (size_t)slot * C.row;
    double acc[NSUM], wj[MAXW], ps[PSUM] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = 0.0;
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wj[j] = 0.0;
    const int k0 = vt * C.tile, kend = min(k0 + C.tile, C.nv);
    VIdx vi = vidx_init<3>(k0 + threadIdx.x, n1, n2);
    for (int k = k0 + threadIdx.x; k < kend; k += BLOCK) {
        const int jx = vi.ix, jy = n0 + vi.iy, jz = n0 + n1 + vi.iz;
        vidx_step<3>(vi, n1, n2);
        const double xi[3] = {t_x[jx], t_x[jy], t_x[jz]};
        const double w = t_w[jx] * t_w[jy] * t_w[jz];
        const double c0 = t_c[jx], c1 = t_c[jy], c2 = t_c[jz];
        const double cc = c0 * c0 + c1 * c1 + c2 * c2;
        const double E = t_e[jx] * t_e[jy] * t_e[jz];
        T v0, v1;
        if (mode == 2) {
            v0 = fr[k];
            v1 = fr[nvp + k];
        } else {
            double f0, f1;
            if (mode == 0) {
                f0 = E * (fx[0] + fx[1] * c0 + fx[2] * c1 + fx[3] * c2 + fx[4] * cc);
                f1 = th * f0;
            } else {
                const double Q2 = sg[0] * c0 * c0 + sg[1] * c1 * c1 + sg[2] * c2 * c2 +
                                  2.0 * (sg[3] * c0 * c1 + sg[4] * c0 * c2 + sg[5] * c1 * c2);
                const double qd = qg[0] * c0 + qg[1] * c1 + qg[2] * c2;
                const double M = A * E;
                f0 = M * (1.0 + Q2 + qd * (0.4 * cc * it - 1.0));
                f1 = th * f0 + (qr[0] * c0 + qr[1] * c1 + qr[2] * c2) * M;
            }
            v0 = (T)f0;
            v1 = (T)f1;
            fr[k] = v0;
            fr[nvp + k] = v1;
        }
        if (mode == 3) continue;
        acc_moments<double, 3>(acc, w, (double)v0, 0.0, c0, c1, c2, cc);
        const double h1 = w * (double)v1;
        ps[0] += h1;
        ps[1] += h1 * c0;
        ps[2] += h1 * c1;
        ps[3] += h1 * c2;
#pragma unroll
        for (int j = 0; j < MAXW; ++j)
            if (j < nw) {
                const double a = xi[0] * wn[j][0] + xi[1] * wn[j][1] + xi[2] * wn[j][2];
                if (a > 0.0) wj[j] += w * a * (double)v0;
            }
    }
    if (vt == 0 && mode != 2)
        for (int kp = C.nv + threadIdx.x; kp < nvp; kp += BLOCK) {
            fr[kp] = (T)0;
            fr[nvp + kp] = (T)0;
        }
    if (mode == 3) return;   // ghost rows carry no sums (block-uniform exit)
#pragma unroll
    for (int j = 0; j < MAXW; ++j)
#pragma unroll
        for (int ww = 0; ww < MAXW; ++ww) acc[S_WALL + ww] += (j < nw && s_wi[j] == ww) ? wj[j] : 0.0;
    block_reduce_store<NSUM>(acc, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
    __syncthreads();
    block_reduce_store<PSUM>(ps, C.psum + ((size_t)slot * C.ntile + vt) * PSUM, red);
}

// GSIS correction of both VDFs (first eq. updatef): f0 += f_eq(W_new) -
// f_eq(W_half), f1 += Th_new f_eq(W_new) - Th_half f_eq(W_half), in place,
// with the partial sums of the corrected rows (relative to the slot's
// reference velocity).  Tensor grid: both Gaussians factorise per axis, so the
// block forms FP64 tables of the offsets and 1D Gaussian factors of the two
// Maxwellians (and the offsets of the reference frame) and a node takes two
// products per Maxwellian, no exp.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_correct_poly(const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    const CaseView &C = *cvp;
    __shared__ double red[(BLOCK / 64) * NSUM];
    __shared__ double wn[MAXW][3];
    __shared__ int s_wi[MAXW], s_nw;
    // per axis node j (axes concatenated): offsets and Gaussian factors of
    // f_eq(W_new) (a) and f_eq(W_half) (b), the reference-frame offset, the
    // node and its weight
    __shared__ double t_ca[3 * MAXA], t_ea[3 * MAXA], t_cb[3 * MAXA], t_eb[3 * MAXA], t_cr[3 * MAXA],
        t_x[3 * MAXA], t_w[3 * MAXA];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin, t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const FeqRec &Fa = C.feq[2 * (size_t)slot];
    const FeqRec &Fb = C.feq[2 * (size_t)slot + 1];
    const double *ur = C.param[slot].u;
    const int n0 = C.n[0], n1 = C.n[1], n2 = C.n[2], NA3 = n0 + n1 + n2;
    if (threadIdx.x == 0) {
        int nw = 0;
        for (int e = C.cf_ptr[cell]; e < C.cf_ptr[cell + 1]; ++e)
            if (C.cf_wall[e] >= 0) {
                for (int d = 0; d < 3; ++d) wn[nw][d] = C.cf_nsv[3 * (size_t)e + d];
                s_wi[nw++] = C.cf_wall[e];
            }
        s_nw = nw;
    }
    for (int j = threadIdx.x; j < NA3; j += BLOCK) {
        const int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        const int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        const double x = C.xv[d * MAXA + jj];
        const double ca = x - Fa.u[d], cb = x - Fb.u[d];
        t_ca[j] = ca;
        t_cb[j] = cb;
        t_ea[j] = exp(-ca * ca * Fa.it);
        t_eb[j] = exp(-cb * cb * Fb.it);
        t_cr[j] = x - ur[d];
        t_x[j] = x;
        t_w[j] = C.wv[d * MAXA + jj];
    }
    __syncthreads();
    const int nw = s_nw;
    const int nvp = C.row / 2;
    T *fr = (T *)C.f[cur] + (size_t)slot * C.row;
    double acc[NSUM], wj[MAXW], ps[PSUM] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = 0.0;
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wj[j] = 0.0;
    const int k0 = vt * C.tile, kend = min(k0 + C.tile, C.nv);
    VIdx vi = vidx_init<3>(k0 + threadIdx.x, n1, n2);
    for (int k = k0 + threadIdx.x; k < kend; k += BLOCK) {
        const int jx = vi.ix, jy = n0 + vi.iy, jz = n0 + n1 + vi.iz;
        vidx_step<3>(vi, n1, n2);
        const double a0 = t_ca[jx], a1 = t_ca[jy], a2 = t_ca[jz];
        const double b0 = t_cb[jx], b1 = t_cb[jy], b2 = t_cb[jz];
        const double aa = a0 * a0 + a1 * a1 + a2 * a2, bb = b0 * b0 + b1 * b1 + b2 * b2;
        const double ma = (t_ea[jx] * t_ea[jy] * t_ea[jz]) *
                          (Fa.fx[0] + Fa.fx[1] * a0 + Fa.fx[2] * a1 + Fa.fx[3] * a2 + Fa.fx[4] * aa);
        const double mb = (t_eb[jx] * t_eb[jy] * t_eb[jz]) *
                          (Fb.fx[0] + Fb.fx[1] * b0 + Fb.fx[2] * b1 + Fb.fx[3] * b2 + Fb.fx[4] * bb);
        const T v0 = (T)((double)fr[k] + (ma - mb));
        const T v1 = (T)((double)fr[nvp + k] + (Fa.Th * ma - Fb.Th * mb));
        fr[k] = v0;
        fr[nvp + k] = v1;
        const double w = t_w[jx] * t_w[jy] * t_w[jz];
        const double c0 = t_cr[jx], c1 = t_cr[jy], c2 = t_cr[jz];
        const double cc = c0 * c0 + c1 * c1 + c2 * c2;
        acc_moments<double, 3>(acc, w, (double)v0, 0.0, c0, c1, c2, cc);
        const double h1 = w * (double)v1;
        ps[0] += h1;
        ps[1] += h1 * c0;
        ps[2] += h1 * c1;
        ps[3] += h1 * c2;
#pragma unroll
        for (int j = 0; j < MAXW; ++j)
            if (j < nw) {
                const double a = t_x[jx] * wn[j][0] + t_x[jy] * wn[j][1] + t_x[jz] * wn[j][2];
                if (a > 0.0) wj[j] += w * a * (double)v0;
            }
    }
#pragma unroll
    for (int j = 0; j < MAXW; ++j)
#pragma unroll
        for (int ww = 0; ww < MAXW; ++ww) acc[S_WALL + ww] += (j < nw && s_wi[j] == ww) ? wj[j] : 0.0;
    block_reduce_store<NSUM>(acc, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
    __syncthreads();
    block_reduce_store<PSUM>(ps, C.psum + ((size_t)slot * C.ntile + vt) * PSUM, red);
}

// the point-Jacobi sweep of both VDFs: one block per (kinetic cell, velocity
// tile), faces as rows with wave-uniform bases -- a kinetic neighbour's
// (f0, f1) rows, or the Grad-13 ghost row of an NS neighbour or the patch row
// of a wall (times rho_w) or far field for f0 with f1 = (d_r T_b / 4) f0; the
// own targets from per-axis Gaussian tables at T_t and T; the loads of a node
// are issued before they are used; FP64 moment sums of both VDFs
template <typename T, int NF, bool VEC>
__global__ __launch_bounds__(BLOCK) void k_sweep_poly(Batch B)
{
    __shared__ double red[(BLOCK / 64) * NSUM];
    // per-axis node tables: FP64 offsets c_d = x_j - u_d and weights (for the
    // sums), nodes and Gaussian factors at T_t and T in the case dtype
    __shared__ double tcd[3 * MAXA], twd[3 * MAXA];
    __shared__ T tx[3 * MAXA], tet[3 * MAXA], ter[3 * MAXA];
    const int nb = gridDim.x;
    const int b = xcd_remap(blockIdx.x, nb);
    int ci = 0;
    while (ci + 1 < B.n && b >= B.start[ci + 1]) ++ci;
    const CaseView &C = *B.cv[ci];
    const int cur = B.cur[ci];
    const int item = b - B.start[ci];
    const int n_kin = (B.start[ci + 1] - B.start[ci]) / C.ntile;
    const int vt = item / n_kin;
    const int t = item - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const PolyRec &R = C.prec[slot];
    const size_t row = (size_t)C.row;
    const int nvp = C.row / 2;
    const T *fold = (const T *)C.f[cur];
    const T *fo = wave_uniform(fold + (size_t)slot * row);
    T *fn = wave_uniform((T *)C.f[cur ^ 1] + (size_t)slot * row);
    // faces: row base, scale (rho_w on walls), n S / V, f1 rule (kinetic row
    // or d_r T_b / 4 times f0), wall-sum index
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    const T *fnb[NF];
    T fsc[NF], fnx[NF], fny[NF], fnz[NF], fkin[NF], fth[NF];
    int fwall[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fnb[l] = fo;
        fsc[l] = fnx[l] = fny[l] = fnz[l] = fkin[l] = fth[l] = (T)0;
        fwall[l] = -1;
        if (l < nf) {
            const int e = e0 + l;
            const int oth = C.cf_other[e];
            fnx[l] = (T)C.cf_nsv[3 * e];
            fny[l] = (T)C.cf_nsv[3 * e + 1];
            fnz[l] = (T)C.cf_nsv[3 * e + 2];
            fsc[l] = (T)1;
            if (oth >= 0 && C.slot_of_cell[oth] >= 0) {
                fnb[l] = fold + (size_t)C.slot_of_cell[oth] * row;
                fkin[l] = (T)1;
            } else if (oth >= 0) {
                // the two-VDF Grad-13 rows of the NS neighbour (f0, f1)
                fnb[l] = (const T *)C.grow + (size_t)C.ghost_slot[oth] * row;
                fkin[l] = (T)1;
            } else {
                const int pi = -1 - oth;
                fnb[l] = (const T *)C.prow + (size_t)pi * row;
                fth[l] = (T)(0.25 * C.dr * C.patch_state[5 * pi + 4]);
                fwall[l] = C.cf_wall[e];
                if (fwall[l] >= 0) fsc[l] = (T)R.rw[fwall[l]];
            }
        }
        fnb[l] = wave_uniform(fnb[l]);
    }
    const int n0 = C.n[0], n1 = C.n[1], n2 = C.n[2], NA3 = n0 + n1 + n2;
    for (int j = threadIdx.x; j < NA3; j += BLOCK) {
        const int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        const int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        const double x = C.xv[d * MAXA + jj], c = x - R.u[d];
        tcd[j] = c;
        twd[j] = C.wv[d * MAXA + jj];
        tx[j] = (T)x;
        tet[j] = (T)exp(-c * c * R.itt);
        ter[j] = (T)exp(-c * c * R.it);
    }
    __syncthreads();
    const T itt = (T)R.itt, it = (T)R.it, itau = (T)R.itau, inv_dt = (T)C.inv_dt;
    const T at = (T)R.at, ar = (T)R.ar, tht = (T)R.tht, thr = (T)R.thr;
    const T kt0 = (T)R.kt[0], kt1 = (T)R.kt[1], kt2 = (T)R.kt[2];
    const T k00 = (T)R.k0[0], k01 = (T)R.k0[1], k02 = (T)R.k0[2];
    const T bt0 = (T)R.bt[0], bt1 = (T)R.bt[1], bt2 = (T)R.bt[2];
    const T br0 = (T)R.br[0], br1 = (T)R.br[1], br2 = (T)R.br[2];
    const T fx0 = (T)R.fx[0], fx1 = (T)R.fx[1], fx2 = (T)R.fx[2], fx3 = (T)R.fx[3], fx4 = (T)R.fx[4];
    double acc[NSUM], wacc[NF], ps[PSUM] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = 0.0;
#pragma unroll
    for (int l = 0; l < NF; ++l) wacc[l] = 0.0;
    const int k0 = vt * C.tile, kend = min(k0 + C.tile, C.nv);
    // one node: the relaxed values of f0 and f1 from the node's own and upwind
    // values, with its moment, balance and wall sums
    auto relax = [&](int jx, int jy, int jz, const T *v0, const T *v1, T o0, T o1, T &n0v, T &n1v) {
        const double wd = twd[jx] * twd[jy] * twd[jz];
        const T x0 = tx[jx], x1 = tx[jy], x2 = tx[jz];
        const double d0 = tcd[jx], d1 = tcd[jy], d2 = tcd[jz];
        const T c0 = (T)d0, c1 = (T)d1, c2 = (T)d2;
        const T cc = c0 * c0 + c1 * c1 + c2 * c2;
        const T Et = tet[jx] * tet[jy] * tet[jz], Er = ter[jx] * ter[jy] * ter[jz];
        const T ht = at * Et * ((T)1 + (kt0 * c0 + kt1 * c1 + kt2 * c2) * (cc * itt - (T)2.5));
        const T hr = ar * Er * ((T)1 + (k00 * c0 + k01 * c1 + k02 * c2) * (cc * it - (T)2.5));
        const T P = fx0 + fx1 * c0 + fx2 * c1 + fx3 * c2 + fx4 * cc;
        const T G0 = P * (ht + hr);
        const T G1 = P * (tht * ht + Et * (bt0 * c0 + bt1 * c1 + bt2 * c2) + thr * hr +
                          Er * (br0 * c0 + br1 * c1 + br2 * c2));
        T den = inv_dt + itau;
        T num0 = itau * G0 + inv_dt * o0;
        T num1 = itau * G1 + inv_dt * o1;
        T ap[NF];
#pragma unroll
        for (int l = 0; l < NF; ++l) {
            const T a = x0 * fnx[l] + x1 * fny[l] + x2 * fnz[l];
            ap[l] = fmax(a, (T)0);
            den += ap[l];
            const T m = fmin(a, (T)0) * fsc[l];
            num0 -= m * v0[l];
            num1 -= m * (fkin[l] * v1[l] + fth[l] * v0[l]);
        }
        const T rden = (T)1 / den;
        n0v = num0 * rden;
        n1v = num1 * rden;
        const double dcc = d0 * d0 + d1 * d1 + d2 * d2;
        acc_moments<double, 3>(acc, wd, (double)n0v, 0.0, d0, d1, d2, dcc);
        const double h1 = wd * (double)n1v;
        ps[0] += h1;
        ps[1] += h1 * d0;
        ps[2] += h1 * d1;
        ps[3] += h1 * d2;
        // moment balance at the old iterate (energy: c^2 f0 + 2 f1)
        const double r0 = wd * (double)(num0 - den * o0);
        acc[S_RES] += r0;
        acc[S_RES + 1] += r0 * d0;
        acc[S_RES + 2] += r0 * d1;
        acc[S_RES + 3] += r0 * d2;
        const double r1 = wd * (double)(num1 - den * o1);
        acc[S_RES + 4] += r0 * dcc + 2.0 * r1;
        ps[4] += r1;
#pragma unroll
        for (int l = 0; l < NF; ++l) wacc[l] += wd * (double)(ap[l] * n0v);
    };
    if (VEC && C.n[2] % 4 == 0 && C.tile % 4 == 0 && C.nv % 4 == 0) {
        // four consecutive z nodes per lane (16-byte loads and stores of every
        // row; n_z, the tile and the rows are multiples of 4 nodes)
        typedef T V4 __attribute__((ext_vector_type(4)));
        for (int k = k0 + 4 * (int)threadIdx.x; k < kend; k += 4 * BLOCK) {
            V4 a0[NF], a1[NF];
#pragma unroll
            for (int l = 0; l < NF; ++l) {
                a0[l] = *(const V4 *)(fnb[l] + k);
                a1[l] = *(const V4 *)(fnb[l] + nvp + k);
            }
            const V4 q0 = *(const V4 *)(fo + k), q1 = *(const V4 *)(fo + nvp + k);
            const int iz = k % n2, r = k / n2, iy = r % n1, ix = r / n1;
            V4 r0v, r1v;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                T v0[NF], v1[NF];
#pragma unroll
                for (int l = 0; l < NF; ++l) {
                    v0[l] = a0[l][jj];
                    v1[l] = a1[l][jj];
                }
                T n0v, n1v;
                relax(ix, n0 + iy, n0 + n1 + iz + jj, v0, v1, q0[jj], q1[jj], n0v, n1v);
                r0v[jj] = n0v;
                r1v[jj] = n1v;
            }
            __builtin_nontemporal_store(r0v, (V4 *)(fn + k));
            __builtin_nontemporal_store(r1v, (V4 *)(fn + nvp + k));
        }
    } else {
        VIdx vi = vidx_init<3>(k0 + threadIdx.x, n1, n2);
        for (int k = k0 + threadIdx.x; k < kend; k += BLOCK) {
            T v0[NF], v1[NF];
#pragma unroll
            for (int l = 0; l < NF; ++l) {
                v0[l] = fnb[l][k];
                v1[l] = fnb[l][nvp + k];
            }
            const T o0 = fo[k], o1 = fo[nvp + k];
            const int jx = vi.ix, jy = n0 + vi.iy, jz = n0 + n1 + vi.iz;
            vidx_step<3>(vi, n1, n2);
            T n0v, n1v;
            relax(jx, jy, jz, v0, v1, o0, o1, n0v, n1v);
            __builtin_nontemporal_store(n0v, &fn[k]);
            __builtin_nontemporal_store(n1v, &fn[nvp + k]);
        }
    }
#pragma unroll
    for (int l = 0; l < NF; ++l)
#pragma unroll
        for (int w = 0; w < MAXW; ++w) acc[S_WALL + w] += (fwall[l] == w) ? wacc[l] : 0.0;
    block_reduce_store<NSUM>(acc, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
    __syncthreads();
    block_reduce_store<PSUM>(ps, C.psum + ((size_t)slot * C.ntile + vt) * PSUM, red);
}

hipError_t launch_param_poly(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_param_poly, dim3((n_kin + 63) / 64), dim3(64), 0, s, cv, n_kin);
    hipLaunchKernelGGL(k_fix_poly, dim3(n_kin), dim3(FIXP_THREADS), 0, s, cv);
    return hipGetLastError();
}

hipError_t launch_fill_poly(const CaseView *cv, const CaseView &h, int mode, int n_items, int cur, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    const int32_t *list = (mode == 1) ? h.new_cell : ((mode == 3) ? h.ghost_cell : h.kin_cell);
    if (mode == 0) hipLaunchKernelGGL(k_feqpar, dim3((n_items + 63) / 64), dim3(64), 0, s, cv, n_items, list, 1);
    dim3 g(n_items * h.ntile);
    if (h.dtype == GSIS_F32)
        hipLaunchKernelGGL((k_fill_poly<float>), g, dim3(BLOCK), 0, s, cv, list, n_items, mode, cur);
    else hipLaunchKernelGGL((k_fill_poly<double>), g, dim3(BLOCK), 0, s, cv, list, n_items, mode, cur);
    return hipGetLastError();
}

hipError_t launch_sweep_poly(const Batch &b, const CaseView &h0, int total, hipStream_t s)
{
    const bool f4 = b.nfmax <= 4;
    if (h0.dtype == GSIS_F32) {
        // 16-byte node groups on the cases whose z axis, tile and node count are
        // multiples of 4 (the kernel checks each case)
        if (poly_vec_on()) {
            if (f4) hipLaunchKernelGGL((k_sweep_poly<float, 4, true>), dim3(total), dim3(BLOCK), 0, s, b);
            else hipLaunchKernelGGL((k_sweep_poly<float, MAXF, true>), dim3(total), dim3(BLOCK), 0, s, b);
        } else {
            if (f4) hipLaunchKernelGGL((k_sweep_poly<float, 4, false>), dim3(total), dim3(BLOCK), 0, s, b);
            else hipLaunchKernelGGL((k_sweep_poly<float, MAXF, false>), dim3(total), dim3(BLOCK), 0, s, b);
        }
    } else {
        if (f4) hipLaunchKernelGGL((k_sweep_poly<double, 4, false>), dim3(total), dim3(BLOCK), 0, s, b);
        else hipLaunchKernelGGL((k_sweep_poly<double, MAXF, false>), dim3(total), dim3(BLOCK), 0, s, b);
    }
    return hipGetLastError();
}

template <typename T, int VD>
static hipError_t launch_sweep_t(const Batch &b, const CaseView &h0, int total, hipStream_t s)
{
    const char *o2g = std::getenv("GSIS_ORDER2_GENERIC");
    if (VD == 3 && (h0.points || (h0.sorder == 2 && !(o2g && o2g[0] == '1')))) {
        // faces as rows: point sets, and 3D tensor grids at order 2 (their
        // node table is filled at bind)
        if (h0.sorder == 2) {
            if (b.nfmax <= 4) hipLaunchKernelGGL((k_sweep_prow<T, 4, true>), dim3(total), dim3(BLOCK), 0, s, b);
            else hipLaunchKernelGGL((k_sweep_prow<T, MAXF, true>), dim3(total), dim3(BLOCK), 0, s, b);
        } else {
            if (b.nfmax <= 4) hipLaunchKernelGGL((k_sweep_prow<T, 4, false>), dim3(total), dim3(BLOCK), 0, s, b);
            else hipLaunchKernelGGL((k_sweep_prow<T, MAXF, false>), dim3(total), dim3(BLOCK), 0, s, b);
        }
        return hipGetLastError();
    }
    int NA3 = h0.n[0] + h0.n[1] + (VD == 3 ? h0.n[2] : 0);
    size_t lds = sizeof(double) * (size_t)NA3 * 2 + sizeof(T) * (size_t)NA3 * (3 + 1 + MAXF);
    if (h0.sorder == 2) {
        // second-order face values on tensor grids: the generic kernel (its
        // per-face branches load neighbour slopes only for incoming values,
        // which measured faster than the row form's unconditional loads)
        hipLaunchKernelGGL((k_sweep<T, VD, false, true>), dim3(total), dim3(BLOCK), lds, s, b);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_sweep<T, VD, false, false>), dim3(total), dim3(BLOCK), lds, s, b);
    return hipGetLastError();
}

hipError_t launch_sweep(const Batch &b, const CaseView &h0, int total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    if (h0.poly) return launch_sweep_poly(b, h0, total, s);
    if (h0.fast) return launch_sweep_fast(b, h0, total, s);
    if (h0.sorder == 2 && b.v4) return launch_sweep_o2v4(b, h0, total, s);
    // all cases of a batch share dtype and vdim; LDS is sized for the largest axes
    if (h0.dtype == GSIS_F32)
        return h0.vdim == 3 ? launch_sweep_t<float, 3>(b, h0, total, s) : launch_sweep_t<float, 2>(b, h0, total, s);
    return h0.vdim == 3 ? launch_sweep_t<double, 3>(b, h0, total, s) : launch_sweep_t<double, 2>(b, h0, total, s);
}

// ---------------------------------------------------------------------------
// GSIS correction (first eq. updatef): f += f_eq(W_new) - f_eq(W_half), in
// place, with the moment epilogue of the corrected f
// ---------------------------------------------------------------------------
template <typename T, int VD, bool PTS>
__global__ __launch_bounds__(BLOCK) void k_correct(const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[(BLOCK / 64) * NSUM];
    __shared__ T wn[MAXW][3];
    __shared__ int s_wi[MAXW], s_nw;
    const CaseView &C = *cvp;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin, t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const int n0 = C.n[0], n1 = C.n[1], n2 = (VD == 3) ? C.n[2] : 0;
    const int NA3 = n0 + n1 + n2;
    T *xs = (T *)smem_raw;
    T *ws = xs + NA3;
    T *tabs = ws + NA3;          // [2][NA3] Gaussian factors of f_eq(W_new), f_eq(W_half)
    T *cts = tabs + 2 * NA3;     // [3][NA3] x_j - u_d for W_new, W_half and the reference frame
    const FeqRec &Fa = C.feq[2 * (size_t)slot];
    const FeqRec &Fb = C.feq[2 * (size_t)slot + 1];
    const ParamRec &P = C.param[slot];
    if (threadIdx.x == 0) {
        int e0 = C.cf_ptr[cell], e1 = C.cf_ptr[cell + 1], nw = 0;
        for (int e = e0; e < e1; ++e)
            if (C.cf_wall[e] >= 0) {
                for (int d = 0; d < 3; ++d) wn[nw][d] = (T)C.cf_nsv[3 * e + d];
                s_wi[nw++] = C.cf_wall[e];
            }
        s_nw = nw;
    }
    for (int j = threadIdx.x; j < (PTS ? 0 : NA3); j += BLOCK) {
        int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        xs[j] = (T)C.xv[d * MAXA + jj];
        ws[j] = (T)C.wv[d * MAXA + jj];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < (PTS ? 0 : 3 * NA3); idx += BLOCK) {
        int src = idx / NA3, j = idx - src * NA3;
        int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        const double x = C.xv[d * MAXA + jj];
        if (src < 2) {
            const FeqRec &F = src ? Fb : Fa;
            double c = x - F.u[d];
            tabs[src * NA3 + j] = (T)exp(-c * c * F.it);
            cts[src * NA3 + j] = (T)c;
        } else {
            cts[2 * NA3 + j] = (T)(x - P.u[d]);
        }
    }
    __syncthreads();
    const T a0 = (T)Fa.fx[0], a1 = (T)Fa.fx[1], a2 = (T)Fa.fx[2], a3 = (T)Fa.fx[3], a4 = (T)Fa.fx[4];
    const T b0 = (T)Fb.fx[0], b1 = (T)Fb.fx[1], b2 = (T)Fb.fx[2], b3 = (T)Fb.fx[3], b4 = (T)Fb.fx[4];
    const T tha = (T)Fa.Th, thb = (T)Fb.Th;
    const int nw = s_nw;
    T *fr = (T *)C.f[cur] + (size_t)slot * C.row;
    const int nvp = C.row / ((VD == 3) ? 1 : 2);
    T acc[NSUM], wj[MAXW];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = (T)0;
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wj[j] = (T)0;
    const int k0 = vt * C.tile;
    const int kend = min(k0 + C.tile, C.nv);
    int k = k0 + threadIdx.x;
    VIdx vi = vidx_init<VD>(PTS ? 0 : k, n1, (VD == 3) ? n2 : 1);
    const T *ta = tabs, *tb = tabs + NA3;
    const T ita = (T)Fa.it, itb = (T)Fb.it;
    for (; k < kend; k += BLOCK) {
        T x0, x1, x2, w, Ea, Eb, da0, da1, da2, db0, db1, db2, c0, c1, c2;
        if constexpr (PTS) {
            // point set: offsets formed in FP64, one exp per node and Maxwellian
            const double *q = C.vpt + 4 * (size_t)k;
            x0 = (T)q[0];
            x1 = (T)q[1];
            x2 = (T)q[2];
            w = (T)q[3];
            da0 = (T)(q[0] - Fa.u[0]);
            da1 = (T)(q[1] - Fa.u[1]);
            da2 = (T)(q[2] - Fa.u[2]);
            db0 = (T)(q[0] - Fb.u[0]);
            db1 = (T)(q[1] - Fb.u[1]);
            db2 = (T)(q[2] - Fb.u[2]);
            Ea = exp(-(da0 * da0 + da1 * da1 + da2 * da2) * ita);
            Eb = exp(-(db0 * db0 + db1 * db1 + db2 * db2) * itb);
            c0 = (T)(q[0] - P.u[0]);
            c1 = (T)(q[1] - P.u[1]);
            c2 = (T)(q[2] - P.u[2]);
        } else {
            x0 = xs[vi.ix];
            x1 = xs[n0 + vi.iy];
            x2 = (VD == 3) ? xs[n0 + n1 + vi.iz] : (T)0;
            w = ws[vi.ix] * ws[n0 + vi.iy] * ((VD == 3) ? ws[n0 + n1 + vi.iz] : (T)1);
            Ea = ta[vi.ix] * ta[n0 + vi.iy] * ((VD == 3) ? ta[n0 + n1 + vi.iz] : (T)1);
            Eb = tb[vi.ix] * tb[n0 + vi.iy] * ((VD == 3) ? tb[n0 + n1 + vi.iz] : (T)1);
            const T *ca = cts, *cb = cts + NA3, *cr = cts + 2 * NA3;
            da0 = ca[vi.ix];
            da1 = ca[n0 + vi.iy];
            da2 = (VD == 3) ? ca[n0 + n1 + vi.iz] : (T)0;
            db0 = cb[vi.ix];
            db1 = cb[n0 + vi.iy];
            db2 = (VD == 3) ? cb[n0 + n1 + vi.iz] : (T)0;
            c0 = cr[vi.ix];
            c1 = cr[n0 + vi.iy];
            c2 = (VD == 3) ? cr[n0 + n1 + vi.iz] : (T)0;
        }
        T Pa, Pb;
        if (VD == 3) {
            Pa = a0 + a1 * da0 + a2 * da1 + a3 * da2 + a4 * (da0 * da0 + da1 * da1 + da2 * da2);
            Pb = b0 + b1 * db0 + b2 * db1 + b3 * db2 + b4 * (db0 * db0 + db1 * db1 + db2 * db2);
        } else {
            Pa = a0 + a1 * da0 + a2 * da1 + a3 * (da0 * da0 + da1 * da1);
            Pb = b0 + b1 * db0 + b2 * db1 + b3 * (db0 * db0 + db1 * db1);
        }
        const T ma = Ea * Pa, mb = Eb * Pb;
        const T v0 = fr[k] + (ma - mb);
        fr[k] = v0;
        T v1 = (T)0;
        if (VD == 2) {
            v1 = fr[nvp + k] + (tha * ma - thb * mb);
            fr[nvp + k] = v1;
        }
        const T cc = c0 * c0 + c1 * c1 + c2 * c2;
        acc_moments<T, VD>(acc, w, v0, v1, c0, c1, c2, cc);
#pragma unroll
        for (int j = 0; j < MAXW; ++j)
            if (j < nw) {
                const T a = x0 * wn[j][0] + x1 * wn[j][1] + x2 * wn[j][2];
                if (a > (T)0) wj[j] += w * a * v0;
            }
        if constexpr (!PTS) vidx_step<VD>(vi, n1, (VD == 3) ? n2 : 1);
    }
#pragma unroll
    for (int j = 0; j < MAXW; ++j)
#pragma unroll
        for (int ww = 0; ww < MAXW; ++ww) acc[S_WALL + ww] += (j < nw && s_wi[j] == ww) ? wj[j] : (T)0;
    double v[NSUM];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) v[i] = (double)acc[i];
    block_reduce_store<NSUM>(v, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
}

hipError_t launch_correct(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    if (h.poly) {
        if (launch_correct_poly_v4(cv, h, n_kin, cur, s)) return hipGetLastError();
        const dim3 g(n_kin * h.ntile);
        if (h.dtype == GSIS_F32) hipLaunchKernelGGL((k_correct_poly<float>), g, dim3(BLOCK), 0, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_correct_poly<double>), g, dim3(BLOCK), 0, s, cv, n_kin, cur);
        return hipGetLastError();
    }
    if (h.fast) return launch_correct_fast(cv, h, n_kin, cur, s);
    int NA3 = h.n[0] + h.n[1] + (h.vdim == 3 ? h.n[2] : 0);
    dim3 g(n_kin * h.ntile);
    if (h.points) {
        if (h.dtype == GSIS_F32) hipLaunchKernelGGL((k_correct<float, 3, true>), g, dim3(BLOCK), 0, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_correct<double, 3, true>), g, dim3(BLOCK), 0, s, cv, n_kin, cur);
        return hipGetLastError();
    }
    if (h.dtype == GSIS_F32) {
        size_t lds = sizeof(float) * NA3 * 7;
        if (h.vdim == 3) hipLaunchKernelGGL((k_correct<float, 3, false>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_correct<float, 2, false>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
    } else {
        size_t lds = sizeof(double) * NA3 * 7;
        if (h.vdim == 3) hipLaunchKernelGGL((k_correct<double, 3, false>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_correct<double, 2, false>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fill the rows of listed cells from a Gaussian source (mode 0: conservation-
// fixed Maxwellian of W, FeqRec slot 0; mode 1: Grad-13 of ghost[cell]) and
// write their moment sums relative to u_ref = source velocity
// ---------------------------------------------------------------------------
template <typename T, int VD, bool PTS>
__global__ __launch_bounds__(BLOCK) void k_fill(const CaseView *__restrict__ cvp, const int32_t *list, int n_items,
                                                int mode, int cur)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[(BLOCK / 64) * NSUM];
    __shared__ T wn[MAXW][3];
    __shared__ int s_wi[MAXW], s_nw;
    const CaseView &C = *cvp;
    const int b = blockIdx.x;
    const int vt = b / n_items, t = b - vt * n_items;
    const int cell = list[t];
    const int slot = (mode == 3) ? C.ghost_slot[cell] : C.slot_of_cell[cell];
    const int n0 = C.n[0], n1 = C.n[1], n2 = (VD == 3) ? C.n[2] : 0;
    const int NA3 = n0 + n1 + n2;
    T *xs = (T *)smem_raw;
    T *ws = xs + NA3;
    T *tabs = ws + NA3;
    // source
    double u[3], it, Th, A = 1.0, fx[5] = {0, 0, 0, 0, 0}, sg[6] = {0, 0, 0, 0, 0, 0}, qg[3] = {0, 0, 0};
    if (mode == 2) {
        const double *W = C.W + 5 * (size_t)cell;
        for (int d = 0; d < 3; ++d) u[d] = W[1 + d];
        if (VD == 2) u[2] = 0.0;
        it = 1.0 / W[4];
        Th = 0.5 * W[4];
    } else if (mode == 0) {
        const FeqRec &F = C.feq[2 * (size_t)slot];
        for (int d = 0; d < 3; ++d) u[d] = F.u[d];
        it = F.it;
        Th = F.Th;
        for (int d = 0; d < 5; ++d) fx[d] = F.fx[d];
    } else {   // modes 1 and 3: Grad-13 of the cell's ghost parameters
        const double *g = C.ghost + (size_t)cell * GSIS_NMOM;
        double rho = g[0], Tg = g[4], p = rho * Tg;
        for (int d = 0; d < 3; ++d) u[d] = g[1 + d];
        if (VD == 2) u[2] = 0.0;
        it = 1.0 / Tg;
        Th = 0.5 * Tg;
        A = (VD == 3) ? rho * pow(M_PI * Tg, -1.5) : rho / (M_PI * Tg);
        for (int d = 0; d < 6; ++d) sg[d] = g[5 + d] / (p * Tg);
        for (int d = 0; d < 3; ++d) qg[d] = 2.0 * g[11 + d] / (p * Tg);
    }
    if (threadIdx.x == 0) {
        if (vt == 0 && mode != 3) {
            for (int d = 0; d < 3; ++d) C.param[slot].u[d] = u[d];
        }
        int e0 = C.cf_ptr[cell], e1 = C.cf_ptr[cell + 1], nw = 0;
        for (int e = e0; e < e1; ++e)
            if (C.cf_wall[e] >= 0) {
                for (int d = 0; d < 3; ++d) wn[nw][d] = (T)C.cf_nsv[3 * e + d];
                s_wi[nw++] = C.cf_wall[e];
            }
        s_nw = nw;
    }
    for (int j = threadIdx.x; j < (PTS ? 0 : NA3); j += BLOCK) {
        int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        xs[j] = (T)C.xv[d * MAXA + jj];
        ws[j] = (T)C.wv[d * MAXA + jj];
    }
    __syncthreads();
    T *cs = tabs + NA3;
    for (int j = threadIdx.x; j < (PTS ? 0 : NA3); j += BLOCK) {
        int d = (j < n0) ? 0 : ((j < n0 + n1) ? 1 : 2);
        int jj = j - ((d == 0) ? 0 : ((d == 1) ? n0 : n0 + n1));
        double c = C.xv[d * MAXA + jj] - u[d];
        tabs[j] = (T)exp(-c * c * it);
        cs[j] = (T)c;
    }
    __syncthreads();
    T *fr = (T *)((mode == 3) ? C.grow : C.f[cur]) + (size_t)slot * C.row;
    const int nvp = C.row / ((VD == 3) ? 1 : 2);
    T acc[NSUM], wj[MAXW];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) acc[i] = (T)0;
#pragma unroll
    for (int j = 0; j < MAXW; ++j) wj[j] = (T)0;
    const int k0 = vt * C.tile;
    const int kend = min(k0 + C.tile, C.nv);
    int k = k0 + threadIdx.x;
    VIdx vi = vidx_init<VD>(PTS ? 0 : k, n1, (VD == 3) ? n2 : 1);
    const int nw = (mode == 3) ? 0 : s_nw;
    const T Tg = (T)(2.0 * Th);
    for (; k < kend; k += BLOCK) {
        T x0, x1, x2, w, E, c0, c1, c2;
        if constexpr (PTS) {
            const double *q = C.vpt + 4 * (size_t)k;
            x0 = (T)q[0];
            x1 = (T)q[1];
            x2 = (T)q[2];
            w = (T)q[3];
            c0 = (T)(q[0] - u[0]);
            c1 = (T)(q[1] - u[1]);
            c2 = (T)(q[2] - u[2]);
            E = exp(-(c0 * c0 + c1 * c1 + c2 * c2) * (T)it);
        } else {
            x0 = xs[vi.ix];
            x1 = xs[n0 + vi.iy];
            x2 = (VD == 3) ? xs[n0 + n1 + vi.iz] : (T)0;
            w = ws[vi.ix] * ws[n0 + vi.iy] * ((VD == 3) ? ws[n0 + n1 + vi.iz] : (T)1);
            E = tabs[vi.ix] * tabs[n0 + vi.iy] * ((VD == 3) ? tabs[n0 + n1 + vi.iz] : (T)1);
            c0 = cs[vi.ix];
            c1 = cs[n0 + vi.iy];
            c2 = (VD == 3) ? cs[n0 + n1 + vi.iz] : (T)0;
        }
        const T cc = c0 * c0 + c1 * c1 + c2 * c2;
        T v0, v1 = (T)0;
        if (mode == 2) {
            v0 = fr[k];
            if (VD == 2) v1 = fr[nvp + k];
        } else if (mode == 0) {
            T Pf = (VD == 3) ? (T)fx[0] + (T)fx[1] * c0 + (T)fx[2] * c1 + (T)fx[3] * c2 + (T)fx[4] * cc
                             : (T)fx[0] + (T)fx[1] * c0 + (T)fx[2] * c1 + (T)fx[3] * cc;
            v0 = E * Pf;
            v1 = (T)Th * v0;
        } else {
            const T Q2 = (T)sg[0] * c0 * c0 + (T)sg[1] * c1 * c1 + (T)sg[2] * c2 * c2 +
                         (T)2 * ((T)sg[3] * c0 * c1 + (T)sg[4] * c0 * c2 + (T)sg[5] * c1 * c2);
            const T qd = (T)qg[0] * c0 + (T)qg[1] * c1 + (T)qg[2] * c2;
            const T Es = (T)A * E;
            if (VD == 3) {
                v0 = Es * ((T)1 + Q2 + qd * ((T)0.4 * cc * (T)it - (T)1));
            } else {
                v0 = Es * ((T)1 + Q2 + (T)Th * (T)sg[2] + qd * ((T)0.4 * cc * (T)it - (T)0.8));
                v1 = (T)Th * Es * ((T)1 + Q2 + (T)1.5 * Tg * (T)sg[2] + qd * ((T)0.4 * cc * (T)it - (T)0.4));
            }
        }
        if (mode != 2) {   // rows read by the next launches only: streaming stores
            __builtin_nontemporal_store(v0, &fr[k]);
            if (VD == 2) __builtin_nontemporal_store(v1, &fr[nvp + k]);
        }
        if (mode != 3) {   // ghost rows carry no sums
            acc_moments<T, VD>(acc, w, v0, v1, c0, c1, c2, cc);
#pragma unroll
            for (int j = 0; j < MAXW; ++j)
                if (j < nw) {
                    const T a = x0 * wn[j][0] + x1 * wn[j][1] + x2 * wn[j][2];
                    if (a > (T)0) wj[j] += w * a * v0;
                }
        }
        if constexpr (!PTS) vidx_step<VD>(vi, n1, (VD == 3) ? n2 : 1);
    }
#pragma unroll
    for (int j = 0; j < MAXW; ++j)
#pragma unroll
        for (int ww = 0; ww < MAXW; ++ww) acc[S_WALL + ww] += (j < nw && s_wi[j] == ww) ? wj[j] : (T)0;
    // zero the padding of this row once
    if (vt == 0 && mode != 2)
        for (int kp = C.nv + threadIdx.x; kp < nvp; kp += BLOCK) {
            fr[kp] = (T)0;
            if (VD == 2) fr[nvp + kp] = (T)0;
        }
    if (mode == 3) return;   // ghost rows carry no sums (block-uniform exit)
    double v[NSUM];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) v[i] = (double)acc[i];
    block_reduce_store<NSUM>(v, C.partial + ((size_t)slot * C.ntile + vt) * NSUM, red);
}

hipError_t launch_fill_poly(const CaseView *cv, const CaseView &h, int mode, int n_items, int cur, hipStream_t s);

// Grad-13 rows of the NS neighbours (mode 3 of k_fill) in the 16-byte-row
// plane layout: a lane keeps one y node and four z nodes and loops over the
// tile's x-planes.  f = A e^{-c^2/T} (1 + c.sigma.c/(pT) + (2/5) q.c/(pT)
// (c^2/T - 5/2)) with c = xi - u; the (y, z) parts of the Gaussian (with A),
// of c^2, of c.sigma.c and of q.c are lane constants formed in FP64 and
// rounded once, the x parts come from an LDS table per plane.  Ghost rows
// carry no sums.  Tiles cover whole x-planes.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ghost_rows_v4(const CaseView *__restrict__ cvp, int n_items)
{
    typedef T V4 __attribute__((ext_vector_type(4)));
    __shared__ T tcx[MAXA], tex[MAXA];
    const CaseView &C = *cvp;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_items, t = b - vt * n_items;
    const int cell = C.ghost_cell[t];
    const int slot = C.ghost_slot[cell];
    const double *g = C.ghost + (size_t)cell * GSIS_NMOM;
    const double rho = g[0], Tg = g[4], p = rho * Tg, it = 1.0 / Tg;
    const double A = rho * pow(M_PI * Tg, -1.5);
    double sg[6], qg[3];
    for (int d = 0; d < 6; ++d) sg[d] = g[5 + d] / (p * Tg);
    for (int d = 0; d < 3; ++d) qg[d] = 2.0 * g[11 + d] / (p * Tg);
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    for (int j = threadIdx.x; j < nx; j += BLOCK) {
        const double c = C.xv[j] - g[1];
        tcx[j] = (T)c;
        tex[j] = (T)exp(-c * c * it);
    }
    const int Q = nz >> 2, PL = ny * Q, G = BLOCK / PL;
    const int xg = threadIdx.x / PL, pr = threadIdx.x - xg * PL;
    const int iy = pr / Q, iz0 = 4 * (pr - iy * Q);
    const double cy = C.xv[MAXA + iy] - g[2];
    const double ey = A * exp(-cy * cy * it);
    T Eyz[4], CC[4], QL[4], QM[4], QD[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double cz = C.xv[2 * MAXA + iz0 + j] - g[3];
        Eyz[j] = (T)(ey * exp(-cz * cz * it));
        CC[j] = (T)(cy * cy + cz * cz);
        QL[j] = (T)(sg[1] * cy * cy + sg[2] * cz * cz + 2.0 * sg[5] * cy * cz);
        QM[j] = (T)(2.0 * (sg[3] * cy + sg[4] * cz));
        QD[j] = (T)(qg[1] * cy + qg[2] * cz);
    }
    const T s0 = (T)sg[0], q0 = (T)qg[0], itT = (T)it;
    __syncthreads();
    T *fr = (T *)C.grow + (size_t)slot * C.row;
    const int P2 = ny * nz;
    const int ix0 = (vt * C.tile) / P2, ix1 = min(nx, ((vt + 1) * C.tile) / P2);
    for (int ix = ix0 + xg; ix < ix1; ix += G) {
        const T c0 = tcx[ix], Ex = tex[ix];
        const T sc = s0 * c0;
        V4 out;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T cc = fma(c0, c0, CC[j]);
            const T Q2 = fma(sc, c0, fma(QM[j], c0, QL[j]));
            const T qd = fma(q0, c0, QD[j]);
            out[j] = (Ex * Eyz[j]) * ((T)1 + Q2 + qd * ((T)0.4 * cc * itT - (T)1));
        }
        __builtin_nontemporal_store(out, (V4 *)(fr + (size_t)ix * P2 + 4 * pr));
    }
}

hipError_t launch_fill(const CaseView *cv, const CaseView &h, int mode, int n_items, int cur, hipStream_t s)
{
    if (n_items <= 0) return hipSuccess;
    if (h.poly) return launch_fill_poly(cv, h, mode, n_items, cur, s);
    const int32_t *list = (mode == 1) ? h.new_cell : ((mode == 3) ? h.ghost_cell : h.kin_cell);
    if (mode == 0) {
        hipLaunchKernelGGL(k_feqpar, dim3((n_items + 63) / 64), dim3(64), 0, s, cv, n_items, list, 1);
        hipError_t e = launch_fix_pts(cv, h, n_items, list, 2, s);
        if (e != hipSuccess) return e;
    }
    int NA3 = h.n[0] + h.n[1] + (h.vdim == 3 ? h.n[2] : 0);
    dim3 g(n_items * h.ntile);
    // Grad-13 ghost rows in 16-byte rows on 3D tensor grids whose (y, z) plane
    // splits into 64-256 lanes of four z nodes and whose tiles cover whole
    // planes (GSIS_FILL_V4=0 keeps the node-per-thread kernel)
    static const bool fill_v4 = [] {
        const char *e = std::getenv("GSIS_FILL_V4");
        return !(e && e[0] == '0');
    }();
    const int P2 = h.n[1] * h.n[2];
    if (mode == 3 && fill_v4 && h.vdim == 3 && !h.points && h.n[2] % 4 == 0 && P2 / 4 >= 64 && P2 / 4 <= BLOCK &&
        BLOCK % (P2 / 4) == 0 && h.tile % P2 == 0) {
        if (h.dtype == GSIS_F32) hipLaunchKernelGGL((k_ghost_rows_v4<float>), g, dim3(BLOCK), 0, s, cv, n_items);
        else hipLaunchKernelGGL((k_ghost_rows_v4<double>), g, dim3(BLOCK), 0, s, cv, n_items);
        return hipGetLastError();
    }
    if (h.points) {
        if (h.dtype == GSIS_F32)
            hipLaunchKernelGGL((k_fill<float, 3, true>), g, dim3(BLOCK), 0, s, cv, list, n_items, mode, cur);
        else hipLaunchKernelGGL((k_fill<double, 3, true>), g, dim3(BLOCK), 0, s, cv, list, n_items, mode, cur);
        return hipGetLastError();
    }
    if (h.dtype == GSIS_F32) {
        size_t lds = sizeof(float) * NA3 * 4;
        if (h.vdim == 3)
            hipLaunchKernelGGL((k_fill<float, 3, false>), g, dim3(BLOCK), lds, s, cv, list, n_items, mode, cur);
        else hipLaunchKernelGGL((k_fill<float, 2, false>), g, dim3(BLOCK), lds, s, cv, list, n_items, mode, cur);
    } else {
        size_t lds = sizeof(double) * NA3 * 4;
        if (h.vdim == 3)
            hipLaunchKernelGGL((k_fill<double, 3, false>), g, dim3(BLOCK), lds, s, cv, list, n_items, mode, cur);
        else hipLaunchKernelGGL((k_fill<double, 2, false>), g, dim3(BLOCK), lds, s, cv, list, n_items, mode, cur);
    }
    return hipGetLastError();
}

hipError_t launch_ghost_rows(const CaseView *cv, const CaseView &h, int n_ghost, hipStream_t s)
{
    return launch_fill(cv, h, 3, n_ghost, 0, s);
}

// wall patches: M(1, u_w, T_w); far-field patches: M(rho, u, T) (FP64, rounded once)
template <typename T>
__global__ void k_patch_rows(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    const int p = blockIdx.y;
    const double *ps = C.patch_state + 5 * p;
    const double rho = (C.patch_kind[p] == GSIS_PATCH_WALL) ? 1.0 : ps[0];
    const double Tp = ps[4], it = 1.0 / Tp;
    const double amp = (C.vdim == 3) ? rho * pow(M_PI * Tp, -1.5) : rho / (M_PI * Tp);
    const int nvp = C.row / C.nfun;
    T *r = (T *)C.prow + (size_t)p * C.row;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nvp; k += gridDim.x * blockDim.x) {
        double v = 0.0;
        if (k < C.nv) {
            double xi[3], w;
            vnode(C, k, xi, w);
            double c0 = xi[0] - ps[1], c1 = xi[1] - ps[2];
            double c2 = (C.vdim == 3) ? xi[2] - ps[3] : 0.0;
            v = amp * exp(-(c0 * c0 + c1 * c1 + c2 * c2) * it);
        }
        r[k] = (T)v;
        if (C.vdim == 2) r[nvp + k] = (T)(0.5 * Tp * v);
    }
}

hipError_t launch_patch_rows(const CaseView *cv, const CaseView &h, hipStream_t s)
{
    if (h.n_patches <= 0) return hipSuccess;
    int nvp = h.row / h.nfun;
    dim3 g((nvp + 255) / 256 < 256 ? (nvp + 255) / 256 : 256, h.n_patches);
    if (h.dtype == GSIS_F32) hipLaunchKernelGGL(k_patch_rows<float>, g, dim3(256), 0, s, cv);
    else hipLaunchKernelGGL(k_patch_rows<double>, g, dim3(256), 0, s, cv);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dense <-> slot-row copies of the VDF (dir 0: workspace -> out, 1: in -> workspace)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gather(const CaseView *__restrict__ cvp, int n_kin, int cur, T *dense, int dir)
{
    const CaseView &C = *cvp;
    const int t = blockIdx.y;
    const int slot = C.slot_of_cell[C.kin_cell[t]];
    const int nvp = C.row / C.nfun;
    T *row = (T *)C.f[cur] + (size_t)slot * C.row;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < C.nfun * C.nv; i += gridDim.x * blockDim.x) {
        int fun = i / C.nv, k = i - fun * C.nv;
        T *d = dense + ((size_t)t * C.nfun + fun) * C.nv + k;
        if (dir == 0) *d = row[fun * nvp + k];
        else row[fun * nvp + k] = *d;
    }
    if (dir == 1 && blockIdx.x == 0)
        for (int fun = 0; fun < C.nfun; ++fun)
            for (int k = C.nv + threadIdx.x; k < nvp; k += blockDim.x) row[fun * nvp + k] = (T)0;
}

hipError_t launch_gather_vdf(const CaseView *cv, const CaseView &h, int n_kin, int cur, void *out, int dir,
                             hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    int gx = (h.nfun * h.nv + 255) / 256;
    if (gx > 64) gx = 64;
    dim3 g(gx, n_kin);
    if (h.dtype == GSIS_F32) hipLaunchKernelGGL(k_gather<float>, g, dim3(256), 0, s, cv, n_kin, cur, (float *)out, dir);
    else hipLaunchKernelGGL(k_gather<double>, g, dim3(256), 0, s, cv, n_kin, cur, (double *)out, dir);
    return hipGetLastError();
}

}  // namespace gsis
