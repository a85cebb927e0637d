// gsis_sweep.hip -- the kinetic sweep of Sec. 3.1 for tensor grids whose
// fastest velocity axis divides the block (the bandwidth-bound hot kernel).
//
// Same update and same outputs as the generic k_sweep (gsis_kinetic.hip):
//   f_i^{n+1/2} = (g_i/tau_i + sum_{a<0} |a| f_j^n) / (1/tau_i + sum_{a>0} a),
//   a = (xi.n) S/V, upwind values from kinetic neighbours, Grad-13 ghosts,
//   diffuse walls or the far field; fused moment, moment-balance and wall sums.
// Every face is a row times a wave-uniform scale: a kinetic neighbour's row of
// f^n, the Grad-13 row of an NS neighbour (built once per sweep), or the
// patch Maxwellian row (built at bind) scaled by the wall density rho_w or 1.
//
// gfx950 mapping.  One block of 256 threads = one (kinetic cell, tile of
// whole x-planes (3D) or x-lines (reduced 2D)).  Because the fastest axis
// (z in 3D, y in 2D) divides 256, every lane keeps the same fastest-axis node
// for all its points: that axis's Gaussian factor, offsets and each face's
// contribution to xi.n are lane constants, and the moment sums only need
// powers of the varying offsets (the lane constant is multiplied in once, in
// FP64, at the end).  Per-axis records (offset c, Gaussian factor E, fix-up
// polynomial part P, Shakhov part K, weight w) are built in FP64 and held in
// LDS.  Face data and neighbour-row bases are wave-uniform (SGPRs); all loads
// of a point are issued before any is consumed.  NF (4 or 8) bounds the faces
// per cell; absent faces read the cell's own row with a zero normal.
#include <math.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "gsis_impl.hpp"

namespace gsis {

// waves per SIMD the FP32 plane kernels are compiled for (caps their VGPRs at
// 512 / waves); the FP64 instantiations are left unconstrained (no spills)
#ifndef SWEEP_WAVES
#define SWEEP_WAVES 4
#endif
#ifndef CORRECT_WAVES
#define CORRECT_WAVES 4
#endif
// largest points per load round of the correction (two planes per pass)
#ifndef CORRECT_UMAX
#define CORRECT_UMAX 2
#endif


namespace {

template <typename T>
using gcptr = const __attribute__((address_space(1))) T *;
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

// a wave-uniform pointer held in SGPRs (the value is the same in every lane)
template <typename P>
__device__ __forceinline__ P uniform_ptr(P p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P)(((uint64_t)hi << 32) | lo);
}

// loads and stores at a 32-bit byte offset from a wave-uniform base (the
// SGPR-base, VGPR-offset addressing form: no 64-bit address arithmetic per access)
template <typename T>
__device__ __forceinline__ T ldb(gcptr<T> p, uint32_t off)
{
    return *(gcptr<T>)((const __attribute__((address_space(1))) char *)p + off);
}
template <typename T>
__device__ __forceinline__ void stb(gptr<T> p, uint32_t off, T v)
{
    // streaming store: the written row is not read again by this launch, so
    // it should not displace neighbour rows from L2
    __builtin_nontemporal_store(v, (gptr<T>)((__attribute__((address_space(1))) char *)p + off));
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// byte offset of the epilogue's LDS area after `tab` table elements of T
template <typename T>
__host__ __device__ constexpr size_t red_offset(size_t tab)
{
    return (sizeof(T) * tab + 15) / 16 * 16;
}

// bytes of the epilogue's LDS area: the raw lane sums, then (reused) the
// per-node partial sums
template <typename T, int NF>
constexpr size_t red_bytes()
{
    return (sizeof(T) * (17 + NF) * BLOCK > sizeof(double) * NSUM * BLOCK / 2)
               ? sizeof(T) * (17 + NF) * BLOCK
               : sizeof(double) * NSUM * BLOCK / 2;
}

// Per-lane moment sums of the plane kernels.  3D: with c_z the lane constant
// and (c_x, c_y) varying, sum_k w f c_x^a c_y^b is kept for the (a, b) the
// moments need; A* = (a, 0), B* = (0, b), C1 = (1, 1), C2 = (2, 1), D2 = (1, 2).
// Reduced 2D (lane constant c_y): A* powers of c_x on phi, Q* on psi.
// R* = moment balance w (num - den f_old) (1, c_x, c_y, c^2 parts), Rp its psi.
template <typename T>
struct PlaneSums {
    T A0 = 0, A1 = 0, A2 = 0, A3 = 0, B1 = 0, B2 = 0, B3 = 0, C1 = 0, C2 = 0, D2 = 0;
    T Q0 = 0, Q1 = 0;
    T R0 = 0, R1 = 0, R2 = 0, R3 = 0, Rp = 0;

    // fold one x-plane's sums of powers of c_y (T*) and its balance sums (S*):
    // x powers from the records, compensated by their low parts
    __device__ __forceinline__ void fold(T cx, T clo, T c2, T c2lo, T c3, T c3lo, T T0, T T1, T T2, T T3, T S0,
                                         T S1, T S2)
    {
        A0 += T0;
        A1 += cx * T0 + clo * T0;
        A2 += c2 * T0 + c2lo * T0;
        A3 += c3 * T0 + c3lo * T0;
        B1 += T1;
        B2 += T2;
        B3 += T3;
        C1 += cx * T1 + clo * T1;
        C2 += c2 * T1 + c2lo * T1;
        D2 += cx * T2 + clo * T2;
        R0 += S0;
        R1 += cx * S0 + clo * S0;
        R2 += S1;
        R3 += c2 * S0 + c2lo * S0 + S2;
    }
};

// Block epilogue.  Lanes that share the fastest-axis node (lane constant)
// first pool their raw sums: every lane writes its 17 + NF FP32 sums to LDS,
// then one thread per node adds its lanes' values in FP64, multiplies in the
// node's offset cl and weight wl, maps to the NSUM layout of the partial sums
// (with the outgoing wall sums of the faces), and the nodes are added in a
// fixed order.  red must hold (17 + NF) * BLOCK values of T and
// NSUM * n_node doubles (it is reused between the two stages).
template <typename T, int VD, int NF>
__device__ __forceinline__ void finish_partials(const PlaneSums<T> &S, const T (&Wf)[NF], const int (&fwall)[NF],
                                                int n_node, const double *xl, const double *wlv, double ul,
                                                double *out, T *red)
{
    constexpr int K = 17 + NF;
    const int tid = threadIdx.x;
    {
        const T raw[17] = {S.A0, S.A1, S.A2, S.A3, S.B1, S.B2, S.B3, S.C1, S.C2, S.D2,
                           S.Q0, S.Q1, S.R0, S.R1, S.R2, S.R3, S.Rp};
#pragma unroll
        for (int k = 0; k < 17; ++k) red[k * BLOCK + tid] = raw[k];
#pragma unroll
        for (int l = 0; l < NF; ++l) red[(17 + l) * BLOCK + tid] = Wf[l];
    }
    __syncthreads();
    double v[NSUM];
    if (tid < n_node) {
        double r[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double acc = 0.0;
            for (int ln = tid; ln < BLOCK; ln += n_node) acc += (double)red[k * BLOCK + ln];
            r[k] = acc;
        }
        const double cl = xl[tid] - ul, wl = wlv[tid], cl2 = cl * cl;
#pragma unroll
        for (int i = 0; i < NSUM; ++i) v[i] = 0.0;
        const double a0 = r[0], a1 = r[1], a2 = r[2], a3 = r[3];
        if (VD == 3) {
            const double b1 = r[4], b2 = r[5], b3 = r[6], c1 = r[7], c2 = r[8], d2 = r[9];
            v[0] = wl * a0;
            v[1] = wl * a1;
            v[2] = wl * b1;
            v[3] = wl * cl * a0;
            v[4] = wl * a2;
            v[5] = wl * b2;
            v[6] = wl * cl2 * a0;
            v[7] = wl * c1;
            v[8] = wl * cl * a1;
            v[9] = wl * cl * b1;
            v[10] = wl * (a3 + d2 + cl2 * a1);
            v[11] = wl * (c2 + b3 + cl2 * b1);
            v[12] = wl * cl * (a2 + b2 + cl2 * a0);
            v[S_RES] = wl * r[12];
            v[S_RES + 1] = wl * r[13];
            v[S_RES + 2] = wl * r[14];
            v[S_RES + 3] = wl * cl * r[12];
            v[S_RES + 4] = wl * (r[15] + cl2 * r[12]);
        } else {
            v[0] = wl * a0;
            v[1] = wl * a1;
            v[2] = wl * cl * a0;
            v[3] = wl * a2;
            v[4] = wl * cl2 * a0;
            v[5] = wl * cl * a1;
            v[6] = wl * (a3 + cl2 * a1);
            v[7] = wl * cl * (a2 + cl2 * a0);
            v[8] = wl * r[10];
            v[9] = wl * r[11];
            v[10] = wl * cl * r[10];
            v[S_RES] = wl * r[12];
            v[S_RES + 1] = wl * r[13];
            v[S_RES + 2] = wl * cl * r[12];
            v[S_RES + 4] = wl * (r[15] + cl2 * r[12] + r[16]);
        }
#pragma unroll
        for (int q2 = 0; q2 < MAXW; ++q2) {
            double sw = 0.0;
#pragma unroll
            for (int l = 0; l < NF; ++l) sw += (fwall[l] == q2) ? r[17 + l] : 0.0;
            v[S_WALL + q2] = wl * sw;
        }
    }
    __syncthreads();
    double *vd = (double *)red;
    if (tid < n_node)
#pragma unroll
        for (int i = 0; i < NSUM; ++i) vd[i * n_node + tid] = v[i];
    __syncthreads();
    if (tid < NSUM) {
        double acc = 0.0;
        for (int z = 0; z < n_node; ++z) acc += vd[tid * n_node + z];
        out[tid] = acc;
    }
}

}  // namespace

template <typename T, int VD, int NF, int U>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? SWEEP_WAVES : 1))) void
k_sweep_fast(Batch B)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];

    // ---- locate the work item -------------------------------------------
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int ci = 0;
    while (ci + 1 < B.n && b >= B.start[ci + 1]) ++ci;
    const CaseView &C = *B.cv[ci];
    const int cur = B.cur[ci];
    const int item = b - B.start[ci];
    const int n_kin = (B.start[ci + 1] - B.start[ci]) / C.ntile;
    int vt, t;
    if (B.order == 2) {   // groups of G consecutive cells, tile-major inside a group
        const int G = B.group;
        const int gi = item / (G * C.ntile);
        const int r = item - gi * G * C.ntile;
        const int gc = min(G, n_kin - gi * G);
        vt = r / gc;
        t = gi * G + (r - vt * gc);
    } else if (B.order) {   // cell-major: the tiles of one cell are consecutive
        t = item / C.ntile;
        vt = item - t * C.ntile;
    } else {         // tile-major
        vt = item / n_kin;
        t = item - vt * n_kin;
    }
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const int nx = C.n[0], ny = C.n[1], nz = (VD == 3) ? C.n[2] : 1;
    const int NA = nx + ny + ((VD == 3) ? nz : 0);
    const size_t row = (size_t)C.row;
    const int nvp = C.row / ((VD == 3) ? 1 : 2);
    gcptr<T> fold = (gcptr<T>)C.f[cur];
    gptr<T> fn = (gptr<T>)C.f[cur ^ 1] + (size_t)slot * row;
    gcptr<T> fo = fold + (size_t)slot * row;

    // ---- LDS: per-axis records of the own target ---------------------------
    T *rc = (T *)smem_raw;       // offset x_j - u_d
    T *rE = rc + NA;             // exp(-c^2 / T)
    T *rP = rE + NA;             // fix-up polynomial part of the axis
    T *rK = rP + NA;             // Shakhov part kq_d c
    T *rw = rK + NA;             // weight
    T *rlo = rw + NA;            // x axis: low part of c, c^2 and its low part, c^3 and its low part
    const size_t red_off = red_offset<T>((size_t)5 * NA + 5 * nx);

    // ---- wave-uniform face data: row, scale, (n S/V), u.n S/V ----------------
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    int fwall[NF];
    T fnx[NF], fny[NF], fnz[NF], fun[NF], fsc[NF];
    gcptr<T> fnb[NF];
    int nw = 0;
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fwall[l] = -1;
        fnx[l] = fny[l] = fnz[l] = fun[l] = (T)0;
        fsc[l] = (T)0;
        fnb[l] = fo;
        if (l < nf) {
            const int e = e0 + l;
            const int oth = C.cf_other[e];
            const double n0 = C.cf_nsv[3 * e], n1 = C.cf_nsv[3 * e + 1], n2 = C.cf_nsv[3 * e + 2];
            fnx[l] = (T)n0;
            fny[l] = (T)n1;
            fnz[l] = (T)n2;
            fun[l] = (T)(P.u[0] * n0 + P.u[1] * n1 + P.u[2] * n2);   // xi.n S/V = c.n S/V + u.n S/V
            fwall[l] = C.cf_wall[e];
            nw += (fwall[l] >= 0);
            fsc[l] = (T)1;
            if (oth >= 0) {
                const int so = C.slot_of_cell[oth];
                fnb[l] = (so >= 0) ? fold + (size_t)so * row
                                   : (gcptr<T>)C.grow + (size_t)C.ghost_slot[oth] * row;
            } else {
                const int pi = -1 - oth;
                fnb[l] = (gcptr<T>)C.prow + (size_t)pi * row;
                if (fwall[l] >= 0) fsc[l] = (T)P.rw[fwall[l]];
            }
        }
    }
    // own-target records: the slot's axis tables (built once per sweep) and weights
    {
        gcptr<T> tb = (gcptr<T>)C.axtab + (size_t)slot * C.tabp;
        for (int j = threadIdx.x; j < 4 * NA; j += BLOCK) rc[j] = tb[j];      // rc, rE, rP, rK
        for (int j = threadIdx.x; j < 5 * nx; j += BLOCK) rlo[j] = tb[4 * NA + j];
        for (int j = threadIdx.x; j < NA; j += BLOCK) {
            const int d = (j < nx) ? 0 : ((j < nx + ny) ? 1 : 2);
            const int jj = j - ((d == 0) ? 0 : ((d == 1) ? nx : nx + ny));
            rw[j] = (T)C.wv[d * MAXA + jj];
        }
    }
    __syncthreads();

    // ---- constants --------------------------------------------------------
    const T it = (T)P.it, Th = (T)P.Th, itau = (T)P.itau, idt = (T)C.inv_dt;
    const T shift0 = (VD == 3) ? (T)2.5 : (T)2, shift1 = (T)1;

    // lane-constant (fastest axis) data
    const int ilc = (VD == 3) ? (int)(threadIdx.x % nz) : (int)(threadIdx.x % ny);
    const int jlc = (VD == 3) ? nx + ny + ilc : nx + ilc;
    const T cL = rc[jlc], EL = rE[jlc], PL = rP[jlc], KL = rK[jlc];
    T AL[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) AL[l] = ((VD == 3) ? fnz[l] : fny[l]) * cL + fun[l];

    // per-lane accumulators
    PlaneSums<T> S;
    T Wf[NF];   // outgoing wall sums
#pragma unroll
    for (int l = 0; l < NF; ++l) Wf[l] = (T)0;

    if (VD == 3) {
        // ---- 3D: lanes own z = ilc; loop x-planes, then the M y-values ----
        // Node k = (ix ny + iy) nz + ilc with iy = yq + m q and q nz = BLOCK, so
        // k = ix ny nz + tid + m BLOCK: every row is addressed by one 32-bit
        // byte offset per round from a wave-uniform base (point u of the round
        // at +u BLOCK elements).
        const int q = BLOCK / nz;
        const int M = ny / q;
        const int yq = threadIdx.x / nz;
        const int ix0 = vt * C.xp, ix1 = min(ix0 + C.xp, nx);
        const uint32_t plane_bytes = (uint32_t)(ny * nz * sizeof(T));
        const uint32_t lane_bytes = (uint32_t)(threadIdx.x * sizeof(T));
        constexpr uint32_t ustep = BLOCK * sizeof(T);
        // the diagonal 1/dt + 1/tau + sum_{a>0} a is written 1/dt + 1/tau - sum_{a<0} a
        // (the cell is closed: sum_l n_l S_l = 0)
        const T den0 = itau + idt;
        gcptr<T> fo_u = uniform_ptr(fo);
        gptr<T> fn_u = uniform_ptr(fn);
        gcptr<T> fnb_u[NF];
#pragma unroll
        for (int l = 0; l < NF; ++l) fnb_u[l] = uniform_ptr(fnb[l]);
        auto planes = [&](auto walls) {
            constexpr bool WALLS = decltype(walls)::value;
            for (int ix = ix0; ix < ix1; ++ix) {
                const T cx = rc[ix], wx = rw[ix];
                const T Exz = itau * rE[ix] * EL, Pxz = rP[ix] + PL, Kxz = rK[ix] + KL;
                const T Axz = (cx * cx + cL * cL) * it - shift0;
                T Ax[NF];
#pragma unroll
                for (int l = 0; l < NF; ++l) Ax[l] = fnx[l] * cx + AL[l];
                T T0 = 0, T1 = 0, T2 = 0, T3 = 0, Z0 = 0, Z1 = 0, Z2 = 0;   // this plane
                uint32_t off = ix * plane_bytes + lane_bytes;
                int jy0 = nx + yq;
                for (int m = 0; m < M; m += U, off += U * ustep, jy0 += U * q) {
                    // every load of the round is in flight before the first is consumed
                    T o[U], v[U][NF];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        o[u] = ldb(fo_u, off + u * ustep);
#pragma unroll
                        for (int l = 0; l < NF; ++l) v[u][l] = ldb(fnb_u[l], off + u * ustep);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int jy = jy0 + u * q;
                        const T cy = rc[jy], Ey = rE[jy], Py = rP[jy], Ky = rK[jy], wy = rw[jy];
                        // relaxation target (1/tau folded into the x-z factor)
                        const T g = Exz * Ey * (Pxz + Py) * ((Kxz + Ky) * (Axz + cy * cy * it) + (T)1);
                        T num = g + idt * o[u];
                        T den = den0;
                        T aw[NF];
#pragma unroll
                        for (int l = 0; l < NF; ++l) {
                            const T a = fny[l] * cy + Ax[l];
                            const T mn = fmin(a, (T)0);
                            den -= mn;
                            if constexpr (WALLS) {
                                aw[l] = a - mn;                      // max(a, 0)
                                num -= (mn * fsc[l]) * v[u][l];
                            } else {
                                num -= mn * v[u][l];
                            }
                        }
                        const T fnv = num * fast_rcp(den);
                        stb(fn_u, off + u * ustep, fnv);
                        // moment sums: powers of c_y only
                        const T w = wx * wy;
                        const T h = w * fnv;
                        T0 += h;
                        const T hy = h * cy;
                        T1 += hy;
                        const T hy2 = hy * cy;
                        T2 += hy2;
                        T3 += hy2 * cy;
                        const T r = w * (num - den * o[u]);
                        Z0 += r;
                        const T ry = r * cy;
                        Z1 += ry;
                        Z2 += ry * cy;
                        if constexpr (WALLS) {
#pragma unroll
                            for (int l = 0; l < NF; ++l)
                                if (fwall[l] >= 0) Wf[l] += h * aw[l];
                        }
                    }
                }
                S.fold(cx, rlo[ix], rlo[nx + ix], rlo[2 * nx + ix], rlo[3 * nx + ix], rlo[4 * nx + ix], T0, T1, T2,
                       T3, Z0, Z1, Z2);
            }
        };
        if (nw > 0) planes(std::true_type{});
        else planes(std::false_type{});
    } else {
        // ---- reduced 2D: lanes own y = ilc; x varies per step --------------
        const int q = BLOCK / ny;
        const int xq = threadIdx.x / ny;
        const int ix0 = vt * C.xp, ix1 = min(ix0 + C.xp, nx);
        for (int ixr = ix0 + xq; ixr < ix1; ixr += U * q) {
          // U lines per round, loads first (lines past the tile are skipped)
          T o0u[U], o1u[U], v0u[U][NF], v1u[U][NF];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int ix = ixr + u * q;
            const int k = ix * ny + ilc;
            if (ix < ix1) {
                o0u[u] = fo[k];
                o1u[u] = fo[nvp + k];
#pragma unroll
                for (int l = 0; l < NF; ++l) {
                    v0u[u][l] = fnb[l][k];
                    v1u[u][l] = fnb[l][nvp + k];
                }
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int ix = ixr + u * q;
            if (ix >= ix1) break;
            const int k = ix * ny + ilc;
            const T o0 = o0u[u], o1 = o1u[u];
            const T *v0 = v0u[u], *v1 = v1u[u];
            const T cx = rc[ix], Ex = rE[ix], Px = rP[ix], Kx = rK[ix], wx = rw[ix];
            const T cc = cx * cx + cL * cL;
            const T EP = Ex * EL * (Px + PL);
            const T Kc = Kx + KL;
            const T g0 = EP * (Kc * (cc * it - shift0) + (T)1);
            const T g1 = Th * EP * (Kc * (cc * it - shift1) + (T)1);
            T num0 = itau * g0 + idt * o0, num1 = itau * g1 + idt * o1;
            T den = itau + idt;
#pragma unroll
            for (int l = 0; l < NF; ++l) {
                const T a = fnx[l] * cx + AL[l];
                den += fmax(a, (T)0);
                const T mn = fmin(a, (T)0) * fsc[l];
                num0 -= mn * v0[l];
                num1 -= mn * v1[l];
            }
            const T rd = fast_rcp(den);
            const T f0 = num0 * rd, f1 = num1 * rd;
            fn[k] = f0;
            fn[nvp + k] = f1;
            const T h = wx * f0;
            S.A0 += h;
            const T hx = h * cx;
            S.A1 += hx;
            const T hx2 = hx * cx;
            S.A2 += hx2;
            S.A3 += hx2 * cx;
            const T hp = wx * f1;
            S.Q0 += hp;
            S.Q1 += hp * cx;
            const T r = wx * (num0 - den * o0);
            S.R0 += r;
            const T rx1 = r * cx;
            S.R1 += rx1;
            S.R3 += rx1 * cx;
            S.Rp += wx * (num1 - den * o1);
            if (nw > 0) {
#pragma unroll
                for (int l = 0; l < NF; ++l)
                    if (fwall[l] >= 0) Wf[l] += h * fmax(fnx[l] * cx + AL[l], (T)0);
            }
          }
        }
    }

    // ---- per-lane constants in FP64, standard partial-sum layout ----------
    const int dl = (VD == 3) ? 2 : 1;
    finish_partials<T, VD, NF>(S, Wf, fwall, (VD == 3) ? nz : ny, C.xv + dl * MAXA, C.wv + dl * MAXA, P.u[dl],
                               C.partial + ((size_t)slot * C.ntile + vt) * NSUM, (T *)(smem_raw + red_off));
}

// ---------------------------------------------------------------------------
// The same sweep on 3D tensor grids whose (y, z) plane splits into 64..256
// lanes of four consecutive z nodes (n_z % 4 == 0, 64 <= n_y n_z / 4 <= 256,
// and n_y n_z / 4 divides 256): the row layout of the plane kernel above, read
// and written as 16-byte vectors (four nodes per lane), with the lane's four
// (y, z) nodes fixed for the whole row and the x-planes looped over.
//
// Per lane, everything that depends on (y, z) only is formed once in FP64:
// the Gaussian factor exp(-(c_y^2 + c_z^2)/T)/tau, the (y, z) parts of the
// fix-up and Shakhov polynomials, and each face's (n_y c_y + n_z c_z + u.n) S/V.
// Per x-plane, the block reads one record from LDS (c_x, its Gaussian, fix-up
// and Shakhov parts, c_x^2/T and the weighted powers w_x c_x^a); the moment
// and balance sums of a node are then four FMAs each.  A face whose
// (xi.n) S/V is >= 0 on every node of a wave's patch of the plane brings
// nothing in: the wave skips its row load and arithmetic (exactly: its
// min(a, 0) is 0 on every node).  Lanes keep FP32 sums over the planes per
// node; the epilogue forms each lane's partial sums in FP64 with its (y, z)
// offsets and weights and reduces them over the block in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec4T;
template <>
struct Vec4T<float> {
    typedef float v __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4T<double> {
    typedef double v __attribute__((ext_vector_type(4)));
};

// per-x-plane record of the v4 sweep (LDS): c, E, P, K, c^2/T, w, w c, w c^2, w c^3
constexpr int XREC = 12;

// one DPP lane move of an FP64 value (both halves; ctrl selects the pattern)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over each 16-lane row, left in every lane of the row: pairs (quad_perm
// 1,0,3,2), quads (2,3,0,1), half rows (row_half_mirror), rows (row_mirror).
// Partners add the same two values, so every lane of a group holds the same
// bits at each level and the order of the additions is fixed.
__device__ __forceinline__ double row_sum16(double x)
{
    x += dpp_f64<0xB1>(x);
    x += dpp_f64<0x4E>(x);
    x += dpp_f64<0x141>(x);
    x += dpp_f64<0x140>(x);
    return x;
}

__device__ __forceinline__ float wave_min(float x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ double wave_min(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o));
    return x;
}

// a value equal in every lane, moved to scalar registers
__device__ __forceinline__ float to_uniform(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double to_uniform(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Block sums of N per-lane FP64 values: DPP row sums of 16 lanes, then the
// block's rows added in a fixed order by thread i < N into out[i].  red holds
// (BLOCK / 16) N doubles; it is free again after the call.
template <int N>
__device__ __forceinline__ void v4_block_sums(const double (&x)[N], double *red, double *out)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();   // red may still be read by an earlier reduction
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double v = row_sum16(x[i]);
        if ((lane & 15) == 0) red[(wave * 4 + (lane >> 4)) * N + i] = v;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double acc = 0.0;
        for (int r = 0; r < BLOCK / 16; ++r) acc += red[r * N + threadIdx.x];
        out[threadIdx.x] = acc;
    }
}

// Epilogue of the 16-byte-row plane kernels.  A lane holds, per node j of its
// four z nodes, FP32 sums over the x-planes of w_x c_x^a f (a = 0..3) in S0..S3,
// the sweep's balance sums in R0..R2 (zero for the correction) and, for cells
// with wall faces, the outgoing wall sums with weight w_x w_z in Wf.  They
// become FP64 partials with the lane's (y, z) offsets, reduced over the wave
// with DPP row sums and over the block's rows in a fixed order, and the NSUM
// partial sums of the (slot, tile) are written to out.
template <typename T, int NF, bool WALLS>
__device__ __forceinline__ void v4_partials(const T (&S0)[4], const T (&S1)[4], const T (&S2)[4], const T (&S3)[4],
                                            const T (&R0)[4], const T (&R1)[4], const T (&R2)[4],
                                            const T (&Wf)[NF], const int (&fwall)[NF], const CaseView &C,
                                            double uz, double cyd, int iy, int iz0, double *red, double *out)
{
    // ---- epilogue: the lane's FP64 partial sums, one at a time, each
    // reduced over the wave in a fixed order; then the waves in order
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double wyd = C.wv[MAXA + iy];
    double wj[4], czj[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        czj[j] = C.xv[2 * MAXA + iz0 + j] - uz;
        wj[j] = wyd * C.wv[2 * MAXA + iz0 + j];
    }
    // row sums (DPP) of 16 lanes, written by the first lane of each row;
    // the 16 rows of the block are added in order below
    auto put = [&](int i, double x) {
        x = row_sum16(x);
        if ((lane & 15) == 0) red[(wave * 4 + (lane >> 4)) * NSUM + i] = x;
    };
    double a, b2, c2, d;
    // mass, and the y moments that are lane constants times it
    a = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) a += wj[j] * (double)S0[j];
    put(0, a);
    put(2, cyd * a);
    put(5, cyd * cyd * a);
    // x moments
    b2 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) b2 += wj[j] * (double)S1[j];
    put(1, b2);
    put(7, cyd * b2);
    c2 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) c2 += wj[j] * (double)S2[j];
    put(4, c2);
    // z moments
    a = 0.0;
    d = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a += wj[j] * czj[j] * (double)S0[j];
        d += wj[j] * czj[j] * czj[j] * (double)S0[j];
    }
    put(3, a);
    put(9, cyd * a);
    put(6, d);
    a = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) a += wj[j] * czj[j] * (double)S1[j];
    put(8, a);
    // heat-flux sums c^2 c_d
    a = 0.0;
    d = 0.0;
    b2 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double yz2 = cyd * cyd + czj[j] * czj[j];
        const double e2 = wj[j] * ((double)S2[j] + yz2 * (double)S0[j]);
        a += wj[j] * ((double)S3[j] + yz2 * (double)S1[j]);
        d += e2;
        b2 += czj[j] * e2;
    }
    put(10, a);
    put(11, cyd * d);
    put(12, b2);
    // moment balance
    a = 0.0;
    d = 0.0;
    b2 = 0.0;
    c2 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double yz2 = cyd * cyd + czj[j] * czj[j];
        a += wj[j] * (double)R0[j];
        d += wj[j] * (double)R1[j];
        b2 += wj[j] * czj[j] * (double)R0[j];
        c2 += wj[j] * ((double)R2[j] + yz2 * (double)R0[j]);
    }
    put(S_RES, a);
    put(S_RES + 1, d);
    put(S_RES + 2, cyd * a);
    put(S_RES + 3, b2);
    put(S_RES + 4, c2);
    // outgoing wall fluxes (weights w_x w_z in the sums, w_y here)
#pragma unroll
    for (int q2 = 0; q2 < MAXW; ++q2) {
        double sw = 0.0;
        if (WALLS) {
#pragma unroll
            for (int l = 0; l < NF; ++l) sw += (fwall[l] == q2) ? (double)Wf[l] : 0.0;
        }
        put(S_WALL + q2, wyd * sw);
    }
    for (int i = S_WALL + MAXW; i < NSUM; ++i) put(i, 0.0);
    __syncthreads();
    if (threadIdx.x < NSUM) {
        double acc = 0.0;
        for (int r = 0; r < BLOCK / 16; ++r) acc += red[r * NSUM + threadIdx.x];
        out[threadIdx.x] = acc;
    }
}

// waves per SIMD of the FP32 16-byte-row sweep (up to 4 faces per cell: 150
// VGPRs without spills at 3; 8 faces take 2)
#ifndef SWEEP_V4_WAVES
#define SWEEP_V4_WAVES 3
#endif
#ifndef SWEEP_V4_U
#define SWEEP_V4_U 2
#endif
template <typename T, int NF, int U>
__global__ __launch_bounds__(BLOCK) __attribute__((
    amdgpu_waves_per_eu(sizeof(T) == 4 ? (NF <= 4 ? SWEEP_V4_WAVES : 2) : 1))) void k_sweep_v4(Batch B)
{
    typedef typename Vec4T<T>::v V4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // ---- locate the work item (as the plane kernel) -------------------------
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int ci = 0;
    while (ci + 1 < B.n && b >= B.start[ci + 1]) ++ci;
    const CaseView &C = *B.cv[ci];
    const int cur = B.cur[ci];
    const int item = b - B.start[ci];
    const int n_kin = (B.start[ci + 1] - B.start[ci]) / C.ntile;
    int vt, t;
    if (B.order == 2) {
        const int G = B.group;
        const int gi = item / (G * C.ntile);
        const int r = item - gi * G * C.ntile;
        const int gc = min(G, n_kin - gi * G);
        vt = r / gc;
        t = gi * G + (r - vt * gc);
    } else if (B.order) {
        t = item / C.ntile;
        vt = item - t * C.ntile;
    } else {
        vt = item / n_kin;
        t = item - vt * n_kin;
    }
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    const size_t row = (size_t)C.row;
    gcptr<T> fold = (gcptr<T>)C.f[cur];
    gptr<T> fn = (gptr<T>)C.f[cur ^ 1] + (size_t)slot * row;
    gcptr<T> fo = fold + (size_t)slot * row;

    // lane -> (x group, y, first of four z nodes)
    const int Q = nz >> 2, PL = ny * Q, G = BLOCK / PL;
    const int xg = threadIdx.x / PL, pr = threadIdx.x - xg * PL;
    const int iy = pr / Q, iz0 = 4 * (pr - iy * Q);

    // ---- LDS: per-plane records, from the slot's axis tables ----------------
    // (offset c, Gaussian factor, fix-up and Shakhov parts, each formed in FP64
    // and rounded once per sweep) and the weighted powers of c
    const int NA = nx + ny + nz;
    gcptr<T> tb = (gcptr<T>)C.axtab + (size_t)slot * C.tabp;
    T *xr = (T *)smem_raw;
    double *red = (double *)(smem_raw + red_offset<T>((size_t)XREC * nx));
    {
        const double ux = P.u[0], it = P.it;
        for (int j = threadIdx.x; j < nx; j += BLOCK) {
            const double c = C.xv[j] - ux, w = C.wv[j];
            T *r = xr + XREC * j;
            r[0] = tb[j];
            r[1] = tb[NA + j];
            r[2] = tb[2 * NA + j];
            r[3] = tb[3 * NA + j];
            r[4] = (T)(c * c * it);
            r[5] = (T)w;
            r[6] = (T)(w * c);
            r[7] = (T)(w * c * c);
            r[8] = (T)(w * c * c * c);
        }
    }

    // ---- faces: row bases (wave-uniform), scales, normals ------------------
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    int fwall[NF];
    T fnx[NF], fsc[NF];
    double fny[NF], fnz[NF], fun[NF];
    gcptr<T> fnb[NF];
    int nw = 0;
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fwall[l] = -1;
        fnx[l] = (T)0;
        fny[l] = fnz[l] = fun[l] = 0.0;
        fsc[l] = (T)0;
        fnb[l] = fo;
        if (l < nf) {
            const int e = e0 + l;
            const int oth = C.cf_other[e];
            const double n0 = C.cf_nsv[3 * e], n1 = C.cf_nsv[3 * e + 1], n2 = C.cf_nsv[3 * e + 2];
            fnx[l] = (T)n0;
            fny[l] = n1;
            fnz[l] = n2;
            fun[l] = P.u[0] * n0 + P.u[1] * n1 + P.u[2] * n2;   // xi.n S/V = c.n S/V + u.n S/V
            fwall[l] = C.cf_wall[e];
            nw += (fwall[l] >= 0);
            fsc[l] = (T)1;
            if (oth >= 0) {
                const int so = C.slot_of_cell[oth];
                fnb[l] = (so >= 0) ? fold + (size_t)so * row : (gcptr<T>)C.grow + (size_t)C.ghost_slot[oth] * row;
            } else {
                const int pi = -1 - oth;
                fnb[l] = (gcptr<T>)C.prow + (size_t)pi * row;
                if (fwall[l] >= 0) fsc[l] = (T)P.rw[fwall[l]];
            }
        }
    }

    // ---- lane constants (FP64, rounded once) --------------------------------
    const double it = P.it;
    const double cyd = C.xv[MAXA + iy] - P.u[1];
    const T Ey = tb[NA + nx + iy], Py = tb[2 * NA + nx + iy], Ky = tb[3 * NA + nx + iy];
    T Eyz[4], Pyz[4], Kyz[4], Ayz[4], wz[4], cz[4], BL[NF];
    T amin[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) BL[l] = (T)(fny[l] * cyd + fun[l]);
#pragma unroll
    for (int l = 0; l < NF; ++l) amin[l] = (T)0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double czd = C.xv[2 * MAXA + iz0 + j] - P.u[2];
        const double r2 = cyd * cyd + czd * czd;
        const int jz = nx + ny + iz0 + j;
        Eyz[j] = ((T)P.itau * Ey) * tb[NA + jz];
        Pyz[j] = Py + tb[2 * NA + jz];
        Kyz[j] = Ky + tb[3 * NA + jz];
        Ayz[j] = (T)(r2 * it - 2.5);
        wz[j] = (T)C.wv[2 * MAXA + iz0 + j];
        cz[j] = (T)czd;
    }
    // a = (xi.n) S/V = n_x c_x + (n_y c_y + u.n) + n_z c_z: the middle term per
    // lane, n_z and n_x per face (uniform)
    T fnzT[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fnzT[l] = (T)fnz[l];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T a = fma(fnzT[l], cz[j], BL[l]);
            amin[l] = (j == 0) ? a : fmin(amin[l], a);
        }
    }
    // smallest (y, z) part of each face's a over the wave: with n_x c_x of the
    // plane it bounds a from below on the wave's whole patch
#pragma unroll
    for (int l = 0; l < NF; ++l) amin[l] = to_uniform(wave_min(amin[l]));
    __syncthreads();

    const T idt = (T)C.inv_dt;
    const T den0 = (T)P.itau + idt;   // 1/dt + 1/tau (the diagonal, with - sum_{a<0} a, as the closed cell allows)
    T S0[4], S1[4], S2[4], S3[4], R0[4], R1[4], R2[4];
    T Wf[NF];
#pragma unroll
    for (int j = 0; j < 4; ++j) S0[j] = S1[j] = S2[j] = S3[j] = R0[j] = R1[j] = R2[j] = (T)0;
#pragma unroll
    for (int l = 0; l < NF; ++l) Wf[l] = (T)0;

    const int ix0 = vt * C.xp, ix1 = min(ix0 + C.xp, nx);
    const uint32_t plane_bytes = (uint32_t)(ny * nz * sizeof(T));
    const uint32_t lane_bytes = (uint32_t)(4 * pr * sizeof(T));
    gcptr<V4> fo_u = (gcptr<V4>)uniform_ptr(fo);
    gptr<V4> fn_u = (gptr<V4>)uniform_ptr(fn);
    gcptr<V4> fnb_u[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) fnb_u[l] = (gcptr<V4>)uniform_ptr(fnb[l]);

    // U x-planes per load round in the common case; cells with a wall face
    // (a few percent) carry the wall sums and take one plane per round
    auto planes = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
        constexpr int UU = WALLS ? 1 : U;
        for (int ixr = ix0 + xg; ixr < ix1; ixr += UU * G) {
            // ---- loads of the round: own rows, and the faces that bring values in
            // A face that brings nothing in on the wave's patch reads the own row
            // instead (the same cache lines as the own load: no extra traffic) and
            // its min(a, 0) is 0 on every node, so the code stays branch-free.
            V4 o[UU], v[UU][NF];
            bool live[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int ix = ixr + u * G;
                live[u] = ix < ix1;
                const int ixc = min(ix, ix1 - 1);
                const uint32_t off = (uint32_t)ixc * plane_bytes + lane_bytes;
                const T cx = xr[XREC * ixc];
                o[u] = ldb(fo_u, off);
#pragma unroll
                for (int l = 0; l < NF; ++l) {
                    // some node may bring a value in: the lower bound of a on the wave's
                    // patch, with a margin that covers the rounding of a itself
                    const T ax = fnx[l] * cx;
                    const int nd = (ax + amin[l] < (T)1e-5 * (fabs(ax) + fabs(amin[l])));
                    const bool need = __builtin_amdgcn_readfirstlane(nd);
                    v[u][l] = ldb(need ? fnb_u[l] : fo_u, off);
                }
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                if (!live[u]) break;
                const int ix = ixr + u * G;
                const T *rx = xr + XREC * ix;
                const T cx = rx[0], Ex = rx[1], Px = rx[2], Kx = rx[3], cx2 = rx[4];
                const T wx = rx[5], wx1 = rx[6], wx2 = rx[7], wx3 = rx[8];
                T AX[NF];
#pragma unroll
                for (int l = 0; l < NF; ++l) AX[l] = fnx[l] * cx + BL[l];
                V4 outv;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const T oj = o[u][j];
                    // relaxation target (1/tau folded into Eyz)
                    const T g = Ex * Eyz[j] * (Px + Pyz[j]) * ((Kx + Kyz[j]) * (cx2 + Ayz[j]) + (T)1);
                    T num = g + idt * oj;
                    T den = den0;
                    T aw[NF];
#pragma unroll
                    for (int l = 0; l < NF; ++l) {
                        const T a = fma(fnzT[l], cz[j], AX[l]);
                        const T mn = fmin(a, (T)0);
                        den -= mn;
                        if constexpr (WALLS) {
                            aw[l] = a - mn;     // max(a, 0)
                            num -= (mn * fsc[l]) * v[u][l][j];
                        } else {
                            num -= mn * v[u][l][j];
                        }
                    }
                    const T f = num * fast_rcp(den);
                    outv[j] = f;
                    S0[j] = fma(wx, f, S0[j]);
                    S1[j] = fma(wx1, f, S1[j]);
                    S2[j] = fma(wx2, f, S2[j]);
                    S3[j] = fma(wx3, f, S3[j]);
                    const T tr = num - den * oj;
                    R0[j] = fma(wx, tr, R0[j]);
                    R1[j] = fma(wx1, tr, R1[j]);
                    R2[j] = fma(wx2, tr, R2[j]);
                    if constexpr (WALLS) {
                        // outgoing wall flux sums, weight w_x w_z here and w_y at the end
                        const T hw = (wx * wz[j]) * f;
#pragma unroll
                        for (int l = 0; l < NF; ++l)
                            if (fwall[l] >= 0) Wf[l] = fma(hw, aw[l], Wf[l]);
                    }
                }
                stb(fn_u, (uint32_t)ix * plane_bytes + lane_bytes, outv);
            }
        }
    };
    auto epilogue = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
        // the sums leave the loop as they are: without this the compiler
        // materialises the zero-trip values of their FP64 conversions before
        // the loop and keeps them live across it (64 registers)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            asm volatile("" : "+v"(S0[j]), "+v"(S1[j]), "+v"(S2[j]), "+v"(S3[j]));
            asm volatile("" : "+v"(R0[j]), "+v"(R1[j]), "+v"(R2[j]));
        }
        if (WALLS) {
#pragma unroll
            for (int l = 0; l < NF; ++l) asm volatile("" : "+v"(Wf[l]));
        }
        v4_partials<T, NF, WALLS>(S0, S1, S2, S3, R0, R1, R2, Wf, fwall, C, P.u[2], cyd, iy, iz0, red,
                                  C.partial + ((size_t)slot * C.ntile + vt) * NSUM);
    };
    if (nw > 0) {
        planes(std::true_type{});
        epilogue(std::true_type{});
    } else {
        planes(std::false_type{});
        epilogue(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// Second-order sweep (Sec. 3, second-order finite volumes, as a deferred
// correction of the first-order implicit update) in the 16-byte-row plane
// layout of k_sweep_v4.  Besides the first-order terms, a node takes
//   - the cell's own increment of every face where the value goes out
//     (num -= max(a, 0) delta_l),
//   - on a face to a kinetic neighbour, the neighbour's increment on the
//     shared face where the value comes in (v = f_nb + delta_nb),
//   - the pseudo-time term damp amax on the diagonal,
// and wall faces scale their Maxwellian row by rho_w with the slope part of
// the outgoing flux.  Per wave and x-plane a face that brings nothing in reads
// neither the neighbour's row nor its increment, and a face that takes
// nothing out does not read the cell's increment (exactly: those terms are
// zero on every node of the wave's patch).  Tiles cover whole x-planes.
// ---------------------------------------------------------------------------
template <typename T, int NF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (NF <= 4 ? 3 : 2) : 1))) void
k_sweep_o2v4(Batch B)
{
    typedef typename Vec4T<T>::v V4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
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
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    const size_t row = (size_t)C.row;
    gcptr<T> fold = (gcptr<T>)C.f[cur];
    gptr<T> fn = (gptr<T>)C.f[cur ^ 1] + (size_t)slot * row;
    gcptr<T> fo = fold + (size_t)slot * row;
    gcptr<T> dl0 = (gcptr<T>)C.slope;

    const int Q = nz >> 2, PL = ny * Q, G = BLOCK / PL;
    const int xg = threadIdx.x / PL, pr = threadIdx.x - xg * PL;
    const int iy = pr / Q, iz0 = 4 * (pr - iy * Q);

    const int NA = nx + ny + nz;
    gcptr<T> tb = (gcptr<T>)C.axtab + (size_t)slot * C.tabp;
    T *xr = (T *)smem_raw;
    double *red = (double *)(smem_raw + red_offset<T>((size_t)XREC * nx));
    {
        const double ux = P.u[0], it = P.it;
        for (int j = threadIdx.x; j < nx; j += BLOCK) {
            const double c = C.xv[j] - ux, w = C.wv[j];
            T *r = xr + XREC * j;
            r[0] = tb[j];
            r[1] = tb[NA + j];
            r[2] = tb[2 * NA + j];
            r[3] = tb[3 * NA + j];
            r[4] = (T)(c * c * it);
            r[5] = (T)w;
            r[6] = (T)(w * c);
            r[7] = (T)(w * c * c);
            r[8] = (T)(w * c * c * c);
        }
    }

    // ---- faces: neighbour rows and increments, own increments, scales -------
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    int fwall[NF];
    T fnx[NF], fsc[NF], qk[NF];
    double fny[NF], fnz[NF], fun[NF];
    gcptr<T> fnb[NF], dnb[NF], dio[NF];
    int nw = 0;
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fwall[l] = -1;
        fnx[l] = fsc[l] = qk[l] = (T)0;
        fny[l] = fnz[l] = fun[l] = 0.0;
        fnb[l] = dnb[l] = dio[l] = fo;
        if (l < nf) {
            const int e = e0 + l;
            const int oth = C.cf_other[e];
            const double n0 = C.cf_nsv[3 * e], n1 = C.cf_nsv[3 * e + 1], n2 = C.cf_nsv[3 * e + 2];
            fnx[l] = (T)n0;
            fny[l] = n1;
            fnz[l] = n2;
            fun[l] = P.u[0] * n0 + P.u[1] * n1 + P.u[2] * n2;
            fsc[l] = (T)1;
            dio[l] = dl0 + ((size_t)slot * C.nfmax + l) * row;
            if (oth >= 0) {
                const int so = C.slot_of_cell[oth];
                if (so >= 0) {
                    fnb[l] = fold + (size_t)so * row;
                    dnb[l] = dl0 + ((size_t)so * C.nfmax + C.cf_back[e]) * row;
                    qk[l] = (T)1;
                } else {
                    fnb[l] = (gcptr<T>)C.grow + (size_t)C.ghost_slot[oth] * row;
                }
            } else {
                fnb[l] = (gcptr<T>)C.prow + (size_t)(-1 - oth) * row;
                fwall[l] = C.cf_wall[e];
                if (fwall[l] >= 0) {
                    // rho_w with the slope part of the outgoing mass flux of f^n
                    double ws = 0.0;
                    for (int tl = 0; tl < C.ntile; ++tl) ws += C.wsl[((size_t)slot * C.ntile + tl) * MAXW + fwall[l]];
                    fsc[l] = (T)(P.rw[fwall[l]] + ws / C.wall_den[e]);
                    ++nw;
                }
            }
        }
    }

    // ---- lane constants (FP64, rounded once) --------------------------------
    const double it = P.it;
    const double cyd = C.xv[MAXA + iy] - P.u[1];
    const T Ey = tb[NA + nx + iy], Py = tb[2 * NA + nx + iy], Ky = tb[3 * NA + nx + iy];
    T Eyz[4], Pyz[4], Kyz[4], Ayz[4], wz[4], cz[4], BL[NF], amin[NF], amx[NF], fnzT[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) BL[l] = (T)(fny[l] * cyd + fun[l]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double czd = C.xv[2 * MAXA + iz0 + j] - P.u[2];
        const double r2 = cyd * cyd + czd * czd;
        const int jz = nx + ny + iz0 + j;
        Eyz[j] = ((T)P.itau * Ey) * tb[NA + jz];
        Pyz[j] = Py + tb[2 * NA + jz];
        Kyz[j] = Ky + tb[3 * NA + jz];
        Ayz[j] = (T)(r2 * it - 2.5);
        wz[j] = (T)C.wv[2 * MAXA + iz0 + j];
        cz[j] = (T)czd;
    }
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fnzT[l] = (T)fnz[l];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T a = fma(fnzT[l], cz[j], BL[l]);
            amin[l] = (j == 0) ? a : fmin(amin[l], a);
            amx[l] = (j == 0) ? a : fmax(amx[l], a);
        }
    }
    // the (y, z) part of each face's a over the wave: with n_x c_x of the plane
    // it bounds a on the wave's whole patch from below and above
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        amin[l] = to_uniform(wave_min(amin[l]));
        amx[l] = to_uniform(-wave_min(-amx[l]));
    }
    __syncthreads();

    const T idt = (T)(C.inv_dt + C.damp2 * C.amax[cell]);
    const T den0 = (T)P.itau + idt;
    T S0[4], S1[4], S2[4], S3[4], R0[4], R1[4], R2[4];
    T Wf[NF];
#pragma unroll
    for (int j = 0; j < 4; ++j) S0[j] = S1[j] = S2[j] = S3[j] = R0[j] = R1[j] = R2[j] = (T)0;
#pragma unroll
    for (int l = 0; l < NF; ++l) Wf[l] = (T)0;

    const int P2 = ny * nz;
    const int ix0 = (vt * C.tile) / P2, ix1 = min(nx, ((vt + 1) * C.tile) / P2);
    const uint32_t plane_bytes = (uint32_t)(P2 * sizeof(T));
    const uint32_t lane_bytes = (uint32_t)(4 * pr * sizeof(T));
    gcptr<V4> fo_u = (gcptr<V4>)uniform_ptr(fo);
    gptr<V4> fn_u = (gptr<V4>)uniform_ptr(fn);
    gcptr<V4> fnb_u[NF], dnb_u[NF], dio_u[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fnb_u[l] = (gcptr<V4>)uniform_ptr(fnb[l]);
        dnb_u[l] = (gcptr<V4>)uniform_ptr(dnb[l]);
        dio_u[l] = (gcptr<V4>)uniform_ptr(dio[l]);
    }

    auto planes = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
        for (int ix = ix0 + xg; ix < ix1; ix += G) {
            const uint32_t off = (uint32_t)ix * plane_bytes + lane_bytes;
            const T cx = xr[XREC * ix];
            const V4 o = ldb(fo_u, off);
            V4 v[NF], dn[NF], di[NF];
#pragma unroll
            for (int l = 0; l < NF; ++l) {
                const T ax = fnx[l] * cx;
                const int ni = (ax + amin[l] < (T)1e-5 * (fabs(ax) + fabs(amin[l])));
                const int no = (ax + amx[l] > (T)-1e-5 * (fabs(ax) + fabs(amx[l])));
                const bool need_in = __builtin_amdgcn_readfirstlane(ni);
                const bool need_out = __builtin_amdgcn_readfirstlane(no);
                v[l] = ldb(need_in ? fnb_u[l] : fo_u, off);
                dn[l] = ldb(need_in ? dnb_u[l] : fo_u, off);
                di[l] = ldb(need_out ? dio_u[l] : fo_u, off);
            }
            const T *rx = xr + XREC * ix;
            const T Ex = rx[1], Px = rx[2], Kx = rx[3], cx2 = rx[4];
            const T wx = rx[5], wx1 = rx[6], wx2 = rx[7], wx3 = rx[8];
            T AX[NF];
#pragma unroll
            for (int l = 0; l < NF; ++l) AX[l] = fnx[l] * cx + BL[l];
            V4 outv;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T oj = o[j];
                const T g = Ex * Eyz[j] * (Px + Pyz[j]) * ((Kx + Kyz[j]) * (cx2 + Ayz[j]) + (T)1);
                T num = g + idt * oj;
                T den = den0;
                T aw[NF];
#pragma unroll
                for (int l = 0; l < NF; ++l) {
                    const T a = fma(fnzT[l], cz[j], AX[l]);
                    const T mn = fmin(a, (T)0);
                    const T ap = a - mn;   // max(a, 0)
                    den -= mn;
                    const T vin = fma(qk[l], dn[l][j], v[l][j]);
                    if constexpr (WALLS) {
                        aw[l] = ap;
                        num -= (mn * fsc[l]) * vin;
                    } else {
                        num -= mn * vin;
                    }
                    num -= ap * di[l][j];
                }
                const T f = num * fast_rcp(den);
                outv[j] = f;
                S0[j] = fma(wx, f, S0[j]);
                S1[j] = fma(wx1, f, S1[j]);
                S2[j] = fma(wx2, f, S2[j]);
                S3[j] = fma(wx3, f, S3[j]);
                const T tr = num - den * oj;
                R0[j] = fma(wx, tr, R0[j]);
                R1[j] = fma(wx1, tr, R1[j]);
                R2[j] = fma(wx2, tr, R2[j]);
                if constexpr (WALLS) {
                    const T hw = (wx * wz[j]) * f;
#pragma unroll
                    for (int l = 0; l < NF; ++l)
                        if (fwall[l] >= 0) Wf[l] = fma(hw, aw[l], Wf[l]);
                }
            }
            stb(fn_u, off, outv);
        }
    };
    auto epilogue = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            asm volatile("" : "+v"(S0[j]), "+v"(S1[j]), "+v"(S2[j]), "+v"(S3[j]));
            asm volatile("" : "+v"(R0[j]), "+v"(R1[j]), "+v"(R2[j]));
        }
        if (WALLS) {
#pragma unroll
            for (int l = 0; l < NF; ++l) asm volatile("" : "+v"(Wf[l]));
        }
        v4_partials<T, NF, WALLS>(S0, S1, S2, S3, R0, R1, R2, Wf, fwall, C, P.u[2], cyd, iy, iz0, red,
                                  C.partial + ((size_t)slot * C.ntile + vt) * NSUM);
    };
    if (nw > 0) {
        planes(std::true_type{});
        epilogue(std::true_type{});
    } else {
        planes(std::false_type{});
        epilogue(std::false_type{});
    }
}

// waves per SIMD of the FP32 16-byte-row correction
#ifndef CORRECT_V4_WAVES
#define CORRECT_V4_WAVES 4
#endif
// x-planes per load round of the 16-byte-row correction (cells without walls)
#ifndef CORRECT_V4_U
#define CORRECT_V4_U 4
#endif

// ---------------------------------------------------------------------------
// GSIS correction (Sec. 3.1) in the 16-byte-row plane layout of k_sweep_v4:
// f += f_eq(W^{n+1}) - f_eq(W^{n+1/2}) in place.  Each f_eq is a
// conservation-fixed Maxwellian E_x E_y E_z (P_x + P_y + P_z) (a_0 in P_x).  A
// lane keeps one y node and four z nodes for the whole row: their (y, z)
// factors E_y E_z and P_y + P_z are formed in FP64 and rounded once; one LDS
// record per x-plane gives c_x, E_x and P_x of both states and w_x c_x^a.  The
// moment and outgoing wall sums are those of the sweep (no balance sums).
// ---------------------------------------------------------------------------
template <typename T, int NF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? CORRECT_V4_WAVES : 1))) void
k_correct_v4(const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    typedef typename Vec4T<T>::v V4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const CaseView &C = *cvp;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin, t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const FeqRec &Fa = C.feq[2 * (size_t)slot];       // f_eq(W^{n+1})
    const FeqRec &Fb = C.feq[2 * (size_t)slot + 1];   // f_eq(W^{n+1/2})
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    gptr<T> fr = (gptr<T>)C.f[cur] + (size_t)slot * C.row;

    // lane -> (x group, y, first of four z nodes), as in the sweep
    const int Q = nz >> 2, PL = ny * Q, G = BLOCK / PL;
    const int xg = threadIdx.x / PL, pr = threadIdx.x - xg * PL;
    const int iy = pr / Q, iz0 = 4 * (pr - iy * Q);

    // ---- LDS: per x-plane c, E_x and P_x of both states, w c^a ---------------
    T *xr = (T *)smem_raw;
    double *red = (double *)(smem_raw + red_offset<T>((size_t)XREC * nx));
    for (int j = threadIdx.x; j < nx; j += BLOCK) {
        const double x = C.xv[j], c = x - P.u[0], w = C.wv[j];
        const double ca = x - Fa.u[0], cb = x - Fb.u[0];
        T *r = xr + XREC * j;
        r[0] = (T)c;
        r[1] = (T)exp(-ca * ca * Fa.it);
        r[2] = (T)(Fa.fx[0] + Fa.fx[1] * ca + Fa.fx[4] * ca * ca);
        r[3] = (T)exp(-cb * cb * Fb.it);
        r[4] = (T)(Fb.fx[0] + Fb.fx[1] * cb + Fb.fx[4] * cb * cb);
        r[5] = (T)w;
        r[6] = (T)(w * c);
        r[7] = (T)(w * c * c);
        r[8] = (T)(w * c * c * c);
    }

    // ---- lane constants (FP64, rounded once) ---------------------------------
    const double yv = C.xv[MAXA + iy];
    const double cyd = yv - P.u[1];
    const double ya = yv - Fa.u[1], yb = yv - Fb.u[1];
    const double Eya = exp(-ya * ya * Fa.it), Pya = Fa.fx[2] * ya + Fa.fx[4] * ya * ya;
    const double Eyb = exp(-yb * yb * Fb.it), Pyb = Fb.fx[2] * yb + Fb.fx[4] * yb * yb;
    T EA[4], PA[4], EB[4], PB[4], wz[4], cz[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double zv = C.xv[2 * MAXA + iz0 + j];
        const double za = zv - Fa.u[2], zb = zv - Fb.u[2];
        EA[j] = (T)(Eya * exp(-za * za * Fa.it));
        PA[j] = (T)(Pya + Fa.fx[3] * za + Fa.fx[4] * za * za);
        EB[j] = (T)(Eyb * exp(-zb * zb * Fb.it));
        PB[j] = (T)(Pyb + Fb.fx[3] * zb + Fb.fx[4] * zb * zb);
        wz[j] = (T)C.wv[2 * MAXA + iz0 + j];
        cz[j] = (T)(zv - P.u[2]);
    }

    // ---- wall faces: a = (xi.n) S/V = n_x c_x + (n_y c_y + u.n) + n_z c_z ------
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    int fwall[NF];
    T fnx[NF], fnzT[NF], BL[NF];
    int nw = 0;
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fwall[l] = -1;
        fnx[l] = fnzT[l] = BL[l] = (T)0;
        if (l < nf) {
            const int e = e0 + l;
            fwall[l] = C.cf_wall[e];
            if (fwall[l] >= 0) {
                const double n0 = C.cf_nsv[3 * e], n1 = C.cf_nsv[3 * e + 1], n2 = C.cf_nsv[3 * e + 2];
                fnx[l] = (T)n0;
                fnzT[l] = (T)n2;
                BL[l] = (T)(n1 * cyd + (P.u[0] * n0 + P.u[1] * n1 + P.u[2] * n2));
                ++nw;
            }
        }
    }
    __syncthreads();

    T S0[4], S1[4], S2[4], S3[4], Z[4], Wf[NF];
#pragma unroll
    for (int j = 0; j < 4; ++j) S0[j] = S1[j] = S2[j] = S3[j] = Z[j] = (T)0;
#pragma unroll
    for (int l = 0; l < NF; ++l) Wf[l] = (T)0;

    const int ix0 = vt * C.xp, ix1 = min(ix0 + C.xp, nx);
    const uint32_t plane_bytes = (uint32_t)(ny * nz * sizeof(T));
    const uint32_t lane_bytes = (uint32_t)(4 * pr * sizeof(T));
    gptr<V4> f_u = (gptr<V4>)uniform_ptr(fr);

    auto planes = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
        constexpr int UU = WALLS ? 1 : CORRECT_V4_U;
        for (int ixr = ix0 + xg; ixr < ix1; ixr += UU * G) {
            V4 o[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int ixc = min(ixr + u * G, ix1 - 1);
                o[u] = ldb(gcptr<V4>(f_u), (uint32_t)ixc * plane_bytes + lane_bytes);
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int ix = ixr + u * G;
                if (ix >= ix1) break;
                const T *rx = xr + XREC * ix;
                const T cx = rx[0], Exa = rx[1], Pxa = rx[2], Exb = rx[3], Pxb = rx[4];
                const T wx = rx[5], wx1 = rx[6], wx2 = rx[7], wx3 = rx[8];
                V4 outv;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const T fv = o[u][j] + (Exa * EA[j] * (Pxa + PA[j]) - Exb * EB[j] * (Pxb + PB[j]));
                    outv[j] = fv;
                    S0[j] = fma(wx, fv, S0[j]);
                    S1[j] = fma(wx1, fv, S1[j]);
                    S2[j] = fma(wx2, fv, S2[j]);
                    S3[j] = fma(wx3, fv, S3[j]);
                    if constexpr (WALLS) {
                        const T hw = (wx * wz[j]) * fv;
#pragma unroll
                        for (int l = 0; l < NF; ++l)
                            if (fwall[l] >= 0) {
                                const T a = fma(fnzT[l], cz[j], fnx[l] * cx + BL[l]);
                                Wf[l] = fma(hw, fmax(a, (T)0), Wf[l]);
                            }
                    }
                }
                stb(f_u, (uint32_t)ix * plane_bytes + lane_bytes, outv);
            }
        }
    };
    auto epilogue = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
#pragma unroll
        for (int j = 0; j < 4; ++j) asm volatile("" : "+v"(S0[j]), "+v"(S1[j]), "+v"(S2[j]), "+v"(S3[j]));
        if (WALLS) {
#pragma unroll
            for (int l = 0; l < NF; ++l) asm volatile("" : "+v"(Wf[l]));
        }
        v4_partials<T, NF, WALLS>(S0, S1, S2, S3, Z, Z, Z, Wf, fwall, C, P.u[2], cyd, iy, iz0, red,
                                  C.partial + ((size_t)slot * C.ntile + vt) * NSUM);
    };
    if (nw > 0) {
        planes(std::true_type{});
        epilogue(std::true_type{});
    } else {
        planes(std::false_type{});
        epilogue(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// Correction of the two-VDF gas (Sec. 3.1, eq. updatef with rho e_r) in the
// 16-byte-row plane layout: per node m_a = f_eq(W^{n+1}) and m_b = f_eq(W^{n+1/2})
// as in k_correct_v4; f0 += m_a - m_b and f1 += th_a m_a - th_b m_b with
// th = d_r T_r / 4 of each state.  Rows hold (f0, f1) with f1 at nvp = row / 2.
// Sums: those of f0 as in the sweep, and of f1 sum w f1, sum w c f1 (PSUM, the
// last entry, the sweep's balance, zero).  A tile must cover whole x-planes.
// ---------------------------------------------------------------------------
template <typename T, int NF>
__global__ __launch_bounds__(BLOCK) __attribute__((
    amdgpu_waves_per_eu(sizeof(T) == 4 ? (NF <= 4 ? CORRECT_V4_WAVES : 2) : 1))) void k_correct_poly_v4(const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    typedef typename Vec4T<T>::v V4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const CaseView &C = *cvp;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin, t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const FeqRec &Fa = C.feq[2 * (size_t)slot];
    const FeqRec &Fb = C.feq[2 * (size_t)slot + 1];
    const int nx = C.n[0], ny = C.n[1], nz = C.n[2];
    gptr<T> fr = (gptr<T>)C.f[cur] + (size_t)slot * C.row;
    const int Q = nz >> 2, PL = ny * Q, G = BLOCK / PL;
    const int xg = threadIdx.x / PL, pr = threadIdx.x - xg * PL;
    const int iy = pr / Q, iz0 = 4 * (pr - iy * Q);

    T *xr = (T *)smem_raw;
    double *red = (double *)(smem_raw + red_offset<T>((size_t)XREC * nx));
    for (int j = threadIdx.x; j < nx; j += BLOCK) {
        const double x = C.xv[j], c = x - P.u[0], w = C.wv[j];
        const double ca = x - Fa.u[0], cb = x - Fb.u[0];
        T *r = xr + XREC * j;
        r[0] = (T)c;
        r[1] = (T)exp(-ca * ca * Fa.it);
        r[2] = (T)(Fa.fx[0] + Fa.fx[1] * ca + Fa.fx[4] * ca * ca);
        r[3] = (T)exp(-cb * cb * Fb.it);
        r[4] = (T)(Fb.fx[0] + Fb.fx[1] * cb + Fb.fx[4] * cb * cb);
        r[5] = (T)w;
        r[6] = (T)(w * c);
        r[7] = (T)(w * c * c);
        r[8] = (T)(w * c * c * c);
    }
    const double yv = C.xv[MAXA + iy];
    const double cyd = yv - P.u[1];
    const double ya = yv - Fa.u[1], yb = yv - Fb.u[1];
    const double Eya = exp(-ya * ya * Fa.it), Pya = Fa.fx[2] * ya + Fa.fx[4] * ya * ya;
    const double Eyb = exp(-yb * yb * Fb.it), Pyb = Fb.fx[2] * yb + Fb.fx[4] * yb * yb;
    T EA[4], PA[4], EB[4], PB[4], wz[4], cz[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double zv = C.xv[2 * MAXA + iz0 + j];
        const double za = zv - Fa.u[2], zb = zv - Fb.u[2];
        EA[j] = (T)(Eya * exp(-za * za * Fa.it));
        PA[j] = (T)(Pya + Fa.fx[3] * za + Fa.fx[4] * za * za);
        EB[j] = (T)(Eyb * exp(-zb * zb * Fb.it));
        PB[j] = (T)(Pyb + Fb.fx[3] * zb + Fb.fx[4] * zb * zb);
        wz[j] = (T)C.wv[2 * MAXA + iz0 + j];
        cz[j] = (T)(zv - P.u[2]);
    }
    const T tha = (T)Fa.Th, thb = (T)Fb.Th;
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    int fwall[NF];
    T fnx[NF], fnzT[NF], BL[NF];
    int nw = 0;
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fwall[l] = -1;
        fnx[l] = fnzT[l] = BL[l] = (T)0;
        if (l < nf) {
            const int e = e0 + l;
            fwall[l] = C.cf_wall[e];
            if (fwall[l] >= 0) {
                const double n0 = C.cf_nsv[3 * e], n1 = C.cf_nsv[3 * e + 1], n2 = C.cf_nsv[3 * e + 2];
                fnx[l] = (T)n0;
                fnzT[l] = (T)n2;
                BL[l] = (T)(n1 * cyd + (P.u[0] * n0 + P.u[1] * n1 + P.u[2] * n2));
                ++nw;
            }
        }
    }
    __syncthreads();

    T S0[4], S1[4], S2[4], S3[4], Q0[4], Q1[4], Z[4], Wf[NF];
#pragma unroll
    for (int j = 0; j < 4; ++j) S0[j] = S1[j] = S2[j] = S3[j] = Q0[j] = Q1[j] = Z[j] = (T)0;
#pragma unroll
    for (int l = 0; l < NF; ++l) Wf[l] = (T)0;

    // the tile's x-planes (tiles cover whole planes)
    const int P2 = ny * nz;
    const int ix0 = (vt * C.tile) / P2, ix1 = min(nx, ((vt + 1) * C.tile) / P2);
    const uint32_t plane_bytes = (uint32_t)(P2 * sizeof(T));
    const uint32_t lane_bytes = (uint32_t)(4 * pr * sizeof(T));
    const uint32_t f1_bytes = (uint32_t)((C.row / 2) * sizeof(T));
    gptr<V4> f_u = (gptr<V4>)uniform_ptr(fr);

    auto planes = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
        constexpr int UU = WALLS ? 1 : 2;
        for (int ixr = ix0 + xg; ixr < ix1; ixr += UU * G) {
            V4 o0[UU], o1[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const uint32_t off = (uint32_t)min(ixr + u * G, ix1 - 1) * plane_bytes + lane_bytes;
                o0[u] = ldb(gcptr<V4>(f_u), off);
                o1[u] = ldb(gcptr<V4>(f_u), off + f1_bytes);
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int ix = ixr + u * G;
                if (ix >= ix1) break;
                const T *rx = xr + XREC * ix;
                const T cx = rx[0], Exa = rx[1], Pxa = rx[2], Exb = rx[3], Pxb = rx[4];
                const T wx = rx[5], wx1 = rx[6], wx2 = rx[7], wx3 = rx[8];
                V4 out0, out1;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const T ma = Exa * EA[j] * (Pxa + PA[j]), mb = Exb * EB[j] * (Pxb + PB[j]);
                    const T v0 = o0[u][j] + (ma - mb);
                    const T v1 = o1[u][j] + (tha * ma - thb * mb);
                    out0[j] = v0;
                    out1[j] = v1;
                    S0[j] = fma(wx, v0, S0[j]);
                    S1[j] = fma(wx1, v0, S1[j]);
                    S2[j] = fma(wx2, v0, S2[j]);
                    S3[j] = fma(wx3, v0, S3[j]);
                    Q0[j] = fma(wx, v1, Q0[j]);
                    Q1[j] = fma(wx1, v1, Q1[j]);
                    if constexpr (WALLS) {
                        const T hw = (wx * wz[j]) * v0;
#pragma unroll
                        for (int l = 0; l < NF; ++l)
                            if (fwall[l] >= 0) {
                                const T a = fma(fnzT[l], cz[j], fnx[l] * cx + BL[l]);
                                Wf[l] = fma(hw, fmax(a, (T)0), Wf[l]);
                            }
                    }
                }
                const uint32_t off = (uint32_t)ix * plane_bytes + lane_bytes;
                stb(f_u, off, out0);
                stb(f_u, off + f1_bytes, out1);
            }
        }
    };
    auto epilogue = [&](auto walls) {
        constexpr bool WALLS = decltype(walls)::value;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            asm volatile("" : "+v"(S0[j]), "+v"(S1[j]), "+v"(S2[j]), "+v"(S3[j]));
            asm volatile("" : "+v"(Q0[j]), "+v"(Q1[j]));
        }
        if (WALLS) {
#pragma unroll
            for (int l = 0; l < NF; ++l) asm volatile("" : "+v"(Wf[l]));
        }
        v4_partials<T, NF, WALLS>(S0, S1, S2, S3, Z, Z, Z, Wf, fwall, C, P.u[2], cyd, iy, iz0, red,
                                  C.partial + ((size_t)slot * C.ntile + vt) * NSUM);
        // the sums of f1: sum w f1 and sum w c f1, then the balance entry (zero)
        const double wyd = C.wv[MAXA + iy];
        double q[PSUM] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double wj = wyd * C.wv[2 * MAXA + iz0 + j];
            const double czj = C.xv[2 * MAXA + iz0 + j] - P.u[2];
            q[0] += wj * (double)Q0[j];
            q[1] += wj * (double)Q1[j];
            q[3] += wj * czj * (double)Q0[j];
        }
        q[2] = cyd * q[0];
        v4_block_sums<PSUM>(q, red, C.psum + ((size_t)slot * C.ntile + vt) * PSUM);
    };
    if (nw > 0) {
        planes(std::true_type{});
        epilogue(std::true_type{});
    } else {
        planes(std::false_type{});
        epilogue(std::false_type{});
    }
}

// ---------------------------------------------------------------------------
// GSIS correction (Sec. 3.1): f += f_eq(W^{n+1}) - f_eq(W^{n+1/2}) on the plane
// layout, with the same fused moment and wall sums as the sweep.  Both f_eq
// are conservation-fixed Maxwellians, separable per axis: E = E_x E_y E_z and
// multiplier P = P_x + P_y + P_z (a_0 folded into P_x), tabulated in FP64 per
// axis and rounded once.
// ---------------------------------------------------------------------------
template <typename T, int VD, int NF, int U>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? CORRECT_WAVES : 1))) void k_correct_fast(
    const CaseView *__restrict__ cvp, int n_kin, int cur)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const CaseView &C = *cvp;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int vt = b / n_kin, t = b - vt * n_kin;
    const int cell = C.kin_cell[t];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const FeqRec &Fa = C.feq[2 * (size_t)slot];       // f_eq(W^{n+1})
    const FeqRec &Fb = C.feq[2 * (size_t)slot + 1];   // f_eq(W^{n+1/2})
    const int nx = C.n[0], ny = C.n[1], nz = (VD == 3) ? C.n[2] : 1;
    const int NA = nx + ny + ((VD == 3) ? nz : 0);
    const int nvp = C.row / ((VD == 3) ? 1 : 2);
    gptr<T> fr = (gptr<T>)C.f[cur] + (size_t)slot * C.row;

    T *rc = (T *)smem_raw;   // x_j - u_d of the moment frame
    T *rw = rc + NA;
    T *Ea = rw + NA, *Pa = Ea + NA, *Eb = Pa + NA, *Pb = Eb + NA;
    T *rlo = Pb + NA;        // x axis: low part of c, c^2 and its low part, c^3 and its low part
    const size_t red_off = red_offset<T>((size_t)6 * NA + 5 * nx);

    // wall faces only (outgoing sums for the next wall density)
    const int e0 = C.cf_ptr[cell];
    const int nf = C.cf_ptr[cell + 1] - e0;
    int fwall[NF];
    T fnx[NF], fny[NF], fnz[NF], fun[NF];
    int nw = 0;
#pragma unroll
    for (int l = 0; l < NF; ++l) {
        fwall[l] = -1;
        fnx[l] = fny[l] = fnz[l] = fun[l] = (T)0;
        if (l < nf) {
            const int e = e0 + l;
            fwall[l] = C.cf_wall[e];
            if (fwall[l] >= 0) {
                const double n0 = C.cf_nsv[3 * e], n1 = C.cf_nsv[3 * e + 1], n2 = C.cf_nsv[3 * e + 2];
                fnx[l] = (T)n0;
                fny[l] = (T)n1;
                fnz[l] = (T)n2;
                fun[l] = (T)(P.u[0] * n0 + P.u[1] * n1 + P.u[2] * n2);
                ++nw;
            }
        }
    }
    {
        const int nq = (VD == 3) ? 4 : 3;   // index of the c^2 coefficient in fx
        for (int j = threadIdx.x; j < NA; j += BLOCK) {
            const int d = (j < nx) ? 0 : ((j < nx + ny) ? 1 : 2);
            const int jj = j - ((d == 0) ? 0 : ((d == 1) ? nx : nx + ny));
            const double x = C.xv[d * MAXA + jj];
            const double c = x - P.u[d];
            rc[j] = (T)c;
            rw[j] = (T)C.wv[d * MAXA + jj];
            const double ca = x - Fa.u[d], cb = x - Fb.u[d];
            Ea[j] = (T)exp(-ca * ca * Fa.it);
            Eb[j] = (T)exp(-cb * cb * Fb.it);
            Pa[j] = (T)(((d == 0) ? Fa.fx[0] : 0.0) + Fa.fx[1 + d] * ca + Fa.fx[nq] * ca * ca);
            Pb[j] = (T)(((d == 0) ? Fb.fx[0] : 0.0) + Fb.fx[1 + d] * cb + Fb.fx[nq] * cb * cb);
            if (d == 0) {
                const double c2 = c * c, c3 = c2 * c;
                rlo[jj] = (T)(c - (double)(T)c);
                rlo[nx + jj] = (T)c2;
                rlo[2 * nx + jj] = (T)(c2 - (double)(T)c2);
                rlo[3 * nx + jj] = (T)c3;
                rlo[4 * nx + jj] = (T)(c3 - (double)(T)c3);
            }
        }
    }
    __syncthreads();

    const int ilc = (VD == 3) ? (int)(threadIdx.x % nz) : (int)(threadIdx.x % ny);
    const int jlc = (VD == 3) ? nx + ny + ilc : nx + ilc;
    const T cL = rc[jlc], EaL = Ea[jlc], PaL = Pa[jlc], EbL = Eb[jlc], PbL = Pb[jlc];
    const T tha = (T)Fa.Th, thb = (T)Fb.Th;
    T AL[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) AL[l] = ((VD == 3) ? fnz[l] : fny[l]) * cL + fun[l];
    PlaneSums<T> S;
    T Wf[NF];
#pragma unroll
    for (int l = 0; l < NF; ++l) Wf[l] = (T)0;
    const int ix0 = vt * C.xp, ix1 = min(ix0 + C.xp, nx);

    if (VD == 3) {
        const int q = BLOCK / nz;
        const int M = ny / q;
        const int yq = threadIdx.x / nz;
        // node k = ix ny nz + tid + m BLOCK (q nz = BLOCK): one 32-bit byte
        // offset per round from the wave-uniform row base
        gptr<T> fr_u = uniform_ptr(fr);
        const uint32_t plane_bytes = (uint32_t)(ny * nz * sizeof(T));
        const uint32_t lane_bytes = (uint32_t)(threadIdx.x * sizeof(T));
        constexpr uint32_t ustep = BLOCK * sizeof(T);
        // two x-planes per pass: the loads of both planes' rounds are in flight together
        auto planes = [&](auto walls) {
            constexpr bool WALLS = decltype(walls)::value;
            for (int ix = ix0; ix < ix1; ix += 2) {
                const int npl = (ix + 1 < ix1) ? 2 : 1;
                T cx[2], wx[2], Exa[2], Pxa[2], Exb[2], Pxb[2], Ax[2][NF], Tp[2][4];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const int jx = (p < npl) ? ix + p : ix;
                    cx[p] = rc[jx];
                    wx[p] = rw[jx];
                    Exa[p] = Ea[jx] * EaL;
                    Pxa[p] = Pa[jx] + PaL;
                    Exb[p] = Eb[jx] * EbL;
                    Pxb[p] = Pb[jx] + PbL;
#pragma unroll
                    for (int l = 0; l < NF; ++l) Ax[p][l] = fnx[l] * cx[p] + AL[l];
#pragma unroll
                    for (int c = 0; c < 4; ++c) Tp[p][c] = (T)0;
                }
                uint32_t off = ix * plane_bytes + lane_bytes;
                int jy0 = nx + yq;
                for (int m = 0; m < M; m += U, off += U * ustep, jy0 += U * q) {
                    T o[2][U];
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            o[p][u] = (p < npl) ? ldb(gcptr<T>(fr_u), off + p * plane_bytes + u * ustep) : (T)0;
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        if (p >= npl) break;
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int jy = jy0 + u * q;
                            const T cy = rc[jy];
                            const T fv = o[p][u] + (Exa[p] * Ea[jy] * (Pxa[p] + Pa[jy]) -
                                                    Exb[p] * Eb[jy] * (Pxb[p] + Pb[jy]));
                            stb(fr_u, off + p * plane_bytes + u * ustep, fv);
                            const T h = wx[p] * rw[jy] * fv;
                            Tp[p][0] += h;
                            const T hy = h * cy;
                            Tp[p][1] += hy;
                            const T hy2 = hy * cy;
                            Tp[p][2] += hy2;
                            Tp[p][3] += hy2 * cy;
                            if constexpr (WALLS) {
#pragma unroll
                                for (int l = 0; l < NF; ++l)
                                    if (fwall[l] >= 0) Wf[l] += h * fmax(fny[l] * cy + Ax[p][l], (T)0);
                            }
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    if (p >= npl) break;
                    const int jx = ix + p;
                    S.fold(cx[p], rlo[jx], rlo[nx + jx], rlo[2 * nx + jx], rlo[3 * nx + jx], rlo[4 * nx + jx],
                           Tp[p][0], Tp[p][1], Tp[p][2], Tp[p][3], (T)0, (T)0, (T)0);
                }
            }
        };
        if (nw > 0) planes(std::true_type{});
        else planes(std::false_type{});
    } else {
        const int q = BLOCK / ny;
        const int xq = threadIdx.x / ny;
        for (int ixr = ix0 + xq; ixr < ix1; ixr += U * q) {
            T o0u[U], o1u[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ix = ixr + u * q;
                const int k = ix * ny + ilc;
                if (ix < ix1) {
                    o0u[u] = fr[k];
                    o1u[u] = fr[nvp + k];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ix = ixr + u * q;
                if (ix >= ix1) break;
                const int k = ix * ny + ilc;
                const T cx = rc[ix], wx = rw[ix];
                const T ma = Ea[ix] * EaL * (Pa[ix] + PaL), mb = Eb[ix] * EbL * (Pb[ix] + PbL);
                const T f0 = o0u[u] + (ma - mb);
                const T f1 = o1u[u] + (tha * ma - thb * mb);
                fr[k] = f0;
                fr[nvp + k] = f1;
                const T h = wx * f0;
                S.A0 += h;
                const T hx = h * cx;
                S.A1 += hx;
                const T hx2 = hx * cx;
                S.A2 += hx2;
                S.A3 += hx2 * cx;
                const T hp = wx * f1;
                S.Q0 += hp;
                S.Q1 += hp * cx;
                if (nw > 0) {
#pragma unroll
                    for (int l = 0; l < NF; ++l)
                        if (fwall[l] >= 0) Wf[l] += h * fmax(fnx[l] * cx + AL[l], (T)0);
                }
            }
        }
    }
    const int dl = (VD == 3) ? 2 : 1;
    finish_partials<T, VD, NF>(S, Wf, fwall, (VD == 3) ? nz : ny, C.xv + dl * MAXA, C.wv + dl * MAXA, P.u[dl],
                               C.partial + ((size_t)slot * C.ntile + vt) * NSUM, (T *)(smem_raw + red_off));
}

// ---------------------------------------------------------------------------
// axis tables of each kinetic slot's relaxation target (FP64, rounded once):
// c = x_j - u_d, E = exp(-c^2 / T), fix-up part (a_0 folded into the x axis),
// Shakhov part kq_d c; then c, c^2, c^3 of the x axis split into rounded value
// and low part for the compensated plane fold
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(128) void k_axtab(const CaseView *__restrict__ cvp)
{
    const CaseView &C = *cvp;
    const int cell = C.kin_cell[blockIdx.x];
    const int slot = C.slot_of_cell[cell];
    const ParamRec &P = C.param[slot];
    const int nx = C.n[0], ny = C.n[1], vd = C.vdim;
    const int NA = nx + ny + ((vd == 3) ? C.n[2] : 0);
    const double it = P.it;
    const double fq = (vd == 3) ? P.fx[4] : P.fx[3];
    T *tb = (T *)C.axtab + (size_t)slot * C.tabp;
    for (int j = threadIdx.x; j < NA; j += blockDim.x) {
        const int d = (j < nx) ? 0 : ((j < nx + ny) ? 1 : 2);
        const int jj = j - ((d == 0) ? 0 : ((d == 1) ? nx : nx + ny));
        const double c = C.xv[d * MAXA + jj] - P.u[d];
        const double pl = (d == 0) ? P.fx[0] + P.fx[1] * c + fq * c * c : P.fx[1 + d] * c + fq * c * c;
        tb[j] = (T)c;
        tb[NA + j] = (T)exp(-c * c * it);
        tb[2 * NA + j] = (T)pl;
        tb[3 * NA + j] = (T)(P.kq[d] * c);
        if (d == 0) {
            const double c2 = c * c, c3 = c2 * c;
            T *lo = tb + 4 * NA;
            lo[jj] = (T)(c - (double)(T)c);
            lo[nx + jj] = (T)c2;
            lo[2 * nx + jj] = (T)(c2 - (double)(T)c2);
            lo[3 * nx + jj] = (T)c3;
            lo[4 * nx + jj] = (T)(c3 - (double)(T)c3);
        }
    }
}

hipError_t launch_axtab(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s)
{
    if (n_kin <= 0) return hipSuccess;
    if (h.dtype == GSIS_F32) hipLaunchKernelGGL(k_axtab<float>, dim3(n_kin), dim3(128), 0, s, cv);
    else hipLaunchKernelGGL(k_axtab<double>, dim3(n_kin), dim3(128), 0, s, cv);
    return hipGetLastError();
}

// table elements in LDS: five per-axis tables and the x axis' low parts
size_t sweep_fast_tab(const CaseView &h)
{
    const int NA = h.n[0] + h.n[1] + (h.vdim == 3 ? h.n[2] : 0);
    return (size_t)5 * NA + 5 * h.n[0];
}

template <typename T, int VD, int U>
void launch_u(const Batch &b, size_t tab, int total, hipStream_t s)
{
    const size_t off = red_offset<T>(tab);
    size_t l4 = off + red_bytes<T, 4>(), l8 = off + red_bytes<T, MAXF>();
    // GSIS_SWEEP_LDS: minimum LDS bytes per block (caps the blocks per CU)
    static const size_t lds_min = [] {
        const char *e = std::getenv("GSIS_SWEEP_LDS");
        return e ? (size_t)std::atol(e) : (size_t)0;
    }();
    l4 = std::max(l4, lds_min);
    l8 = std::max(l8, lds_min);
    if (b.nfmax <= 4) hipLaunchKernelGGL((k_sweep_fast<T, VD, 4, U>), dim3(total), dim3(BLOCK), l4, s, b);
    else hipLaunchKernelGGL((k_sweep_fast<T, VD, MAXF, U>), dim3(total), dim3(BLOCK), l8, s, b);
}

// points per load round: 3D, the largest of 4, 2, 1 that divides M, the
// y-values per lane and plane (M = n_y n_z / 256; for a batch, the gcd over
// its cases); reduced 2D, 4 lines (guarded); at most 2 for FP64 or 8-face
// meshes (register budget)
int rounds_u(int vdim, int mdiv, size_t es, int nfmax)
{
    int U = 4;
    if (vdim == 3) U = (mdiv % 4 == 0) ? 4 : ((mdiv % 2 == 0) ? 2 : 1);
    if (es == 8 || nfmax > 4) U = (U > 2) ? 2 : U;
    return U;
}

template <typename T, int VD>
void launch_nf(const Batch &b, const CaseView &h0, size_t lds, int total, hipStream_t s)
{
    const int U = rounds_u(h0.vdim, b.mdiv, sizeof(T), b.nfmax);
    if (U == 4) launch_u<T, VD, 4>(b, lds, total, s);
    else if (U == 2) launch_u<T, VD, 2>(b, lds, total, s);
    else launch_u<T, VD, 1>(b, lds, total, s);
}

// the 16-byte-row sweep covers 3D grids with n_z % 4 == 0 and a (y, z) plane
// of 64..256 four-node lanes that divides the block
bool sweep_v4_fits(int ny, int nz)
{
    if (nz % 4) return false;
    const int P = ny * nz / 4;
    return P >= 64 && P <= BLOCK && BLOCK % P == 0;
}

template <typename T>
void launch_v4(const Batch &b, const CaseView &h0, int total, hipStream_t s)
{
    const size_t lds = red_offset<T>((size_t)XREC * h0.n[0]) + sizeof(double) * (BLOCK / 16) * NSUM;
    if (b.nfmax <= 4) hipLaunchKernelGGL((k_sweep_v4<T, 4, SWEEP_V4_U>), dim3(total), dim3(BLOCK), lds, s, b);
    else hipLaunchKernelGGL((k_sweep_v4<T, MAXF, 1>), dim3(total), dim3(BLOCK), lds, s, b);
}

// second-order cases the 16-byte-row sweep takes: 3D tensor grids whose (y, z)
// plane splits into 64-256 lanes of four z nodes and whose tiles cover whole
// x-planes (GSIS_O2_V4=0 keeps the node-per-thread sweep)
bool o2_v4_fits(const CaseView &h)
{
    static const bool on = [] {
        const char *e = std::getenv("GSIS_O2_V4");
        return !(e && e[0] == '0');
    }();
    return on && h.sorder == 2 && h.vdim == 3 && !h.points && !h.poly && sweep_v4_fits(h.n[1], h.n[2]) &&
           h.tile % (h.n[1] * h.n[2]) == 0;
}

hipError_t launch_sweep_o2v4(const Batch &b, const CaseView &h0, int total, hipStream_t s)
{
    const size_t lds_f = red_offset<float>((size_t)XREC * h0.n[0]) + sizeof(double) * (BLOCK / 16) * NSUM;
    const size_t lds_d = red_offset<double>((size_t)XREC * h0.n[0]) + sizeof(double) * (BLOCK / 16) * NSUM;
    if (h0.dtype == GSIS_F32) {
        if (b.nfmax <= 4) hipLaunchKernelGGL((k_sweep_o2v4<float, 4>), dim3(total), dim3(BLOCK), lds_f, s, b);
        else hipLaunchKernelGGL((k_sweep_o2v4<float, MAXF>), dim3(total), dim3(BLOCK), lds_f, s, b);
    } else {
        if (b.nfmax <= 4) hipLaunchKernelGGL((k_sweep_o2v4<double, 4>), dim3(total), dim3(BLOCK), lds_d, s, b);
        else hipLaunchKernelGGL((k_sweep_o2v4<double, MAXF>), dim3(total), dim3(BLOCK), lds_d, s, b);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_fast(const Batch &b, const CaseView &h0, int total, hipStream_t s)
{
    if (b.v4) {
        if (h0.dtype == GSIS_F32) launch_v4<float>(b, h0, total, s);
        else launch_v4<double>(b, h0, total, s);
        return hipGetLastError();
    }
    if (h0.dtype == GSIS_F32) {
        const size_t lds = sweep_fast_tab(h0);
        if (h0.vdim == 3) launch_nf<float, 3>(b, h0, lds, total, s);
        else launch_nf<float, 2>(b, h0, lds, total, s);
    } else {
        const size_t lds = sweep_fast_tab(h0);
        if (h0.vdim == 3) launch_nf<double, 3>(b, h0, lds, total, s);
        else launch_nf<double, 2>(b, h0, lds, total, s);
    }
    return hipGetLastError();
}

template <typename T, int VD, int U>
void launch_correct_u(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    const int NA = h.n[0] + h.n[1] + (VD == 3 ? h.n[2] : 0);
    const size_t off = red_offset<T>((size_t)6 * NA + 5 * h.n[0]);
    dim3 g(n_kin * h.ntile);
    const size_t l4 = off + red_bytes<T, 4>(), l8 = off + red_bytes<T, MAXF>();
    if (h.nfmax <= 4) hipLaunchKernelGGL((k_correct_fast<T, VD, 4, U>), g, dim3(BLOCK), l4, s, cv, n_kin, cur);
    else hipLaunchKernelGGL((k_correct_fast<T, VD, MAXF, U>), g, dim3(BLOCK), l8, s, cv, n_kin, cur);
}

template <typename T, int VD>
void launch_correct_t(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    int U = rounds_u(h.vdim, h.n[1] * h.n[2] / BLOCK, sizeof(T), h.nfmax);
    static const int umax = [] {
        const char *e = std::getenv("GSIS_CORRECT_U");
        return e ? std::atoi(e) : CORRECT_UMAX;
    }();
    while (U > 1 && U > umax) U /= 2;
    if (U == 4) launch_correct_u<T, VD, 4>(cv, h, n_kin, cur, s);
    else if (U == 2) launch_correct_u<T, VD, 2>(cv, h, n_kin, cur, s);
    else launch_correct_u<T, VD, 1>(cv, h, n_kin, cur, s);
}

// 16-byte rows for the correction where the sweep takes them (GSIS_CORRECT_V4=0
// keeps 4-byte rows)
static bool correct_v4_on()
{
    static const bool on = [] {
        const char *e = std::getenv("GSIS_CORRECT_V4");
        return !(e && e[0] == '0');
    }();
    return on;
}

template <typename T>
void launch_correct_v4(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    const size_t lds = red_offset<T>((size_t)XREC * h.n[0]) + sizeof(double) * (BLOCK / 16) * NSUM;
    const dim3 g(n_kin * h.ntile);
    if (h.nfmax <= 4) hipLaunchKernelGGL((k_correct_v4<T, 4>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
    else hipLaunchKernelGGL((k_correct_v4<T, MAXF>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
}

// the two-VDF correction in 16-byte rows, where the tile covers whole
// x-planes; false leaves the case to the per-node kernel
bool launch_correct_poly_v4(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    if (!(h.vdim == 3 && sweep_v4_fits(h.n[1], h.n[2]) && h.tile % (h.n[1] * h.n[2]) == 0 && correct_v4_on()))
        return false;
    const dim3 g(n_kin * h.ntile);
    if (h.dtype == GSIS_F32) {
        const size_t lds = red_offset<float>((size_t)XREC * h.n[0]) + sizeof(double) * (BLOCK / 16) * NSUM;
        if (h.nfmax <= 4) hipLaunchKernelGGL((k_correct_poly_v4<float, 4>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_correct_poly_v4<float, MAXF>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
    } else {
        const size_t lds = red_offset<double>((size_t)XREC * h.n[0]) + sizeof(double) * (BLOCK / 16) * NSUM;
        if (h.nfmax <= 4) hipLaunchKernelGGL((k_correct_poly_v4<double, 4>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
        else hipLaunchKernelGGL((k_correct_poly_v4<double, MAXF>), g, dim3(BLOCK), lds, s, cv, n_kin, cur);
    }
    return true;
}

hipError_t launch_correct_fast(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s)
{
    if (h.vdim == 3 && sweep_v4_fits(h.n[1], h.n[2]) && correct_v4_on()) {
        if (h.dtype == GSIS_F32) launch_correct_v4<float>(cv, h, n_kin, cur, s);
        else launch_correct_v4<double>(cv, h, n_kin, cur, s);
        return hipGetLastError();
    }
    if (h.dtype == GSIS_F32) {
        if (h.vdim == 3) launch_correct_t<float, 3>(cv, h, n_kin, cur, s);
        else launch_correct_t<float, 2>(cv, h, n_kin, cur, s);
    } else {
        if (h.vdim == 3) launch_correct_t<double, 3>(cv, h, n_kin, cur, s);
        else launch_correct_t<double, 2>(cv, h, n_kin, cur, s);
    }
    return hipGetLastError();
}

}  // namespace gsis
