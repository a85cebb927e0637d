// gsis_impl.hpp -- internal declarations shared by the library's HIP sources.
//
// A bound case lives entirely inside one caller-owned device workspace.  The
// device-side view of that workspace is a CaseView (plain pointers and
// sizes), itself stored at the start of the workspace so that kernels, graph
// replays and batched launches can find every array from one pointer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsis.h"

namespace gsis {

constexpr int BLOCK = 256;             // threads per block of the streaming kernels
constexpr int MAXF = GSIS_MAX_FACES;
constexpr int MAXW = GSIS_MAX_WALL_FACES;
constexpr int MAXA = GSIS_MAX_AXIS;
constexpr int NSUM = 24;               // per (slot, tile) partial sums, see below
constexpr int MAX_BATCH = 64;          // cases per batched launch (the batch structures stay under 4 KB of kernel arguments)
// per-slot moment record: the GSIS_NMOM moments, the MAXW outgoing wall
// fluxes, then (polyatomic gas) T_r and q_r
constexpr int MOMS = GSIS_NMOM + MAXW + 4;
constexpr int MOM_INT = GSIS_NMOM + MAXW;

// Partial sums written by every kernel that produces a VDF (init, sweep,
// correction), per (slot, velocity tile), relative to the slot's reference
// velocity u_ref = ParamRec::u:
//   3D: [0] sum w f, [1..3] sum w f c, [4..9] sum w f c_d c_e (xx yy zz xy xz yz),
//       [10..12] sum w f c^2 c_d
//   2D: [0] sum w phi, [1..2] sum w phi c, [3..5] (xx yy xy), [6..7] sum w phi c^2 c_d,
//       [8] sum w psi, [9..10] sum w psi c_d
//   [13..17] moment balance of the kinetic scheme at the old iterate
//       sum w D (f_new - f_old) (1, c_x, c_y, c_z, c^2 [+ psi]) (sweep only)
//   [18..21] sum_{a > 0} w a phi per wall face of the cell (a = xi.n S/V)
enum { S_RES = 13, S_WALL = 18 };
constexpr int PSUM = 5;                // per (slot, tile) sums of the second function (two-VDF gas)

// Per-slot parameters of the relaxation target (FP64; Sec. 2 reference
// distribution specialised to d_r = 0, with the conservation fix-up).
struct ParamRec {
    double u[3];      // mean velocity of f^n (reference frame of the sums)
    double it;        // 1 / T
    double Th;        // T / 2 (psi factor of the reduced pair)
    double itau;      // 1 / tau
    double kq[3];     // K q_d, K = (4/5)(1 - Pr) / (p T)
    double fx[5];     // fix-up multiplier (a0, a_x, a_y, [a_z], b), amplitude folded in
    double rw[MAXW];  // densities of the diffuse-wall faces (Jacobi: from f^n)
    double pad[3];
};

// Polyatomic gas (Sec. 2 two-VDF model): per-slot coefficients of the targets
//   G0 = P(c) [at Et (1 + kt.c (c^2/T_t - 5/2)) + ar Er (1 + k0.c (c^2/T - 5/2))]
//   G1 = P(c) [tht at Et (...) + Et bt.c + thr ar Er (...) + Er br.c]
// with Et = exp(-c^2/T_t), Er = exp(-c^2/T), c = xi - u and the fix-up
// P(c) = fx0 + fx.c + fx4 c^2; the (1 - 1/Z_r) and 1/Z_r weights are folded
// into at, bt and ar, br.
struct PolyRec {
    double u[3];
    double itt, it;      // 1 / T_t, 1 / T
    double itau;         // 1 / tau, tau = mu(T_t) / p_t
    double at, ar;       // rho (pi T_t)^-3/2 (1 - 1/Z_r), rho (pi T)^-3/2 / Z_r
    double kt[3], k0[3]; // (4/15) q_t / (T_t p_t), (4/15) q_0 / (T p)
    double tht, thr;     // d_r T_r / 4, d_r T / 4
    double bt[3], br[3]; // (pi T_t)^-3/2 (1 - 1/Z_r) q_r / T_t, (pi T)^-3/2 q_1 / (T Z_r)
    double fx[5];
    double rw[MAXW];     // wall densities (Jacobi: from f0^n)
};

// Conservation-fixed Maxwellian f_eq(W) (Sec. 3.2): amplitude-folded
// multiplier (a0 + a.c + b c^2) times exp(-c^2/T), c = xi - u.
struct FeqRec {
    double u[3];
    double it;
    double Th;
    double fx[5];
};

// Grad-13 source coefficients (Sec. 3.2 eq. G13_VDF) for one cell state.
struct G13Rec {
    double A;         // rho (pi T)^(-3/2)  [2D: rho / (pi T)]
    double u[3];
    double it, T;
    double s[6];      // sigma / (p T)   (xx yy zz xy xz yz)
    double q[3];      // 2 q / (p T)
};

struct CaseView {
    // sizes
    int32_t n_cells, n_faces, n_patches, dim, nnz;
    int32_t vdim, nfun, n[3], nv, row;      // row = nfun * nv_pad (elements per slot)
    int32_t tile, ntile;        // velocity nodes per tile (a contiguous k range), tiles per row
    int32_t fast, xp;           // fast sweep layout: x-planes (3D) or x-lines (2D) per tile
    int32_t capacity;
    int32_t dtype;
    double Kn, omega, Pr, inv_dt;
    // mesh
    const int32_t *cf_ptr;      // [n_cells + 1]
    const int32_t *cf_face;     // [nnz] face id
    const int32_t *cf_other;    // [nnz] neighbour cell, or -1 - patch
    const int32_t *cf_wall;     // [nnz] wall-sum index of the face in its cell, -1 otherwise
    const double *cf_nsv;       // [nnz][3] outward n S / V
    const double *lsq;          // [2][nnz][3] least-squares coefficients (all faces / no wall faces)
    const double *cf_fs;        // [nnz] -S_f if the cell owns the face, +S_f otherwise
    const double *cell_sS;      // [n_cells][2] sum S_f, sum S_f / d_f
    const double *wall_den;     // [nnz] sum_{xi.n<0} w |xi.n| M(1, u_w, T_w) (wall faces)
    const int32_t *face_cells;  // [n_faces][2]
    const double *face_normal;  // [n_faces][3]
    const double *face_area;
    const double *face_center;  // [n_faces][3]
    const double *face_dist;    // [n_faces] normal distance between centroids (interior) or twice
                                // the centroid-face normal distance (boundary)
    const double *face_dx;      // [n_faces][3] x_R - x_L between the centroids (interior faces), 0 on boundaries
    const double *cell_volume;
    const double *cell_center;  // [n_cells][3]
    const int32_t *patch_kind;
    const double *patch_state;  // [n_patches][5]
    const int32_t *wall_face;   // [n_wall] boundary faces on diffuse walls, ascending id
    int32_t n_wall, pad_w;
    const double *xv;           // [3][MAXA] nodes
    const double *wv;           // [3][MAXA] weights
    const double *vpt;          // point-set grids: [nv][4] node (3) and weight
    const float *vptf;          // the same rounded to FP32 (node tables of the FP32 kernels)
    int32_t points, pad_p;      // 1: the velocity grid is the point set vpt
    // region
    int32_t *flags;             // [n_cells] 1 = kinetic
    int32_t *slot_of_cell;      // [n_cells], -1 for NS cells
    int32_t *kin_cell;          // [capacity] ascending cell id
    int32_t *n_kin_dev;         // device copy of the kinetic count
    int32_t *new_cell;          // [capacity] cells that became kinetic at the last update
    int32_t *n_new_dev;
    int32_t *scan_tmp;          // [max(n_cells, capacity) + 1024] scratch for scans
    int32_t *status;            // [4] sticky error flags (0 nonfinite, 1 capacity)
    // boundary rows used by the fast sweep: every face is a row times a scale
    void *prow;                 // [n_patches][row] wall: M(1, u_w, T_w); far field: M(rho, u, T)
    void *grow;                 // [gcap][row] Grad-13 rows of NS cells next to the kinetic region
    int32_t *ghost_slot;        // [n_cells] row of the cell in grow, -1 otherwise
    int32_t *ghost_cell;        // [gcap] ascending cell id
    int32_t *n_ghost_dev;
    int32_t gcap, nfmax;
    // per-slot axis tables of the relaxation target for the plane sweep, in the
    // case dtype: offsets c, Gaussian factors E, fix-up parts P, Shakhov parts K
    // (each [NA]), then the x axis' low parts (5 nx); tabp elements per slot
    void *axtab;
    int32_t tabp, order;        // order: sweep blocks 0 = tile-major, 1 = cell-major,
                                // 2 = groups of `group` cells, tile-major inside a group
    int32_t group, pad_g;
    // spatial order 2 (second-order face values): the reconstruction increments
    // of every face of every kinetic cell, slope [capacity][nfmax][row] in the
    // case dtype (delta_l = phi g . (x_face_l - x_cell) per VDF value), each
    // cell's largest outflow rate amax [n_cells], per (slot, tile) sums over the
    // wall faces wsl [capacity][ntile][MAXW] of sum_{a>0} w a delta (the
    // reconstruction part of the next wall densities), and cf_back [nnz], the
    // local index of each face in the neighbour's face list (-1 on boundaries)
    int32_t sorder, pad_o;
    double damp2;
    // polyatomic gas (d_r > 0): rows hold (f0, f1); per-slot target records and
    // per (slot, tile) sums of the second function [PSUM]: sum w f1, sum w c f1
    // (3), and (sweep only) the balance sum w D (f1_new - f1_old) at the old iterate
    int32_t poly, pad_p2;
    double dr, Zr, A[4];
    PolyRec *prec;
    double *psum;
    void *slope;
    double *amax;
    double *wsl;
    const int32_t *cf_back;
    // kinetic state
    void *f[2];                 // VDF double buffer [capacity][row]
    ParamRec *param;            // [capacity]
    FeqRec *feq;                // [capacity][2] (new, half)
    double *partial;            // [capacity][ntile][NSUM]
    double *mom;                // [capacity][MOMS]
    // macroscopic state (FP64, every cell)
    double *W;                  // [n_cells][5] current W^n
    double *Wh;                 // [n_cells][5] W^{n+1/2}
    double *Wn;                 // [n_cells][5] work / W^{n+1}
    double *U;                  // [n_cells][5] conserved
    double *grad;               // [n_cells][6][3]  (ux uy uz T rho |u|)
    double *ghost;              // [n_cells][GSIS_NMOM] Grad-13 parameters
    double *hot;                // [n_cells][9]
    double *src;                // [n_cells][5]
    double *Rk;                 // [n_cells][5] kinetic moment balance per unit volume
    double *Rm;                 // [n_cells][5]
    double *fflux;              // [n_faces][5]
    double *hface;              // [n_faces][4] face means of the high-order terms: sigma.n (3), q.n (1)
    double *dloc;               // [n_cells]
    double *red;                // [1024 * 8] reduction scratch
    double *eps;                // [8]
    // range limit of the Grad-13 rows (<= 0: unlimited), the factor each cell's
    // (sigma, q) was scaled by at the last Grad-13 build [n_cells], and the
    // cumulative limiter counters (see gsis_limiter_stats): rows built and rows
    // limited for ghosts [0, 1] and new cells [2, 3], corrections applied and
    // cut [4, 5]
    double g13_rmax;
    double *g13_th;
    unsigned long long *lim;
    // two-VDF gas, synthetic side (Sec. 2 eq. macroscopic_equation_2, last line):
    // the internal temperature T_r of W^n, W^{n+1/2} and W^{n+1} [n_cells] each,
    // rho e_r during the pseudo-time steps, its source, kinetic and synthetic
    // balances [n_cells], face fluxes and HoT face means of rho e_r [n_faces],
    // HoT of q_r [n_cells][3], the gradient of T_r [n_cells][3] and the Grad-13
    // parameters T_r, q_r of every cell [n_cells][4]
    double *Tr, *Trh, *Trn, *Ur, *srcr, *Rkr, *Rmr;
    double *fr, *hfr, *hotr, *gTr, *ghr;
};

// Logical index of workgroup b of nb.  Workgroups are dispatched round-robin
// over the 8 XCDs; this gives XCD x the contiguous range [x q + min(x, rem), ...)
// of logical blocks, so that the work of neighbouring blocks (cells of a
// locality-ordered mesh, their rows and faces) shares that XCD's L2.  A
// bijection on [0, nb): blocks keep their work, so results do not change.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int X = 8;
    const int x = b % X, r = b / X, q = nb / X, rem = nb % X;
    return x * q + min(x, rem) + r;
}

struct Batch {
    const CaseView *cv[MAX_BATCH];
    int32_t start[MAX_BATCH + 1];   // prefix of work items (blocks) per case
    int32_t n;
    int32_t nfmax;                  // largest faces-per-cell over the cases
    int32_t mdiv;                   // plane kernel, 3D: gcd over the cases of the y-values per lane
                                    // and plane, M = n_y n_z / 256 (load rounds must divide it)
    int32_t cur[MAX_BATCH];         // per case: the buffer holding f^n (the sweep writes the other)
    int32_t order;                  // 0: blocks tile-major, 1: cell-major (all tiles of a cell together),
                                    // 2: groups of `group` consecutive cells, tile-major inside each group
    int32_t group;
    int32_t v4;                     // 3D plane layout read as 16-byte rows (every case fits sweep_v4_fits)
};

// Cases of one batched macroscopic launch: each case owns whole blocks
// (cell kernels: MBLOCK cells per block, face kernels: MBLOCK_F faces), so the
// case of a block is block-uniform.
constexpr int MBLOCK = 256;
constexpr int MBLOCK_F = 128;
constexpr int MCELLS_Q = 64;     // cells per block of the lane-per-face kernels
struct MBatch {
    const CaseView *cv[MAX_BATCH];
    double *W[MAX_BATCH];            // state advanced by the pseudo-time steps
    double *Tr[MAX_BATCH];           // two-VDF gas: its internal temperature (else null)
    const double *hot[MAX_BATCH];    // [n_cells][9] high-order terms
    const double *src[MAX_BATCH];    // [n_cells][5] sources per unit volume, or null
    int32_t bc[MAX_BATCH + 1];       // prefix of cell blocks
    int32_t bf[MAX_BATCH + 1];       // prefix of face blocks
    int32_t bq[MAX_BATCH + 1];       // prefix of cell-group blocks (MCELLS_Q cells, one lane per face)
    int32_t n;
    int32_t nfmax;
    int32_t poly;                    // the cases are two-VDF gases (synthetic equations with rho e_r)
};

// velocity node k and its weight: tensor grids (k = (ix n1 + iy) n2 + iz, or
// ix n1 + iy reduced) or point sets
__device__ __forceinline__ void vnode(const CaseView &C, int k, double *xi, double &w)
{
    if (C.points) {
        const double *q = C.vpt + 4 * (size_t)k;
        xi[0] = q[0];
        xi[1] = q[1];
        xi[2] = q[2];
        w = q[3];
        return;
    }
    int ix, iy, iz = 0;
    if (C.vdim == 3) {
        iz = k % C.n[2];
        iy = (k / C.n[2]) % C.n[1];
        ix = k / (C.n[2] * C.n[1]);
    } else {
        iy = k % C.n[1];
        ix = k / C.n[1];
    }
    xi[0] = C.xv[ix];
    xi[1] = C.xv[MAXA + iy];
    xi[2] = (C.vdim == 3) ? C.xv[2 * MAXA + iz] : 0.0;
    w = C.wv[ix] * C.wv[MAXA + iy] * ((C.vdim == 3) ? C.wv[2 * MAXA + iz] : 1.0);
}

// --- binding (gsis_api.cpp, gsis_static.hip) ----------------------------------
gsis_status bind_impl(gsis_case c, void *ws, size_t bytes, int64_t cap, void *stream, bool with_events);
void unbind_case(gsis_case c);
gsis_status set_error(gsis_status code, const char *msg);
// forget c as the holder of a device's static workspace (destroy, re-bind)
void static_release(gsis_case c);

// --- launch wrappers (gsis_kinetic.hip) ---------------------------------------
hipError_t launch_wall_den(const CaseView *cv, const CaseView &h, hipStream_t s);
// mode 0: conservation-fixed Maxwellian of W on the kinetic cells; mode 1:
// Grad-13 of ghost[] on the new cells; mode 2: keep the rows, recompute sums
hipError_t launch_fill(const CaseView *cv, const CaseView &h, int mode, int n_items, int cur, hipStream_t s);
hipError_t launch_reduce(const CaseView *cv, const CaseView &h, int n_kin, int with_res, hipStream_t s);
hipError_t launch_param(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);
hipError_t launch_feqpar(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);
hipError_t launch_sweep(const Batch &b, const CaseView &h0, int total_items, hipStream_t s);
// (gsis_sweep.hip) tensor grids whose fastest axis divides the block
hipError_t launch_sweep_fast(const Batch &b, const CaseView &h0, int total_items, hipStream_t s);
bool sweep_v4_fits(int ny, int nz);
bool o2_v4_fits(const CaseView &h);
hipError_t launch_sweep_o2v4(const Batch &b, const CaseView &h0, int total, hipStream_t s);
hipError_t launch_axtab(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);
// spatial order 2: largest outflow rate per cell (at bind), limited slopes of f[cur]
hipError_t launch_amax(const CaseView *cv, const CaseView &h, hipStream_t s);
hipError_t launch_slope(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s);
hipError_t launch_correct(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s);
bool launch_correct_poly_v4(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s);
hipError_t launch_correct_fast(const CaseView *cv, const CaseView &h, int n_kin, int cur, hipStream_t s);
hipError_t launch_patch_rows(const CaseView *cv, const CaseView &h, hipStream_t s);
hipError_t launch_ghost_rows(const CaseView *cv, const CaseView &h, int n_ghost, hipStream_t s);
hipError_t launch_gather_vdf(const CaseView *cv, const CaseView &h, int n_kin, int cur, void *out, int dir,
                             hipStream_t s);

// --- launch wrappers (gsis_macro.hip) ----------------------------------------
hipError_t launch_lsq(const CaseView *cv, const CaseView &h, const double *W, int nvar, hipStream_t s);
hipError_t launch_lsq_batch(const MBatch &b, int nvar, hipStream_t s);
hipError_t launch_ghost(const CaseView *cv, const CaseView &h, const double *W, hipStream_t s);
// add to the limiter counters lim[2 which], lim[2 which + 1] the n cells of
// list and those whose Grad-13 pair was scaled (list and n from the host)
hipError_t launch_count_g13(const CaseView *cv, const int32_t *list, int n, int which, hipStream_t s);
hipError_t launch_hot(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);
hipError_t launch_whalf(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);
hipError_t launch_macro_residual(const CaseView *cv, const CaseView &h, const double *W, const double *hot,
                                 double *Rout, hipStream_t s);
hipError_t launch_src(const CaseView *cv, const CaseView &h, int n_kin, hipStream_t s);
// n_inner pseudo-time steps for every case of a batch (cfl > 0 local steps,
// cfl < 0 one global step per case)
hipError_t launch_macro_steps_batch(const MBatch &b, int n_inner, double cfl, hipStream_t s);
void mbatch_add(MBatch &b, const CaseView *cv, const CaseView &h, double *W, const double *hot, const double *src,
                double *Tr = nullptr);
hipError_t launch_macro_steps(const CaseView *cv, const CaseView &h, double *W, const double *hot,
                              const double *src, int n_inner, double cfl, hipStream_t s);
hipError_t launch_eps(const CaseView *cv, const CaseView &h, const double *Wnew, const double *Wold,
                      hipStream_t s);
hipError_t launch_flags(const CaseView *cv, const CaseView &h, double Kn_ref, int layers, hipStream_t s);
hipError_t launch_compact(const CaseView *cv, const CaseView &h, hipStream_t s);   // also builds the ghost list
hipError_t launch_copy_W(double *dst, const double *src, int n, hipStream_t s);
// flags NULL: every cell gets `fill`
hipError_t launch_set_flags(const CaseView *cv, const CaseView &h, const uint8_t *flags, int fill, hipStream_t s);
hipError_t launch_get_flags(const CaseView *cv, const CaseView &h, uint8_t *flags, hipStream_t s);
hipError_t launch_moments_out(const CaseView *cv, const CaseView &h, int n_kin, double *out, int32_t *kc,
                              hipStream_t s);
// polyatomic gas: T_r, q_r per kinetic cell [n_kin][4]
hipError_t launch_internal_out(const CaseView *cv, const CaseView &h, int n_kin, double *out, hipStream_t s);
hipError_t launch_W_from_mom(const CaseView *cv, const CaseView &h, int n_kin, double *W, hipStream_t s);
// surface quantities of the wall faces (GSIS_NSURF per face) and optional totals
hipError_t launch_surface(const CaseView *cv, const CaseView &h, int cur, double *out, double *totals, hipStream_t s);
hipError_t launch_check_W(const CaseView *cv, const CaseView &h, const double *W, hipStream_t s);

// --- two-VDF gas, synthetic side (gsis_poly.hip) -----------------------------
// Grad-13 parameters (ghost, ghr) of every cell from W, Tr and their gradients
// (grad rows of W from launch_lsq, the T_r gradient computed here)
hipError_t launch_ghost_poly(const CaseView *cv, const CaseView &h, const double *W, const double *Tr, hipStream_t s);
// HoT of sigma, q_t (hot) and q_r (hotr) on kinetic cells at W^{n+1/2}
hipError_t launch_hot_poly(const CaseView *cv, const CaseView &h, hipStream_t s);
hipError_t launch_surface_ns_poly(const CaseView *cv, const CaseView &h, double *out, hipStream_t s);
// out = T_r of the moments on kinetic cells, Tr elsewhere (out may be Tr)
hipError_t launch_tr_half(const CaseView *cv, const CaseView &h, double *out, hipStream_t s);
// synthetic residual per unit volume at (W, Tr), with the exchange source
hipError_t launch_macro_residual_poly(const CaseView *cv, const CaseView &h, const double *W, const double *Tr,
                                      const double *hot, double *Rout, double *Rrout, hipStream_t s);
hipError_t launch_src_poly(const CaseView *cv, const CaseView &h, hipStream_t s);
hipError_t launch_macro_steps_poly(const MBatch &b, int n_inner, double cfl, hipStream_t s);
hipError_t launch_copy_d(double *dst, const double *src, int n, hipStream_t s);
// out[i] = T_t of W (every cell)
hipError_t launch_tt_copy(const CaseView *cv, const CaseView &h, double *out, hipStream_t s);

}  // namespace gsis
