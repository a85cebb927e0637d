// gsis_api.cpp -- host side of the C ABI declared in include/gsis.h.
//
// Validates arguments, builds the per-cell face lists, lays a bound case out
// inside the caller's device workspace, and sequences the kernels of one
// outer iteration of the method (Sec. 3.4 of arXiv 2501.02245).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "gsis_impl.hpp"

using namespace gsis;

namespace {

thread_local std::string g_err;

gsis_status fail(gsis_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(GSIS_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct Segment {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

}  // namespace

struct gsis_mesh_s {
    int32_t dim, n_cells, n_faces, n_patches, nnz, max_faces = 0;
    std::vector<int32_t> face_cells, cf_ptr, cf_face, cf_other, cf_wall, patch_kind;
    std::vector<int32_t> cf_back;      // [nnz] local index of the face in the neighbour's list, -1 on boundaries
    std::vector<int32_t> wall_faces;   // boundary faces on diffuse-wall patches, ascending id
    std::vector<double> face_normal, face_area, face_center, cell_volume, cell_center, cf_nsv, face_dist,
        face_dx, patch_state;
    // geometry-only factors of the macroscopic kernels
    std::vector<double> lsq;      // [2][nnz][3] least-squares coefficients: all faces / no wall faces
    std::vector<double> cf_fs;    // [nnz] -S (owner) or +S: the face's sign and area in the cell balance
    std::vector<double> cell_sS;  // [n_cells][2] sum S, sum S / d over the cell's faces
    int refs = 0;
};

struct gsis_case_s {
    gsis_mesh mesh = nullptr;
    gsis_gas gas{};
    int32_t dtype = GSIS_F32;
    int32_t vdim = 0, n[3] = {0, 0, 0}, nv = 0;
    double xv[3][MAXA], wv[3][MAXA];
    std::vector<double> vpt;    // point-set grid: [nv][4] = xi (3), w
    std::vector<double> vt;     // node table the kernels read (see node_table), kept with the grid
    std::vector<float> vtf;     // the same rounded to FP32
    bool points = false;
    int32_t order = 1;          // spatial order of the kinetic face values
    double damp2 = 2.0;         // pseudo-time factor of the order-2 iteration
    double dr = 0.0, Zr = 1.0, A[4] = {0, 0, 0, 0};   // polyatomic gas (dr > 0)
    double g13_rmax = 0.5;      // range limit of the Grad-13 rows (<= 0: none)
    bool grid_set = false, bound = false, state_set = false;
    int32_t capacity = 0, tile = 0, ntile = 0, row = 0;
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    CaseView hv{};             // host copy of the device view
    CaseView *cv = nullptr;    // device view inside the workspace
    int n_kin = 0, n_ghost = 0, cur = 0, iter = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
};

namespace {
void drop_graphs_of(gsis_case c);   // captured synthetic solves that use the case
void refresh_node_table(gsis_case c);   // node tables of the kernels, rebuilt when grid or order change
}  // namespace

extern "C" const char *gsis_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// mesh
// ---------------------------------------------------------------------------
namespace {

// Gauss elimination with partial pivoting (n <= 3); false if a pivot vanishes
bool solve_small_host(int n, double *A, double *b)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
        if (!(std::fabs(A[piv * n + col]) > 0.0)) return false;
        if (piv != col) {
            for (int j = 0; j < n; ++j) std::swap(A[col * n + j], A[piv * n + j]);
            std::swap(b[col], b[piv]);
        }
        for (int r = col + 1; r < n; ++r) {
            double fac = A[r * n + col] / A[col * n + col];
            for (int j = col; j < n; ++j) A[r * n + j] -= fac * A[col * n + j];
            b[r] -= fac * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double v = b[r];
        for (int j = r + 1; j < n; ++j) v -= A[r * n + j] * b[j];
        b[r] = v / A[r * n + r];
    }
    return true;
}

// Least-squares gradient (Sec. 3.4 Step 2) as fixed per-face coefficients:
// grad phi_i = sum_e c_e (phi_e - phi_i), c_e = A^-1 w_e dx_e with
// A = sum_e w_e dx_e dx_e^T, w_e = 1/|dx_e|^2, dx_e to the neighbour centroid
// (or the face centre on a boundary).  Variant 1 leaves out wall faces (no
// density is prescribed there).  A singular system gives a zero gradient.
// Also the signed face areas of the cell balance and the per-cell sums
// sum S and sum S/d of the local pseudo-time step.
void build_macro_factors(gsis_mesh_s *m)
{
    const int dim = m->dim;
    m->lsq.assign(6 * (size_t)m->nnz, 0.0);
    m->cf_fs.assign(m->nnz, 0.0);
    m->cell_sS.assign(2 * (size_t)m->n_cells, 0.0);
    for (int i = 0; i < m->n_cells; ++i) {
        const int e0 = m->cf_ptr[i], e1 = m->cf_ptr[i + 1];
        for (int var = 0; var < 2; ++var) {
            double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            double dxs[MAXF][3], wgt[MAXF];
            bool use[MAXF];
            for (int e = e0; e < e1; ++e) {
                const int l = e - e0, oth = m->cf_other[e];
                use[l] = !(var == 1 && oth < 0 && m->patch_kind[-1 - oth] == GSIS_PATCH_WALL);
                const double *xo = (oth >= 0) ? &m->cell_center[3 * (size_t)oth]
                                              : &m->face_center[3 * (size_t)m->cf_face[e]];
                double r2 = 0.0;
                for (int d = 0; d < 3; ++d) dxs[l][d] = xo[d] - m->cell_center[3 * (size_t)i + d];
                for (int d = 0; d < dim; ++d) r2 += dxs[l][d] * dxs[l][d];
                wgt[l] = 1.0 / r2;
                if (!use[l]) continue;
                for (int a = 0; a < dim; ++a)
                    for (int c = 0; c < dim; ++c) A[a * dim + c] += wgt[l] * dxs[l][a] * dxs[l][c];
            }
            double Ainv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            bool ok = true;
            for (int col = 0; col < dim && ok; ++col) {
                double Ac[9], b[3] = {0, 0, 0};
                std::copy(A, A + 9, Ac);
                b[col] = 1.0;
                ok = solve_small_host(dim, Ac, b);
                for (int r = 0; r < dim; ++r) Ainv[r * dim + col] = b[r];
            }
            if (!ok) continue;
            for (int e = e0; e < e1; ++e) {
                const int l = e - e0;
                if (!use[l]) continue;
                for (int a = 0; a < dim; ++a) {
                    double v = 0.0;
                    for (int c = 0; c < dim; ++c) v += Ainv[a * dim + c] * wgt[l] * dxs[l][c];
                    m->lsq[3 * ((size_t)var * m->nnz + e) + a] = v;
                }
            }
        }
        for (int e = e0; e < e1; ++e) {
            const int f = m->cf_face[e];
            const double S = m->face_area[f];
            m->cf_fs[e] = (m->face_cells[2 * f] == i) ? -S : S;
            m->cell_sS[2 * (size_t)i] += S;
            m->cell_sS[2 * (size_t)i + 1] += S / m->face_dist[f];
        }
    }
}

}  // namespace

extern "C" gsis_status gsis_create_mesh(const gsis_mesh_desc *d, gsis_mesh *out)
{
    if (!d || !out) return fail(GSIS_E_ARG, "null argument");
    *out = nullptr;
    if (d->dim < 1 || d->dim > 3) return fail(GSIS_E_ARG, "dim must be 1, 2 or 3");
    if (d->n_cells <= 0 || d->n_faces < 0 || d->n_patches < 0) return fail(GSIS_E_ARG, "bad sizes");
    if (d->n_faces > 0 && (!d->face_cells || !d->face_normal || !d->face_area || !d->face_center))
        return fail(GSIS_E_ARG, "null face array");
    if (!d->cell_volume || !d->cell_center) return fail(GSIS_E_ARG, "null cell array");
    if (d->n_patches > 0 && !d->patches) return fail(GSIS_E_ARG, "null patches");
    auto *m = new gsis_mesh_s();
    m->dim = d->dim;
    m->n_cells = d->n_cells;
    m->n_faces = d->n_faces;
    m->n_patches = d->n_patches;
    const int nc = d->n_cells, nf = d->n_faces;
    m->face_cells.assign(d->face_cells, d->face_cells + 2 * nf);
    m->face_normal.assign(d->face_normal, d->face_normal + 3 * nf);
    m->face_area.assign(d->face_area, d->face_area + nf);
    m->face_center.assign(d->face_center, d->face_center + 3 * nf);
    m->cell_volume.assign(d->cell_volume, d->cell_volume + nc);
    m->cell_center.assign(d->cell_center, d->cell_center + 3 * nc);
    for (int p = 0; p < d->n_patches; ++p) {
        const gsis_patch &P = d->patches[p];
        if (P.kind != GSIS_PATCH_WALL && P.kind != GSIS_PATCH_FAR) {
            delete m;
            return fail(GSIS_E_ARG, "patch %d: unknown kind %d", p, P.kind);
        }
        if (!(P.T > 0) || (P.kind == GSIS_PATCH_FAR && !(P.rho > 0))) {
            delete m;
            return fail(GSIS_E_ARG, "patch %d: non-positive state", p);
        }
        m->patch_kind.push_back(P.kind);
        m->patch_state.insert(m->patch_state.end(), {P.rho, P.u[0], P.u[1], P.u[2], P.T});
    }
    // validate and build the per-cell face lists
    std::vector<int32_t> cnt(nc + 1, 0);
    for (int f = 0; f < nf; ++f) {
        int a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
        if (a < 0 || a >= nc || b >= nc || (b < 0 && -1 - b >= d->n_patches) || a == b) {
            delete m;
            return fail(GSIS_E_MESH, "face %d: bad cell/patch index (%d, %d)", f, a, b);
        }
        if (!(m->face_area[f] > 0)) {
            delete m;
            return fail(GSIS_E_MESH, "face %d: area must be positive", f);
        }
        double nn = 0;
        for (int k = 0; k < 3; ++k) nn += m->face_normal[3 * f + k] * m->face_normal[3 * f + k];
        if (std::fabs(nn - 1.0) > 1e-9) {
            delete m;
            return fail(GSIS_E_MESH, "face %d: normal is not unit", f);
        }
        cnt[a + 1]++;
        if (b >= 0) cnt[b + 1]++;
    }
    for (int i = 0; i < nc; ++i) {
        if (!(m->cell_volume[i] > 0)) {
            delete m;
            return fail(GSIS_E_MESH, "cell %d: volume must be positive", i);
        }
        if (cnt[i + 1] > MAXF) {
            delete m;
            return fail(GSIS_E_MESH, "cell %d has %d faces (max %d)", i, cnt[i + 1], MAXF);
        }
        cnt[i + 1] += cnt[i];
    }
    m->nnz = cnt[nc];
    for (int i = 0; i < nc; ++i) m->max_faces = std::max(m->max_faces, cnt[i + 1] - cnt[i]);
    m->cf_ptr = cnt;
    m->cf_face.assign(m->nnz, 0);
    m->cf_other.assign(m->nnz, 0);
    m->cf_wall.assign(m->nnz, -1);
    m->cf_back.assign(m->nnz, -1);
    m->cf_nsv.assign(3 * (size_t)m->nnz, 0.0);
    std::vector<int32_t> pos(cnt.begin(), cnt.end() - 1);
    for (int f = 0; f < nf; ++f) {
        int a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
        int e = pos[a]++;
        m->cf_face[e] = f;
        m->cf_other[e] = b;
        for (int k = 0; k < 3; ++k) m->cf_nsv[3 * e + k] = m->face_normal[3 * f + k] * m->face_area[f] / m->cell_volume[a];
        if (b >= 0) {
            const int ea = e;
            e = pos[b]++;
            m->cf_back[ea] = e - cnt[b];
            m->cf_back[e] = ea - cnt[a];
            m->cf_face[e] = f;
            m->cf_other[e] = a;
            for (int k = 0; k < 3; ++k)
                m->cf_nsv[3 * e + k] = -m->face_normal[3 * f + k] * m->face_area[f] / m->cell_volume[b];
        }
    }
    // closure, wall-face numbering, face distances
    for (int i = 0; i < nc; ++i) {
        double s[3] = {0, 0, 0}, A = 0;
        int nw = 0;
        for (int e = m->cf_ptr[i]; e < m->cf_ptr[i + 1]; ++e) {
            int f = m->cf_face[e];
            for (int k = 0; k < 3; ++k) s[k] += m->cf_nsv[3 * e + k] * m->cell_volume[i];
            A += m->face_area[f];
            int b = m->cf_other[e];
            if (b < 0 && m->patch_kind[-1 - b] == GSIS_PATCH_WALL) {
                if (nw >= MAXW) {
                    delete m;
                    return fail(GSIS_E_MESH, "cell %d has more than %d wall faces", i, MAXW);
                }
                m->cf_wall[e] = nw++;
            }
        }
        double sn = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        if (sn > 1e-9 * A) {
            delete m;
            return fail(GSIS_E_MESH, "cell %d is not closed (|sum n S| = %g)", i, sn);
        }
    }
    m->face_dist.assign(nf, 0.0);
    m->face_dx.assign(3 * (size_t)nf, 0.0);
    for (int f = 0; f < nf; ++f) {
        int a = m->face_cells[2 * f], b = m->face_cells[2 * f + 1];
        double dd = 0;
        if (b >= 0) {
            // normal distance between the centroids
            for (int k = 0; k < 3; ++k) {
                m->face_dx[3 * (size_t)f + k] = m->cell_center[3 * b + k] - m->cell_center[3 * a + k];
                dd += m->face_dx[3 * (size_t)f + k] * m->face_normal[3 * f + k];
            }
        } else {
            for (int k = 0; k < 3; ++k) dd += (m->face_center[3 * f + k] - m->cell_center[3 * a + k]) * m->face_normal[3 * f + k];
            dd *= 2.0;
        }
        if (!(dd > 0)) {
            delete m;
            return fail(GSIS_E_MESH, "face %d: centroids do not straddle the face", f);
        }
        m->face_dist[f] = dd;
    }
    build_macro_factors(m);
    for (int f = 0; f < nf; ++f) {
        int b = m->face_cells[2 * f + 1];
        if (b < 0 && m->patch_kind[-1 - b] == GSIS_PATCH_WALL) m->wall_faces.push_back(f);
    }
    *out = m;
    return GSIS_OK;
}

extern "C" gsis_status gsis_destroy_mesh(gsis_mesh m)
{
    if (!m) return fail(GSIS_E_ARG, "null mesh");
    if (m->refs > 0) return fail(GSIS_E_STATE, "mesh still used by %d case(s)", m->refs);
    delete m;
    return GSIS_OK;
}

// ---------------------------------------------------------------------------
// case
// ---------------------------------------------------------------------------
extern "C" gsis_status gsis_create_case(gsis_mesh mesh, const gsis_gas *gas, int32_t vdf_dtype, gsis_case *out)
{
    if (!mesh || !gas || !out) return fail(GSIS_E_ARG, "null argument");
    if (vdf_dtype != GSIS_F32 && vdf_dtype != GSIS_F64) return fail(GSIS_E_ARG, "vdf_dtype must be GSIS_F32 or GSIS_F64");
    if (!(gas->Kn > 0) || !(gas->Pr > 0) || !(gas->Pr <= 1.0) || !std::isfinite(gas->omega))
        return fail(GSIS_E_ARG, "bad gas parameters");
    auto *c = new gsis_case_s();
    c->mesh = mesh;
    c->gas = *gas;
    c->dtype = vdf_dtype;
    mesh->refs++;
    *out = c;
    return GSIS_OK;
}

extern "C" gsis_status gsis_destroy_case(gsis_case c)
{
    if (!c) return fail(GSIS_E_ARG, "null case");
    static_release(c);
    drop_graphs_of(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    c->mesh->refs--;
    delete c;
    return GSIS_OK;
}

extern "C" gsis_status gsis_set_velocity_grid(gsis_case c, int32_t vdim, const int32_t n[3],
                                              const double *const nodes[3], const double *const weights[3])
{
    if (!c || !n || !nodes || !weights) return fail(GSIS_E_ARG, "null argument");
    if (c->bound) return fail(GSIS_E_STATE, "velocity grid must be set before binding");
    if (vdim != 2 && vdim != 3) return fail(GSIS_E_ARG, "vdim must be 2 or 3");
    int64_t nv = 1;
    for (int d = 0; d < vdim; ++d) {
        if (n[d] < 2 || n[d] > MAXA) return fail(GSIS_E_ARG, "axis %d: %d nodes (need 2..%d)", d, n[d], MAXA);
        if (!nodes[d] || !weights[d]) return fail(GSIS_E_ARG, "axis %d: null array", d);
        for (int j = 0; j < n[d]; ++j)
            if (!(weights[d][j] > 0) || !std::isfinite(nodes[d][j])) return fail(GSIS_E_ARG, "axis %d: bad node %d", d, j);
        nv *= n[d];
    }
    if (nv > (1 << 24)) return fail(GSIS_E_ARG, "too many velocity nodes");
    c->vdim = vdim;
    std::memset(c->xv, 0, sizeof c->xv);
    std::memset(c->wv, 0, sizeof c->wv);
    for (int d = 0; d < 3; ++d) {
        c->n[d] = (d < vdim) ? n[d] : 1;
        if (d < vdim)
            for (int j = 0; j < n[d]; ++j) {
                c->xv[d][j] = nodes[d][j];
                c->wv[d][j] = weights[d][j];
            }
    }
    c->nv = (int32_t)nv;
    c->points = false;
    c->vt.clear();
    c->vpt.clear();
    c->grid_set = true;
    refresh_node_table(c);
    return GSIS_OK;
}

extern "C" gsis_status gsis_set_velocity_points(gsis_case c, int32_t np, const double *xi, const double *w)
{
    if (!c || !xi || !w) return fail(GSIS_E_ARG, "null argument");
    if (c->bound) return fail(GSIS_E_STATE, "velocity grid must be set before binding");
    if (np < 1 || np > (1 << 24)) return fail(GSIS_E_ARG, "%d points (need 1..2^24)", np);
    c->vpt.assign(4 * (size_t)np, 0.0);
    for (int k = 0; k < np; ++k) {
        for (int d = 0; d < 3; ++d) {
            if (!std::isfinite(xi[3 * (size_t)k + d])) return fail(GSIS_E_ARG, "point %d: non-finite node", k);
            c->vpt[4 * (size_t)k + d] = xi[3 * (size_t)k + d];
        }
        if (!(w[k] > 0) || !std::isfinite(w[k])) return fail(GSIS_E_ARG, "point %d: weight must be positive", k);
        c->vpt[4 * (size_t)k + 3] = w[k];
    }
    c->vdim = 3;
    std::memset(c->xv, 0, sizeof c->xv);
    std::memset(c->wv, 0, sizeof c->wv);
    for (int d = 0; d < 3; ++d) c->n[d] = 1;
    c->nv = np;
    c->points = true;
    c->grid_set = true;
    refresh_node_table(c);
    return GSIS_OK;
}

extern "C" gsis_status gsis_set_internal_dof(gsis_case c, double d_r, double Z_r, const double *A)
{
    if (!c || !A) return fail(GSIS_E_ARG, "null argument");
    if (c->bound) return fail(GSIS_E_STATE, "internal degrees of freedom must be set before binding");
    if (!(d_r >= 0.0) || !std::isfinite(d_r)) return fail(GSIS_E_ARG, "d_r must be finite and >= 0");
    if (!(Z_r >= 1.0) || !std::isfinite(Z_r)) return fail(GSIS_E_ARG, "Z_r must be finite and >= 1");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(A[i])) return fail(GSIS_E_ARG, "A must be finite");
    c->dr = d_r;
    c->Zr = Z_r;
    for (int i = 0; i < 4; ++i) c->A[i] = A[i];
    return GSIS_OK;
}

extern "C" gsis_status gsis_set_g13_limit(gsis_case c, double rmax)
{
    if (!c) return fail(GSIS_E_ARG, "null case");
    if (c->bound) return fail(GSIS_E_STATE, "the Grad-13 limit must be set before binding");
    if (!std::isfinite(rmax)) return fail(GSIS_E_ARG, "rmax must be finite");
    c->g13_rmax = rmax;
    return GSIS_OK;
}

extern "C" gsis_status gsis_limiter_stats(gsis_case c, int64_t *out, void *stream)
{
    if (!c || !out) return fail(GSIS_E_ARG, "null argument");
    if (!c->bound) return fail(GSIS_E_STATE, "case is not bound to a workspace");
    unsigned long long v[6];
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(v, c->hv.lim, sizeof v, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < 6; ++i) out[i] = (int64_t)v[i];
    return GSIS_OK;
}

extern "C" gsis_status gsis_set_spatial_order(gsis_case c, int32_t order, double damp)
{
    if (!c) return fail(GSIS_E_ARG, "null case");
    if (c->bound) return fail(GSIS_E_STATE, "spatial order must be set before binding");
    if (order != 1 && order != 2) return fail(GSIS_E_ARG, "spatial order must be 1 or 2");
    if (!(damp >= 0.0) || !std::isfinite(damp)) return fail(GSIS_E_ARG, "damp must be finite and >= 0");
    c->order = order;
    c->damp2 = damp;
    if (c->grid_set) refresh_node_table(c);
    return GSIS_OK;
}

namespace {

struct Layout {
    size_t cv, cf_ptr, cf_face, cf_other, cf_wall, cf_nsv, lsq, cf_fs, cell_sS, wall_den, face_cells, face_normal, face_area, face_center,
        face_dist, face_dx, cell_volume, cell_center, patch_kind, patch_state, wallf, xv, wv, vpt, vptf, flags, slot, kin, nkin, newc, nnew, scan,
        status, lim, g13th, prow, grow, gslot, gcell, ngh, axtab, slope, amax, wsl, cf_back, prec, psum, f0, f1, param, feq, partial, mom, W, Wh, Wn, U, grad, ghost, hot, src, Rk, Rm, fflux, hface, dloc, red, eps,
        Tr, Trh, Trn, Ur, srcr, Rkr, Rmr, fr, hfr, hotr, gTr, ghr;
    size_t total;
};

// Tile of the sweep: a contiguous range of velocity nodes per block.  When
// the fastest velocity axis divides the block (3D: n2 | 256 and 256 | n1 n2;
// reduced 2D: n1 | 256) the fast kernel handles whole x-planes / x-lines;
// otherwise the generic kernel takes any contiguous range.
struct TileChoice {
    int tile, ntile, fast, xp;
};

TileChoice choose_tile(const gsis_case_s *c, int64_t cap)
{
    // Default: the largest power-of-two tile (at most a whole row) that still
    // gives at least 4096 blocks at full capacity.  Fewer, longer blocks
    // amortise each block's set-up and final reduction.
    const char *env = std::getenv("GSIS_TILE");
    int target = 32768;
    while (target > 1024 && cap * (int64_t)((c->nv + target - 1) / target) < 4096) target /= 2;
    if (env) target = std::atoi(env);
    if (target < BLOCK) target = BLOCK;
    const char *gen = std::getenv("GSIS_GENERIC_SWEEP");
    const bool allow_fast = !(gen && gen[0] == '1') && !c->points && c->order == 1 && !(c->dr > 0);
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
    TileChoice t{};
    if (allow_fast && c->vdim == 3 && BLOCK % nz == 0 && (ny * nz) % BLOCK == 0) {
        const int P = ny * nz;
        t.fast = 1;
        t.xp = std::max(1, target / P);
        t.tile = t.xp * P;
        t.ntile = (nx + t.xp - 1) / t.xp;
    } else if (allow_fast && c->vdim == 2 && BLOCK % ny == 0) {
        const int q = BLOCK / ny;
        t.fast = 1;
        t.xp = std::max(q, (target / ny) / q * q);
        t.tile = t.xp * ny;
        t.ntile = (nx + t.xp - 1) / t.xp;
    } else {
        target = (target / BLOCK) * BLOCK;
        t.fast = 0;
        t.xp = 0;
        t.tile = c->nv <= target ? c->nv : target;
        t.ntile = (c->nv + t.tile - 1) / t.tile;
    }
    return t;
}

// elements per slot of the plane sweep's axis tables (4 NA + 5 nx, padded to 64)
int axtab_len(const gsis_case_s *c)
{
    const int NA = c->n[0] + c->n[1] + (c->vdim == 3 ? c->n[2] : 0);
    return (4 * NA + 5 * c->n[0] + 63) / 64 * 64;
}

// doubles of the per-node table [nv][4] (node, weight): the point set itself,
// or for a 3D tensor grid at spatial order 2 (whose sweep reads the nodes per
// point, faces as rows) the tensor nodes in row order
size_t node_table_len(const gsis_case_s *c)
{
    if (c->points) return c->vpt.size();
    if (c->order == 2 && c->vdim == 3) return 4 * (size_t)c->nv;
    return 0;
}

std::vector<double> node_table(const gsis_case_s *c);

void refresh_node_table(gsis_case c)
{
    c->vt = node_table(c);
    c->vtf.assign(c->vt.begin(), c->vt.end());
}

std::vector<double> node_table(const gsis_case_s *c)
{
    if (c->points) return c->vpt;
    std::vector<double> t(node_table_len(c));
    if (t.empty()) return t;
    const int n1 = c->n[1], n2 = c->n[2];
    for (int k = 0; k < c->nv; ++k) {
        const int iz = k % n2, iy = (k / n2) % n1, ix = k / (n2 * n1);
        t[4 * (size_t)k + 0] = c->xv[0][ix];
        t[4 * (size_t)k + 1] = c->xv[1][iy];
        t[4 * (size_t)k + 2] = c->xv[2][iz];
        t[4 * (size_t)k + 3] = c->wv[0][ix] * c->wv[1][iy] * c->wv[2][iz];
    }
    return t;
}

// rows reserved for the Grad-13 ghosts of NS cells next to the kinetic region
size_t ghost_capacity(int64_t n_cells, int64_t cap)
{
    return (size_t)std::min<int64_t>(n_cells, std::max<int64_t>(cap, 256));
}

Layout make_layout(const gsis_case_s *c, int64_t cap, int *tile, int *ntile, int *row, int *fast = nullptr,
                   int *xp = nullptr)
{
    const gsis_mesh_s *m = c->mesh;
    const size_t nc = m->n_cells, nf = m->n_faces, nnz = m->nnz, np = std::max(1, m->n_patches);
    const int nfun = (c->vdim == 3 && !(c->dr > 0)) ? 1 : 2;
    const int nvp = (c->nv + 63) / 64 * 64;
    *row = nfun * nvp;
    TileChoice tc = choose_tile(c, cap);
    *tile = tc.tile;
    *ntile = tc.ntile;
    if (fast) *fast = tc.fast;
    if (xp) *xp = tc.xp;
    const size_t es = (c->dtype == GSIS_F32) ? 4 : 8;
    Segment S;
    Layout L;
    L.cv = S.take(sizeof(CaseView));
    L.cf_ptr = S.take(4 * (nc + 1));
    L.cf_face = S.take(4 * nnz);
    L.cf_other = S.take(4 * nnz);
    L.cf_wall = S.take(4 * nnz);
    L.cf_nsv = S.take(24 * nnz);
    L.lsq = S.take(48 * nnz);
    L.cf_fs = S.take(8 * nnz);
    L.cell_sS = S.take(16 * nc);
    L.wall_den = S.take(8 * nnz);
    L.face_cells = S.take(8 * nf);
    L.face_normal = S.take(24 * nf);
    L.face_area = S.take(8 * nf);
    L.face_center = S.take(24 * nf);
    L.face_dist = S.take(8 * nf);
    L.face_dx = S.take(24 * nf);
    L.cell_volume = S.take(8 * nc);
    L.cell_center = S.take(24 * nc);
    L.patch_kind = S.take(4 * np);
    L.patch_state = S.take(40 * np);
    L.wallf = S.take(4 * std::max<size_t>(1, m->wall_faces.size()));
    L.xv = S.take(8 * 3 * MAXA);
    L.wv = S.take(8 * 3 * MAXA);
    L.vpt = S.take(8 * std::max<size_t>(4, node_table_len(c)));
    L.vptf = S.take(4 * std::max<size_t>(4, node_table_len(c)));
    L.flags = S.take(4 * nc);
    L.slot = S.take(4 * nc);
    L.kin = S.take(4 * (size_t)cap);
    L.nkin = S.take(16);
    L.newc = S.take(4 * (size_t)cap);
    L.nnew = S.take(16);
    L.scan = S.take(4 * (2 * nc + 2 * (size_t)cap + 1024));
    L.status = S.take(16);
    L.lim = S.take(64);
    L.g13th = S.take(8 * nc);
    const size_t gcap = ghost_capacity(m->n_cells, cap);
    L.prow = S.take(es * np * (*row));
    L.grow = S.take(es * gcap * (*row));
    L.gslot = S.take(4 * nc);
    L.gcell = S.take(4 * gcap);
    L.ngh = S.take(16);
    L.axtab = S.take(es * (size_t)cap * axtab_len(c));
    const bool o2 = c->order == 2;
    L.slope = S.take(o2 ? es * (size_t)m->max_faces * (size_t)cap * (*row) : 0);
    L.amax = S.take(o2 ? 8 * nc : 0);
    L.wsl = S.take(o2 ? 8 * (size_t)cap * (*ntile) * MAXW : 0);
    L.cf_back = S.take(o2 ? 4 * nnz : 0);
    const bool poly = c->dr > 0;
    L.prec = S.take(poly ? sizeof(PolyRec) * (size_t)cap : 0);
    L.psum = S.take(poly ? 8 * PSUM * (size_t)cap * (*ntile) : 0);
    L.f0 = S.take(es * (size_t)cap * (*row));
    L.f1 = S.take(es * (size_t)cap * (*row));
    L.param = S.take(sizeof(ParamRec) * (size_t)cap);
    L.feq = S.take(2 * sizeof(FeqRec) * (size_t)cap);
    L.partial = S.take(8 * (size_t)cap * (*ntile) * NSUM);
    L.mom = S.take(8 * (size_t)cap * MOMS);
    L.W = S.take(40 * nc);
    L.Wh = S.take(40 * nc);
    L.Wn = S.take(40 * nc);
    L.U = S.take(40 * nc);
    L.grad = S.take(144 * nc);
    L.ghost = S.take(8 * GSIS_NMOM * nc);
    L.hot = S.take(72 * nc);
    L.src = S.take(40 * nc);
    L.Rk = S.take(40 * nc);
    L.Rm = S.take(40 * nc);
    L.fflux = S.take(40 * std::max<size_t>(nf, 1));
    L.hface = S.take(32 * std::max<size_t>(nf, 1));
    L.dloc = S.take(8 * nc);
    L.red = S.take(8 * std::max<size_t>(8192, 8 + 6 * (nc / 256 + 2) + 256));
    L.eps = S.take(64);
    // two-VDF gas, synthetic side
    const size_t pc = poly ? nc : 0, pf = poly ? std::max<size_t>(nf, 1) : 0;
    L.Tr = S.take(8 * pc);
    L.Trh = S.take(8 * pc);
    L.Trn = S.take(8 * pc);
    L.Ur = S.take(8 * pc);
    L.srcr = S.take(8 * pc);
    L.Rkr = S.take(8 * pc);
    L.Rmr = S.take(8 * pc);
    L.fr = S.take(8 * pf);
    L.hfr = S.take(8 * pf);
    L.hotr = S.take(24 * pc);
    L.gTr = S.take(24 * pc);
    L.ghr = S.take(32 * pc);
    L.total = S.off;
    return L;
}

gsis_status sync_status(gsis_case c, hipStream_t s)
{
    int32_t st[4];
    HIPCHK(hipMemcpyAsync(st, c->hv.status, sizeof st, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (st[0]) return fail(GSIS_E_NONFINITE, "non-finite or non-positive state detected on the device");
    if (st[1]) return fail(GSIS_E_CAPACITY, "kinetic region exceeds the bound capacity (%d)", c->capacity);
    return GSIS_OK;
}

gsis_status check_ready(gsis_case c)
{
    if (!c) return fail(GSIS_E_ARG, "null case");
    if (!c->bound) return fail(GSIS_E_STATE, "case is not bound to a workspace");
    if (!c->state_set) return fail(GSIS_E_STATE, "state not set (call gsis_set_state)");
    return GSIS_OK;
}

// read n_kin / n_new after a compaction (synchronises)
gsis_status read_counts(gsis_case c, hipStream_t s, int *n_new)
{
    int32_t v[3];
    HIPCHK(hipMemcpyAsync(&v[0], c->hv.n_kin_dev, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&v[1], c->hv.n_new_dev, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&v[2], c->hv.n_ghost_dev, 4, hipMemcpyDeviceToHost, s));
    gsis_status st = sync_status(c, s);
    if (st) {
        // the region lists may be partial: no further sweep until set_state
        c->state_set = false;
        return st;
    }
    c->n_kin = v[0];
    c->n_ghost = v[2];
    if (n_new) *n_new = v[1];
    return GSIS_OK;
}

}  // namespace

namespace {
// combinations of grid, order and gas the kernels support
gsis_status check_config(const gsis_case_s *c)
{
    if (c->dr > 0 && (c->vdim != 3 || c->points || c->order != 1))
        return fail(GSIS_E_ARG, "the polyatomic gas needs a 3D tensor velocity grid and spatial order 1");
    return GSIS_OK;
}

gsis_status refuse_poly(gsis_case c, const char *what)
{
    if (c && c->dr > 0) return fail(GSIS_E_ARG, "%s: not available for the two-VDF (polyatomic) gas", what);
    return GSIS_OK;
}
}  // namespace

extern "C" gsis_status gsis_case_footprint(gsis_case c, int64_t cap, size_t *bytes)
{
    if (!c || !bytes) return fail(GSIS_E_ARG, "null argument");
    if (!c->grid_set) return fail(GSIS_E_STATE, "velocity grid not set");
    if (cap <= 0 || cap > c->mesh->n_cells) return fail(GSIS_E_ARG, "capacity must be in 1..n_cells");
    if (gsis_status st = check_config(c)) return st;
    int tile, ntile, row;
    *bytes = make_layout(c, cap, &tile, &ntile, &row).total;
    return GSIS_OK;
}

namespace gsis {
// Lay the case out in the device buffer ws of `bytes` (256-byte aligned) and
// copy the mesh and grid; with_events creates the sweep timing events.
gsis_status bind_impl(gsis_case c, void *ws, size_t bytes, int64_t cap, void *stream, bool with_events)
{
    if (!c || !ws) return fail(GSIS_E_ARG, "null argument");
    if (!c->grid_set) return fail(GSIS_E_STATE, "velocity grid not set");
    if (cap <= 0 || cap > c->mesh->n_cells) return fail(GSIS_E_ARG, "capacity must be in 1..n_cells");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GSIS_E_ARG, "workspace must be 256-byte aligned");
    if (gsis_status st = check_config(c)) return st;
    int tile, ntile, row, fast, xp;
    Layout L = make_layout(c, cap, &tile, &ntile, &row, &fast, &xp);
    if (bytes < L.total) return fail(GSIS_E_NOMEM, "workspace of %zu bytes < footprint %zu", bytes, L.total);
    drop_graphs_of(c);   // captured launches point into the previous workspace
    hipStream_t s = (hipStream_t)stream;
    const gsis_mesh_s *m = c->mesh;
    unsigned char *B = (unsigned char *)ws;
    c->ws = B;
    c->ws_bytes = bytes;
    c->capacity = (int32_t)cap;
    c->tile = tile;
    c->ntile = ntile;
    c->row = row;
    CaseView &h = c->hv;
    std::memset(&h, 0, sizeof h);
    h.n_cells = m->n_cells;
    h.n_faces = m->n_faces;
    h.n_patches = m->n_patches;
    h.dim = m->dim;
    h.nnz = m->nnz;
    h.vdim = c->vdim;
    h.nfun = (c->vdim == 3 && !(c->dr > 0)) ? 1 : 2;
    for (int d = 0; d < 3; ++d) h.n[d] = c->n[d];
    h.nv = c->nv;
    h.row = row;
    h.tile = tile;
    h.ntile = ntile;
    h.fast = fast;
    h.xp = xp;
    h.capacity = (int32_t)cap;
    h.dtype = c->dtype;
    h.Kn = c->gas.Kn;
    h.omega = c->gas.omega;
    h.Pr = c->gas.Pr;
    h.inv_dt = 0.0;
#define P(T, name, off) h.name = (T)(B + L.off)
    P(const int32_t *, cf_ptr, cf_ptr);
    P(const int32_t *, cf_face, cf_face);
    P(const int32_t *, cf_other, cf_other);
    P(const int32_t *, cf_wall, cf_wall);
    P(const double *, cf_nsv, cf_nsv);
    P(const double *, lsq, lsq);
    P(const double *, cf_fs, cf_fs);
    P(const double *, cell_sS, cell_sS);
    P(const double *, wall_den, wall_den);
    P(const int32_t *, face_cells, face_cells);
    P(const double *, face_normal, face_normal);
    P(const double *, face_area, face_area);
    P(const double *, face_center, face_center);
    P(const double *, face_dist, face_dist);
    P(const double *, face_dx, face_dx);
    P(const double *, cell_volume, cell_volume);
    P(const double *, cell_center, cell_center);
    P(const int32_t *, patch_kind, patch_kind);
    P(const double *, patch_state, patch_state);
    P(const int32_t *, wall_face, wallf);
    h.n_wall = (int32_t)m->wall_faces.size();
    P(const double *, xv, xv);
    P(const double *, wv, wv);
    P(const double *, vpt, vpt);
    P(const float *, vptf, vptf);
    h.points = c->points ? 1 : 0;
    P(int32_t *, flags, flags);
    P(int32_t *, slot_of_cell, slot);
    P(int32_t *, kin_cell, kin);
    P(int32_t *, n_kin_dev, nkin);
    P(int32_t *, new_cell, newc);
    P(int32_t *, n_new_dev, nnew);
    P(int32_t *, scan_tmp, scan);
    P(int32_t *, status, status);
    P(unsigned long long *, lim, lim);
    P(double *, g13_th, g13th);
    P(void *, prow, prow);
    P(void *, grow, grow);
    P(int32_t *, ghost_slot, gslot);
    P(int32_t *, ghost_cell, gcell);
    P(int32_t *, n_ghost_dev, ngh);
    h.gcap = (int32_t)ghost_capacity(m->n_cells, cap);
    h.nfmax = m->max_faces;
    P(void *, axtab, axtab);
    h.tabp = axtab_len(c);
    {
        const char *env = std::getenv("GSIS_SWEEP_ORDER");
        h.order = env ? std::atoi(env) : 0;
        const char *genv = std::getenv("GSIS_SWEEP_GROUP");
        h.group = genv ? std::max(1, std::atoi(genv)) : 256;
    }
    h.sorder = c->order;
    h.damp2 = c->damp2;
    h.g13_rmax = c->g13_rmax;
    h.poly = c->dr > 0 ? 1 : 0;
    h.dr = c->dr;
    h.Zr = c->Zr;
    for (int i = 0; i < 4; ++i) h.A[i] = c->A[i];
    if (h.poly) {
        P(PolyRec *, prec, prec);
        P(double *, psum, psum);
        P(double *, Tr, Tr);
        P(double *, Trh, Trh);
        P(double *, Trn, Trn);
        P(double *, Ur, Ur);
        P(double *, srcr, srcr);
        P(double *, Rkr, Rkr);
        P(double *, Rmr, Rmr);
        P(double *, fr, fr);
        P(double *, hfr, hfr);
        P(double *, hotr, hotr);
        P(double *, gTr, gTr);
        P(double *, ghr, ghr);
    }
    if (c->order == 2) {
        P(void *, slope, slope);
        P(double *, amax, amax);
        P(double *, wsl, wsl);
        P(const int32_t *, cf_back, cf_back);
    }
    P(ParamRec *, param, param);
    P(FeqRec *, feq, feq);
    P(double *, partial, partial);
    P(double *, mom, mom);
    P(double *, W, W);
    P(double *, Wh, Wh);
    P(double *, Wn, Wn);
    P(double *, U, U);
    P(double *, grad, grad);
    P(double *, ghost, ghost);
    P(double *, hot, hot);
    P(double *, src, src);
    P(double *, Rk, Rk);
    P(double *, Rm, Rm);
    P(double *, fflux, fflux);
    P(double *, hface, hface);
    P(double *, dloc, dloc);
    P(double *, red, red);
    P(double *, eps, eps);
#undef P
    h.f[0] = B + L.f0;
    h.f[1] = B + L.f1;
    c->cv = (CaseView *)(B + L.cv);
    auto put = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(B + off, src, n, hipMemcpyHostToDevice, s);
    };
    const size_t nnz = m->nnz, nf = m->n_faces, nc = m->n_cells;
    HIPCHK(put(L.cv, &h, sizeof h));
    HIPCHK(put(L.cf_ptr, m->cf_ptr.data(), 4 * (nc + 1)));
    HIPCHK(put(L.cf_face, m->cf_face.data(), 4 * nnz));
    HIPCHK(put(L.cf_other, m->cf_other.data(), 4 * nnz));
    HIPCHK(put(L.cf_wall, m->cf_wall.data(), 4 * nnz));
    HIPCHK(put(L.cf_nsv, m->cf_nsv.data(), 24 * nnz));
    HIPCHK(put(L.lsq, m->lsq.data(), 48 * nnz));
    HIPCHK(put(L.cf_fs, m->cf_fs.data(), 8 * nnz));
    HIPCHK(put(L.cell_sS, m->cell_sS.data(), 16 * nc));
    HIPCHK(put(L.face_cells, m->face_cells.data(), 8 * nf));
    HIPCHK(put(L.face_normal, m->face_normal.data(), 24 * nf));
    HIPCHK(put(L.face_area, m->face_area.data(), 8 * nf));
    HIPCHK(put(L.face_center, m->face_center.data(), 24 * nf));
    HIPCHK(put(L.face_dist, m->face_dist.data(), 8 * nf));
    HIPCHK(put(L.face_dx, m->face_dx.data(), 24 * nf));
    HIPCHK(put(L.cell_volume, m->cell_volume.data(), 8 * nc));
    HIPCHK(put(L.cell_center, m->cell_center.data(), 24 * nc));
    HIPCHK(put(L.patch_kind, m->patch_kind.data(), 4 * m->n_patches));
    HIPCHK(put(L.patch_state, m->patch_state.data(), 40 * m->n_patches));
    HIPCHK(put(L.wallf, m->wall_faces.data(), 4 * m->wall_faces.size()));
    HIPCHK(put(L.xv, c->xv, sizeof c->xv));
    HIPCHK(put(L.wv, c->wv, sizeof c->wv));
    HIPCHK(put(L.vpt, c->vt.data(), 8 * c->vt.size()));
    HIPCHK(put(L.vptf, c->vtf.data(), 4 * c->vtf.size()));
    HIPCHK(hipMemsetAsync(B + L.slot, 0xff, 4 * nc, s));
    HIPCHK(hipMemsetAsync(B + L.flags, 0, 4 * nc, s));
    HIPCHK(hipMemsetAsync(B + L.status, 0, 16, s));
    HIPCHK(hipMemsetAsync(B + L.lim, 0, 64, s));
    HIPCHK(hipMemsetAsync(B + L.gslot, 0xff, 4 * nc, s));
    HIPCHK(hipMemsetAsync(B + L.ngh, 0, 16, s));
    HIPCHK(hipMemsetAsync(B + L.prow, 0, L.gslot - L.prow, s));
    HIPCHK(hipMemsetAsync(B + L.wall_den, 0, 8 * nnz, s));
    HIPCHK(hipMemsetAsync(B + L.hot, 0, 72 * nc, s));
    if (h.poly) HIPCHK(hipMemsetAsync(B + L.hotr, 0, 24 * nc, s));
    // padding of the VDF rows stays zero
    HIPCHK(hipMemsetAsync(B + L.f0, 0, L.f1 - L.f0, s));
    HIPCHK(hipMemsetAsync(B + L.f1, 0, L.param - L.f1, s));
    HIPCHK(launch_wall_den(c->cv, h, s));
    HIPCHK(launch_patch_rows(c->cv, h, s));
    if (c->order == 2) {
        HIPCHK(put(L.cf_back, m->cf_back.data(), 4 * nnz));
        HIPCHK(hipMemsetAsync(B + L.wsl, 0, L.cf_back - L.wsl, s));
        HIPCHK(launch_amax(c->cv, h, s));
    }
    if (with_events && !c->ev0) {
        HIPCHK(hipEventCreate(&c->ev0));
        HIPCHK(hipEventCreate(&c->ev1));
    }
    HIPCHK(hipStreamSynchronize(s));
    c->bound = true;
    c->state_set = false;
    c->n_kin = 0;
    c->cur = 0;
    c->timed = false;
    return GSIS_OK;
}

// the case no longer holds a workspace (another case took the static one)
void unbind_case(gsis_case c)
{
    drop_graphs_of(c);
    c->bound = false;
    c->state_set = false;
    c->ws = nullptr;
    c->ws_bytes = 0;
}

gsis_status set_error(gsis_status code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace gsis

extern "C" gsis_status gsis_case_bind(gsis_case c, void *ws, size_t bytes, int64_t cap, void *stream)
{
    if (c) static_release(c);
    return bind_impl(c, ws, bytes, cap, stream, true);
}

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
extern "C" gsis_status gsis_set_state(gsis_case c, const double *W_dev, const void *vdf_dev, const uint8_t *flags_dev,
                                      void *stream)
{
    if (!c || !W_dev) return fail(GSIS_E_ARG, "null argument");
    if (!c->bound) return fail(GSIS_E_STATE, "case is not bound to a workspace");
    hipStream_t s = (hipStream_t)stream;
    CaseView &h = c->hv;
    c->state_set = false;
    HIPCHK(hipMemsetAsync(h.status, 0, 16, s));
    HIPCHK(hipMemsetAsync(h.lim, 0, 64, s));
    HIPCHK(launch_copy_W(h.W, W_dev, h.n_cells, s));
    HIPCHK(launch_check_W(c->cv, h, h.W, s));
    HIPCHK(hipMemsetAsync(h.slot_of_cell, 0xff, 4 * (size_t)h.n_cells, s));
    HIPCHK(launch_set_flags(c->cv, h, flags_dev, 1, s));
    HIPCHK(launch_compact(c->cv, h, s));
    gsis_status st = read_counts(c, s, nullptr);
    if (st) return st;
    c->cur = 0;
    // two-VDF gas: the internal temperature starts at T_t on every cell
    if (h.poly) HIPCHK(launch_tt_copy(c->cv, h, h.Tr, s));
    if (vdf_dev) {
        HIPCHK(launch_gather_vdf(c->cv, h, c->n_kin, 0, const_cast<void *>(vdf_dev), 1, s));
        HIPCHK(launch_fill(c->cv, h, 2, c->n_kin, 0, s));
    } else {
        HIPCHK(launch_fill(c->cv, h, 0, c->n_kin, 0, s));
    }
    HIPCHK(launch_reduce(c->cv, h, c->n_kin, 0, s));
    // W (and T_r) on kinetic cells = moments of the VDF
    HIPCHK(launch_W_from_mom(c->cv, h, c->n_kin, h.W, s));
    if (h.poly) HIPCHK(launch_tr_half(c->cv, h, h.Tr, s));
    st = sync_status(c, s);
    if (st) return st;
    c->state_set = true;
    c->iter = 0;
    return GSIS_OK;
}

extern "C" gsis_status gsis_n_kinetic(gsis_case c, int64_t *n)
{
    if (!c || !n) return fail(GSIS_E_ARG, "null argument");
    *n = c->n_kin;
    return GSIS_OK;
}

// ---------------------------------------------------------------------------
// sweeps
// ---------------------------------------------------------------------------
namespace {

bool has_ns_cells(gsis_case c) { return c->n_kin < c->hv.n_cells; }

// per-case preparation of one sweep: relaxation parameters from the current
// moments, Grad-13 ghosts of NS neighbours from W
gsis_status prepare_sweep(gsis_case c, hipStream_t s)
{
    CaseView &h = c->hv;
    HIPCHK(launch_param(c->cv, h, c->n_kin, s));
    if (h.fast || o2_v4_fits(h)) HIPCHK(launch_axtab(c->cv, h, c->n_kin, s));
    if (has_ns_cells(c)) {
        HIPCHK(launch_lsq(c->cv, h, h.W, 4, s));
        if (h.poly) HIPCHK(launch_ghost_poly(c->cv, h, h.W, h.Tr, s));
        else HIPCHK(launch_ghost(c->cv, h, h.W, s));
        HIPCHK(launch_count_g13(c->cv, h.ghost_cell, c->n_ghost, 0, s));
        if (h.fast || h.points || (h.sorder == 2 && h.vdim == 3) || h.poly)
            HIPCHK(launch_ghost_rows(c->cv, h, c->n_ghost, s));
    }
    return GSIS_OK;
}

// the launch batch of cases [i0, i0 + m): work-item prefixes, buffers, layout
Batch make_batch(gsis_case const *cases, int i0, int m)
{
    Batch b{};
    b.n = m;
    b.start[0] = 0;
    for (int j = 0; j < m; ++j) {
        gsis_case c = cases[i0 + j];
        b.cv[j] = c->cv;
        b.start[j + 1] = b.start[j] + c->n_kin * c->ntile;
        b.nfmax = std::max(b.nfmax, c->hv.nfmax);
        if (c->vdim == 3) b.mdiv = std::gcd(b.mdiv, c->n[1] * c->n[2] / BLOCK);
    }
    // every case sweeps its own f^n buffer (cur) into the other one
    for (int j = 0; j < m; ++j) b.cur[j] = cases[i0 + j]->cur;
    b.order = cases[i0]->hv.order;
    b.group = cases[i0]->hv.group;
    // 16-byte rows when every case's (y, z) plane fits (GSIS_SWEEP_V4=0 keeps 4-byte rows)
    {
        const bool v4_on = [] {
            const char *e = std::getenv("GSIS_SWEEP_V4");
            return !(e && e[0] == '0');
        }();
        b.v4 = v4_on;
        for (int j = 0; j < m; ++j) {
            const CaseView &hj = cases[i0 + j]->hv;
            if (!(hj.fast && hj.vdim == 3 && !hj.poly && sweep_v4_fits(hj.n[1], hj.n[2]))) b.v4 = 0;
        }
        // order 2: the 16-byte-row sweep when every case fits it
        if (cases[i0]->hv.sorder == 2) {
            b.v4 = 1;
            for (int j = 0; j < m; ++j)
                if (!o2_v4_fits(cases[i0 + j]->hv)) b.v4 = 0;
        }
    }
    return b;
}

gsis_status batched_sweep(gsis_case const *cases, int n, hipStream_t s, bool timed)
{
    // A case is swept by the kernel it gets alone (16-byte rows or not): cases
    // of the two kinds never share a launch, so its rows do not depend on the
    // batch it comes in.  Within a launch the LDS is sized for the largest
    // axes of its cases.
    std::vector<gsis_case> part[2];
    for (int j = 0; j < n; ++j) {
        gsis_case one[1] = {cases[j]};
        part[make_batch(one, 0, 1).v4 ? 1 : 0].push_back(cases[j]);
    }
    bool first = true;
    for (int k = 1; k >= 0; --k) {
        const std::vector<gsis_case> &pc = part[k];
        for (size_t i0 = 0; i0 < pc.size(); i0 += MAX_BATCH) {
            const int m = (int)std::min<size_t>(MAX_BATCH, pc.size() - i0);
            Batch b = make_batch(pc.data(), (int)i0, m);
            CaseView hs = pc[i0]->hv;
            for (int j = 1; j < m; ++j)
                for (int d = 0; d < 3; ++d) hs.n[d] = std::max(hs.n[d], pc[i0 + j]->hv.n[d]);
            if (timed && first && cases[0]->ev0) HIPCHK(hipEventRecord(cases[0]->ev0, s));
            first = false;
            // order 2: limited slopes of every case's f^n (the sweep reads its own
            // and its neighbours')
            for (int j = 0; j < m; ++j) {
                gsis_case c = pc[i0 + j];
                if (c->order == 2) HIPCHK(launch_slope(c->cv, c->hv, c->n_kin, c->cur, s));
            }
            HIPCHK(launch_sweep(b, hs, b.start[m], s));
        }
    }
    if (timed && cases[0]->ev1) HIPCHK(hipEventRecord(cases[0]->ev1, s));
    // the events time the whole batched launch; they belong to the first case
    for (int j = 0; j < n; ++j) {
        cases[j]->cur ^= 1;
        cases[j]->timed = false;
    }
    cases[0]->timed = timed && cases[0]->ev0;
    return GSIS_OK;
}

// the kinetic moment balance of the case's current rows (f^{n+1/2} after a
// sweep): the targets and wall densities from their moments, then one sweep
// of them into the other buffer (f^n, no longer needed), whose fused balance
// sums are the balance at its input (the fix-up makes the collision term's
// conserved moments vanish); the buffers do not swap and the rows written are
// discarded.  Rk <- the balance (the moments stay those of the rows).
gsis_status balance_of_current(gsis_case c, hipStream_t s)
{
    CaseView &h = c->hv;
    HIPCHK(launch_param(c->cv, h, c->n_kin, s));
    if (h.fast || o2_v4_fits(h)) HIPCHK(launch_axtab(c->cv, h, c->n_kin, s));
    if (c->order == 2) HIPCHK(launch_slope(c->cv, h, c->n_kin, c->cur, s));
    gsis_case one[1] = {c};
    Batch b = make_batch(one, 0, 1);
    HIPCHK(launch_sweep(b, h, b.start[1], s));
    HIPCHK(launch_reduce(c->cv, h, c->n_kin, 2, s));
    return GSIS_OK;
}

gsis_status check_batch(gsis_case const *cases, int n)
{
    if (!cases || n <= 0) return fail(GSIS_E_ARG, "no cases");
    for (int j = 0; j < n; ++j) {
        gsis_status st = check_ready(cases[j]);
        if (st) return st;
        if (cases[j]->dtype != cases[0]->dtype || cases[j]->vdim != cases[0]->vdim ||
            cases[j]->hv.fast != cases[0]->hv.fast || cases[j]->points != cases[0]->points ||
            cases[j]->order != cases[0]->order || (cases[j]->dr > 0) != (cases[0]->dr > 0))
            return fail(GSIS_E_ARG, "batched cases must share dtype, vdim, grid kind, spatial order, gas kind and sweep layout");
        for (int d = 0; d < 3; ++d)
            if (cases[j]->n[d] > cases[0]->n[d] && j > 0) {
                // LDS is sized from the first case: put the largest grid first
                return fail(GSIS_E_ARG, "batched cases: the first case must have the largest velocity axes");
            }
        for (int i = 0; i < j; ++i)
            if (cases[i] == cases[j]) return fail(GSIS_E_ARG, "a case appears twice in the batch");
    }
    return GSIS_OK;
}

}  // namespace

extern "C" gsis_status gsis_kinetic_sweep(gsis_case const *cases, int32_t n_cases, int32_t n_sweeps, void *stream)
{
    gsis_status st = check_batch(cases, n_cases);
    if (st) return st;
    if (n_sweeps < 0) return fail(GSIS_E_ARG, "n_sweeps < 0");
    hipStream_t s = (hipStream_t)stream;
    for (int it = 0; it < n_sweeps; ++it) {
        for (int j = 0; j < n_cases; ++j)
            if ((st = prepare_sweep(cases[j], s))) return st;
        if ((st = batched_sweep(cases, n_cases, s, true))) return st;
        for (int j = 0; j < n_cases; ++j) {
            gsis_case c = cases[j];
            HIPCHK(launch_reduce(c->cv, c->hv, c->n_kin, 1, s));
            HIPCHK(launch_W_from_mom(c->cv, c->hv, c->n_kin, c->hv.W, s));
            if (c->hv.poly) HIPCHK(launch_tr_half(c->cv, c->hv, c->hv.Tr, s));
        }
    }
    return GSIS_OK;
}

extern "C" gsis_status gsis_sweep_layout(gsis_case c, int32_t *fast, int32_t *tile, int32_t *n_tiles)
{
    if (!c) return fail(GSIS_E_ARG, "null case");
    if (!c->bound) return fail(GSIS_E_STATE, "case is not bound to a workspace");
    if (fast) *fast = c->hv.fast;
    if (tile) *tile = c->hv.tile;
    if (n_tiles) *n_tiles = c->hv.ntile;
    return GSIS_OK;
}

extern "C" gsis_status gsis_last_sweep_ms(gsis_case c, float *ms)
{
    if (!c || !ms) return fail(GSIS_E_ARG, "null argument");
    if (!c->timed) return fail(GSIS_E_STATE, "no timed sweep on this case");
    HIPCHK(hipEventSynchronize(c->ev1));
    HIPCHK(hipEventElapsedTime(ms, c->ev0, c->ev1));
    return GSIS_OK;
}

extern "C" gsis_status gsis_internal_moments(gsis_case c, double *out, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!(c->dr > 0)) return fail(GSIS_E_ARG, "the gas has no internal degrees of freedom");
    if (!out && c->n_kin > 0) return fail(GSIS_E_ARG, "null output");
    HIPCHK(launch_internal_out(c->cv, c->hv, c->n_kin, out, (hipStream_t)stream));
    return GSIS_OK;
}

extern "C" gsis_status gsis_get_internal_temperature(gsis_case c, double *out, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!(c->dr > 0)) return fail(GSIS_E_ARG, "the gas has no internal degrees of freedom");
    if (!out) return fail(GSIS_E_ARG, "null output");
    HIPCHK(launch_copy_d(out, c->hv.Tr, c->hv.n_cells, (hipStream_t)stream));
    return GSIS_OK;
}

extern "C" gsis_status gsis_moments(gsis_case c, double *out, int32_t *kc, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!out && c->n_kin > 0) return fail(GSIS_E_ARG, "null output");
    HIPCHK(launch_moments_out(c->cv, c->hv, c->n_kin, out, kc, (hipStream_t)stream));
    return GSIS_OK;
}

extern "C" gsis_status gsis_get_vdf(gsis_case c, void *out, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!out && c->n_kin > 0) return fail(GSIS_E_ARG, "null output");
    HIPCHK(launch_gather_vdf(c->cv, c->hv, c->n_kin, c->cur, out, 0, (hipStream_t)stream));
    return GSIS_OK;
}

extern "C" gsis_status gsis_get_state(gsis_case c, double *W, uint8_t *flags, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (W) HIPCHK(launch_copy_W(W, c->hv.W, c->hv.n_cells, s));
    if (flags) HIPCHK(launch_get_flags(c->cv, c->hv, flags, s));
    return GSIS_OK;
}

// ---------------------------------------------------------------------------
// regions
// ---------------------------------------------------------------------------
extern "C" gsis_status gsis_update_regions(gsis_case c, double Kn_ref, int32_t layers, int64_t *n_host, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!(Kn_ref >= 0) || layers < 0) return fail(GSIS_E_ARG, "bad Kn_ref or layers");
    hipStream_t s = (hipStream_t)stream;
    CaseView &h = c->hv;
    HIPCHK(launch_flags(c->cv, h, Kn_ref, layers, s));
    HIPCHK(launch_compact(c->cv, h, s));
    int n_new = 0;
    if ((st = read_counts(c, s, &n_new))) return st;
    if (n_new > 0) {
        // Grad-13 of the current W (gradients of u, T are in grad after launch_flags)
        if (h.poly) HIPCHK(launch_ghost_poly(c->cv, h, h.W, h.Tr, s));
        else HIPCHK(launch_ghost(c->cv, h, h.W, s));
        HIPCHK(launch_count_g13(c->cv, h.new_cell, n_new, 1, s));
        HIPCHK(launch_fill(c->cv, h, 1, n_new, c->cur, s));
    }
    HIPCHK(launch_reduce(c->cv, h, c->n_kin, 0, s));
    if (n_host) *n_host = c->n_kin;
    return sync_status(c, s);
}

// ---------------------------------------------------------------------------
// outer iteration
// ---------------------------------------------------------------------------
namespace {

// after the sweep, up to the synthetic solve: moments of f^{n+1/2}, W^{n+1/2},
// high-order terms, the source of eq. macro, W^{n+1} <- W^n (GSIS/aGSIS);
// W^{n+1} <- W^{n+1/2} (DVM)
gsis_status pre_macro(gsis_case c, const gsis_solve_params *p, hipStream_t s)
{
    CaseView &h = c->hv;
    HIPCHK(launch_reduce(c->cv, h, c->n_kin, 1, s));
    if (p->mode == GSIS_MODE_DVM) {
        HIPCHK(launch_copy_W(h.Wn, h.W, h.n_cells, s));
        HIPCHK(launch_W_from_mom(c->cv, h, c->n_kin, h.Wn, s));
        if (h.poly) HIPCHK(launch_tr_half(c->cv, h, h.Trn, s));
        return GSIS_OK;
    }
    HIPCHK(launch_whalf(c->cv, h, c->n_kin, s));
    if (h.poly) HIPCHK(launch_tr_half(c->cv, h, h.Trh, s));
    // high-order terms from f^{n+1/2} and gradients of W^{n+1/2}
    HIPCHK(launch_lsq(c->cv, h, h.Wh, 4, s));
    if (h.poly) HIPCHK(launch_hot_poly(c->cv, h, s));
    else HIPCHK(launch_hot(c->cv, h, c->n_kin, s));
    if (p->source_half) {
        // source at the half step: the balance of f^{n+1/2} minus the synthetic
        // residual at W^{n+1/2}; the solve starts from W^{n+1/2}
        gsis_status st = balance_of_current(c, s);
        if (st) return st;
        HIPCHK(launch_macro_residual(c->cv, h, h.Wh, h.hot, h.Rm, s));
        HIPCHK(launch_src(c->cv, h, c->n_kin, s));
        HIPCHK(launch_copy_W(h.Wn, h.Wh, h.n_cells, s));
        return GSIS_OK;
    }
    // source: kinetic moment balance at f^n minus synthetic residual at W^n
    if (h.poly) {
        HIPCHK(launch_macro_residual_poly(c->cv, h, h.W, h.Tr, h.hot, h.Rm, h.Rmr, s));
        HIPCHK(launch_src_poly(c->cv, h, s));
        HIPCHK(launch_copy_d(h.Trn, h.Tr, h.n_cells, s));
    } else {
        HIPCHK(launch_macro_residual(c->cv, h, h.W, h.hot, h.Rm, s));
        HIPCHK(launch_src(c->cv, h, c->n_kin, s));
    }
    HIPCHK(launch_copy_W(h.Wn, h.W, h.n_cells, s));
    return GSIS_OK;
}

// ---------------------------------------------------------------------------
// HIP graphs of the synthetic solve: the n_inner pseudo-time steps of a batch
// (3-5 launches each) are captured once per batch composition on a private
// stream and replayed on the caller's stream.  Every pointer a captured launch
// uses lives in the cases' workspaces, so a graph stays valid while its cases
// stay bound; binding again or destroying a case drops its graphs.  Set
// GSIS_GRAPHS=0 to launch eagerly.
// ---------------------------------------------------------------------------
struct MacroGraph {
    std::vector<gsis_case> cases;
    int n_inner;
    double cfl;
    bool with_src;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
};

std::mutex g_graph_mu;
std::vector<MacroGraph> g_graphs;
hipStream_t g_capture_stream = nullptr;
uint64_t g_graph_clock = 0;
constexpr size_t MAX_GRAPHS = 64;

bool graphs_enabled()
{
    const char *env = std::getenv("GSIS_GRAPHS");
    return !(env && env[0] == '0');
}

// Whole outer iterations from HIP graphs (GSIS_STEP_GRAPHS=1): everything a
// step launches before its region update -- relaxation parameters, ghosts,
// the batched sweep, moments, HoT, the synthetic solve, the correction and
// the residual -- is captured once per batch composition, parameters, kinetic
// and ghost counts and buffer parity, and replayed while those stay the same
// (between region updates).  The region update and the residual read-back
// stay eager.  Sweep timing events are not recorded in this mode.
struct StepGraph {
    std::vector<gsis_case> cases;
    std::vector<int32_t> nk, ng, cur;
    gsis_solve_params p;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
};
std::vector<StepGraph> g_step_graphs;

bool step_graphs_enabled()
{
    const char *env = std::getenv("GSIS_STEP_GRAPHS");
    return env && env[0] == '1';
}

void drop_graphs_of(gsis_case c)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t k = 0; k < g_graphs.size();) {
        MacroGraph &G = g_graphs[k];
        if (std::find(G.cases.begin(), G.cases.end(), c) != G.cases.end()) {
            (void)hipGraphExecDestroy(G.exec);
            (void)hipGraphDestroy(G.graph);
            g_graphs.erase(g_graphs.begin() + k);
        } else {
            ++k;
        }
    }
    for (size_t k = 0; k < g_step_graphs.size();) {
        StepGraph &G = g_step_graphs[k];
        if (std::find(G.cases.begin(), G.cases.end(), c) != G.cases.end()) {
            (void)hipGraphExecDestroy(G.exec);
            (void)hipGraphDestroy(G.graph);
            g_step_graphs.erase(g_step_graphs.begin() + k);
        } else {
            ++k;
        }
    }
}

// n_inner pseudo-time steps of the cases' synthetic equations, W <- Wn
gsis_status run_macro_batch(gsis_case const *cases, int n, int n_inner, double cfl, bool with_src, hipStream_t s)
{
    MBatch b{};
    for (int j = 0; j < n; ++j) {
        CaseView &h = cases[j]->hv;
        mbatch_add(b, cases[j]->cv, h, h.Wn, h.hot, with_src ? h.src : nullptr, h.poly ? h.Trn : nullptr);
    }
    if (!graphs_enabled() || n_inner <= 0) {
        HIPCHK(launch_macro_steps_batch(b, n_inner, cfl, s));
        return GSIS_OK;
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    std::vector<gsis_case> key(cases, cases + n);
    MacroGraph *hit = nullptr;
    for (auto &G : g_graphs)
        if (G.cases == key && G.n_inner == n_inner && G.cfl == cfl && G.with_src == with_src) hit = &G;
    if (!hit) {
        if (!g_capture_stream) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
        if (g_graphs.size() >= MAX_GRAPHS) {
            auto lru = std::min_element(g_graphs.begin(), g_graphs.end(),
                                        [](const MacroGraph &a, const MacroGraph &c) { return a.last_use < c.last_use; });
            (void)hipGraphExecDestroy(lru->exec);
            (void)hipGraphDestroy(lru->graph);
            g_graphs.erase(lru);
        }
        MacroGraph G{key, n_inner, cfl, with_src, nullptr, nullptr, 0};
        HIPCHK(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_macro_steps_batch(b, n_inner, cfl, g_capture_stream);
        hipError_t e2 = hipStreamEndCapture(g_capture_stream, &G.graph);
        HIPCHK(e);
        HIPCHK(e2);
        HIPCHK(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
        g_graphs.push_back(G);
        hit = &g_graphs.back();
    }
    hit->last_use = ++g_graph_clock;
    HIPCHK(hipGraphLaunch(hit->exec, s));
    return GSIS_OK;
}

// the synthetic solves of a batch: one launch per kernel and pseudo-time step
// for all cases (up to 16 per launch)
gsis_status macro_solves(gsis_case const *cases, int n, const gsis_solve_params *p, hipStream_t s,
                         bool capturing = false)
{
    if (p->mode == GSIS_MODE_DVM) return GSIS_OK;
    gsis_status st;
    for (int j0 = 0; j0 < n; j0 += MAX_BATCH) {
        const int m = std::min(MAX_BATCH, n - j0);
        if (capturing) {
            // inside a whole-step capture: the launches themselves (no nested graph)
            MBatch b{};
            for (int j = 0; j < m; ++j) {
                CaseView &h = cases[j0 + j]->hv;
                mbatch_add(b, cases[j0 + j]->cv, h, h.Wn, h.hot, h.src, h.poly ? h.Trn : nullptr);
            }
            HIPCHK(launch_macro_steps_batch(b, p->n_macro_inner, p->cfl, s));
        } else if ((st = run_macro_batch(cases + j0, m, p->n_macro_inner, p->cfl, true, s))) {
            return st;
        }
    }
    return GSIS_OK;
}

// after the synthetic solve: GSIS correction f += f_eq(W^{n+1}) - f_eq(W^{n+1/2}),
// moments of f^{n+1}, the residual, W <- W^{n+1}
gsis_status post_macro(gsis_case c, const gsis_solve_params *p, hipStream_t s)
{
    CaseView &h = c->hv;
    if (p->mode != GSIS_MODE_DVM) {
        HIPCHK(launch_feqpar(c->cv, h, c->n_kin, s));
        HIPCHK(launch_correct(c->cv, h, c->n_kin, c->cur, s));
        HIPCHK(launch_reduce(c->cv, h, c->n_kin, 0, s));
    }
    HIPCHK(launch_eps(c->cv, h, h.Wn, h.W, s));
    HIPCHK(launch_copy_W(h.W, h.Wn, h.n_cells, s));
    if (h.poly) HIPCHK(launch_copy_d(h.Tr, h.Trn, h.n_cells, s));
    return GSIS_OK;
}

// everything one outer iteration launches before its region update
gsis_status step_body(gsis_case const *cases, int n, const gsis_solve_params *p, hipStream_t s, bool capturing)
{
    gsis_status st;
    for (int j = 0; j < n; ++j)
        if ((st = prepare_sweep(cases[j], s))) return st;
    if ((st = batched_sweep(cases, n, s, !capturing))) return st;
    for (int j = 0; j < n; ++j)
        if ((st = pre_macro(cases[j], p, s))) return st;
    if ((st = macro_solves(cases, n, p, s, capturing))) return st;
    for (int j = 0; j < n; ++j)
        if ((st = post_macro(cases[j], p, s))) return st;
    return GSIS_OK;
}

bool same_params(const gsis_solve_params &a, const gsis_solve_params &b)
{
    return a.mode == b.mode && a.n_macro_inner == b.n_macro_inner && a.cfl == b.cfl && a.source_half == b.source_half;
}

gsis_status step_from_graph(gsis_case const *cases, int n, const gsis_solve_params *p, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    std::vector<gsis_case> key(cases, cases + n);
    std::vector<int32_t> nk(n), ng(n), cur(n);
    for (int j = 0; j < n; ++j) {
        nk[j] = cases[j]->n_kin;
        ng[j] = cases[j]->n_ghost;
        cur[j] = cases[j]->cur;
    }
    StepGraph *hit = nullptr;
    for (auto &G : g_step_graphs)
        if (G.cases == key && G.nk == nk && G.ng == ng && G.cur == cur && same_params(G.p, *p)) hit = &G;
    if (hit) {
        hit->last_use = ++g_graph_clock;
        HIPCHK(hipGraphLaunch(hit->exec, s));
        // the host bookkeeping of the captured sweep
        for (int j = 0; j < n; ++j) {
            cases[j]->cur ^= 1;
            cases[j]->timed = false;
        }
        return GSIS_OK;
    }
    if (!g_capture_stream) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    if (g_step_graphs.size() >= MAX_GRAPHS) {
        auto lru = std::min_element(g_step_graphs.begin(), g_step_graphs.end(),
                                    [](const StepGraph &a, const StepGraph &c) { return a.last_use < c.last_use; });
        (void)hipGraphExecDestroy(lru->exec);
        (void)hipGraphDestroy(lru->graph);
        g_step_graphs.erase(lru);
    }
    StepGraph G{key, nk, ng, cur, *p, nullptr, nullptr, 0};
    // the capture stream starts after the work already on s
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, s));
    HIPCHK(hipStreamWaitEvent(g_capture_stream, ev, 0));
    HIPCHK(hipEventDestroy(ev));
    HIPCHK(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    gsis_status st = step_body(cases, n, p, g_capture_stream, true);
    hipError_t e2 = hipStreamEndCapture(g_capture_stream, &G.graph);
    if (st) {
        if (G.graph) (void)hipGraphDestroy(G.graph);
        return st;
    }
    HIPCHK(e2);
    HIPCHK(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
    G.last_use = ++g_graph_clock;
    g_step_graphs.push_back(G);
    HIPCHK(hipGraphLaunch(G.exec, s));
    return GSIS_OK;
}

gsis_status check_params(const gsis_solve_params *p)
{
    if (!p) return fail(GSIS_E_ARG, "null params");
    if (p->mode < GSIS_MODE_DVM || p->mode > GSIS_MODE_AGSIS) return fail(GSIS_E_ARG, "bad mode");
    if (p->mode != GSIS_MODE_DVM && (p->n_macro_inner < 0 || p->cfl == 0 || !std::isfinite(p->cfl)))
        return fail(GSIS_E_ARG, "bad macro parameters");
    if (p->source_half != 0 && p->source_half != 1) return fail(GSIS_E_ARG, "source_half must be 0 or 1");
    return GSIS_OK;
}

// the half-step source is defined for the monatomic gas
gsis_status check_source(gsis_case const *cases, int n, const gsis_solve_params *p)
{
    if (p->source_half && p->mode != GSIS_MODE_DVM)
        for (int j = 0; j < n; ++j)
            if (cases[j]->dr > 0) return fail(GSIS_E_ARG, "source_half is defined for the monatomic gas");
    return GSIS_OK;
}

}  // namespace

extern "C" gsis_status gsis_step(gsis_case const *cases, int32_t n, const gsis_solve_params *p, double *eps_host,
                                 void *stream)
{
    gsis_status st = check_batch(cases, n);
    if (st) return st;
    if ((st = check_params(p))) return st;
    if ((st = check_source(cases, n, p))) return st;
    hipStream_t s = (hipStream_t)stream;
    if (step_graphs_enabled()) {
        if ((st = step_from_graph(cases, n, p, s))) return st;
    } else if ((st = step_body(cases, n, p, s, false))) {
        return st;
    }
    // per-case endings: a case whose region update or state check fails is
    // reported with NaN residuals; the others complete the step
    gsis_status first = GSIS_OK;
    std::string first_msg;
    for (int j = 0; j < n; ++j) {
        gsis_case c = cases[j];
        c->iter++;
        st = GSIS_OK;
        const int k = p->region_update_every;
        if (p->mode == GSIS_MODE_AGSIS && ((k > 0 && c->iter % k == 0) || (k < 0 && c->iter == -k)))
            st = gsis_update_regions(c, p->Kn_ref, p->force_wall_layers, nullptr, stream);
        double e[3] = {NAN, NAN, NAN};
        if (!st && eps_host) {
            HIPCHK(hipMemcpyAsync(e, c->hv.eps, sizeof e, hipMemcpyDeviceToHost, s));
            st = sync_status(c, s);
            if (st) e[0] = e[1] = e[2] = NAN;
        }
        if (st && !first) {
            first = st;
            first_msg = "case " + std::to_string(j) + " of the batch: " + g_err;
        }
        if (eps_host)
            for (int k = 0; k < 3; ++k) eps_host[3 * j + k] = st ? NAN : e[k];
    }
    if (first) return fail(first, "%s", first_msg.c_str());
    return GSIS_OK;
}

extern "C" gsis_status gsis_correct(gsis_case c, const double *W_new, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if ((st = refuse_poly(c, "gsis_correct"))) return st;
    if (!W_new) return fail(GSIS_E_ARG, "null W_new");
    hipStream_t s = (hipStream_t)stream;
    CaseView &h = c->hv;
    HIPCHK(launch_whalf(c->cv, h, c->n_kin, s));
    HIPCHK(launch_copy_W(h.Wn, W_new, h.n_cells, s));
    HIPCHK(launch_check_W(c->cv, h, h.Wn, s));
    HIPCHK(launch_feqpar(c->cv, h, c->n_kin, s));
    HIPCHK(launch_correct(c->cv, h, c->n_kin, c->cur, s));
    HIPCHK(launch_reduce(c->cv, h, c->n_kin, 0, s));
    HIPCHK(launch_copy_W(h.W, h.Wn, h.n_cells, s));
    return GSIS_OK;
}

extern "C" gsis_status gsis_correct_internal(gsis_case c, const double *W_new, const double *Tr_new, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!(c->dr > 0)) return fail(GSIS_E_ARG, "gsis_correct_internal: a monatomic case (use gsis_correct)");
    if (!W_new || !Tr_new) return fail(GSIS_E_ARG, "null W_new or Tr_new");
    hipStream_t s = (hipStream_t)stream;
    CaseView &h = c->hv;
    // W^{n+1/2} and T_r^{n+1/2}: the moments of the current rows on kinetic cells
    HIPCHK(launch_whalf(c->cv, h, c->n_kin, s));
    HIPCHK(launch_tr_half(c->cv, h, h.Trh, s));
    HIPCHK(launch_copy_W(h.Wn, W_new, h.n_cells, s));
    HIPCHK(launch_copy_d(h.Trn, Tr_new, h.n_cells, s));
    HIPCHK(launch_check_W(c->cv, h, h.Wn, s));
    HIPCHK(launch_feqpar(c->cv, h, c->n_kin, s));
    HIPCHK(launch_correct(c->cv, h, c->n_kin, c->cur, s));
    HIPCHK(launch_reduce(c->cv, h, c->n_kin, 0, s));
    HIPCHK(launch_copy_W(h.W, h.Wn, h.n_cells, s));
    HIPCHK(launch_copy_d(h.Tr, h.Trn, h.n_cells, s));
    return GSIS_OK;
}

extern "C" gsis_status gsis_n_wall_faces(gsis_case c, int32_t *n_wall)
{
    if (!c || !n_wall) return fail(GSIS_E_ARG, "null argument");
    *n_wall = (int32_t)c->mesh->wall_faces.size();
    return GSIS_OK;
}

extern "C" gsis_status gsis_surface(gsis_case c, int32_t *face_dev, double *out, double *totals, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if (!out) return fail(GSIS_E_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    CaseView &h = c->hv;
    if (face_dev && h.n_wall > 0)
        HIPCHK(hipMemcpyAsync(face_dev, h.wall_face, 4 * (size_t)h.n_wall, hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_surface(c->cv, h, c->cur, out, totals, s));
    return GSIS_OK;
}

extern "C" gsis_status gsis_force_coefficients(const double *totals, double rho_inf, const double *u_inf, double area,
                                               double *out)
{
    if (!totals || !u_inf || !out) return fail(GSIS_E_ARG, "null argument");
    const double U = std::sqrt(u_inf[0] * u_inf[0] + u_inf[1] * u_inf[1] + u_inf[2] * u_inf[2]);
    if (!(U > 0) || !(rho_inf > 0) || !(area > 0) || !std::isfinite(U))
        return fail(GSIS_E_ARG, "bad free stream or reference area");
    const double e[3] = {u_inf[0] / U, u_inf[1] / U, u_inf[2] / U};
    const double el[3] = {-e[1], e[0], 0.0};
    const double q = rho_inf * U * U * area;
    out[0] = (totals[0] * e[0] + totals[1] * e[1] + totals[2] * e[2]) / q;
    out[1] = (totals[0] * el[0] + totals[1] * el[1] + totals[2] * el[2]) / q;
    out[2] = totals[3] / (q * U);
    return GSIS_OK;
}

extern "C" gsis_status gsis_macro_solve(gsis_case c, double *W, const double *hot, const double *src, int32_t n_inner,
                                        double cfl, void *stream)
{
    if (!c || !W || !hot) return fail(GSIS_E_ARG, "null argument");
    if (!c->bound) return fail(GSIS_E_STATE, "case is not bound to a workspace");
    if (n_inner < 0 || cfl == 0 || !std::isfinite(cfl)) return fail(GSIS_E_ARG, "bad n_inner or cfl");
    if (c->dr > 0) return fail(GSIS_E_ARG, "gsis_macro_solve: the two-VDF gas's synthetic solve runs inside gsis_step");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(c->hv.status, 0, 16, s));
    HIPCHK(launch_check_W(c->cv, c->hv, W, s));
    HIPCHK(launch_macro_steps(c->cv, c->hv, W, hot, src, n_inner, cfl, s));
    return sync_status(c, s);
}

extern "C" gsis_status gsis_macro_solve_internal(gsis_case c, double *W, double *Tr, const double *hot,
                                                 const double *hot_r, const double *src, const double *src_r,
                                                 int32_t n_inner, double cfl, void *stream)
{
    if (!c || !W || !Tr || !hot) return fail(GSIS_E_ARG, "null argument");
    if (!c->bound) return fail(GSIS_E_STATE, "case is not bound to a workspace");
    if (!(c->dr > 0)) return fail(GSIS_E_ARG, "gsis_macro_solve_internal: a monatomic case (use gsis_macro_solve)");
    if (n_inner < 0 || cfl == 0 || !std::isfinite(cfl)) return fail(GSIS_E_ARG, "bad n_inner or cfl");
    hipStream_t s = (hipStream_t)stream;
    CaseView &h = c->hv;
    const size_t nc = (size_t)h.n_cells;
    HIPCHK(hipMemsetAsync(h.status, 0, 16, s));
    HIPCHK(launch_check_W(c->cv, h, W, s));
    // the q_r high-order terms and the rho e_r source live in the workspace
    if (hot_r) HIPCHK(hipMemcpyAsync(h.hotr, hot_r, 24 * nc, hipMemcpyDeviceToDevice, s));
    else HIPCHK(hipMemsetAsync(h.hotr, 0, 24 * nc, s));
    if (src) {
        if (src_r) HIPCHK(hipMemcpyAsync(h.srcr, src_r, 8 * nc, hipMemcpyDeviceToDevice, s));
        else HIPCHK(hipMemsetAsync(h.srcr, 0, 8 * nc, s));
    }
    MBatch b{};
    mbatch_add(b, c->cv, h, W, hot, src, Tr);
    HIPCHK(launch_macro_steps_poly(b, n_inner, cfl, s));
    return sync_status(c, s);
}

extern "C" gsis_status gsis_ns_init(gsis_case const *cases, int32_t n, const gsis_solve_params *p, int32_t *chunks,
                                    void *stream)
{
    if (!cases || n <= 0 || n > 1024) return fail(GSIS_E_ARG, "bad case list");
    gsis_status st;
    if ((st = check_params(p))) return st;
    if (p->mode != GSIS_MODE_AGSIS) return fail(GSIS_E_ARG, "the NS start belongs to aGSIS");
    for (int j = 0; j < n; ++j) {
        if ((st = check_ready(cases[j]))) return st;
        for (int i = 0; i < j; ++i)
            if (cases[i] == cases[j]) return fail(GSIS_E_ARG, "a case appears twice");
    }
    hipStream_t s = (hipStream_t)stream;
    // Step 1: every cell NS, the synthetic solve alone (HoT = 0) to eps < 1e-6
    const double ns_tol = 1e-6;
    for (int j = 0; j < n; ++j) {
        gsis_case c = cases[j];
        CaseView &h = c->hv;
        HIPCHK(launch_set_flags(c->cv, h, nullptr, 0, s));
        HIPCHK(launch_compact(c->cv, h, s));
        if ((st = read_counts(c, s, nullptr))) return st;
        HIPCHK(hipMemsetAsync(h.hot, 0, 72 * (size_t)h.n_cells, s));
        if (h.poly) HIPCHK(hipMemsetAsync(h.hotr, 0, 24 * (size_t)h.n_cells, s));
        if (chunks) chunks[j] = 0;
    }
    std::vector<gsis_case> active(cases, cases + n);
    std::vector<int> idx(n);
    for (int j = 0; j < n; ++j) idx[j] = j;
    const int max_chunks = p->ns_init_max_chunks > 0 ? p->ns_init_max_chunks : 1000;
    for (int k = 0; k < max_chunks && !active.empty(); ++k) {
        for (gsis_case c : active) {
            HIPCHK(launch_copy_W(c->hv.Wn, c->hv.W, c->hv.n_cells, s));
            if (c->hv.poly) HIPCHK(launch_copy_d(c->hv.Trn, c->hv.Tr, c->hv.n_cells, s));
        }
        for (size_t j0 = 0; j0 < active.size(); j0 += MAX_BATCH)
            if ((st = run_macro_batch(active.data() + j0, (int)std::min<size_t>(MAX_BATCH, active.size() - j0),
                                      p->n_macro_inner, p->cfl, false, s)))
                return st;
        std::vector<double> e(3 * active.size());
        for (size_t j = 0; j < active.size(); ++j) {
            CaseView &h = active[j]->hv;
            HIPCHK(launch_eps(active[j]->cv, h, h.Wn, h.W, s));
            HIPCHK(launch_copy_W(h.W, h.Wn, h.n_cells, s));
            if (h.poly) HIPCHK(launch_copy_d(h.Tr, h.Trn, h.n_cells, s));
            HIPCHK(hipMemcpyAsync(&e[3 * j], h.eps, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipStreamSynchronize(s));
        std::vector<gsis_case> still;
        std::vector<int> still_idx;
        for (size_t j = 0; j < active.size(); ++j) {
            if ((st = sync_status(active[j], s))) return st;
            if (chunks) chunks[idx[j]] = k + 1;
            if (std::max(e[3 * j], std::max(e[3 * j + 1], e[3 * j + 2])) >= ns_tol) {
                still.push_back(active[j]);
                still_idx.push_back(idx[j]);
            }
        }
        active.swap(still);
        idx.swap(still_idx);
    }
    // Step 2: first flagging; every kinetic cell is new and starts from Grad-13.
    // A case whose flagging fails (a region beyond its capacity) is marked with
    // chunks[j] = -1 and the others complete; the first error is returned.
    gsis_status first = GSIS_OK;
    std::string first_msg;
    for (int j = 0; j < n; ++j) {
        if ((st = gsis_update_regions(cases[j], p->Kn_ref, p->force_wall_layers, nullptr, stream))) {
            if (chunks) chunks[j] = -1;
            if (!first) {
                first = st;
                first_msg = "case " + std::to_string(j) + " of the batch: " + g_err;
            }
        }
    }
    if (first) return fail(first, "%s", first_msg.c_str());
    return GSIS_OK;
}

extern "C" gsis_status gsis_solve_steady(gsis_case c, const gsis_solve_params *p, gsis_solve_result *r, void *stream)
{
    gsis_status st = check_ready(c);
    if (st) return st;
    if ((st = check_params(p))) return st;
    if ((st = check_source(&c, 1, p))) return st;
    if (!r) return fail(GSIS_E_ARG, "null result");
    const bool ns_init = p->mode == GSIS_MODE_AGSIS && p->ns_init;
    if (!(p->tol > 0) || p->max_iter < 0 || (p->max_iter == 0 && !ns_init))
        return fail(GSIS_E_ARG, "bad tol or max_iter");
    std::memset(r, 0, sizeof *r);
    if (ns_init) {
        if ((st = gsis_ns_init(&c, 1, p, nullptr, stream))) return st;
        r->n_kinetic = c->n_kin;
        if (p->max_iter == 0) return GSIS_OK;
    }
    double eps[3] = {1, 1, 1};
    for (int it = 0; it < p->max_iter; ++it) {
        if ((st = gsis_step(&c, 1, p, eps, stream))) return st;
        r->iterations = it + 1;
        for (int k = 0; k < 3; ++k) r->eps[k] = eps[k];
        r->n_kinetic = c->n_kin;
        if (std::max(eps[0], std::max(eps[1], eps[2])) < p->tol) return GSIS_OK;
    }
    return fail(GSIS_E_NOCONV, "not converged after %d iterations (eps %g %g %g)", p->max_iter, eps[0], eps[1], eps[2]);
}
