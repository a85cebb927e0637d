"""FP64 CPU oracle for the adaptive GSIS kinetic sweep -- TEST INFRASTRUCTURE.

Only tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library (``paper_2501_02245_amd``): the numerical pieces live in
``gsis_oracle.c`` (plain loops, FP64), and this module strings them together
in the order of the paper's algorithm (Zhang, Zeng & Wu, arXiv 2501.02245,
Sec. 3.1-3.4).  Inputs come from ``gsis_inputs`` only.

Functions with no pin against an independent result are marked
"parity unpinned" in their docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
NMOM = 14
PI = np.pi


def build(force: bool = False) -> str:
    """Compile gsis_oracle.c into liboracle.so with gcc (FP64, OpenMP)."""
    src = os.path.join(_HERE, "gsis_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_cells", C.c_int32), ("n_faces", C.c_int32),
                ("n_patches", C.c_int32),
                ("face_cells", C.c_void_p), ("face_normal", C.c_void_p), ("face_area", C.c_void_p),
                ("face_center", C.c_void_p), ("cell_volume", C.c_void_p), ("cell_center", C.c_void_p),
                ("patch_kind", C.c_void_p), ("patch_state", C.c_void_p)]


class _Grid(C.Structure):
    _fields_ = [("vdim", C.c_int32), ("n", C.c_int32 * 3), ("x", C.c_void_p * 3), ("w", C.c_void_p * 3),
                ("npts", C.c_int32), ("pts", C.c_void_p), ("pw", C.c_void_p)]


class _Gas(C.Structure):
    _fields_ = [("Kn", C.c_double), ("omega", C.c_double), ("Pr", C.c_double), ("inv_dt", C.c_double),
                ("damp2", C.c_double),
                ("dr", C.c_double), ("Zr", C.c_double), ("A", C.c_double * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.oc_nv.restype = C.c_int32
        _lib.oc_threads.restype = C.c_int32
        _lib.oc_tau.restype = C.c_double
        for name in ("oc_fixup", "oc_equilibrium", "oc_feq", "oc_sweep", "oc_macro"):
            getattr(_lib, name).restype = C.c_int32
        _lib.oc_tau.argtypes = [P, C.c_double, C.c_double]
        _lib.oc_fixup.argtypes = [P, C.c_double, P, C.c_double, P, P]
        _lib.oc_maxwellian.argtypes = [P, C.c_double, P, C.c_double, P]
        _lib.oc_shakhov.argtypes = [P, C.c_double, P, P]
        _lib.oc_lsq_gradients.argtypes = [P, C.c_int32, P, P, P]
        _lib.oc_nsf.argtypes = [P, C.c_double, P, P, P, P]
        _lib.oc_sweep.argtypes = [P, P, P, C.c_int32, P, P, P, P, P]
        _lib.oc_macro.argtypes = [P, P, P, P, C.c_int32, C.c_double, P]
        _lib.oc_macro_residual.restype = C.c_int32
        _lib.oc_macro_residual.argtypes = [P, P, P, P, P]
        _lib.oc_kinetic_residual.restype = C.c_int32
        _lib.oc_kinetic_residual.argtypes = [P, P, C.c_int32, P, P, P, P, P]
        for name in ("oc_kinetic_slopes", "oc_sweep2", "oc_kinetic_residual2", "oc_poly_target", "oc_sweep_poly"):
            getattr(_lib, name).restype = C.c_int32
        _lib.oc_moments_poly.argtypes = [P, C.c_double, P, P]
        _lib.oc_g13_poly.argtypes = [P, C.c_double, P, P]
        _lib.oc_nsf_poly.argtypes = [P, C.c_double, P, P, P, P, P, P]
        for name in ("oc_kinetic_residual_poly", "oc_macro_residual_poly", "oc_macro_poly"):
            getattr(_lib, name).restype = C.c_int32
        _lib.oc_kinetic_residual_poly.argtypes = [P, P, P, C.c_int32, P, P, P, P, P]
        _lib.oc_macro_residual_poly.argtypes = [P, P, P, P, P]
        _lib.oc_macro_poly.argtypes = [P, P, P, P, C.c_int32, C.c_double, P]
        _lib.oc_poly_target.argtypes = [P, P, P, P]
        _lib.oc_sweep_poly.argtypes = [P, P, P, C.c_int32, P, P, P, P, P]
        _lib.oc_kinetic_slopes.argtypes = [P, P, C.c_int32, P, P, P, P]
        _lib.oc_sweep2.argtypes = [P, P, P, C.c_int32, P, P, P, P, P, P]
        _lib.oc_kinetic_residual2.argtypes = [P, P, C.c_int32, P, P, P, P, P, P]
    return _lib


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Plain FP64 implementation of one steady problem (mesh + gas + grid).

    order 2: second-order face values (limited least-squares slopes of every
    discrete-velocity value, deferred correction of the first-order implicit
    sweep) with the pseudo-time factor damp2 of that iteration.

    dr > 0: the polyatomic two-VDF gas (Sec. 2) with internal collision number
    Zr and heat-flux matrix A = (A_tt, A_tr, A_rt, A_rr); rows are (f0, f1) on
    a 3D velocity grid and moments carry T_r and q_r after the 14 of f0.
    """

    def __init__(self, mesh, grid, Kn, omega=0.5, Pr=2.0 / 3.0, inv_dt=0.0, order=1, damp2=2.0,
                 dr=0.0, Zr=1.0, A=None, g13_rmax=0.5):
        L = lib()
        # range limit of the Grad-13 rows (reading; None: unlimited)
        self.g13_rmax = g13_rmax
        self.last_g13_limited = None
        if order not in (1, 2):
            raise ValueError("spatial order must be 1 or 2")
        self.order = order
        self.mesh, self.grid = mesh, grid
        self.vdim = grid["vdim"]
        self.nfun = 1 if self.vdim == 3 else 2
        self._keep = []
        k = self._keep.append
        fc = np.ascontiguousarray(mesh["face_cells"], dtype=np.int32); k(fc)
        arrs = [_f64(mesh[n]) for n in ("face_normal", "face_area", "face_center", "cell_volume", "cell_center")]
        for a in arrs:
            k(a)
        pk = np.array([0 if p["kind"] == "wall" else 1 for p in mesh["patches"]], dtype=np.int32); k(pk)
        ps = np.array([[p["rho"], *p["u"], p["T"]] for p in mesh["patches"]], dtype=np.float64).reshape(-1, 5); k(ps)
        self.patch_state = ps
        self.patch_kind = pk
        self.cm = _Mesh(mesh["dim"], mesh["n_cells"], mesh["n_faces"], len(mesh["patches"]),
                        fc.ctypes.data, *[a.ctypes.data for a in arrs], pk.ctypes.data, ps.ctypes.data)
        self.cg = _Grid()
        self.cg.vdim = self.vdim
        if grid.get("kind") == "points":
            # a point set with its own weights (non-tensor velocity grid)
            pts, pw = _f64(grid["points"]).reshape(-1, 3), _f64(grid["pweights"])
            k(pts); k(pw)
            self.cg.npts = len(pw)
            self.cg.pts = pts.ctypes.data
            self.cg.pw = pw.ctypes.data
        for d in range(3):
            if grid.get("kind") == "points":
                self.cg.n[d] = 1
            elif d < self.vdim:
                x, w = _f64(grid["nodes"][d]), _f64(grid["weights"][d])
                k(x); k(w)
                self.cg.n[d] = len(x)
                self.cg.x[d] = x.ctypes.data
                self.cg.w[d] = w.ctypes.data
            else:
                self.cg.n[d] = 1
        self.nv = L.oc_nv(C.byref(self.cg))
        self.poly = dr > 0
        if self.poly and (self.vdim != 3 or order != 1):
            raise ValueError("the polyatomic gas needs a 3D velocity grid and first-order face values")
        if self.poly:
            self.nfun = 2
        Av = (C.c_double * 4)(*([Pr, 0.0, 0.0, 1.0] if A is None else [float(a) for a in A]))
        self.gas = _Gas(Kn, omega, Pr, inv_dt, damp2, dr, Zr, Av)
        self.Kn, self.omega, self.Pr = Kn, omega, Pr
        self.dr, self.Zr = dr, Zr
        # per-node velocities and weights (for tests and diagnostics)
        self.xi, self.w = self._nodes()

    def _nodes(self):
        g = self.grid
        if g.get("kind") == "points":
            return np.array(g["points"], dtype=np.float64).reshape(-1, 3), np.array(g["pweights"], dtype=np.float64)
        if self.vdim == 3:
            X, Y, Z = np.meshgrid(*g["nodes"], indexing="ij")
            WX, WY, WZ = np.meshgrid(*g["weights"], indexing="ij")
            xi = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
            w = (WX * WY * WZ).ravel()
        else:
            X, Y = np.meshgrid(*g["nodes"], indexing="ij")
            WX, WY = np.meshgrid(*g["weights"], indexing="ij")
            xi = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], 1)
            w = (WX * WY).ravel()
        return xi, w

    # --- single-cell pieces -------------------------------------------------
    def row_shape(self):
        return (self.nfun, self.nv)

    def moments(self, f):
        """Moments of rows f[..., nfun, nv] -> [..., 14] (Sec. 2, getmoment);
        polyatomic: [..., 18] with T_r, q_r appended (T and q are T_t, q_t)."""
        f = _f64(f)
        lead = f.shape[:-2]
        fr = f.reshape(-1, self.nfun * self.nv)
        nm = NMOM + 4 if self.poly else NMOM
        out = np.empty((fr.shape[0], nm))
        for i in range(fr.shape[0]):
            row = np.ascontiguousarray(fr[i])
            if self.poly:
                lib().oc_moments_poly(C.byref(self.cg), float(self.dr), _p(row), _p(out[i]))
            else:
                lib().oc_moments(C.byref(self.cg), _p(row), _p(out[i]))
        return out.reshape(*lead, nm)

    def poly_target(self, mom):
        """Polyatomic relaxation targets (G0, G1) with the conservation fix-up, [2, nv]."""
        out = np.empty((2, self.nv))
        m = _f64(mom)
        if lib().oc_poly_target(C.byref(self.cg), C.byref(self.gas), _p(m), _p(out)) != 0:
            raise FloatingPointError("fix-up system singular")
        return out

    def maxwellian(self, rho, u, T):
        out = np.empty(self.row_shape())
        uu = _f64(np.asarray(u, dtype=np.float64).reshape(3))
        lib().oc_maxwellian(C.byref(self.cg), float(rho), _p(uu), float(T), _p(out))
        return out

    def shakhov(self, mom):
        out = np.empty(self.row_shape())
        m = _f64(mom)
        lib().oc_shakhov(C.byref(self.cg), float(self.Pr), _p(m), _p(out))
        return out

    def fixup(self, g, rho, u, T):
        g = _f64(g).copy()
        coef = np.zeros(5)
        uu = _f64(np.asarray(u, dtype=np.float64).reshape(3))
        r = lib().oc_fixup(C.byref(self.cg), float(rho), _p(uu), float(T), _p(g), _p(coef))
        if r != 0:
            raise FloatingPointError("fix-up system singular")
        return g, coef[: self.vdim + 2]

    def equilibrium(self, mom):
        out = np.empty(self.row_shape())
        m = _f64(mom)
        if lib().oc_equilibrium(C.byref(self.cg), C.byref(self.gas), _p(m), _p(out)) != 0:
            raise FloatingPointError("fix-up system singular")
        return out

    def feq(self, W5):
        """Conservation-fixed Maxwellian of W (Sec. 3.2) at (rho, u, T).
        Polyatomic, W = (rho, u, T_t, T_r): f0 at T_t, and f1 = (d_r T_r / 4) f0
        (f_eq,1 = (d_r/2) R T_r f_eq); a five-component W uses T_r = T_t."""
        out = np.empty(self.row_shape())
        w = _f64(W5)
        if lib().oc_feq(C.byref(self.cg), _p(np.ascontiguousarray(w[:5])), _p(out)) != 0:
            raise FloatingPointError("fix-up system singular")
        if self.poly:
            Tr = w[5] if len(w) > 5 else w[4]
            out[1] = 0.25 * self.dr * Tr * out[0]
        return out

    def g13(self, mom):
        """Grad-13 rows (Sec. 3.2 eq. G13_VDF) of parameters mom; polyatomic:
        the 18 parameters of ghost_params (T_r and q_r last)."""
        out = np.empty(self.row_shape())
        m = _f64(mom)
        if self.poly:
            lib().oc_g13_poly(C.byref(self.cg), float(self.dr), _p(m), _p(out))
        else:
            lib().oc_g13(C.byref(self.cg), _p(m), _p(out))
        return out

    def tau(self, rho, T):
        return lib().oc_tau(C.byref(self.gas), float(rho), float(T))

    # --- field-level pieces -------------------------------------------------
    def sweep(self, f_old, kin_cell, slot_of_cell, ghost=None, slope=None):
        """One point-Jacobi kinetic sweep (Sec. 3.1).  f_old [n_slots, nfun, nv].
        Order 2: `slope` [n_slots, nfun, nv, 3] (default: the slopes of f_old over
        kin_cell; pass them to sweep a subset of cells whose neighbours' slopes
        come from a larger list)."""
        f_old = _f64(f_old)
        f_new = np.zeros_like(f_old)
        kc = np.ascontiguousarray(kin_cell, dtype=np.int32)
        sc = np.ascontiguousarray(slot_of_cell, dtype=np.int32)
        if ghost is None:
            ghost = np.zeros((self.mesh["n_cells"], NMOM + 4 if self.poly else NMOM))
        gh = _f64(ghost)
        if self.poly:
            r = lib().oc_sweep_poly(C.byref(self.cm), C.byref(self.cg), C.byref(self.gas), len(kc), _p(kc),
                                    _p(sc), _p(f_old), _p(gh), _p(f_new))
            if r != 0:
                raise FloatingPointError("oracle sweep failed (%d)" % r)
            return f_new
        sl = None
        if self.order == 2:
            sl = self.slopes(f_old, kc, sc) if slope is None else np.ascontiguousarray(slope, dtype=np.float64)
        r = lib().oc_sweep2(C.byref(self.cm), C.byref(self.cg), C.byref(self.gas), len(kc), _p(kc), _p(sc),
                            _p(f_old), _p(gh), _p(sl), _p(f_new))
        if r != 0:
            raise FloatingPointError("oracle sweep failed (%d)" % r)
        return f_new

    def slopes(self, f, kin_cell, slot_of_cell):
        """Limited least-squares slopes of every discrete-velocity value of the
        kinetic cells (second-order face values): [n_slots, nfun, nv, 3]."""
        f = _f64(f)
        out = np.zeros(f.shape + (3,))
        kc = np.ascontiguousarray(kin_cell, dtype=np.int32)
        sc = np.ascontiguousarray(slot_of_cell, dtype=np.int32)
        lib().oc_kinetic_slopes(C.byref(self.cm), C.byref(self.cg), len(kc), _p(kc), _p(sc), _p(f), _p(out))
        return out

    def lsq(self, phi, bnd):
        """LSQ gradients (Sec. 3.4 Step 2). phi [n_cells, nvar], bnd [n_patches, nvar]."""
        phi = _f64(phi)
        nvar = phi.shape[1]
        bnd = _f64(bnd).reshape(len(self.mesh["patches"]), nvar)
        grad = np.zeros((phi.shape[0], nvar, 3))
        lib().oc_lsq_gradients(C.byref(self.cm), nvar, _p(phi), _p(bnd), _p(grad))
        return grad

    def nsf(self, T, grad_u, grad_T):
        s = np.zeros(6)
        q = np.zeros(3)
        gu = _f64(grad_u).reshape(9)
        gt = _f64(grad_T).reshape(3)
        lib().oc_nsf(C.byref(self.gas), float(T), _p(gu), _p(gt), _p(s), _p(q))
        return s, q

    def primitive_gradients(self, W):
        """LSQ gradients of (ux, uy, uz, T, rho, |u|) with patch values at faces;
        polyatomic W (6 columns): a seventh row, the gradient of T_r (patch
        value T)."""
        cols = [W[:, 1:5], W[:, :1], np.linalg.norm(W[:, 1:4], axis=1)[:, None]]
        poly = W.shape[1] > 5
        if poly:
            cols.append(W[:, 5:6])
        phi = np.concatenate(cols, 1)
        bnd = np.full((len(self.mesh["patches"]), phi.shape[1]), np.nan)
        for p, pt in enumerate(self.mesh["patches"]):
            bnd[p, 0:3] = pt["u"]
            bnd[p, 3] = pt["T"]
            bnd[p, 5] = np.linalg.norm(pt["u"])
            if poly:
                bnd[p, 6] = pt["T"]
            if pt["kind"] == "far":
                bnd[p, 4] = pt["rho"]
        return self.lsq(phi, bnd)

    def nsf_field(self, W, grad=None):
        """sigma_NSF, q_NSF on every cell from LSQ gradients of W (Sec. 2
        NSF_constitutive); polyatomic W: [n, 12] = sigma, q_t, q_r (eq. mu_kappa)."""
        if grad is None:
            grad = self.primitive_gradients(W)
        if W.shape[1] > 5:
            out = np.zeros((len(W), 12))
            for i in range(len(W)):
                s, qt, qr = np.zeros(6), np.zeros(3), np.zeros(3)
                gu = _f64(grad[i, 0:3, :]).reshape(9)
                lib().oc_nsf_poly(C.byref(self.gas), float(W[i, 4]), _p(gu), _p(_f64(grad[i, 3, :])),
                                  _p(_f64(grad[i, 6, :])), _p(s), _p(qt), _p(qr))
                out[i, :6], out[i, 6:9], out[i, 9:] = s, qt, qr
            return out
        out = np.zeros((len(W), 9))
        for i in range(len(W)):
            s, q = self.nsf(W[i, 4], grad[i, 0:3, :], grad[i, 3, :])
            out[i, :6] = s
            out[i, 6:] = q
        return out

    def ghost_params(self, W, grad=None):
        """Grad-13 parameters (rho, u, T, sigma_NSF, q_NSF) per cell (Sec. 3.2).

        Reading: the Grad expansion is used inside its range of validity.  With
        r = max(max_ij |sigma_ij| / p, |q| / (p sqrt(T))), p = rho T, the pair
        (sigma, q) is scaled by min(1, rmax / r), rmax = g13_rmax (0.5 by
        default, None: no limit), so that the polynomial factor of the Grad-13
        distribution stays of order one at thermal speeds (an unlimited one
        from a strongly sheared NS field is negative over much of velocity
        space).  The cells whose pair was scaled are left in
        ``last_g13_limited`` (bool per cell)."""
        if self.poly and W.shape[1] == 5:
            W = np.concatenate([W, W[:, 4:5]], 1)   # internal modes at T_t
        nsf = self.nsf_field(W, grad)
        p = W[:, 0] * W[:, 4]
        r = np.maximum(np.abs(nsf[:, :6]).max(axis=1) / p, np.linalg.norm(nsf[:, 6:9], axis=1) / (p * np.sqrt(W[:, 4])))
        if W.shape[1] > 5:
            # two-VDF gas: the q_r term of f1 (q_r.c/(rho T_t) M at thermal
            # speed sqrt(T_t)) relative to its equilibrium part (d_r T_r/4) M
            r = np.maximum(r, 4.0 * np.linalg.norm(nsf[:, 9:12], axis=1) /
                           (self.dr * W[:, 0] * W[:, 5] * np.sqrt(W[:, 4])))
        rmax = self.g13_rmax
        if rmax is None:
            theta = np.ones(len(W))
        else:
            theta = np.where(r > rmax, rmax / np.where(r > 0, r, 1.0), 1.0)
        self.last_g13_limited = theta < 1.0
        poly = W.shape[1] > 5
        gh = np.zeros((len(W), NMOM + 4 if poly else NMOM))
        gh[:, 0:5] = W[:, :5]
        gh[:, 5:11] = nsf[:, :6] * theta[:, None]
        gh[:, 11:14] = nsf[:, 6:9] * theta[:, None]
        if poly:
            gh[:, 14] = W[:, 5]
            gh[:, 15:18] = nsf[:, 9:12] * theta[:, None]
        if self.vdim == 2:
            gh[:, 3] = 0.0
            gh[:, 9:11] = 0.0
            gh[:, 13] = 0.0
        return gh

    def kn_gll(self, W, grad=None):
        """Gradient-length local Kn (Sec. 3.2 eq. Kn_Gll).

        Reading: lambda = Kn T^(omega - 1/2) / rho (scaled mean free path),
        |grad U| / max(U, a) with a = sqrt(5 T / 6) so that U -> 0 stays finite.
        """
        if grad is None:
            grad = self.primitive_gradients(W)
        rho, T = W[:, 0], W[:, 4]
        U = np.linalg.norm(W[:, 1:4], axis=1)
        a = np.sqrt(5.0 * T / 6.0)
        lam = self.Kn * T ** (self.omega - 0.5) / rho
        gr = np.linalg.norm(grad[:, 4, :], axis=1) / rho
        gu = np.linalg.norm(grad[:, 5, :], axis=1) / np.maximum(U, a)
        gt = np.linalg.norm(grad[:, 3, :], axis=1) / T
        return lam * np.maximum(np.maximum(gr, gu), gt)

    def wall_layers(self, n_layers):
        """Cells within n_layers face-neighbour hops of a wall (reading of the forced wall layers)."""
        m = self.mesh
        fc = m["face_cells"]
        mark = np.zeros(m["n_cells"], dtype=bool)
        wall_p = [p for p, pt in enumerate(m["patches"]) if pt["kind"] == "wall"]
        bnd = fc[:, 1] < 0
        for p in wall_p:
            mark[fc[bnd & (fc[:, 1] == -1 - p), 0]] = True
        inner = fc[:, 1] >= 0
        a, b = fc[inner, 0], fc[inner, 1]
        cur = mark.copy()
        for _ in range(max(n_layers - 1, 0)):
            nxt = cur.copy()
            nxt[b[cur[a]]] = True
            nxt[a[cur[b]]] = True
            cur = nxt
        return cur if n_layers > 0 else np.zeros_like(mark)

    def flags(self, W, Kn_ref, force_wall_layers=0, grad=None):
        """DVM region flag = Kn_Gll >= Kn_ref (Sec. 3.2 second eq. updatef; ties are kinetic)."""
        k = self.kn_gll(W, grad) >= Kn_ref
        return (k | self.wall_layers(force_wall_layers)).astype(np.uint8)

    def macro(self, W, hot, n_inner, cfl=0.5, src=None):
        """Synthetic macroscopic solve (Sec. 3.1 eq. macro); see oc_macro for
        the reading.  Polyatomic: W [n, 6], hot [n, 12], src [n, 6] (oc_macro_poly,
        with the internal-energy equation of Sec. 2 eq. macroscopic_equation_2)."""
        Wio = _f64(W).copy()
        h = _f64(hot)
        sr = _f64(src) if src is not None else None
        fn = lib().oc_macro_poly if self.poly else lib().oc_macro
        r = fn(C.byref(self.cm), C.byref(self.gas), _p(h), _p(sr), int(n_inner), float(cfl), _p(Wio))
        if r != 0:
            raise FloatingPointError("macro solve produced a non-positive state")
        return Wio

    def macro_residual(self, W, hot):
        """Per-unit-volume residual of the synthetic equations at W (monatomic:
        no source; polyatomic: with the internal relaxation source)."""
        Wc = _f64(W)
        h = _f64(hot)
        out = np.zeros((len(Wc), 6 if self.poly else 5))
        fn = lib().oc_macro_residual_poly if self.poly else lib().oc_macro_residual
        if fn(C.byref(self.cm), C.byref(self.gas), _p(h), _p(Wc), _p(out)) != 0:
            raise FloatingPointError("non-positive state")
        return out

    def wall_faces(self):
        """Boundary faces on diffuse-wall patches, ascending face id."""
        fc = self.mesh["face_cells"]
        kinds = self.patch_kind
        return np.array([f for f in range(len(fc)) if fc[f, 1] < 0 and kinds[-1 - fc[f, 1]] == 0], dtype=np.int64)

    def surface(self, f, slot_of_cell, W, grad=None):
        """Surface quantities on every diffuse-wall face (Sec. 4.2/4.3: surface
        pressure, heat flux, aerodynamic forces), rows [n_wall][9]:
        stress tau = P.n exerted by the gas (3), p = tau.n, shear tau - p n (3),
        heat flux into the wall, net mass flux.  n points out of the gas.

        Kinetic wall cell (slot >= 0), in the wall frame c = xi - u_w:
        incoming velocities (c.n > 0) carry the cell's distribution, reflected
        ones rho_w M(u_w, T_w) with rho_w making the net mass flux zero (the
        diffuse wall of the sweep); tau = 2 sum w c (c.n) f (P = 2 int c c f in
        these units), q = sum w (c.n) |c|^2 f, reduced 2D q = sum w (c.n)
        (|c|^2 phi + psi).  NS wall cell: tau = rho T n + sigma.n and
        q = q.n with the NSF laws at T_w evaluated on the LSQ cell gradient
        whose normal part is replaced by the one-sided difference to the wall
        values (the wall flux of the synthetic equations).

        Two-VDF gas (W with T_r as a sixth column): the energy carried is
        |c|^2 f0 + 2 f1 (the total energy of the scaled units), the reflected
        f1 is (d_r T_w / 4) rho_w M (internal modes in equilibrium with the
        wall), and an NS wall cell's heat flux is (q_t + q_r).n of the
        two-temperature NSF laws with T_r also held at T_w.
        """
        m = self.mesh
        fc = m["face_cells"]
        faces = self.wall_faces()
        out = np.zeros((len(faces), 9))
        if grad is None:
            grad = self.primitive_gradients(W)
        for j, fi in enumerate(faces):
            L = fc[fi, 0]
            pt = m["patches"][-1 - fc[fi, 1]]
            n = np.asarray(m["face_normal"][fi], dtype=np.float64)
            uw = np.asarray(pt["u"], dtype=np.float64)
            Tw = float(pt["T"])
            s = slot_of_cell[L]
            if s >= 0:
                c = self.xi.copy()
                c[:, : self.vdim] -= uw[: self.vdim]
                a = c @ n
                c2 = np.sum(c * c, axis=1)
                M = self.maxwellian(1.0, uw, Tw).reshape(self.nfun, self.nv)
                if self.poly:
                    M[1] = 0.25 * self.dr * Tw * M[0]
                row = np.asarray(f[s], dtype=np.float64).reshape(self.nfun, self.nv)
                inc, ref = a > 0, a < 0
                rho_w = np.sum(self.w[inc] * a[inc] * row[0, inc]) / np.sum(self.w[ref] * -a[ref] * M[0, ref])
                g = np.where(inc[None, :], row, np.where(ref[None, :], rho_w * M, 0.0))
                tau = 2.0 * np.sum((self.w * a * g[0])[:, None] * c, axis=0)
                if self.poly:
                    e = c2 * g[0] + 2.0 * g[1]
                else:
                    e = c2 * g[0] + (g[1] if self.nfun == 2 else 0.0)
                q = np.sum(self.w * a * e)
                mass = np.sum(self.w * a * g[0])
            else:
                dn = float(np.dot(m["face_center"][fi] - m["cell_center"][L], n))
                wall = np.concatenate([uw, [Tw]])
                cellv = np.concatenate([W[L, 1:4], [W[L, 4]]])
                G = grad[L, 0:4, :].copy()
                for v in range(4):
                    G[v] += ((wall[v] - cellv[v]) / dn - np.dot(G[v], n)) * n
                if self.poly:
                    Gr = grad[L, 6, :].copy()
                    Gr += ((Tw - W[L, 5]) / dn - np.dot(Gr, n)) * n
                    sg, qt, qr = np.zeros(6), np.zeros(3), np.zeros(3)
                    gu, gt, gr = _f64(G[0:3]).reshape(9).copy(), _f64(G[3]).copy(), _f64(Gr).copy()
                    lib().oc_nsf_poly(C.byref(self.gas), float(Tw), _p(gu), _p(gt), _p(gr), _p(sg), _p(qt), _p(qr))
                    qv = qt + qr
                else:
                    sg, qv = self.nsf(Tw, G[0:3], G[3])
                S = np.array([[sg[0], sg[3], sg[4]], [sg[3], sg[1], sg[5]], [sg[4], sg[5], sg[2]]])
                tau = W[L, 0] * W[L, 4] * n + S @ n
                q = float(np.dot(qv, n))
                mass = 0.0
            p = float(np.dot(tau, n))
            out[j, 0:3] = tau
            out[j, 3] = p
            out[j, 4:7] = tau - p * n
            out[j, 7] = q
            out[j, 8] = mass
        return faces, out

    def kinetic_residual(self, f, kin_cell, slot_of_cell, ghost=None):
        """Moment balance (mass, momentum, energy per unit volume) of the kinetic
        scheme at f; polyatomic: [n, 6] with the internal energy (face fluxes and
        the exchange term of the sweep's targets)."""
        f = _f64(f)
        kc = np.ascontiguousarray(kin_cell, dtype=np.int32)
        sc = np.ascontiguousarray(slot_of_cell, dtype=np.int32)
        if self.poly:
            gh = _f64(ghost if ghost is not None else np.zeros((self.mesh["n_cells"], NMOM + 4)))
            out = np.zeros((self.mesh["n_cells"], 6))
            if lib().oc_kinetic_residual_poly(C.byref(self.cm), C.byref(self.cg), C.byref(self.gas), len(kc),
                                              _p(kc), _p(sc), _p(f), _p(gh), _p(out)) != 0:
                raise FloatingPointError("fix-up system singular")
            return out
        gh = _f64(ghost if ghost is not None else np.zeros((self.mesh["n_cells"], NMOM)))
        out = np.zeros((self.mesh["n_cells"], 5))
        sl = self.slopes(f, kc, sc) if self.order == 2 else None
        lib().oc_kinetic_residual2(C.byref(self.cm), C.byref(self.cg), len(kc), _p(kc), _p(sc), _p(f), _p(gh),
                                   _p(sl), _p(out))
        return out

    # --- drivers -------------------------------------------------------------
    def residual(self, W_new, W_old):
        """Convergence measure of Sec. 4 (volume-weighted relative change of rho, u, T_t).

        Reading: u is taken as a vector; a vanishing denominator falls back to
        the absolute change.
        """
        V = self.mesh["cell_volume"]
        out = []
        for sl in (slice(0, 1), slice(1, 4), slice(4, 5)):
            num = np.sum(np.sum((W_new[:, sl] - W_old[:, sl]) ** 2, axis=1) * V)
            den = np.sum(np.sum(W_old[:, sl] ** 2, axis=1) * V)
            out.append(np.sqrt(num / den) if den > 1e-30 else np.sqrt(num))
        return np.array(out)


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oc_threads())


def set_threads(n):
    """Threads of the oracle's parallel loops from now on (n >= 1)."""
    lib().oc_set_threads(int(n))


def regions_from_flags(flags, old_slot_of_cell=None):
    """Compacted kinetic list (ascending cell id) and slot assignment.

    Cells that stay kinetic keep their slot; leaving cells free theirs; new
    cells take free slots lowest-first in ascending cell id.  Returns
    (kin_cell, slot_of_cell, new_cells).
    """
    flags = np.asarray(flags).astype(bool)
    n = len(flags)
    kin = np.nonzero(flags)[0].astype(np.int32)
    if old_slot_of_cell is None:
        slot = np.full(n, -1, dtype=np.int32)
        slot[kin] = np.arange(len(kin), dtype=np.int32)
        return kin, slot, kin.copy()
    slot = np.where(flags, old_slot_of_cell, -1).astype(np.int32)
    used = set(int(s) for s in slot[slot >= 0])
    new = np.nonzero(flags & (np.asarray(old_slot_of_cell) < 0))[0].astype(np.int32)
    free = (s for s in range(n) if s not in used)
    for c in new:
        slot[c] = next(free)
    return kin, slot, new


def conductivities(A, d_r):
    """kappa_t/(mu R), kappa_r/(mu R) from eq. (mu_kappa): (1/2) A^{-1} [5, d_r].

    For d_r = 0 the system reduces to kappa_t = (mu R / 2) 5 / A_tt.
    """
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    rhs = np.array([5.0, float(d_r)])[: A.shape[0]]
    return 0.5 * np.linalg.solve(A, rhs)


def eucken_factors(A, d_r):
    """Eucken factors f = kappa / (mu c_v) with c_v,t = 3R/2 and c_v,r = d_r R / 2."""
    k = conductivities(A, d_r)
    out = [k[0] / 1.5]
    if len(k) > 1:
        out.append(k[1] / (0.5 * d_r))
    return np.array(out)


def one_cell_mesh():
    """A single closed cell with no faces (homogeneous relaxation)."""
    return {"dim": 3, "n_cells": 1, "n_faces": 0,
            "face_cells": np.zeros((0, 2), dtype=np.int32), "face_normal": np.zeros((0, 3)),
            "face_area": np.zeros(0), "face_center": np.zeros((0, 3)),
            "cell_volume": np.ones(1), "cell_center": np.zeros((1, 3)), "patches": []}


def _cons(W, dr=0.0):
    """Conserved variables of W = (rho, u, T[, T_r]): (rho, rho u, E[, rho e_r]),
    E = rho |u|^2 + (3/2) rho T (+ rho e_r, rho e_r = (d_r/2) rho T_r)."""
    rho = W[0]
    E = rho * (W[1] ** 2 + W[2] ** 2 + W[3] ** 2) + 1.5 * rho * W[4]
    if len(W) > 5:
        er = 0.5 * dr * rho * W[5]
        return np.array([rho, rho * W[1], rho * W[2], rho * W[3], E + er, er])
    return np.array([rho, rho * W[1], rho * W[2], rho * W[3], E])


def _prim(U, dr=0.0):
    rho = U[0]
    u = U[1:4] / rho
    if len(U) > 5:
        return np.array([rho, u[0], u[1], u[2], (U[4] - rho * np.dot(u, u) - U[5]) / (1.5 * rho),
                         U[5] / (0.5 * dr * rho)])
    return np.array([rho, u[0], u[1], u[2], (U[4] - rho * np.dot(u, u)) / (1.5 * rho)])


def limit_correction(Wh, Wn, factor=2.0, halvings=10, with_theta=False, dr=0.0):
    """Limiter of the GSIS correction (reading; inactive at convergence).

    The conserved-variable change from W^{n+1/2} to W^{n+1} of a kinetic cell
    is halved (at most ten times, then dropped) until the new density and
    temperature lie within a factor 2 of those of W^{n+1/2}, so that the
    corrected distribution stays resolvable on the velocity grid.
    with_theta: also return the fraction of the change kept (1 = inactive,
    0 = dropped).  Two-VDF gas (six-component W, d_r = dr): the conserved
    variables include rho e_r, and T_r is held to the same range.
    """
    Uh, Un = _cons(Wh, dr), _cons(Wn, dr)
    th = 1.0
    for _ in range(halvings + 1):
        W = _prim(Uh + th * (Un - Uh), dr)
        ok = (Wh[0] / factor <= W[0] <= Wh[0] * factor) and (Wh[4] / factor <= W[4] <= Wh[4] * factor)
        if len(W) > 5:
            ok = ok and (Wh[5] / factor <= W[5] <= Wh[5] * factor)
        if ok:
            return (W, th) if with_theta else W
        th *= 0.5
    W = np.array(Wh, dtype=np.float64)
    return (W, 0.0) if with_theta else W


class SteadySolver:
    """Outer iteration of Sec. 3.4 (Steps 1-4), one plain step at a time.

    mode 'dvm'  : f^{n+1} = f^{n+1/2} (conventional iteration, no synthetic step)
    mode 'gsis' : every cell kinetic; Sec. 3.1 synthetic step and correction
    mode 'agsis': kinetic cells chosen by Kn_Gll >= Kn_ref (Sec. 3.2), NS elsewhere;
                  region_every k > 0 re-flags every k iterations, k < 0 once after
                  |k| iterations (Sec. 3.4 Step 3 takes five GSIS iterations first)

    State: W [n_cells, 5] primitive (rho, u, T) on every cell; flags; kinetic
    list and slots; f [n_slots, nfun, nv] for the kinetic cells.

    source_half (monatomic gas): the source of eq. macro is the kinetic
    balance at f^{n+1/2} minus the synthetic residual at W^{n+1/2}, and the
    synthetic solve starts from W^{n+1/2}; the synthetic equation is then
    the usual GSIS one, fed by the sweep's new non-equilibrium moments.
    Default: the balance at f^n and the residual at W^n, the solve from W^n.
    """

    def __init__(self, O, mode="gsis", Kn_ref=0.01, n_inner=400, cfl=0.5,
                 region_every=1, force_wall_layers=0, capacity=None, source_half=False):
        if source_half and O.poly:
            raise ValueError("source_half is defined for the monatomic gas")
        self.source_half = bool(source_half)
        self.O, self.mode = O, mode
        self.Kn_ref, self.n_inner, self.cfl = Kn_ref, n_inner, cfl
        self.region_every, self.layers = region_every, force_wall_layers
        self.n = O.mesh["n_cells"]
        self.capacity = capacity if capacity is not None else self.n
        self.it = 0
        # limiter activity of the last step and region update (readings R19b, R24):
        # Grad-13 ghost rows and new-cell rows whose (sigma, q) were scaled, and
        # kinetic cells whose correction was cut
        self.stats = {"g13_ghost_limited": 0, "g13_ghosts": 0, "g13_new_limited": 0, "g13_new": 0,
                      "corrections_limited": 0}

    # -- initial state ---------------------------------------------------------
    def _W_of(self, mom):
        """W of kinetic cells from their moments: (rho, u, T[_t]) [, T_r]."""
        if self.O.poly:
            return np.concatenate([mom[:, :5], mom[:, 14:15]], 1)
        return mom[:, :5]

    def set_state(self, W, f=None, flags=None):
        """W on all cells ((rho, u, T); two-VDF gas: (rho, u, T_t, T_r), a
        missing T_r is taken equal to T_t); f (rows for the kinetic cells in
        ascending id) or None to start kinetic cells from the
        conservation-fixed Maxwellian of W."""
        O = self.O
        self.W = np.array(W, dtype=np.float64)
        if O.poly and self.W.shape[1] == 5:
            self.W = np.concatenate([self.W, self.W[:, 4:5]], 1)
        if flags is None:
            flags = np.ones(self.n, np.uint8)
        self.flags = np.asarray(flags, dtype=np.uint8).copy()
        self.kin, self.slot, _ = regions_from_flags(self.flags)
        self.f = np.zeros((self.capacity,) + O.row_shape())
        if f is None:
            for c in self.kin:
                self.f[self.slot[c]] = O.feq(self.W[c])
        else:
            self.f[self.slot[self.kin]] = np.asarray(f, dtype=np.float64)
        # W on kinetic cells is the moments of their distribution
        if len(self.kin):
            self.W[self.kin] = self._W_of(O.moments(self.f[self.slot[self.kin]]))

    def ns_init(self, tol=1e-6, chunk=None, max_chunks=1000):
        """Step 1 (Sec. 3.4): every cell NS, the macroscopic (NSF) solve alone,
        HoT = 0, to eps < tol; then the first flagging (Step 2), so that every
        kinetic cell starts from the Grad-13 distribution of the NS field."""
        O = self.O
        self.flags = np.zeros(self.n, np.uint8)
        self.kin, self.slot, _ = regions_from_flags(self.flags)
        chunk = chunk or self.n_inner
        hot = np.zeros((self.n, 12 if O.poly else 9))
        k, eps = max_chunks, None
        for j in range(max_chunks):
            Wn = O.macro(self.W, hot, chunk, self.cfl)
            eps = O.residual(Wn, self.W)
            self.W = Wn
            if eps.max() < tol:
                k = j + 1
                break
        self.update_regions()
        return k, eps

    def update_regions(self):
        """Step 2/3: LSQ gradients, Kn_Gll flags, compaction, G13 init of new cells."""
        O = self.O
        grad = O.primitive_gradients(self.W)
        fl = O.flags(self.W, self.Kn_ref, self.layers, grad)
        kin, slot, new = regions_from_flags(fl, self.slot)
        if len(kin) > self.capacity:
            raise MemoryError("kinetic region exceeds capacity")
        gh = O.ghost_params(self.W, grad)
        for c in new:
            self.f[slot[c]] = O.g13(gh[c])
        self.stats["g13_new"] = len(new)
        self.stats["g13_new_limited"] = int(O.last_g13_limited[new].sum()) if len(new) else 0
        self.flags, self.kin, self.slot = fl, kin, slot
        return len(kin)

    def ghost_cells(self):
        """NS cells with a kinetic face neighbour (the cells whose Grad-13 rows a sweep reads)."""
        fc = self.O.mesh["face_cells"]
        inner = fc[:, 1] >= 0
        a, b = fc[inner, 0], fc[inner, 1]
        k = self.flags.astype(bool)
        mark = np.zeros(self.n, dtype=bool)
        mark[a[k[b] & ~k[a]]] = True
        mark[b[k[a] & ~k[b]]] = True
        return np.nonzero(mark)[0]

    # -- one outer iteration ---------------------------------------------------
    def step(self):
        O = self.O
        kin, slot = self.kin, self.slot
        rows = slot[kin]
        ghost = O.ghost_params(self.W) if self.mode == "agsis" else None
        if ghost is not None:
            gc = self.ghost_cells()
            self.stats["g13_ghosts"] = len(gc)
            self.stats["g13_ghost_limited"] = int(O.last_g13_limited[gc].sum())
        if self.mode != "dvm" and not self.source_half:
            Rk = O.kinetic_residual(self.f, kin, slot, ghost)
        f_half = O.sweep(self.f, kin, slot, ghost)
        mom_half = O.moments(f_half[rows])
        W_old = self.W
        W_half = W_old.copy()
        W_half[kin] = self._W_of(mom_half)
        if self.mode == "dvm":
            W_new = W_half
            self.f = f_half
        else:
            # high-order terms on kinetic cells (eq. full_constitutive)
            nsf = O.nsf_field(W_half)
            hot = np.zeros((self.n, nsf.shape[1]))
            hot[kin, :6] = mom_half[:, 5:11] - nsf[kin, :6]
            hot[kin, 6:9] = mom_half[:, 11:14] - nsf[kin, 6:9]
            if O.poly:
                # HoT of the internal heat flux (eq. full_constitutive, third line)
                hot[kin, 9:12] = mom_half[:, 15:18] - nsf[kin, 9:12]
            # Source Q of eq. macro (reading): on kinetic cells, the kinetic
            # scheme's own moment balance at f^n minus the synthetic residual
            # at W^n.  The synthetic solve then starts from W^n and acts as a
            # Newton-like corrector of the conserved moments, and its fixed
            # point is the fixed point of the kinetic iteration.
            src = np.zeros((self.n, W_old.shape[1]))
            if self.source_half:
                # the same at the half step: the sweep's f^{n+1/2} and W^{n+1/2}
                # (NS cells keep W^n, and their Grad-13 rows are those of the sweep)
                Rk = O.kinetic_residual(f_half, kin, slot, ghost)
                src[kin] = Rk[kin] - O.macro_residual(W_half, hot)[kin]
                W_new = O.macro(W_half, hot, self.n_inner, self.cfl, src)
            else:
                src[kin] = Rk[kin] - O.macro_residual(W_old, hot)[kin]
                W_new = O.macro(W_old, hot, self.n_inner, self.cfl, src)
            # GSIS correction (first eq. updatef), with the change of the
            # conserved moments limited on each kinetic cell
            cut = 0
            for c in kin:
                W_new[c], th = limit_correction(W_half[c], W_new[c], with_theta=True, dr=O.dr)
                cut += th < 1.0
                f_half[slot[c]] += O.feq(W_new[c]) - O.feq(W_half[c])
            self.stats["corrections_limited"] = int(cut)
            self.f = f_half
        eps = O.residual(W_new, W_old)
        self.W = W_new
        self.it += 1
        self.last_mom = mom_half
        k = self.region_every
        if self.mode == "agsis" and ((k > 0 and self.it % k == 0) or (k < 0 and self.it == -k)):
            self.update_regions()
        return eps

    def solve(self, tol=1e-6, max_iter=1000, callback=None):
        for _ in range(max_iter):
            eps = self.step()
            if callback:
                callback(self, eps)
            if eps.max() < tol:
                return self.it, eps
        return self.it, eps
