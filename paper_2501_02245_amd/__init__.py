"""Python binding of the MI355X adaptive-GSIS kinetic-sweep library (libgsis.so).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI of ``include/gsis.h``.  PyTorch provides device memory (the
case workspace and state buffers) and the HIP stream.  Importing this module
does not touch the GPU; the library is loaded on first use and its absence
raises an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsis.so")

OK, E_ARG, E_MESH, E_STATE, E_NOMEM, E_CAPACITY, E_HIP, E_NONFINITE, E_NOCONV = 0, -1, -2, -3, -4, -5, -6, -7, -8
F32, F64 = 0, 1
PATCH_WALL, PATCH_FAR = 0, 1
MODE_DVM, MODE_GSIS, MODE_AGSIS = 0, 1, 2
NMOM = 14
NSURF = 9
MAX_FACES, MAX_WALL_FACES, MAX_AXIS = 8, 4, 128

EXPORTS = [
    "gsis_last_error", "gsis_create_mesh", "gsis_destroy_mesh", "gsis_create_case", "gsis_destroy_case",
    "gsis_set_velocity_grid", "gsis_case_footprint", "gsis_case_bind", "gsis_set_state", "gsis_kinetic_sweep",
    "gsis_moments", "gsis_n_kinetic", "gsis_update_regions", "gsis_step", "gsis_solve_steady", "gsis_get_vdf",
    "gsis_get_state", "gsis_correct", "gsis_macro_solve", "gsis_last_sweep_ms",
    "gsis_sweep_layout", "gsis_ns_init", "gsis_n_wall_faces", "gsis_surface", "gsis_set_velocity_points",
    "gsis_set_spatial_order", "gsis_set_internal_dof", "gsis_internal_moments",
    "gsis_set_g13_limit", "gsis_limiter_stats", "gsis_case_bind_static", "gsis_get_internal_temperature",
    "gsis_force_coefficients", "gsis_correct_internal", "gsis_macro_solve_internal",
]


def force_coefficients(totals, rho_inf, u_inf, area):
    """Drag, lift and heat coefficients (Sec. 4.3) from surface totals
    [Fx, Fy, Fz, Q] (gsis_force_coefficients)."""
    t = np.ascontiguousarray(np.asarray(totals, dtype=np.float64)[:4])
    u = np.ascontiguousarray(np.asarray(u_inf, dtype=np.float64)[:3])
    out = np.zeros(3)
    _check(lib().gsis_force_coefficients(C.c_void_p(t.ctypes.data), C.c_double(rho_inf), C.c_void_p(u.ctypes.data),
                                         C.c_double(area), C.c_void_p(out.ctypes.data)))
    return {"C_d": float(out[0]), "C_l": float(out[1]), "C_h": float(out[2])}


class GsisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gsis error %d: %s" % (code, msg))
        self.code = code


class _Patch(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rho", C.c_double), ("u", C.c_double * 3), ("T", C.c_double)]


class _MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_cells", C.c_int32), ("n_faces", C.c_int32), ("n_patches", C.c_int32),
                ("face_cells", C.c_void_p), ("face_normal", C.c_void_p), ("face_area", C.c_void_p),
                ("face_center", C.c_void_p), ("cell_volume", C.c_void_p), ("cell_center", C.c_void_p),
                ("patches", C.c_void_p)]


class _Gas(C.Structure):
    _fields_ = [("Kn", C.c_double), ("omega", C.c_double), ("Pr", C.c_double)]


class SolveParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("Kn_ref", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("region_update_every", C.c_int32), ("n_macro_inner", C.c_int32), ("cfl", C.c_double),
                ("force_wall_layers", C.c_int32), ("ns_init", C.c_int32), ("ns_init_max_chunks", C.c_int32),
                ("source_half", C.c_int32)]

    def __init__(self, mode=MODE_GSIS, Kn_ref=0.01, tol=1e-6, max_iter=1000, region_update_every=1,
                 n_macro_inner=400, cfl=0.5, force_wall_layers=0, ns_init=0, ns_init_max_chunks=1000,
                 source_half=0):
        super().__init__(mode, Kn_ref, tol, max_iter, region_update_every, n_macro_inner, cfl, force_wall_layers,
                         ns_init, ns_init_max_chunks, int(source_half))


class SolveResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("eps", C.c_double * 3), ("n_kinetic", C.c_int64)]


_lib = None


def lib():
    """Load libgsis.so (built in-tree by ``paper_2501_02245_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgsis.so is not built (run python -m paper_2501_02245_amd.build)")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.gsis_last_error.restype = C.c_char_p
        sig = {
            "gsis_create_mesh": [P, P], "gsis_destroy_mesh": [P], "gsis_create_case": [P, P, I32, P],
            "gsis_destroy_case": [P], "gsis_set_velocity_grid": [P, I32, P, P, P],
            "gsis_case_footprint": [P, I64, P], "gsis_case_bind": [P, P, C.c_size_t, I64, P],
            "gsis_set_state": [P, P, P, P, P], "gsis_kinetic_sweep": [P, I32, I32, P],
            "gsis_moments": [P, P, P, P], "gsis_n_kinetic": [P, P], "gsis_update_regions": [P, D, I32, P, P],
            "gsis_step": [P, I32, P, P, P], "gsis_solve_steady": [P, P, P, P], "gsis_get_vdf": [P, P, P],
            "gsis_get_state": [P, P, P, P], "gsis_correct": [P, P, P], "gsis_macro_solve": [P, P, P, P, I32, D, P],
            "gsis_last_sweep_ms": [P, P],
            "gsis_sweep_layout": [P, P, P, P],
            "gsis_ns_init": [P, I32, P, P, P],
            "gsis_n_wall_faces": [P, P], "gsis_surface": [P, P, P, P, P],
            "gsis_set_velocity_points": [P, I32, P, P],
            "gsis_set_spatial_order": [P, I32, D],
            "gsis_set_internal_dof": [P, D, D, P], "gsis_internal_moments": [P, P, P],
            "gsis_get_internal_temperature": [P, P, P],
            "gsis_force_coefficients": [P, D, P, D, P],
            "gsis_set_g13_limit": [P, D], "gsis_limiter_stats": [P, P, P],
            "gsis_case_bind_static": [P, I64, P],
            "gsis_correct_internal": [P, P, P, P],
            "gsis_macro_solve_internal": [P, P, P, P, P, P, P, I32, D, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = I32
        _lib = L
    return _lib


def _check(code, allow=()):
    if code != OK and code not in allow:
        raise GsisError(code, lib().gsis_last_error().decode())
    return code


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(a, dtype):
    """numpy / torch -> contiguous CUDA tensor of `dtype`."""
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


class Mesh:
    """Host-side mesh handle (gsis_create_mesh); see gsis_inputs for the dictionary layout."""

    def __init__(self, m):
        self._arrays = [np.ascontiguousarray(m["face_cells"], dtype=np.int32)]
        for k in ("face_normal", "face_area", "face_center", "cell_volume", "cell_center"):
            self._arrays.append(np.ascontiguousarray(m[k], dtype=np.float64))
        pt = (_Patch * max(1, len(m["patches"])))()
        for i, p in enumerate(m["patches"]):
            pt[i].kind = PATCH_WALL if p["kind"] == "wall" else PATCH_FAR
            pt[i].rho = p["rho"]
            for d in range(3):
                pt[i].u[d] = float(p["u"][d])
            pt[i].T = p["T"]
        self._patches = pt
        a = self._arrays
        desc = _MeshDesc(m["dim"], m["n_cells"], m["n_faces"], len(m["patches"]),
                         *[x.ctypes.data for x in a], C.addressof(pt))
        h = C.c_void_p()
        _check(lib().gsis_create_mesh(C.byref(desc), C.byref(h)))
        self.handle = h
        self.n_cells = m["n_cells"]
        self.n_faces = m["n_faces"]
        self.dict = m

    def close(self):
        if self.handle:
            _check(lib().gsis_destroy_mesh(self.handle))
            self.handle = None


def _set_grid(h, grid):
    """Pass a velocity grid to a case: a tensor grid (dict vdim, nodes, weights)
    or a point set (dict kind="points", points [nv, 3], pweights [nv]).
    Returns the host arrays (kept alive by the caller during the call)."""
    if grid.get("kind") == "points":
        pts = np.ascontiguousarray(grid["points"], dtype=np.float64).reshape(-1, 3)
        pw = np.ascontiguousarray(grid["pweights"], dtype=np.float64)
        _check(lib().gsis_set_velocity_points(h, len(pw), C.c_void_p(pts.ctypes.data), C.c_void_p(pw.ctypes.data)))
        return (pts, pw)
    vdim = grid["vdim"]
    n = (C.c_int32 * 3)(*[len(grid["nodes"][d]) if d < vdim else 1 for d in range(3)])
    xs_ = [np.ascontiguousarray(grid["nodes"][d] if d < vdim else [0.0], dtype=np.float64) for d in range(3)]
    ws_ = [np.ascontiguousarray(grid["weights"][d] if d < vdim else [1.0], dtype=np.float64) for d in range(3)]
    xs = (C.c_void_p * 3)(*[x.ctypes.data for x in xs_])
    ws = (C.c_void_p * 3)(*[x.ctypes.data for x in ws_])
    _check(lib().gsis_set_velocity_grid(h, vdim, n, xs, ws))
    return (xs_, ws_)


def grid_nv(grid):
    """Velocity nodes of a tensor grid or a point set."""
    if grid.get("kind") == "points":
        return int(len(grid["pweights"]))
    return int(np.prod([len(grid["nodes"][d]) for d in range(grid["vdim"])]))


def footprint(mesh: Mesh, grid, Kn, dtype=F32, capacity=None, omega=0.5, Pr=2.0 / 3.0):
    """Device bytes a case of this mesh, grid and kinetic capacity binds (no allocation)."""
    h = C.c_void_p()
    _check(lib().gsis_create_case(mesh.handle, C.byref(_Gas(Kn, omega, Pr)), dtype, C.byref(h)))
    try:
        _keep = _set_grid(h, grid)
        nbytes = C.c_size_t()
        _check(lib().gsis_case_footprint(h, int(capacity or mesh.n_cells), C.byref(nbytes)))
        return nbytes.value
    finally:
        _check(lib().gsis_destroy_case(h))


class Case:
    """One steady problem bound to a torch-allocated device workspace."""

    def __init__(self, mesh: Mesh, grid, Kn, omega=0.5, Pr=2.0 / 3.0, dtype=F32, capacity=None,
                 order=1, damp2=2.0, dr=0.0, Zr=1.0, A=None, g13_rmax=0.5, static=False):
        """order 2: second-order face values with pseudo-time factor damp2
        (gsis_set_spatial_order); dr > 0: the polyatomic gas with Zr and the
        heat-flux matrix A (gsis_set_internal_dof); g13_rmax: range limit of
        the Grad-13 rows (gsis_set_g13_limit; None or <= 0: unlimited);
        static: bind to the library's static device workspace
        (gsis_case_bind_static) instead of a torch allocation."""
        import torch
        self.mesh = mesh
        self.dtype = dtype
        self.vdim = grid["vdim"]
        self.nfun = 1 if self.vdim == 3 else 2
        h = C.c_void_p()
        _check(lib().gsis_create_case(mesh.handle, C.byref(_Gas(Kn, omega, Pr)), dtype, C.byref(h)))
        self.handle = h
        self._grid = _set_grid(h, grid)
        self.order = int(order)
        _check(lib().gsis_set_spatial_order(h, self.order, C.c_double(damp2)))
        self.poly = dr > 0
        if self.poly:
            Av = np.ascontiguousarray(A if A is not None else (Pr, 0.0, 0.0, 1.0), dtype=np.float64)
            _check(lib().gsis_set_internal_dof(h, C.c_double(dr), C.c_double(Zr), C.c_void_p(Av.ctypes.data)))
            self.nfun = 2
        _check(lib().gsis_set_g13_limit(h, C.c_double(0.0 if g13_rmax is None else g13_rmax)))
        self.points = grid.get("kind") == "points"
        self.nv = grid_nv(grid)
        self.capacity = int(capacity or mesh.n_cells)
        nbytes = C.c_size_t()
        _check(lib().gsis_case_footprint(h, self.capacity, C.byref(nbytes)))
        self.footprint = nbytes.value
        if static:
            self.workspace = None
            _check(lib().gsis_case_bind_static(h, self.capacity, _stream()))
        else:
            self.workspace = torch.empty(self.footprint, dtype=torch.uint8, device="cuda")
            _check(lib().gsis_case_bind(h, _ptr(self.workspace), self.footprint, self.capacity, _stream()))

    @property
    def torch_dtype(self):
        import torch
        return torch.float32 if self.dtype == F32 else torch.float64

    def close(self):
        if self.handle:
            _check(lib().gsis_destroy_case(self.handle))
            self.handle = None
            self.workspace = None

    def set_state(self, W, vdf=None, flags=None):
        import torch
        Wd = _dev(W, torch.float64)
        vd = _dev(vdf, self.torch_dtype) if vdf is not None else None
        fd = _dev(flags, torch.uint8) if flags is not None else None
        _check(lib().gsis_set_state(self.handle, _ptr(Wd), _ptr(vd), _ptr(fd), _stream()))

    @property
    def n_kin(self):
        n = C.c_int64()
        _check(lib().gsis_n_kinetic(self.handle, C.byref(n)))
        return n.value

    def sweep(self, n_sweeps=1):
        arr = (C.c_void_p * 1)(self.handle)
        _check(lib().gsis_kinetic_sweep(arr, 1, n_sweeps, _stream()))

    def moments(self):
        import torch
        n = self.n_kin
        out = torch.empty((n, NMOM), dtype=torch.float64, device="cuda")
        kc = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().gsis_moments(self.handle, _ptr(out), _ptr(kc), _stream()))
        return out, kc

    def internal_moments(self):
        """Polyatomic gas: T_r and q_r per kinetic cell [n_kin, 4] (device, FP64)."""
        import torch
        out = torch.empty((self.n_kin, 4), dtype=torch.float64, device="cuda")
        _check(lib().gsis_internal_moments(self.handle, _ptr(out), _stream()))
        return out

    def internal_temperature(self):
        """Polyatomic gas: T_r of every cell [n_cells] (device, FP64)."""
        import torch
        out = torch.empty(self.mesh.n_cells, dtype=torch.float64, device="cuda")
        _check(lib().gsis_get_internal_temperature(self.handle, _ptr(out), _stream()))
        return out

    def limiter_stats(self):
        """Cumulative limiter activity since bind / set_state (gsis_limiter_stats)."""
        v = (C.c_int64 * 6)()
        _check(lib().gsis_limiter_stats(self.handle, v, _stream()))
        keys = ("g13_ghosts", "g13_ghost_limited", "g13_new", "g13_new_limited", "corrections",
                "corrections_limited")
        return dict(zip(keys, [int(x) for x in v]))

    def get_vdf(self):
        import torch
        out = torch.empty((self.n_kin, self.nfun, self.nv), dtype=self.torch_dtype, device="cuda")
        _check(lib().gsis_get_vdf(self.handle, _ptr(out), _stream()))
        return out

    def get_state(self):
        import torch
        W = torch.empty((self.mesh.n_cells, 5), dtype=torch.float64, device="cuda")
        fl = torch.empty(self.mesh.n_cells, dtype=torch.uint8, device="cuda")
        _check(lib().gsis_get_state(self.handle, _ptr(W), _ptr(fl), _stream()))
        return W, fl

    def surface(self, totals=True):
        """Wall-face surface quantities (Sec. 4.2/4.3): (face ids [n_wall] int32,
        rows [n_wall][9] FP64: tau (3), p, shear (3), heat flux, mass flux,
        totals [4] = sum tau S, sum q S or None), device tensors."""
        import torch
        n = C.c_int32()
        _check(lib().gsis_n_wall_faces(self.handle, C.byref(n)))
        faces = torch.empty(max(n.value, 1), dtype=torch.int32, device="cuda")
        out = torch.empty((max(n.value, 1), NSURF), dtype=torch.float64, device="cuda")
        tot = torch.empty(4, dtype=torch.float64, device="cuda") if totals else None
        _check(lib().gsis_surface(self.handle, _ptr(faces), _ptr(out), _ptr(tot) if totals else None, _stream()))
        return faces[: n.value], out[: n.value], tot

    def update_regions(self, Kn_ref, force_wall_layers=0):
        n = C.c_int64()
        _check(lib().gsis_update_regions(self.handle, Kn_ref, force_wall_layers, C.byref(n), _stream()))
        return n.value

    def step(self, params: SolveParams):
        eps = (C.c_double * 3)()
        arr = (C.c_void_p * 1)(self.handle)
        _check(lib().gsis_step(arr, 1, C.byref(params), eps, _stream()))
        return np.array(eps[:])

    def solve(self, params: SolveParams, allow_noconv=False):
        r = SolveResult()
        code = lib().gsis_solve_steady(self.handle, C.byref(params), C.byref(r), _stream())
        _check(code, allow=(E_NOCONV,) if allow_noconv else ())
        return r.iterations, np.array(r.eps[:]), r.n_kinetic

    def correct(self, W_new):
        import torch
        Wd = _dev(W_new, torch.float64)
        _check(lib().gsis_correct(self.handle, _ptr(Wd), _stream()))

    def correct_internal(self, W_new, Tr_new):
        """Two-VDF gas: the correction with the internal temperature (gsis_correct_internal)."""
        import torch
        Wd = _dev(W_new, torch.float64)
        Td = _dev(Tr_new, torch.float64)
        _check(lib().gsis_correct_internal(self.handle, _ptr(Wd), _ptr(Td), _stream()))

    def macro_solve_internal(self, W, Tr, hot, hot_r=None, src=None, src_r=None, n_inner=1, cfl=0.5):
        """Two-VDF gas: the synthetic solve alone (gsis_macro_solve_internal); returns (W, T_r) on the device."""
        import torch
        Wd = _dev(W, torch.float64)
        Td = _dev(Tr, torch.float64)
        args = [_dev(a, torch.float64) if a is not None else None for a in (hot, hot_r, src, src_r)]
        _check(lib().gsis_macro_solve_internal(self.handle, _ptr(Wd), _ptr(Td), *[_ptr(a) if a is not None else None
                                                                                  for a in args],
                                               n_inner, cfl, _stream()))
        return Wd, Td

    def macro_solve(self, W, hot, src=None, n_inner=1, cfl=0.5):
        import torch
        Wd = _dev(W, torch.float64)
        hd = _dev(hot, torch.float64)
        sd = _dev(src, torch.float64) if src is not None else None
        _check(lib().gsis_macro_solve(self.handle, _ptr(Wd), _ptr(hd), _ptr(sd), n_inner, cfl, _stream()))
        return Wd

    def sweep_layout(self):
        """(fast, tile, n_tiles) of the sweep kernel chosen at bind."""
        v = [C.c_int32() for _ in range(3)]
        _check(lib().gsis_sweep_layout(self.handle, *[C.byref(x) for x in v]))
        return tuple(int(x.value) for x in v)

    def last_sweep_ms(self):
        ms = C.c_float()
        _check(lib().gsis_last_sweep_ms(self.handle, C.byref(ms)))
        return ms.value


def kinetic_sweep(cases, n_sweeps=1):
    """One batched launch per sweep over several cases (same dtype and vdim)."""
    arr = (C.c_void_p * len(cases))(*[c.handle for c in cases])
    _check(lib().gsis_kinetic_sweep(arr, len(cases), n_sweeps, _stream()))


def ns_init(cases, params: SolveParams):
    """Steps 1-2 (NS start, first flagging) for several aGSIS cases with batched
    launches; returns the chunks each case ran.  On failure the GsisError
    carries `chunks`: -1 marks the cases whose first flagging failed; the
    others completed their start."""
    arr = (C.c_void_p * len(cases))(*[c.handle for c in cases])
    chunks = (C.c_int32 * len(cases))()
    code = lib().gsis_ns_init(arr, len(cases), C.byref(params), chunks, _stream())
    try:
        _check(code)
    except GsisError as e:
        e.chunks = list(chunks)
        raise
    return list(chunks)


def step(cases, params: SolveParams):
    """One outer iteration for a batch of cases; returns eps [n_cases, 3].

    On failure the GsisError carries `eps`: NaN rows mark the cases that
    failed; the others completed the step."""
    eps = (C.c_double * (3 * len(cases)))()
    arr = (C.c_void_p * len(cases))(*[c.handle for c in cases])
    code = lib().gsis_step(arr, len(cases), C.byref(params), eps, _stream())
    out = np.array(eps[:]).reshape(len(cases), 3)
    if code != OK:
        err = GsisError(code, lib().gsis_last_error().decode())
        if not np.isnan(out).any():   # failed before the per-case endings: every case
            out[:] = np.nan
        err.eps = out
        raise err
    return out
