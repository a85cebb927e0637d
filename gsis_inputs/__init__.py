"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module builds the *inputs* of the method and nothing else: unstructured
meshes (face lists with normals, areas, volumes, centroids), tensor-product
velocity quadratures, macroscopic fields W = (rho, u, T) and random
perturbation factors.  It contains none of the method's arithmetic (no
equilibrium, no moments, no sweep), so both sides of every parity test start
from the same arrays without sharing any step of the computation.

Units are the dimensionless ones used throughout: lengths scaled by L,
velocities by the most-probable speed sqrt(2 R T0), temperature by T0 and
density by rho0.

Mesh dictionary (all numpy, C-contiguous):
    dim          spatial dimension (1, 2 or 3); gradients use the first `dim`
                 components only
    face_cells   int32 [n_faces, 2]  owner, other; other < 0 encodes the
                 boundary patch id p as -1 - p
    face_normal  float64 [n_faces, 3] unit normal pointing owner -> other
    face_area    float64 [n_faces]
    face_center  float64 [n_faces, 3]
    cell_volume  float64 [n_cells]
    cell_center  float64 [n_cells, 3]
    patches      list of dicts {kind: 'wall'|'far', rho, u (3,), T}
"""
from __future__ import annotations

import math

import numpy as np

WALL = 0
FAR = 1


# ---------------------------------------------------------------------------
# velocity quadratures
# ---------------------------------------------------------------------------
def uniform_axis(n: int, half_width: float):
    """n equispaced nodes on [-V, V] with trapezoid weights."""
    x = np.linspace(-half_width, half_width, n)
    h = x[1] - x[0]
    w = np.full(n, h)
    w[0] = w[-1] = 0.5 * h
    return x, w


def stretched_axis(n: int, half_width: float, alpha: float = 0.4):
    """Nonuniform nodes clustered near zero velocity.

    xi(eta) = V (alpha eta + (1 - alpha) eta^3) with eta equispaced on [-1, 1];
    weights are the trapezoid rule in eta times d xi / d eta.  With n even no
    node sits at xi = 0.
    """
    eta = np.linspace(-1.0, 1.0, n)
    h = eta[1] - eta[0]
    x = half_width * (alpha * eta + (1.0 - alpha) * eta ** 3)
    jac = half_width * (alpha + 3.0 * (1.0 - alpha) * eta ** 2)
    w = np.full(n, h) * jac
    w[0] *= 0.5
    w[-1] *= 0.5
    return x, w


def velocity_grid(vdim: int, n, half_width, kind: str = "uniform", alpha: float = 0.4):
    """Tensor-product grid: dict(vdim, nodes=[x_d], weights=[w_d]).

    vdim == 3: full velocity space, axes (x, y, z), z fastest in memory.
    vdim == 2: reduced distributions over (xi_x, xi_y), y fastest.
    `n` and `half_width` may be scalars or per-axis sequences.
    """
    ns = [n] * vdim if np.isscalar(n) else list(n)
    hw = [half_width] * vdim if np.isscalar(half_width) else list(half_width)
    nodes, weights = [], []
    for d in range(vdim):
        if kind == "uniform":
            x, w = uniform_axis(int(ns[d]), float(hw[d]))
        elif kind == "stretched":
            x, w = stretched_axis(int(ns[d]), float(hw[d]), alpha)
        else:
            raise ValueError(kind)
        nodes.append(np.ascontiguousarray(x, dtype=np.float64))
        weights.append(np.ascontiguousarray(w, dtype=np.float64))
    return {"vdim": vdim, "nodes": nodes, "weights": weights, "kind": kind}


def ball_grid(n, half_width, kind: str = "uniform", radius=None, alpha: float = 0.4):
    """Non-tensor 3D velocity set: the nodes of the tensor grid
    velocity_grid(3, n, half_width, kind) that lie in the ball |xi| <= radius
    (default: the half-width), each keeping its tensor weight.  Returned as a
    point set: dict(vdim=3, kind="points", points [nv, 3], pweights [nv]), in
    the tensor grid's row-major order."""
    g = velocity_grid(3, n, half_width, kind, alpha)
    X = np.meshgrid(*g["nodes"], indexing="ij")
    Wt = np.meshgrid(*g["weights"], indexing="ij")
    pts = np.stack([x.ravel() for x in X], 1)
    w = (Wt[0] * Wt[1] * Wt[2]).ravel()
    r = float(np.max(half_width) if radius is None else radius)
    keep = np.sum(pts * pts, axis=1) <= r * r * (1.0 + 1e-12)
    return {"vdim": 3, "kind": "points", "points": np.ascontiguousarray(pts[keep]),
            "pweights": np.ascontiguousarray(w[keep])}


def grid_size(grid) -> int:
    if grid.get("kind") == "points":
        return int(len(grid["pweights"]))
    return int(np.prod([len(x) for x in grid["nodes"]]))


# ---------------------------------------------------------------------------
# mesh helpers
# ---------------------------------------------------------------------------
def _patch(kind, rho=1.0, u=(0.0, 0.0, 0.0), T=1.0):
    return {"kind": kind, "rho": float(rho), "u": np.asarray(u, dtype=np.float64), "T": float(T)}


def _finish(dim, face_cells, normal, area, fcenter, volume, ccenter, patches):
    m = {
        "dim": int(dim),
        "face_cells": np.ascontiguousarray(face_cells, dtype=np.int32),
        "face_normal": np.ascontiguousarray(normal, dtype=np.float64),
        "face_area": np.ascontiguousarray(area, dtype=np.float64),
        "face_center": np.ascontiguousarray(fcenter, dtype=np.float64),
        "cell_volume": np.ascontiguousarray(volume, dtype=np.float64),
        "cell_center": np.ascontiguousarray(ccenter, dtype=np.float64),
        "patches": patches,
    }
    m["n_cells"] = len(m["cell_volume"])
    m["n_faces"] = len(m["face_area"])
    return m


def renumber_cells(mesh, order):
    """Return a copy of `mesh` whose cell k is old cell order[k]."""
    order = np.asarray(order, dtype=np.int64)
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    fc = mesh["face_cells"].astype(np.int64).copy()
    fc[:, 0] = inv[fc[:, 0]]
    inner = fc[:, 1] >= 0
    fc[inner, 1] = inv[fc[inner, 1]]
    # keep faces sorted by owner for locality
    key = fc[:, 0] * (len(order) + 1) + np.where(inner, fc[:, 1], len(order))
    fo = np.argsort(key, kind="stable")
    return _finish(mesh["dim"], fc[fo], mesh["face_normal"][fo], mesh["face_area"][fo],
                   mesh["face_center"][fo], mesh["cell_volume"][order],
                   mesh["cell_center"][order], mesh["patches"])


def morton_order(mesh, bits: int = 20):
    """Order of the cells along a Z-order (Morton) curve of their centroids.

    Consecutive cells are spatially clustered at every scale, so face
    neighbours mostly sit a short distance apart in the numbering: streaming
    kernels that visit cells in order then find neighbour data in cache."""
    x = mesh["cell_center"][:, : max(mesh["dim"], 1)]
    lo, hi = x.min(axis=0), x.max(axis=0)
    q = ((x - lo) / np.maximum(hi - lo, 1e-300) * ((1 << bits) - 1)).astype(np.uint64)
    code = np.zeros(len(x), dtype=np.uint64)
    nd = x.shape[1]
    for b in range(bits):
        for d in range(nd):
            code |= ((q[:, d] >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * nd + d)
    return np.argsort(code, kind="stable")


def rcm_order(mesh):
    """Reverse Cuthill-McKee order of the cell adjacency graph (locality)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    fc = mesh["face_cells"]
    inner = fc[:, 1] >= 0
    a, b = fc[inner, 0], fc[inner, 1]
    n = mesh["n_cells"]
    g = sp.coo_matrix((np.ones(2 * len(a)), (np.r_[a, b], np.r_[b, a])), shape=(n, n)).tocsr()
    return np.asarray(reverse_cuthill_mckee(g, symmetric_mode=True), dtype=np.int64)


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------
def slab_1d(n_cells: int, left, right, x0: float = 0.0, x1: float = 1.0):
    """Uniform 1D slab [x0, x1] in x, unit cross-section; `left`/`right` are patches."""
    xf = np.linspace(x0, x1, n_cells + 1)
    h = np.diff(xf)
    xc = 0.5 * (xf[1:] + xf[:-1])
    fc, nrm, fcen = [], [], []
    # left boundary face: owner cell 0, normal -x (points out of the gas)
    fc.append((0, -1)); nrm.append((-1.0, 0.0, 0.0)); fcen.append((xf[0], 0.0, 0.0))
    for i in range(n_cells - 1):
        fc.append((i, i + 1)); nrm.append((1.0, 0.0, 0.0)); fcen.append((xf[i + 1], 0.0, 0.0))
    fc.append((n_cells - 1, -2)); nrm.append((1.0, 0.0, 0.0)); fcen.append((xf[-1], 0.0, 0.0))
    cc = np.zeros((n_cells, 3)); cc[:, 0] = xc
    return _finish(1, fc, nrm, np.ones(len(fc)), fcen, h, cc, [left, right])


def couette_1d(n_cells: int = 64, wall_speed: float = 0.1, T_wall: float = 1.0):
    """Planar Couette: x = 0 wall moves -U y, x = 1 wall moves +U y, both diffuse at T_wall."""
    return slab_1d(n_cells, _patch("wall", u=(0.0, -wall_speed, 0.0), T=T_wall),
                   _patch("wall", u=(0.0, wall_speed, 0.0), T=T_wall))


def fourier_1d(n_cells: int = 64, T_left: float = 1.0, T_right: float = 1.1):
    """Planar Fourier: stationary diffuse walls at T_left and T_right."""
    return slab_1d(n_cells, _patch("wall", T=T_left), _patch("wall", T=T_right))


def hex_box_3d(nx: int = 5, ny: int = 5, nz: int = 5, wall_speed: float = 0.2, T_wall: float = 1.0,
               free=(1.0, (0.5, 0.0, 0.0), 1.0)):
    """Structured box [0,1]^3 of nx ny nz hexahedra as a face list (six faces per
    interior cell).  The x = 0 and x = 1 faces are diffuse walls at T_wall moving
    -wall_speed and +wall_speed in y (patches 0 and 1); the y and z faces are
    far field at free = (rho, u, T) (patch 2).  Interior face normals point from
    the lower to the higher cell index along their axis; boundary normals point
    out of the gas."""
    n = (nx, ny, nz)
    h = (1.0 / nx, 1.0 / ny, 1.0 / nz)

    def cid(i, j, k):
        return (i * ny + j) * nz + k

    fc, nrm, area, fcen = [], [], [], []
    for ax in range(3):
        a1, a2 = [d for d in range(3) if d != ax]
        for idx in np.ndindex(*n):
            i = idx[ax]
            cen = [(idx[d] + 0.5) * h[d] for d in range(3)]
            e = [0.0, 0.0, 0.0]
            e[ax] = 1.0
            fa = h[a1] * h[a2]
            c = cid(*idx)
            if i == 0:   # lower boundary face of the box on this axis
                p = 0 if ax == 0 else 2
                fcx = list(cen); fcx[ax] = 0.0
                fc.append((c, -1 - p)); nrm.append(tuple(-x for x in e)); area.append(fa); fcen.append(tuple(fcx))
            if i < n[ax] - 1:
                nb = list(idx); nb[ax] += 1
                fcx = list(cen); fcx[ax] = (i + 1) * h[ax]
                fc.append((c, cid(*nb))); nrm.append(tuple(e)); area.append(fa); fcen.append(tuple(fcx))
            else:        # upper boundary face
                p = 1 if ax == 0 else 2
                fcx = list(cen); fcx[ax] = 1.0
                fc.append((c, -1 - p)); nrm.append(tuple(e)); area.append(fa); fcen.append(tuple(fcx))
    ncell = nx * ny * nz
    cc = np.array([[(i + 0.5) * h[0], (j + 0.5) * h[1], (k + 0.5) * h[2]]
                   for i in range(nx) for j in range(ny) for k in range(nz)])
    vol = np.full(ncell, h[0] * h[1] * h[2])
    rho, u, T = free
    patches = [_patch("wall", u=(0.0, -wall_speed, 0.0), T=T_wall), _patch("wall", u=(0.0, wall_speed, 0.0), T=T_wall),
               _patch("far", rho=rho, u=u, T=T)]
    return _finish(3, fc, nrm, np.asarray(area), fcen, vol, cc, patches)


def quad_cavity_2d(nx: int = 64, ny: int = 64, lid_speed: float = 0.1, T_wall: float = 1.0):
    """Lid-driven cavity on [0,1]^2 as an unstructured quad face list.

    Cell id = j * nx + i (row-major).  Patches: 0 stationary walls
    (left, right, bottom), 1 lid at y = 1 moving +lid_speed x.
    """
    hx, hy = 1.0 / nx, 1.0 / ny
    cid = lambda i, j: j * nx + i
    fc, nrm, area, fcen = [], [], [], []
    for j in range(ny):
        for i in range(nx):
            c = cid(i, j)
            # east face
            if i + 1 < nx:
                fc.append((c, cid(i + 1, j)))
            else:
                fc.append((c, -1))
            nrm.append((1.0, 0.0, 0.0)); area.append(hy); fcen.append(((i + 1) * hx, (j + 0.5) * hy, 0.0))
            # north face
            if j + 1 < ny:
                fc.append((c, cid(i, j + 1)))
            else:
                fc.append((c, -2))
            nrm.append((0.0, 1.0, 0.0)); area.append(hx); fcen.append(((i + 0.5) * hx, (j + 1) * hy, 0.0))
            if i == 0:
                fc.append((c, -1)); nrm.append((-1.0, 0.0, 0.0)); area.append(hy)
                fcen.append((0.0, (j + 0.5) * hy, 0.0))
            if j == 0:
                fc.append((c, -1)); nrm.append((0.0, -1.0, 0.0)); area.append(hx)
                fcen.append(((i + 0.5) * hx, 0.0, 0.0))
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
    cc = np.zeros((nx * ny, 3))
    cc[:, 0] = ((ii + 0.5) * hx).ravel()
    cc[:, 1] = ((jj + 0.5) * hy).ravel()
    vol = np.full(nx * ny, hx * hy)
    patches = [_patch("wall", T=T_wall), _patch("wall", u=(lid_speed, 0.0, 0.0), T=T_wall)]
    fc = np.asarray(fc)
    # sort faces by owner for locality
    o = np.argsort(fc[:, 0], kind="stable")
    return _finish(2, fc[o], np.asarray(nrm)[o], np.asarray(area)[o], np.asarray(fcen)[o], vol, cc, patches)


def _simplex_faces(simplices, pts, dim):
    """Face list of a simplicial mesh: returns (face_cells, normal, area, center)."""
    nc, nv = simplices.shape
    # local faces: each omits one vertex
    loc = [tuple(v for v in range(nv) if v != k) for k in range(nv)]
    faces = np.concatenate([simplices[:, l] for l in loc], axis=0)        # [nv*nc, nv-1]
    owner = np.tile(np.arange(nc), nv)
    opp = np.concatenate([simplices[:, k] for k in range(nv)])            # vertex not on the face
    key = np.sort(faces, axis=1)
    order = np.lexsort(key.T[::-1])
    key, faces, owner, opp = key[order], faces[order], owner[order], opp[order]
    same = np.all(key[1:] == key[:-1], axis=1)
    first = np.ones(len(key), dtype=bool)
    first[1:] = ~same
    idx = np.nonzero(first)[0]
    other = np.full(len(idx), -1, dtype=np.int64)
    pair = np.zeros(len(key), dtype=bool)
    pair[:-1] = same
    # for paired faces (idx[k], idx[k]+1)
    sel = pair[idx]
    other[sel] = owner[idx[sel] + 1]
    F = faces[idx]
    own = owner[idx]
    op = pts[opp[idx]]
    P = pts[F]                                                         # [nf, nv-1, 3]
    center = P.mean(axis=1)
    if dim == 2:
        t = P[:, 1] - P[:, 0]
        n = np.stack([t[:, 1], -t[:, 0], np.zeros(len(t))], axis=1)
        area = np.linalg.norm(n[:, :2], axis=1)
    else:
        n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        area = 0.5 * np.linalg.norm(n, axis=1)
    n = n / np.linalg.norm(n, axis=1)[:, None]
    # orient owner -> outside: normal points away from the owner's opposite vertex
    s = np.einsum("ij,ij->i", n, center - op)
    n[s < 0] *= -1.0
    return own, other, n, area, center


def cylinder_tri_2d(n_theta: int = 160, n_rings: int = 62, first_layer: float = 0.005,
                    r_in: float = 0.5, r_out: float = 5.0, seed: int = 12345,
                    wall_T: float = 1.0, free=(1.0, (4.564, 0.0, 0.0), 1.0)):
    """Seeded Delaunay triangulation around a unit-diameter cylinder.

    Rings graded geometrically from the wall (first spacing `first_layer`) to
    r_out, jittered in angle and radius from `seed`; triangles inside the
    cylinder are removed.  Patch 0 = diffuse wall (stationary, wall_T),
    patch 1 = far field (free-stream rho, u, T).
    """
    from scipy.spatial import Delaunay

    rng = np.random.Generator(np.random.PCG64(seed))
    # geometric ring spacing
    lo, hi = 1.0, 2.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        tot = first_layer * (q ** n_rings - 1.0) / (q - 1.0)
        if tot > r_out - r_in:
            hi = q
        else:
            lo = q
    q = 0.5 * (lo + hi)
    radii = r_in + first_layer * (q ** np.arange(n_rings + 1) - 1.0) / (q - 1.0)
    radii[-1] = r_out
    pts = []
    for k, r in enumerate(radii):
        th = 2 * np.pi * (np.arange(n_theta) + 0.5 * (k % 2)) / n_theta
        if 0 < k < n_rings:
            dr = min(radii[k + 1] - r, r - radii[k - 1])
            th = th + rng.uniform(-0.2, 0.2, n_theta) * 2 * np.pi / n_theta
            r = r + rng.uniform(-0.1, 0.1, n_theta) * dr
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], axis=1))
    pts = np.concatenate(pts)
    tri = Delaunay(pts)
    S = tri.simplices
    cen = pts[S].mean(axis=1)
    keep = np.hypot(cen[:, 0], cen[:, 1]) > r_in
    S = S[keep]
    P3 = np.zeros((len(pts), 3)); P3[:, :2] = pts
    own, other, n, area, fcen = _simplex_faces(S, P3, 2)
    bnd = other < 0
    rf = np.hypot(fcen[:, 0], fcen[:, 1])
    other[bnd & (rf < 0.5 * (r_in + r_out))] = -1       # wall
    other[bnd & (rf >= 0.5 * (r_in + r_out))] = -2      # far field
    a, b, c = P3[S[:, 0]], P3[S[:, 1]], P3[S[:, 2]]
    vol = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    cc = (a + b + c) / 3.0
    rho_f, u_f, T_f = free
    patches = [_patch("wall", T=wall_T), _patch("far", rho=rho_f, u=u_f, T=T_f)]
    m = _finish(2, np.stack([own, other], 1), n, area, fcen, vol, cc, patches)
    return renumber_cells(m, morton_order(m))


def sphere_tet_3d(h_wall: float = 0.05, growth: float = 0.27, h_max: float = 1.0,
                  r_in: float = 0.5, r_out: float = 5.0, seed: int = 2024,
                  wall_T: float = 1.0, free=(1.0, (4.564, 0.0, 0.0), 1.0)):
    """Seeded tetrahedral mesh around a unit-diameter sphere.

    Points are the perturbed leaf centres of an octree over [-r_out, r_out]^3
    refined toward the sphere (target size h_wall + growth * distance, capped
    at h_max), plus Fibonacci points on the sphere and on the outer shell.
    Delaunay tetrahedralisation; tetrahedra inside the sphere are removed.
    Patch 0 = diffuse wall, patch 1 = far field.
    """
    from scipy.spatial import Delaunay

    rng = np.random.Generator(np.random.PCG64(seed))
    leaves = []
    stack = [(np.zeros(3), 2.0 * r_out)]
    while stack:
        c, s = stack.pop()
        d = abs(np.linalg.norm(c) - r_in)
        # distance to the sphere surface from anywhere in the cube is >= d - s*sqrt(3)/2
        dmin = max(d - 0.5 * math.sqrt(3.0) * s, 0.0)
        if s > min(h_wall + growth * dmin, h_max):
            for dx in (-0.25, 0.25):
                for dy in (-0.25, 0.25):
                    for dz in (-0.25, 0.25):
                        stack.append((c + s * np.array([dx, dy, dz]), 0.5 * s))
        else:
            leaves.append((c, s))
    C = np.array([c for c, _ in leaves])
    Sz = np.array([s for _, s in leaves])
    C = C + rng.uniform(-0.1, 0.1, C.shape) * Sz[:, None]
    r = np.linalg.norm(C, axis=1)
    keep = (r > r_in + 0.5 * Sz) & (r < r_out - 0.5 * Sz)
    C = C[keep]

    def fib(n, rad):
        i = np.arange(n) + 0.5
        phi = np.arccos(1 - 2 * i / n)
        th = np.pi * (1 + 5 ** 0.5) * i
        return rad * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)

    n_in = int(4 * np.pi * r_in ** 2 / (h_wall ** 2) * 1.15)
    n_out = int(4 * np.pi * r_out ** 2 / (h_max ** 2) * 1.15)
    pts = np.concatenate([fib(n_in, r_in), C, fib(n_out, r_out)])
    tri = Delaunay(pts)
    S = tri.simplices
    P = pts[S]
    cen = P.mean(axis=1)
    keep = np.linalg.norm(cen, axis=1) > r_in
    S = S[keep]
    P = pts[S]
    vol = np.abs(np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6.0
    own, other, n, area, fcen = _simplex_faces(S, pts, 3)
    bnd = other < 0
    rf = np.linalg.norm(fcen, axis=1)
    other[bnd & (rf < 0.5 * (r_in + r_out))] = -1
    other[bnd & (rf >= 0.5 * (r_in + r_out))] = -2
    rho_f, u_f, T_f = free
    patches = [_patch("wall", T=wall_T), _patch("far", rho=rho_f, u=u_f, T=T_f)]
    m = _finish(3, np.stack([own, other], 1), n, area, fcen, vol, cen[keep], patches)
    return renumber_cells(m, morton_order(m))


# ---------------------------------------------------------------------------
# fields and regions
# ---------------------------------------------------------------------------
def rng_of(seed: int):
    return np.random.Generator(np.random.PCG64(seed))


def couette_initial_W(n_cells: int = 64, seed: int = 0, amp: float = 1e-3):
    """Global Maxwellian state with density 1 + amp * N(0,1) per cell, u = 0, T = 1.

    Returns W [n_cells, 5] = (rho, ux, uy, uz, T).
    """
    W = np.zeros((n_cells, 5))
    W[:, 0] = 1.0 + amp * rng_of(seed).standard_normal(n_cells)
    W[:, 4] = 1.0
    return W


def uniform_W(n_cells: int, rho=1.0, u=(0.0, 0.0, 0.0), T=1.0):
    W = np.zeros((n_cells, 5))
    W[:, 0] = rho
    W[:, 1:4] = u
    W[:, 4] = T
    return W


def random_W(n_cells: int, seed: int, u_scale: float = 0.3, dT: float = 0.2, drho: float = 0.2):
    """Smoothly random positive states for parity tests."""
    g = rng_of(seed)
    W = np.zeros((n_cells, 5))
    W[:, 0] = 1.0 + drho * g.uniform(-1, 1, n_cells)
    W[:, 1:4] = u_scale * g.uniform(-1, 1, (n_cells, 3))
    W[:, 4] = 1.0 + dT * g.uniform(-1, 1, n_cells)
    return W


def perturbation(shape, seed: int, amp: float = 0.1):
    """Multiplicative factors 1 + amp * U(-1, 1) (used to make non-equilibrium VDFs)."""
    return 1.0 + amp * rng_of(seed).uniform(-1.0, 1.0, shape)


def hypersonic_field(mesh, mach: float = 5.0, gamma: float = 5.0 / 3.0, seed: int = 7):
    """Macroscopic field shaped like a blunt-body flow, for throughput runs.

    Free stream (rho 1, u = Ma sqrt(gamma/2) x, T 1) outside a bow-shock
    shell; a hot, dense, slow post-shock layer inside it.  Returns W [n, 5].
    """
    u_inf = mach * math.sqrt(gamma / 2.0)
    T_stag = 1.0 + 0.5 * (gamma - 1.0) * mach ** 2
    x = mesh["cell_center"]
    r = np.linalg.norm(x, axis=1)
    shock = 0.5 + 0.35 + 0.25 * np.clip(x[:, 0], 0, None) ** 1.2
    s = 1.0 / (1.0 + np.exp((r - shock) / 0.05))                   # 1 inside the shell
    wake = np.clip(x[:, 0] / 5.0, 0, 1)
    W = np.zeros((mesh["n_cells"], 5))
    W[:, 0] = 1.0 + 3.0 * s * (1 - 0.7 * wake)
    W[:, 1] = u_inf * (1 - s * (1 - 0.6 * wake))
    W[:, 2] = 0.05 * u_inf * s * np.sign(x[:, 1]) * np.abs(x[:, 1]) / np.maximum(r, 1e-3)
    W[:, 4] = 1.0 + (T_stag - 1.0) * s * (1 - 0.5 * wake)
    g = rng_of(seed)
    W[:, 0] *= 1.0 + 0.01 * g.uniform(-1, 1, len(W))
    return W


def synthetic_region(mesh, fraction: float, seed: int = 11):
    """Seeded kinetic flags covering ~`fraction` of the cells.

    Union of a wall band (cells nearest the body), a shock shell and a wake
    cone, grown until the requested fraction is reached.  Returns uint8 flags.
    """
    x = mesh["cell_center"]
    r = np.linalg.norm(x, axis=1)
    g = rng_of(seed)
    score = np.minimum.reduce([
        (r - 0.5) / 0.5,                                   # wall band
        np.abs(r - (0.9 + 0.3 * np.clip(x[:, 0], 0, None))) / 0.4,   # shock shell
        np.where(x[:, 0] > 0, np.hypot(x[:, 1], x[:, 2] if x.shape[1] > 2 else 0) / (0.5 + 0.2 * x[:, 0]), 9.0),
    ]) + 0.05 * g.uniform(0, 1, len(r))
    k = int(round(fraction * mesh["n_cells"]))
    flags = np.zeros(mesh["n_cells"], dtype=np.uint8)
    flags[np.argsort(score, kind="stable")[:k]] = 1
    return flags


def node_velocities(grid):
    """Velocity nodes [nv, 3] and weights [nv]: a tensor grid row-major (last
    axis fastest), or a point set as given."""
    if grid.get("kind") == "points":
        return np.asarray(grid["points"], dtype=np.float64), np.asarray(grid["pweights"], dtype=np.float64)
    xs = list(grid["nodes"]) + [np.zeros(1)] * (3 - grid["vdim"])
    ws = list(grid["weights"]) + [np.ones(1)] * (3 - grid["vdim"])
    X = np.meshgrid(*xs, indexing="ij")
    Wt = np.meshgrid(*ws, indexing="ij")
    return np.stack([x.ravel() for x in X], 1), (Wt[0] * Wt[1] * Wt[2]).ravel()


def gaussian_rows(grid, W, seed: int, amp: float = 0.05, dtype=np.float32):
    """Random positive VDF rows shaped like local Gaussians: [n, nfun, nv].

    Row i is rho (pi T)^(-3/2) exp(-|xi - u|^2 / T) (for vdim 2: the reduced
    pair with the second function scaled by T/2) times independent factors
    1 + amp * U(-1, 1).  A test input only: its moments are not W exactly.
    """
    xi, _ = node_velocities(grid)
    W = np.atleast_2d(W)
    g = rng_of(seed)
    nfun = 1 if grid["vdim"] == 3 else 2
    out = np.empty((len(W), nfun, len(xi)), dtype=dtype)
    for i, w in enumerate(W):
        d = xi - w[1:4][None, :]
        if grid["vdim"] == 2:
            d[:, 2] = 0.0
        c2 = np.sum(d * d, axis=1)
        if grid["vdim"] == 3:
            base = w[0] * (np.pi * w[4]) ** -1.5 * np.exp(-c2 / w[4])
            out[i, 0] = base * (1.0 + amp * g.uniform(-1, 1, len(xi)))
        else:
            base = w[0] / (np.pi * w[4]) * np.exp(-c2 / w[4])
            out[i, 0] = base * (1.0 + amp * g.uniform(-1, 1, len(xi)))
            out[i, 1] = 0.5 * w[4] * base * (1.0 + amp * g.uniform(-1, 1, len(xi)))
    return out


def separable_row_factors(grid, W, cells, seed: int, amp: float = 0.05):
    """Per-axis factors (3D grids) of random Gaussian-shaped rows, one set per
    listed cell, drawn from a stream keyed by (seed, cell id) so that any
    subset of cells can be regenerated alone.

    Row of cell c = a_x[c] (x) a_y[c] (x) a_z[c] (outer product, x slowest),
    a_d[j] = s exp(-(xi_{d,j} - u_d)^2 / T) (1 + amp U(-1, 1)),
    s = (rho (pi T)^(-3/2))^(1/3); returned in FP32: ([n, nx], [n, ny], [n, nz]).
    """
    assert grid["vdim"] == 3
    out = [np.empty((len(cells), len(grid["nodes"][d])), dtype=np.float32) for d in range(3)]
    for i, c in enumerate(np.asarray(cells, dtype=np.int64)):
        w = W[c]
        g = np.random.Generator(np.random.PCG64([seed, int(c)]))
        s = (w[0] * (np.pi * w[4]) ** -1.5) ** (1.0 / 3.0)
        for d in range(3):
            x = grid["nodes"][d]
            f = s * np.exp(-(x - w[1 + d]) ** 2 / w[4]) * (1.0 + amp * g.uniform(-1, 1, len(x)))
            out[d][i] = f.astype(np.float32)
    return out


def assemble_separable_rows(ax, ay, az):
    """Rows [n, 1, nx ny nz] = (a_x a_y) a_z in FP32, in that association order."""
    r = (ax[:, :, None, None] * ay[:, None, :, None]) * az[:, None, None, :]
    return r.reshape(len(ax), 1, -1)


def sphere_workload(nv1d: int = 32, mach: float = 5.0):
    """Mach-5 sphere at the benchmark size: mesh (~192k tetrahedra, Morton
    order), stretched nv1d^3 velocity grid on [-15, 15]^3 and the synthetic
    starting field."""
    u_inf = mach * np.sqrt(5.0 / 6.0)
    mesh = sphere_tet_3d(free=(1.0, (u_inf, 0.0, 0.0), 1.0))
    grid = velocity_grid(3, nv1d, 15.0, "stretched")
    return mesh, grid, hypersonic_field(mesh, mach=mach)


def resolving_size(nv: int, sizes, V: float, u: float, max_spacing: float = 0.7, alpha: float = 0.4) -> int:
    """Smallest axis size >= nv that resolves a unit-temperature Maxwellian
    centred at u on the stretched axis of half-width V: node spacing at u at
    most max_spacing (the Maxwellian exp(-c^2) has standard deviation 0.71).
    Sizes beyond the listed ones double the largest; coarser axes leave the
    conservation-fixed Maxwellian of the free stream negative in its tails."""
    eta = abs(u) / V
    for _ in range(60):      # invert xi(eta) = V (alpha eta + (1 - alpha) eta^3) by Newton
        f = alpha * eta + (1.0 - alpha) * eta ** 3 - abs(u) / V
        eta -= f / (alpha + 3.0 * (1.0 - alpha) * eta * eta)
    slope = V * (alpha + 3.0 * (1.0 - alpha) * eta * eta)
    cands = sorted(x for x in sizes if x >= nv)
    while True:
        for n in cands:
            if slope * 2.0 / (n - 1) <= max_spacing:
                return int(n)
        cands = [2 * cands[-1]]


def serving_requests(n: int, rate: float, seed: int = 7, kinds=("couette", "fourier", "cylinder"),
                     cells_1d=(32, 512), nv_1d=(16, 32), cells_2d=(2000, 20000), nv_2d=(32, 64),
                     Kn_range=(1e-3, 1.0), mach_range=(1.0, 8.0)):
    """Seeded steady-solve requests with Poisson arrivals (`rate` per second).

    Each request is a dict: arrival time, kind, mesh, velocity grid, Kn, Mach,
    starting field, forced wall layers and kinetic capacity (fraction of cells).
      couette : walls moving -+Ma a0/2 (a0 = sqrt(5/6)) at T = 1, uniform start;
      fourier : stationary walls at T = 1 and 1 + 0.1 Ma, linear-T start;
      cylinder: Mach-Ma flow past a unit cylinder, synthetic start, 2 wall layers.
    The 1D boxes are solved fully kinetic (GSIS, global pseudo-time step); the
    cylinder adaptively (aGSIS from the NS start).
    Cells log-uniform in the given ranges; Kn log-uniform; Mach uniform; the
    velocity range is max(5 or 15, u + 4 sqrt(T_stag)), T_stag = 1 + Ma^2/3;
    the drawn axis size grows (resolving_size) until the unit-temperature
    Maxwellian of the free stream or the moving walls is resolved.
    """
    g = rng_of(seed)
    t = 0.0
    out = []
    a0 = math.sqrt(5.0 / 6.0)
    for i in range(n):
        t += g.exponential(1.0 / rate)
        kind = kinds[int(g.integers(len(kinds)))]
        Kn = float(10 ** g.uniform(math.log10(Kn_range[0]), math.log10(Kn_range[1])))
        Ma = float(g.uniform(*mach_range))
        T_stag = 1.0 + Ma * Ma / 3.0
        if kind in ("couette", "fourier"):
            nc = int(round(math.exp(g.uniform(math.log(cells_1d[0]), math.log(cells_1d[1])))))
            nv = int(nv_1d[int(g.integers(len(nv_1d)))])
            if kind == "couette":
                U = 0.5 * Ma * a0
                mesh = couette_1d(nc, U)
                V = max(5.0, U + 4.0 * math.sqrt(T_stag))
                W0 = uniform_W(nc)
            else:
                TR = 1.0 + 0.1 * Ma
                mesh = fourier_1d(nc, 1.0, TR)
                V = max(5.0, 4.0 * math.sqrt(TR) + 1.0)
                W0 = uniform_W(nc)
                W0[:, 4] = 1.0 + (TR - 1.0) * mesh["cell_center"][:, 0]
            nv = resolving_size(nv, nv_1d, V, U if kind == "couette" else 0.0)
            grid = velocity_grid(3, nv, V, "stretched")
            # closed box, every cell kinetic: GSIS with one global (conservative) step
            layers, cap, mode, cfl = 0, 1.0, "gsis", -0.5
        else:
            nc = math.exp(g.uniform(math.log(cells_2d[0]), math.log(cells_2d[1])))
            nt = max(24, int(round(math.sqrt(nc / 0.8))))
            nr = max(8, int(round(0.4 * nt)))
            u = Ma * a0
            mesh = cylinder_tri_2d(n_theta=nt, n_rings=nr, free=(1.0, (u, 0.0, 0.0), 1.0),
                                   seed=int(g.integers(1 << 30)))
            nv = int(nv_2d[int(g.integers(len(nv_2d)))])
            V = max(15.0, u + 4.0 * math.sqrt(T_stag))
            nv = resolving_size(nv, nv_2d, V, u)
            grid = velocity_grid(2, nv, V, "stretched")
            W0 = hypersonic_field(mesh, mach=Ma)
            W0[:, 3] = 0.0
            # open domain: aGSIS from the NS start, local steps
            layers, cap, mode, cfl = 2, 0.4, "agsis", 0.5
        out.append({"rid": i, "arrival": t, "kind": kind, "mesh": mesh, "grid": grid, "Kn": Kn, "mach": Ma,
                    "W0": W0, "layers": layers, "capacity": cap, "mode": mode, "cfl": cfl})
    return out
