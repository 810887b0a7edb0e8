"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only builds *inputs*: polygonal meshes of the unit square or of a
basin section (vertex coordinates, CCW vertex lists, a fluid/solid flag per cell)
and piecewise-constant material fields.  It holds none of the discretisation's
arithmetic (no bases, no quadrature, no operators), so that both the FP64
oracle and the HIP path can consume the very same meshes.

Mesh conventions (paper Sec. 3.1): cells are polygons with planar faces aligned
with the fluid/solid partition; hanging nodes are kept as ordinary polygon
vertices, so a square next to two refined squares becomes a pentagon and a
triangle next to one becomes a quadrilateral.

Returned meshes are dicts with
    xy        float64 [n_vertices, 2]
    cell_ptr  int32   [n_cells + 1]   CSR offsets into cell_vtx
    cell_vtx  int32   [cell_ptr[-1]]  counter-clockwise vertex ids
    medium    uint8   [n_cells]       0 = fluid (acoustic), 1 = solid (elastic)
and, after ``with_materials``, rho, a, b (float64 [n_cells]): fluid a = c
(sound speed), b unused (0); solid a = lambda, b = mu.
"""
from __future__ import annotations

import numpy as np

FLUID = 0
SOLID = 1


def _lattice_mesh(nx, ny, x0, x1, y0, y1, refine, p_split, rng):
    """Build a 2:1 refined square lattice, optionally split into triangles.

    The lattice works in integer half-step coordinates so that the midpoint of
    any coarse edge is an exact lattice point.  ``refine`` is a bool array
    [nx, ny] (coarse square (i, j) refined into four children) or None.
    Each leaf square is kept with probability 1 - p_split, otherwise it is cut
    along one of its two diagonals, chosen at random.
    """
    if refine is None:
        refine = np.zeros((nx, ny), dtype=bool)
    hx = (x1 - x0) / nx
    hy = (y1 - y0) / ny
    # leaf squares in half-step lattice coordinates: (I, J, size) with size 1 or 2
    leaves = []
    for j in range(ny):
        for i in range(nx):
            if refine[i, j]:
                for b in (0, 1):
                    for a in (0, 1):
                        leaves.append((2 * i + a, 2 * j + b, 1))
            else:
                leaves.append((2 * i, 2 * j, 2))
    nl = len(leaves)
    split_u = rng.random(nl) if p_split > 0 else np.ones(nl)
    diag_u = rng.random(nl) if p_split > 0 else np.zeros(nl)
    polys = []
    for idx, (I, J, s) in enumerate(leaves):
        c00, c10, c11, c01 = (I, J), (I + s, J), (I + s, J + s), (I, J + s)
        if split_u[idx] < p_split:
            if diag_u[idx] < 0.5:   # diagonal c00 - c11
                polys.append([c00, c10, c11])
                polys.append([c00, c11, c01])
            else:                   # diagonal c10 - c01
                polys.append([c00, c10, c01])
                polys.append([c10, c11, c01])
        else:
            polys.append([c00, c10, c11, c01])
    used = set()
    for P in polys:
        used.update(P)
    # insert hanging nodes: used lattice points strictly inside axis-aligned edges of length 2
    cells = []
    for P in polys:
        out = []
        n = len(P)
        for t in range(n):
            a = P[t]
            b = P[(t + 1) % n]
            out.append(a)
            dI, dJ = b[0] - a[0], b[1] - a[1]
            if (abs(dI) == 2 and dJ == 0) or (abs(dJ) == 2 and dI == 0):
                m = (a[0] + dI // 2, a[1] + dJ // 2)
                if m in used:
                    out.append(m)
        cells.append(out)
    ids = {}
    order = sorted(used, key=lambda q: (q[1], q[0]))
    for q in order:
        ids[q] = len(ids)
    xy = np.empty((len(order), 2))
    for q, v in ids.items():
        xy[v, 0] = x0 + q[0] * hx / 2
        xy[v, 1] = y0 + q[1] * hy / 2
    cell_ptr = np.zeros(len(cells) + 1, dtype=np.int32)
    cell_ptr[1:] = np.cumsum([len(c) for c in cells])
    cell_vtx = np.fromiter((ids[q] for c in cells for q in c), dtype=np.int32,
                           count=int(cell_ptr[-1]))
    return dict(xy=xy, cell_ptr=cell_ptr, cell_vtx=cell_vtx, h=hx)


def _barycentres(mesh):
    xy, ptr, vtx = mesh["xy"], mesh["cell_ptr"], mesh["cell_vtx"]
    cnt = np.diff(ptr)
    sx = np.add.reduceat(xy[vtx, 0], ptr[:-1])
    sy = np.add.reduceat(xy[vtx, 1], ptr[:-1])
    return np.stack([sx / cnt, sy / cnt], axis=1)   # vertex average: only used to classify media


def unit_square(n, p_split=0.0, seed=0, interface_y=0.5, refine=None):
    """n x n squares on [0,1]^2, solid below y = interface_y, fluid above.

    ``p_split`` = probability that a square is cut into two triangles (the
    hybrid meshes of the benchmark workloads use 0.5).  ``refine`` is an
    optional [n, n] bool mask of squares refined 2:1 (hanging nodes).
    """
    rng = np.random.default_rng(seed)
    m = _lattice_mesh(n, n, 0.0, 1.0, 0.0, 1.0, refine, p_split, rng)
    bc = _barycentres(m)
    m["medium"] = np.where(bc[:, 1] > interface_y, FLUID, SOLID).astype(np.uint8)
    return m


def single_medium(n, medium, p_split=0.0, seed=0, refine=None):
    """n x n squares on [0,1]^2 filled with one medium (pure acoustic / elastic)."""
    rng = np.random.default_rng(seed)
    m = _lattice_mesh(n, n, 0.0, 1.0, 0.0, 1.0, refine, p_split, rng)
    m["medium"] = np.full(len(m["cell_ptr"]) - 1, medium, dtype=np.uint8)
    return m


def bilayer_vertical(n, p_split=0.0, seed=0):
    """The CFL test geometry: solid (-1,0)x(0,1), fluid (0,1)x(0,1), interface x = 0.

    Uses 2n x n squares of side 1/n.
    """
    rng = np.random.default_rng(seed)
    m = _lattice_mesh(2 * n, n, -1.0, 1.0, 0.0, 1.0, None, p_split, rng)
    bc = _barycentres(m)
    m["medium"] = np.where(bc[:, 0] > 0.0, FLUID, SOLID).astype(np.uint8)
    return m


def _clip(poly, axis, value, keep_below):
    """Sutherland-Hodgman clip of an integer polygon by x_axis <= value (keep_below) or >= value.
    Crossing points are computed exactly (the honeycomb only meets its clip lines at lattice
    points or along edges)."""
    out = []
    n = len(poly)
    inside = (lambda q: q[axis] <= value) if keep_below else (lambda q: q[axis] >= value)
    for t in range(n):
        a, b = poly[t], poly[(t + 1) % n]
        ia, ib = inside(a), inside(b)
        if ia:
            out.append(a)
        if ia != ib:
            da, db = a[axis] - value, b[axis] - value
            num = [a[c] * (db) - b[c] * (da) for c in range(2)]
            den = db - da
            q = [num[0] // den if num[0] % den == 0 else None, num[1] // den if num[1] % den == 0 else None]
            if q[0] is None or q[1] is None:
                raise ValueError("clip crossing off the lattice")
            q = tuple(q)
            if not out or out[-1] != q:
                out.append(q)
    # drop repeated vertices
    res = []
    for q in out:
        if not res or res[-1] != q:
            res.append(q)
    if len(res) > 1 and res[0] == res[-1]:
        res.pop()
    return res


def honeycomb_bilayer(X=30):
    """Regular hexagons (pointy-top) on the CFL geometry: solid for x < 0, fluid for x > 0,
    x in (-1, 1), y in (0, H) with H the lattice height closest to 1.  Hexagons are built on an
    integer lattice (centres (2i + j mod 2, 3j), vertices at (c_x, c_y -+ 2), (c_x +- 1, c_y -+ 1)),
    clipped by the domain and split along x = 0, which all pass through lattice points, then
    scaled by (1/X, 1/(sqrt(3) X)) so that every hexagon is regular.  Cells cut by the boundary or
    the interface are quadrilaterals or pentagons.  X must be even."""
    if X % 2:
        raise ValueError("X must be even")
    J = max(1, int(round(X / np.sqrt(3.0))))
    Y = 3 * J
    cells = []
    for j in range(-1, J + 2):
        for cx in range(-X - 2, X + 3):
            if (cx - j) % 2:
                continue
            cy = 3 * j
            hexv = [(cx, cy - 2), (cx + 1, cy - 1), (cx + 1, cy + 1), (cx, cy + 2), (cx - 1, cy + 1), (cx - 1, cy - 1)]
            P = hexv
            for axis, value, below in ((0, X, True), (0, -X, False), (1, Y, True), (1, 0, False)):
                if len(P) < 3:
                    break
                P = _clip(P, axis, value, below)
            if len(P) < 3:
                continue
            for half in (_clip(P, 0, 0, True), _clip(P, 0, 0, False)):
                if len(half) < 3:
                    continue
                area2 = sum(half[t][0] * half[(t + 1) % len(half)][1] - half[(t + 1) % len(half)][0] * half[t][1]
                            for t in range(len(half)))
                if area2 > 0:
                    cells.append(half)
    ids = {}
    for c in cells:
        for q in c:
            ids.setdefault(q, len(ids))
    sx = 1.0 / X
    sy = sx / np.sqrt(3.0)
    xy = np.empty((len(ids), 2))
    for q, v in ids.items():
        xy[v] = (q[0] * sx, q[1] * sy)
    cell_ptr = np.zeros(len(cells) + 1, dtype=np.int32)
    cell_ptr[1:] = np.cumsum([len(c) for c in cells])
    cell_vtx = np.fromiter((ids[q] for c in cells for q in c), dtype=np.int32, count=int(cell_ptr[-1]))
    m = dict(xy=xy, cell_ptr=cell_ptr, cell_vtx=cell_vtx, h=float(np.sqrt(2.0 * np.sqrt(3.0)) / X))
    bc = _barycentres(m)
    m["medium"] = np.where(bc[:, 0] > 0.0, FLUID, SOLID).astype(np.uint8)
    return m


def perturbed_square(n, amount=0.15, p_split=0.5, seed=0, interface_y=0.5, x_max=None):
    """unit_square(n, p_split) with every vertex moved by a seeded uniform offset of up to
    amount * h per coordinate, except along the constraints: corners stay, other boundary
    vertices and vertices on the interface y = interface_y move only along their line.  Every
    cell then has its own shape (no two cells are translates of each other), like a mesh from an
    unstructured generator.  With x_max set only the vertices left of x = x_max move, so the
    cells right of that line keep the lattice shapes."""
    m = unit_square(n, p_split=p_split, seed=seed, interface_y=interface_y)
    h = 1.0 / n
    rng = np.random.default_rng(seed + 7)
    xy = m["xy"].copy()
    d = rng.uniform(-amount * h, amount * h, xy.shape)
    on_x = (np.abs(xy[:, 0]) < 1e-12) | (np.abs(xy[:, 0] - 1.0) < 1e-12)
    on_y = (np.abs(xy[:, 1]) < 1e-12) | (np.abs(xy[:, 1] - 1.0) < 1e-12) | (np.abs(xy[:, 1] - interface_y) < 1e-12)
    d[on_x, 0] = 0.0
    d[on_y, 1] = 0.0
    if x_max is not None:
        d[xy[:, 0] >= x_max - 1e-12] = 0.0
    out = dict(m)
    out["xy"] = xy + d
    return out


def with_materials(mesh, rho_f=1.0, c_f=1.0, rho_s=1.0, cp_s=np.sqrt(3.0), cs_s=1.0,
                   perturb=0.0, seed=None):
    """Attach per-cell (rho, a, b).  Each physical parameter (rho, c for fluid
    cells; rho, cP, cS for solid cells) is multiplied by 1 + U[-perturb, perturb]
    independently per cell; solid Lame parameters follow from
    mu = rho cS^2 and lambda = rho cP^2 - 2 mu."""
    nc = len(mesh["cell_ptr"]) - 1
    med = mesh["medium"]
    rng = np.random.default_rng(seed)
    f = (lambda: 1.0 + rng.uniform(-perturb, perturb, nc)) if perturb > 0 else (lambda: np.ones(nc))
    rho = np.where(med == FLUID, rho_f, rho_s) * f()
    c1 = np.where(med == FLUID, c_f, cp_s) * f()
    c2 = np.where(med == FLUID, 0.0, cs_s) * f()
    mu = rho * c2 ** 2
    lam = rho * c1 ** 2 - 2.0 * mu
    a = np.where(med == FLUID, c1, lam)
    b = np.where(med == FLUID, 0.0, mu)
    out = dict(mesh)
    out.update(rho=rho.astype(np.float64), a=a.astype(np.float64), b=b.astype(np.float64))
    return out


def max_wave_speed(mesh):
    """Largest wave speed over the cells (c for fluid, cP for solid)."""
    med, rho, a, b = mesh["medium"], mesh["rho"], mesh["a"], mesh["b"]
    cp = np.where(med == FLUID, a, np.sqrt(np.maximum(a + 2.0 * b, 0.0) / rho))
    return float(cp.max())


# --------------------------------------------------------------------------------------
# Named workloads (sizes and seeds of the benchmark configurations)
# --------------------------------------------------------------------------------------

def manufactured_square(n=16):
    """Unit square, 16 x 16 quads, fluid rho = 1, c = 1 above y = 1/2; solid rho = 1,
    cP = sqrt(3), cS = 1 below (lambda = mu = 1)."""
    return with_materials(unit_square(n))


def hybrid_square(n=256, mesh_seed=2001, mat_seed=2002, perturb=0.10):
    """n x n squares, each kept or cut along a random diagonal with probability 1/2,
    per-cell materials perturbed by U[-10 %, +10 %]."""
    return with_materials(unit_square(n, p_split=0.5, seed=mesh_seed),
                          perturb=perturb, seed=mat_seed)


def hanging_square(n=8, seed=7, p_split=0.5, frac=0.25):
    """Hybrid unit-square mesh where a random set of squares is refined 2:1,
    producing pentagons, hexagons and quadrilaterals with hanging nodes."""
    rng = np.random.default_rng(seed + 1)
    refine = rng.random((n, n)) < frac
    return with_materials(unit_square(n, p_split=p_split, seed=seed, refine=refine))


def basin(nx=1120, ny=280, seed=3001, p_split=0.5):
    """Synthetic sedimentary basin: x in [0, 20] km, y in [-4, 1] km, water above
    y = 0 (c = 1500 m/s, rho = 1000), layered solid below with a Gaussian-profile
    low-velocity basin (depth 1 km * exp(-((x - 12 km)/2.5 km)^2)); the squares
    intersecting the basin plus a one-square margin are refined 2:1."""
    L, y0, y1 = 20000.0, -4000.0, 1000.0
    hx = L / nx
    xs = (np.arange(nx) + 0.5) * hx
    ys = y0 + (np.arange(ny) + 0.5) * (y1 - y0) / ny
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    d = 1000.0 * np.exp(-((X - 12000.0) / 2500.0) ** 2)
    inside = (Y < 0) & (-Y < d + hx)
    refine = inside.copy()
    refine[1:, :] |= inside[:-1, :]
    refine[:-1, :] |= inside[1:, :]
    refine[:, 1:] |= inside[:, :-1]
    refine[:, :-1] |= inside[:, 1:]
    refine &= (Y < 0)
    rng = np.random.default_rng(seed)
    m = _lattice_mesh(nx, ny, 0.0, L, y0, y1, refine, p_split, rng)
    bc = _barycentres(m)
    med = np.where(bc[:, 1] > 0.0, FLUID, SOLID).astype(np.uint8)
    z = -bc[:, 1]
    cs = np.select([z < 500, z < 1500, z < 2500], [1200.0, 1800.0, 2400.0], 3000.0)
    rho = np.select([z < 500, z < 1500, z < 2500], [2100.0, 2300.0, 2500.0], 2700.0)
    db = 1000.0 * np.exp(-((bc[:, 0] - 12000.0) / 2500.0) ** 2)
    inb = (z > 0) & (z < db)
    cs = np.where(inb, 300.0 + 600.0 * z / np.maximum(db, 1e-9), cs)
    rho = np.where(inb, 1800.0 + 200.0 * z / np.maximum(db, 1e-9), rho)
    cp = np.sqrt(3.0) * cs
    mu = rho * cs ** 2
    lam = rho * cp ** 2 - 2.0 * mu
    m["medium"] = med
    m["rho"] = np.where(med == FLUID, 1000.0, rho)
    m["a"] = np.where(med == FLUID, 1500.0, lam)
    m["b"] = np.where(med == FLUID, 0.0, mu)
    return m


def adjoint_square(n=128, mesh_seed=5001):
    """The adjoint workload: n x n hybrid squares (random diagonal cuts, p = 1/2) with the
    unperturbed two-material setting as the model being evaluated."""
    return with_materials(unit_square(n, p_split=0.5, seed=mesh_seed))


def adjoint_receivers(n_each=16):
    """Receivers of the adjoint workload: n_each recording p at y = 0.75 (fluid) and n_each
    recording v at y = 0.40 (solid)."""
    xy = np.concatenate([receiver_line(n_each, 0.75), receiver_line(n_each, 0.40)])
    field = np.concatenate([np.zeros(n_each, np.int32), np.ones(n_each, np.int32)])
    return xy, field


def perturbed_model(mesh, seed=5002, amount=0.05):
    """Copy of mesh with every per-cell parameter times (1 + U[-amount, amount])."""
    out = dict(mesh)
    rng = np.random.default_rng(seed)
    for key in ("rho", "a", "b"):
        out[key] = np.asarray(mesh[key], float) * (1 + rng.uniform(-amount, amount, len(mesh["rho"])))
    return out


def batch_meshes(n_meshes=16, c_min=2.0e4, c_max=3.0e5):
    """Sizes of the multi-mesh batch: target cell counts log-spaced between
    c_min and c_max, n_i = round(sqrt(C_i / 1.5)) squares per side, split seed
    4000 + i, degree k_i = 1 + (i mod 3)."""
    out = []
    for i in range(n_meshes):
        ci = c_min * (c_max / c_min) ** (i / max(n_meshes - 1, 1))
        n = int(round(np.sqrt(ci / 1.5)))
        n += n % 2
        out.append(dict(n=n, seed=4000 + i, k=1 + (i % 3)))
    return out


def shot_positions(n, seed, box=(0.1, 0.9, 0.1, 0.4)):
    """Seeded source positions, uniform in the given box of the solid part."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(box[0], box[1], n)
    y = rng.uniform(box[2], box[3], n)
    return np.stack([x, y], axis=1)


def receiver_line(n, y, x0=0.05, x1=0.95):
    """n receivers equally spaced on the horizontal line at height y."""
    return np.stack([np.linspace(x0, x1, n), np.full(n, y)], axis=1)


def random_state(ndof_per_cell, seed, scale=1.0):
    """Seeded random cell coefficients (one value per cell degree of freedom)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(int(np.sum(ndof_per_cell)))


def granite_water(nx=161, ny_s=68, ny_f=42):
    """The granite-water bilayer of the paper's explicit/implicit timing study (Sec. 5.2,
    Table tab::cfl_cpu): x in (-1.9, 1.9) km, granite (rho = 2690, cP = 6000 m/s,
    cS = 3000 m/s) below the interface, water (rho = 1025, c = 1500 m/s) above, squares of
    23.6 m.  The 2.6 km height is split into ny_s + ny_f = 110 rows of 23.64 m so that the
    interface is a row line: it lies at y = 7.3 m instead of y = 0 (68 rows of granite below,
    42 of water above)."""
    ny = ny_s + ny_f
    L, H = 3800.0, 2600.0
    y0 = -1600.0
    rng = np.random.default_rng(0)
    m = _lattice_mesh(nx, ny, -L / 2, L / 2, y0, y0 + H, None, 0.0, rng)
    y_int = y0 + ny_s * H / ny
    bc = _barycentres(m)
    m["medium"] = np.where(bc[:, 1] > y_int, FLUID, SOLID).astype(np.uint8)
    return with_materials(m, rho_f=1025.0, c_f=1500.0, rho_s=2690.0, cp_s=6000.0, cs_s=3000.0)


def pressure_pulse(mesh, k, center=(0.0, 200.0), sigma=50.0, k_primal=None):
    """Initial state with a Gaussian pressure bump exp(-|x - center|^2 / (2 sigma^2)) in the
    fluid: the lowest (constant) coefficient of p per fluid cell, scaled by sqrt(area) (the
    constant function of an orthonormal cell basis is 1/sqrt(area)); everything else zero.
    External layout: per cell in input order, [p | m_x | m_y] (fluid) or [v_x | v_y | s]
    (solid), N = (k+1)(k+2)/2 coefficients per field, or N' = (k'+1)(k'+2)/2 for p and v when
    k_primal = k' is given (cell degree k' of the primal fields, k of the dual ones)."""
    N = (k + 1) * (k + 2) // 2
    kp = k if k_primal is None else k_primal
    Np = (kp + 1) * (kp + 2) // 2
    med = np.asarray(mesh["medium"])
    per = np.where(med == FLUID, Np + 2 * N, 2 * Np + 3 * N)
    off = np.concatenate([[0], np.cumsum(per)[:-1]])
    xy, ptr, vtx = mesh["xy"], mesh["cell_ptr"], mesh["cell_vtx"]
    U = np.zeros(int(per.sum()))
    bc = _barycentres(mesh)
    for c in np.flatnonzero(med == FLUID):
        p = xy[vtx[ptr[c]:ptr[c + 1]]]
        area = 0.5 * abs(np.dot(p[:, 0], np.roll(p[:, 1], -1)) - np.dot(p[:, 1], np.roll(p[:, 0], -1)))
        r2 = (bc[c, 0] - center[0]) ** 2 + (bc[c, 1] - center[1]) ** 2
        U[off[c]] = np.exp(-r2 / (2 * sigma ** 2)) * np.sqrt(area)
    return U


# ----------------------------------------------------------------------------- three dimensions
# Three-dimensional meshes are dicts with xyz float64 [n_vertices, 3], cell_ptr / cell_vtx (4 ids
# per tetrahedron; 6 per triangular prism: 0-2 around the bottom triangle, 3-5 above them; 8 per
# hexahedron: 0-3 around the bottom face counter-clockwise seen from above, 4-7 above them), medium,
# and after with_materials3d rho, a, b.

# the six tetrahedra of a cube around its diagonal from corner 0 to corner 6
_KUHN = ((0, 1, 2, 6), (0, 2, 3, 6), (0, 3, 7, 6), (0, 7, 4, 6), (0, 4, 5, 6), (0, 5, 1, 6))


def unit_cube(n, tets=True, jitter=0.0, seed=0, interface_z=0.5, shear=None, kind=None):
    """n^3 cubes on [0, 1]^3, solid below z = interface_z and fluid above (cell centres).  kind
    (default "tets" if tets else "hexes"): "tets" cuts every cube into six tetrahedra, "hexes" keeps
    it, "prisms" cuts it into two triangular prisms along a diagonal of its base (the same diagonal
    in every cube), "hybrid" keeps every vertical column of cubes as hexahedra or cuts it into prisms
    along a random diagonal, each with probability 1/2 (seeded).  jitter: interior vertices off the
    interface plane moved by U[-jitter, jitter] h per coordinate (seeded; tetrahedra only).  shear:
    a 3 x 3 matrix applied to every vertex (hexahedra and prisms keep planar faces)."""
    kind = kind or ("tets" if tets else "hexes")
    tets = kind == "tets"
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(i, j, l):
        return (i * (n + 1) + j) * (n + 1) + l

    cells = []
    col_rng = np.random.default_rng(seed + 7919)
    for i in range(n):
        for j in range(n):
            # column kind: 0 hexahedra, 1 / 2 prisms cut along the diagonal from base vertex 0 / 1
            col = {"hexes": 0, "prisms": 1, "tets": 0}.get(kind, 0)
            if kind == "hybrid":
                col = 0 if col_rng.random() < 0.5 else 1 + int(col_rng.integers(2))
            for l in range(n):
                h = (vid(i, j, l), vid(i + 1, j, l), vid(i + 1, j + 1, l), vid(i, j + 1, l),
                     vid(i, j, l + 1), vid(i + 1, j, l + 1), vid(i + 1, j + 1, l + 1), vid(i, j + 1, l + 1))
                if tets:
                    cells += [tuple(h[t] for t in tt) for tt in _KUHN]
                elif col == 0:
                    cells.append(h)
                elif col == 1:
                    cells += [(h[0], h[1], h[2], h[4], h[5], h[6]), (h[0], h[2], h[3], h[4], h[6], h[7])]
                else:
                    cells += [(h[0], h[1], h[3], h[4], h[5], h[7]), (h[1], h[2], h[3], h[5], h[6], h[7])]
    if kind == "hybrid" or kind == "prisms":
        ptr = np.concatenate([[0], np.cumsum([len(c) for c in cells])]).astype(np.int32)
        vtx = np.concatenate([np.asarray(c) for c in cells]).astype(np.int32)
        cent = np.array([xyz[list(c)].mean(axis=0) for c in cells])
        medium = np.where(cent[:, 2] < interface_z, SOLID, FLUID).astype(np.uint8)
        if shear is not None:
            xyz = xyz @ np.asarray(shear, float).T
        return dict(xyz=xyz, cell_ptr=ptr, cell_vtx=vtx, medium=medium)
    cells = np.array(cells, np.int64)
    cent = xyz[cells].mean(axis=1)
    medium = np.where(cent[:, 2] < interface_z, SOLID, FLUID).astype(np.uint8)
    if jitter > 0.0:
        if not tets:
            raise ValueError("jitter keeps faces planar only for tetrahedra")
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, xyz.shape) / n
        fixed = np.zeros(len(xyz), bool)
        for ax in range(3):
            fixed |= (np.abs(xyz[:, ax]) < 1e-12) | (np.abs(xyz[:, ax] - 1.0) < 1e-12)
        fixed |= np.abs(xyz[:, 2] - interface_z) < 1e-12
        xyz = xyz + np.where(fixed[:, None], 0.0, d)
    if shear is not None:
        xyz = xyz @ np.asarray(shear, float).T
    if tets:  # positive orientation
        P = xyz[cells]
        det = np.einsum("ij,ij->i", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))
        flip = det < 0
        cells[flip, 1], cells[flip, 2] = cells[flip, 2].copy(), cells[flip, 1].copy()
    nv = cells.shape[1]
    return dict(xyz=xyz, cell_ptr=np.arange(0, nv * len(cells) + 1, nv, dtype=np.int32),
                cell_vtx=cells.reshape(-1).astype(np.int32), medium=medium)


def with_materials3d(mesh, rho_f=1.0, c_f=1.0, rho_s=1.0, lam=1.0, mu=1.0, perturb=0.0, seed=0):
    """Piecewise-constant materials: fluid (rho_f, c_f), solid (rho_s, lambda, mu); with perturb, every
    per-cell parameter times (1 + U[-perturb, perturb]) (seeded)."""
    med = np.asarray(mesh["medium"])
    nc = len(med)
    rng = np.random.default_rng(seed)
    f = (lambda: 1.0 + rng.uniform(-perturb, perturb, nc)) if perturb > 0 else (lambda: np.ones(nc))
    rho = np.where(med == FLUID, rho_f, rho_s) * f()
    a = np.where(med == FLUID, c_f, lam) * f()
    b = np.where(med == FLUID, 0.0, mu) * f()
    out = dict(mesh)
    out.update(rho=rho, a=a, b=b)
    return out


def max_wave_speed3d(mesh):
    """Largest wave speed of a three-dimensional mesh with materials (c_P in the solid)."""
    med = np.asarray(mesh["medium"])
    rho, a, b = (np.asarray(mesh[k_]) for k_ in ("rho", "a", "b"))
    c = np.where(med == FLUID, a, np.sqrt(np.maximum(a + 2.0 * b, 0.0) / rho))
    return float(c.max())
