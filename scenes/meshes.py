"""Seeded synthetic geometry: surface meshes, coarse embedding grids and the
barycentric embedding matrix W.

This module builds *inputs* only (meshes, node positions, W, displacement
fields).  It holds none of the contact-stage arithmetic: no distances, no
barrier, no reduction and no CCD.  Both the CPU oracle and the HIP library are
fed from what it returns.

Embedding construction follows the paper's embedding section (Eq. 13-14): every
surface vertex lies in one tetrahedron of a coarse tet mesh and is written as a
barycentric combination of that tetrahedron's four nodes.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Surface meshes
# ---------------------------------------------------------------------------

_ICO_T = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array([
    [-1, _ICO_T, 0], [1, _ICO_T, 0], [-1, -_ICO_T, 0], [1, -_ICO_T, 0],
    [0, -1, _ICO_T], [0, 1, _ICO_T], [0, -1, -_ICO_T], [0, 1, -_ICO_T],
    [_ICO_T, 0, -1], [_ICO_T, 0, 1], [-_ICO_T, 0, -1], [-_ICO_T, 0, 1]],
    dtype=np.float64)
_ICO_F = np.array([
    [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
    [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
    [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
    [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)

_GEODESIC_CACHE: dict[int, tuple[np.ndarray, np.ndarray]] = {}


def geodesic_sphere(nu: int) -> tuple[np.ndarray, np.ndarray]:
    """Unit geodesic sphere of frequency ``nu`` (class I subdivision of the
    icosahedron).  V = 10 nu^2 + 2, F = 20 nu^2, E = 30 nu^2.  Faces are
    oriented with outward normals.  nu = 16 is the level-4 icosphere."""
    if nu in _GEODESIC_CACHE:
        v, f = _GEODESIC_CACHE[nu]
        return v.copy(), f.copy()
    if nu < 1:
        raise ValueError("nu must be >= 1")
    key_to_id: dict[tuple, int] = {}
    pts: list[np.ndarray] = []

    def vid(a: int, b: int, c: int, i: int, j: int) -> int:
        # point = ((nu-i-j) A + i B + j C) / nu, keyed exactly by its integer
        # weights on the icosahedron corners (shared edges get one id)
        w = {}
        for corner, wt in ((a, nu - i - j), (b, i), (c, j)):
            if wt:
                w[corner] = w.get(corner, 0) + wt
        key = tuple(sorted(w.items()))
        got = key_to_id.get(key)
        if got is None:
            p = sum(_ICO_V[k] * (wt / nu) for k, wt in key)
            got = len(pts)
            key_to_id[key] = got
            pts.append(p / np.linalg.norm(p))
        return got

    faces = []
    for a, b, c in _ICO_F:
        grid = {}
        for i in range(nu + 1):
            for j in range(nu + 1 - i):
                grid[i, j] = vid(a, b, c, i, j)
        for i in range(nu):
            for j in range(nu - i):
                faces.append((grid[i, j], grid[i + 1, j], grid[i, j + 1]))
                if i + j < nu - 1:
                    faces.append((grid[i + 1, j], grid[i + 1, j + 1], grid[i, j + 1]))
    v = np.array(pts, dtype=np.float64)
    f = np.array(faces, dtype=np.int32)
    # orient outward
    c = v[f].mean(axis=1)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    flip = np.einsum("ij,ij->i", n, c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    _GEODESIC_CACHE[nu] = (v, f)
    return v.copy(), f.copy()


def unique_edges(faces: np.ndarray) -> np.ndarray:
    """Unique undirected edges (a < b) of a triangle list, sorted
    lexicographically, int32 [n_edge, 2]."""
    f = np.asarray(faces, dtype=np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def grid_quad_mesh(nx: int, ny: int, x0, x1, y0, y1, z: float, up: bool = True):
    """Flat rectangle split into 2 nx ny triangles at height z."""
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    v = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)
    idx = np.arange((nx + 1) * (ny + 1)).reshape(nx + 1, ny + 1)
    f = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = idx[i, j], idx[i + 1, j], idx[i + 1, j + 1], idx[i, j + 1]
            f.append((a, b, c))
            f.append((a, c, d))
    f = np.array(f, dtype=np.int32)
    if not up:
        f = f[:, [0, 2, 1]]
    return v, f


def cylinder_mesh(radius: float, length: float, n_around: int, n_along: int):
    """Closed cylinder along +x from 0 to ``length`` with fan caps.
    Triangles = 2 n_around n_along + 2 n_around."""
    th = 2 * np.pi * np.arange(n_around) / n_around
    xs = np.linspace(0.0, length, n_along + 1)
    ring = np.stack([np.cos(th), np.sin(th)], axis=1) * radius
    v = []
    for x in xs:
        for c, s in ring:
            v.append((x, c, s))
    v.append((0.0, 0.0, 0.0))
    v.append((length, 0.0, 0.0))
    v = np.array(v, dtype=np.float64)
    c0 = len(v) - 2
    c1 = len(v) - 1

    def rid(i, k):
        return i * n_around + (k % n_around)

    f = []
    for i in range(n_along):
        for k in range(n_around):
            a, b, c, d = rid(i, k), rid(i + 1, k), rid(i + 1, k + 1), rid(i, k + 1)
            f.append((a, c, b))
            f.append((a, d, c))
    for k in range(n_around):
        f.append((c0, rid(0, k + 1), rid(0, k)))
        f.append((c1, rid(n_along, k), rid(n_along, k + 1)))
    f = np.array(f, dtype=np.int32)
    # orient outward (convex body: compare with the centroid)
    cen = v.mean(axis=0)
    fc = v[f].mean(axis=1)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    flip = np.einsum("ij,ij->i", n, fc - cen) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def disc_plate_mesh(radius: float, thickness: float, spacing: float):
    """Closed thin disc: two structured triangulated faces (grid clipped to
    the circle, boundary vertices snapped to it) joined by a rim strip.
    The plate lies in z in [-thickness/2, thickness/2], centred at the origin."""
    n = int(np.ceil(radius / spacing))
    coords = np.arange(-n, n + 1) * spacing
    X, Y = np.meshgrid(coords, coords, indexing="ij")
    inside = (X ** 2 + Y ** 2) <= radius ** 2
    # keep grid cells whose 4 corners are inside; snap nothing inside
    idx = -np.ones(X.shape, dtype=np.int64)
    idx[inside] = np.arange(inside.sum())
    pts2 = np.stack([X[inside], Y[inside]], axis=1)
    tris = []
    m = X.shape[0]
    for i in range(m - 1):
        for j in range(m - 1):
            a, b, c, d = idx[i, j], idx[i + 1, j], idx[i + 1, j + 1], idx[i, j + 1]
            if min(a, b, c, d) < 0:
                continue
            tris.append((a, b, c))
            tris.append((a, c, d))
    tris = np.array(tris, dtype=np.int64)
    # boundary loop of the clipped grid region: edges used by one triangle
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    key = np.sort(e, axis=1)
    uniq, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    bmask = cnt[inv.ravel()] == 1
    bedges = e[bmask]  # directed as in the (ccw) triangles
    nxt = {int(a): int(b) for a, b in bedges}
    start = int(bedges[0, 0])
    loop = [start]
    cur = nxt[start]
    while cur != start:
        loop.append(cur)
        cur = nxt[cur]
    loop = np.array(loop)
    # snap boundary vertices radially onto the circle
    p = pts2.copy()
    r = np.linalg.norm(p[loop], axis=1)
    p[loop] = p[loop] * (radius / r)[:, None]
    nv = len(p)
    top = np.concatenate([p, np.full((nv, 1), thickness / 2)], axis=1)
    bot = np.concatenate([p, np.full((nv, 1), -thickness / 2)], axis=1)
    v = np.concatenate([top, bot])
    f_top = tris
    f_bot = tris[:, [0, 2, 1]] + nv
    rim = []
    L = len(loop)
    for k in range(L):
        a, b = loop[k], loop[(k + 1) % L]
        # boundary edge a->b is ccw seen from +z; outward rim faces
        rim.append((a, a + nv, b + nv))
        rim.append((a, b + nv, b))
    f = np.concatenate([f_top, f_bot, np.array(rim, dtype=np.int64)]).astype(np.int32)
    return v, f


# ---------------------------------------------------------------------------
# Coarse embedding grid and barycentric W (paper Eq. 13-14)
# ---------------------------------------------------------------------------

# The 6 tetrahedra of the Kuhn (Freudenthal) split of a unit cube.  Each is
# [c000, c000+e_a, c000+e_a+e_b, c111] for a permutation (a, b, c) of axes.
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


class CoarseGrid:
    """Regular nx x ny x nz node grid over a box, 6 Kuhn tets per cell."""

    def __init__(self, lo, hi, dims):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.dims = tuple(int(d) for d in dims)
        nx, ny, nz = self.dims
        if min(self.dims) < 2:
            raise ValueError("grid needs >= 2 nodes per axis")
        self.h = (self.hi - self.lo) / (np.array(self.dims) - 1)
        gx = np.linspace(self.lo[0], self.hi[0], nx)
        gy = np.linspace(self.lo[1], self.hi[1], ny)
        gz = np.linspace(self.lo[2], self.hi[2], nz)
        X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
        self.nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        tets = []
        for i in range(nx - 1):
            for j in range(ny - 1):
                for k in range(nz - 1):
                    for perm in _KUHN_PERMS:
                        c = np.array([i, j, k])
                        ids = [self.nid(*c)]
                        for ax in perm:
                            c = c.copy()
                            c[ax] += 1
                            ids.append(self.nid(*c))
                        tets.append(ids)
        self.tets = np.array(tets, dtype=np.int32)

    @property
    def n_node(self) -> int:
        return len(self.nodes)

    def nid(self, i, j, k) -> int:
        nx, ny, nz = self.dims
        return (i * ny + j) * nz + k

    def cell_of(self, x: np.ndarray) -> np.ndarray:
        c = np.floor((x - self.lo) / self.h).astype(np.int64)
        return np.clip(c, 0, np.array(self.dims) - 2)

    def embed(self, x: np.ndarray, node_pos: np.ndarray | None = None, with_tet: bool = False):
        """Barycentric weights of points x in the grid's tets.

        Reading of the 'unique containing tetrahedron' rule: the point is
        assigned to the cell that contains it (floor of the grid coordinate,
        clamped), and within that cell to the first of its 6 Kuhn tets (in
        the fixed order above) whose smallest barycentric coordinate is
        >= -1e-12.  Returns (tet_nodes int32[n,4], weights f64[n,4]) and,
        with with_tet, the tet indices int64[n] too."""
        if node_pos is None:
            node_pos = self.nodes
        nx, ny, nz = self.dims
        cells = self.cell_of(x)
        cidx = (cells[:, 0] * (ny - 1) + cells[:, 1]) * (nz - 1) + cells[:, 2]
        n = len(x)
        best_tet = -np.ones(n, dtype=np.int64)
        best_w = np.zeros((n, 4))
        for t in range(6):
            tid = cidx * 6 + t
            tn = self.tets[tid]
            p0 = node_pos[tn[:, 0]]
            D = np.stack([node_pos[tn[:, 1]] - p0, node_pos[tn[:, 2]] - p0,
                          node_pos[tn[:, 3]] - p0], axis=2)
            lam = np.linalg.solve(D, (x - p0)[:, :, None])[:, :, 0]
            w = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
            ok = (w.min(axis=1) >= -1e-12) & (best_tet < 0)
            best_tet[ok] = tid[ok]
            best_w[ok] = w[ok]
        if (best_tet < 0).any():
            raise ValueError("some points lie outside the embedding grid")
        if with_tet:
            return self.tets[best_tet].astype(np.int32), best_w, best_tet
        return self.tets[best_tet].astype(np.int32), best_w


def padded_grid(points: np.ndarray, dims, pad: float = 0.01) -> CoarseGrid:
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    ext = hi - lo
    return CoarseGrid(lo - pad * ext, hi + pad * ext, dims)


def near_cubic_dims(box_ext: np.ndarray, n_target: int) -> tuple[int, int, int]:
    """Node counts (>= 2 each) proportional to the box extent whose product
    is closest to n_target."""
    best = None
    ext = np.maximum(np.asarray(box_ext, dtype=np.float64), 1e-12)
    for s in np.linspace(0.2, 4.0, 400):
        base = (n_target / np.prod(ext / ext.max())) ** (1 / 3) * s / 2
        d = np.maximum(2, np.round(ext / ext.max() * base * 2)).astype(int)
        err = abs(int(np.prod(d)) - n_target)
        if best is None or err < best[0]:
            best = (err, tuple(int(v) for v in d))
    return best[1]


def build_W(tet_nodes: np.ndarray, weights: np.ndarray, n_rows: int,
            row_ids: np.ndarray, node_offset: int = 0):
    """CSR pieces for rows ``row_ids`` (each with 4 nnz) of an n_rows-row W."""
    return row_ids, tet_nodes.astype(np.int64) + node_offset, weights


def assemble_csr(n_vert: int, entries: list[tuple[np.ndarray, np.ndarray, np.ndarray]]):
    """Assemble CSR (rowptr int32, col int32, val f64) from per-body pieces
    (row_ids, cols[n,k], vals[n,k]).  Rows not listed are empty (static or
    kinematic vertices)."""
    counts = np.zeros(n_vert, dtype=np.int64)
    for rows, cols, vals in entries:
        counts[rows] += cols.shape[1]
    rowptr = np.zeros(n_vert + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(counts)
    nnz = int(rowptr[-1])
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float64)
    for rows, cols, vals in entries:
        k = cols.shape[1]
        for j in range(k):
            col[rowptr[rows] + j] = cols[:, j]
            val[rowptr[rows] + j] = vals[:, j]
    if nnz >= 2 ** 31:
        raise ValueError("W too large for int32 CSR")
    return rowptr.astype(np.int32), col, val
