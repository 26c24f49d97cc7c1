"""Scene container and the seeded scene recipes.

Recipes (sizes and value distributions follow the paper's experiments and
the workloads the contact stage is measured on):

* ``config1``: icosphere of frequency 16 (2,562 v / 5,120 f, r = 0.05 m)
  embedded in a 5x5x5-node Kuhn-split grid, on a static 2-triangle ground.
* ``config2``: soft-bubble grasp: a spherical-harmonic blob (frequency 71,
  100,820 f) between two conformed ellipsoidal membranes (frequency 32,
  20,480 f each).
* ``config3``: thin disc plate (about 60k f) over a static rack of 40
  cylinders (4,992 f each), near-parallel edges.
* ``tiny_scene``: two small convex bodies separated by a plane, for exact
  comparisons on inputs small enough for brute force.
* ``batch_scenes``: many grasp scenes of uneven size.
* ``mixed_scale_scene``: a fine sheet over coarse static plates whose
  triangles are tens to hundreds of times larger than the sheet's, so that
  the broad phase meets primitives of very different sizes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .meshes import (CoarseGrid, assemble_csr, cylinder_mesh, disc_plate_mesh,
                     geodesic_sphere, near_cubic_dims, padded_grid, unique_edges)


def rng_for(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


@dataclasses.dataclass
class Scene:
    name: str
    n_node: int
    faces: np.ndarray            # int32 [n_face, 3]
    edges: np.ndarray            # int32 [n_edge, 2], a < b, sorted
    W_rowptr: np.ndarray         # int32 [n_vert + 1]
    W_col: np.ndarray            # int32 [nnz]
    W_val: np.ndarray            # f64 [nnz]
    x_off: np.ndarray | None     # f64 [n_vert, 3] or None
    x_rest: np.ndarray | None    # f64 [n_vert, 3] or None
    q: np.ndarray                # f64 [3 n_node]
    dq: np.ndarray               # f64 [3 n_node]
    dx_off: np.ndarray | None    # f64 [n_vert, 3] or None
    dhat: float
    kappa: float
    seed: int = 0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_vert(self) -> int:
        return len(self.W_rowptr) - 1

    @property
    def n_face(self) -> int:
        return len(self.faces)

    @property
    def n_edge(self) -> int:
        return len(self.edges)

    def summary(self) -> str:
        return (f"{self.name}: n_vert={self.n_vert} n_face={self.n_face} "
                f"n_edge={self.n_edge} n_node={self.n_node} nnz={len(self.W_col)} "
                f"dhat={self.dhat:g} kappa={self.kappa:g} seed={self.seed}")


def _wq(rowptr, col, val, q):
    """Plain W q used only to place bodies while generating inputs."""
    q3 = q.reshape(-1, 3)
    n = len(rowptr) - 1
    x = np.zeros((n, 3))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    np.add.at(x, rows, val[:, None] * q3[col])
    return x


@dataclasses.dataclass
class Body:
    verts: np.ndarray            # rest positions [n, 3]
    faces: np.ndarray            # local indices [m, 3]
    grid: CoarseGrid | None      # None: static / kinematic (empty W rows)
    full_space: bool = False     # W = I rows (one node per vertex)


def _assemble(bodies: list[Body]):
    """Concatenate bodies into one scene: vertex, face and node numbering in
    body order.  Returns faces, edges, W pieces, q0, x_off, x_rest."""
    v_off = 0
    n_off = 0
    faces = []
    entries = []
    q_parts = []
    x_off_parts = []
    any_static = False
    for b in bodies:
        n = len(b.verts)
        faces.append(b.faces.astype(np.int64) + v_off)
        rows = np.arange(v_off, v_off + n)
        if b.full_space:
            entries.append((rows, (np.arange(n) + n_off)[:, None], np.ones((n, 1))))
            q_parts.append(b.verts.reshape(-1))
            n_off += n
            x_off_parts.append(np.zeros((n, 3)))
        elif b.grid is not None:
            tn, w = b.grid.embed(b.verts)
            entries.append((rows, tn.astype(np.int64) + n_off, w))
            q_parts.append(b.grid.nodes.reshape(-1))
            n_off += b.grid.n_node
            x_off_parts.append(np.zeros((n, 3)))
        else:
            any_static = True
            x_off_parts.append(b.verts.copy())
        v_off += n
    n_vert = v_off
    faces = np.concatenate(faces).astype(np.int32)
    edges = unique_edges(faces)
    rowptr, col, val = assemble_csr(n_vert, entries)
    q0 = np.concatenate(q_parts) if q_parts else np.zeros(0)
    x_off = np.concatenate(x_off_parts) if any_static else None
    x_rest = np.concatenate([b.verts for b in bodies])
    return faces, edges, rowptr, col, val, q0, n_off, x_off, x_rest


def _make(name, bodies, q, dq, dhat, kappa, seed, dx_off=None, meta=None,
          assembled=None):
    faces, edges, rowptr, col, val, q0, n_node, x_off, x_rest = assembled or _assemble(bodies)
    return Scene(name=name, n_node=n_node, faces=faces, edges=edges,
                 W_rowptr=rowptr, W_col=col, W_val=val, x_off=x_off,
                 x_rest=x_rest, q=np.ascontiguousarray(q, dtype=np.float64),
                 dq=np.ascontiguousarray(dq, dtype=np.float64), dx_off=dx_off,
                 dhat=float(dhat), kappa=float(kappa), seed=seed, meta=meta or {})


# ---------------------------------------------------------------------------
# Config 1: icosphere on a ground plane
# ---------------------------------------------------------------------------

def config1(seed: int = 0, literal: bool = False, grid_dims=(5, 5, 5),
            noise: float = 1e-4) -> Scene:
    """Icosphere (frequency 16, r = 0.05 m) in a padded 5x5x5 Kuhn grid over
    a static ground made of 2 triangles spanning [-0.2, 0.2]^2 at z = 0.

    The bottom node layer is moved toward the next layer by sigma = 0.077
    (an exact vertical compression of the bottom cell layer) so that about
    300 vertices end within dhat of the ground; ``literal=True`` skips it.
    q gets N(0, noise) per coordinate, then the body is shifted in z so the
    lowest vertex sits at 1e-4 m.  dq ~ N(0, 5e-3 m) from a second stream.
    dhat = 1e-3 m, kappa = 1e3."""
    r = 0.05
    v_unit, f = geodesic_sphere(16)
    v = r * v_unit
    grid = padded_grid(v, grid_dims)
    ground_v = np.array([[-0.2, -0.2, 0.0], [0.2, -0.2, 0.0],
                         [0.2, 0.2, 0.0], [-0.2, 0.2, 0.0]])
    ground_f = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    bodies = [Body(v, f, grid), Body(ground_v, ground_f, None)]
    asm = _assemble(bodies)
    faces, edges, rowptr, col, val, q0, n_node, x_off, x_rest = asm
    q = q0.reshape(-1, 3).copy()
    nz = grid.dims[2]
    k = np.arange(grid.n_node) % nz
    if not literal:
        z0 = q[k == 0, 2]
        z1 = q[k == 1, 2]
        q[k == 0, 2] = z1 + 0.077 * (z0 - z1)
    rng = rng_for(seed, 0)
    q += rng.normal(0.0, noise, q.shape)
    x = _wq(rowptr, col, val, q.reshape(-1))
    zmin = x[:len(v), 2].min()
    q[:, 2] += 1e-4 - zmin
    dq = rng_for(seed, 1).normal(0.0, 5e-3, q.size)
    return _make("config1" + ("_literal" if literal else ""), bodies, q.reshape(-1), dq,
                 1e-3, 1e3, seed, assembled=asm,
                 meta={"grid_dims": grid_dims, "squash": not literal})


# ---------------------------------------------------------------------------
# Tiny two-body scenes (brute-force sized)
# ---------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    qv = rng.normal(size=4)
    qv /= np.linalg.norm(qv)
    w, x, y, z = qv
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


class SingleTet:
    """One tetrahedron enclosing a point set (the paper's affine-body special
    case): a regular tetrahedron around the points' bounding sphere."""

    def __init__(self, points: np.ndarray, margin: float = 1.5):
        c = points.mean(axis=0)
        r = np.linalg.norm(points - c, axis=1).max() * margin
        # regular tetrahedron with insphere radius r: vertices at distance 3r
        d = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        self.nodes = c + 3.0 * r * d
        self.tets = np.array([[0, 1, 2, 3]], dtype=np.int32)

    @property
    def n_node(self) -> int:
        return 4

    def embed(self, x: np.ndarray):
        p0 = self.nodes[0]
        D = np.stack([self.nodes[1] - p0, self.nodes[2] - p0, self.nodes[3] - p0], axis=1)
        lam = np.linalg.solve(D, (x - p0).T).T
        w = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
        if w.min() < -1e-12:
            raise ValueError("point outside the enclosing tetrahedron")
        return np.repeat(self.tets, len(x), axis=0), w


def tiny_scene(seed: int, dhat: float | None = None, mode: str = "grid") -> Scene:
    """Two small convex bodies (geodesic spheres of frequency 1-3 with random
    anisotropic scale and rotation) on opposite sides of a random plane,
    separated by a gap g (so they cannot intersect), with dhat = g U(2, 12).

    ``mode``: 'grid' (both embedded in small Kuhn grids), 'static' (body B
    static), 'full' (body B full-space, W = I rows), 'full_both' (both
    full-space: the paper's full-space IPC special case), 'tet' (body A in
    one enclosing tetrahedron: the affine-body special case; B static)."""
    rng = rng_for(seed, 0)
    bodies = []
    nrm = rng.normal(size=3)
    nrm /= np.linalg.norm(nrm)
    gap = 10 ** rng.uniform(-4.0, -3.0)
    for side in (-1.0, 1.0):
        nu = int(rng.integers(1, 4))
        v, f = geodesic_sphere(nu)
        v = v * (0.01 * rng.uniform(0.6, 1.6, size=3))
        v = v @ _random_rotation(rng).T
        # put the body on its side of the plane n.x = 0 at distance gap/2
        h = v @ nrm
        if side < 0:
            v = v - nrm * (h.max() + gap / 2)
        else:
            v = v - nrm * (h.min() - gap / 2)
        bodies.append((v, f))
    # slide B along the plane so its extreme vertex faces A's extreme vertex:
    # the closest distance is then exactly the gap
    va, vb = bodies[0][0], bodies[1][0]
    pa = va[np.argmax(va @ nrm)]
    pb = vb[np.argmin(vb @ nrm)]
    t = pa - pb
    t = t - nrm * (t @ nrm)
    bodies[1] = (vb + t, bodies[1][1])
    dhat_v = float(dhat) if dhat is not None else gap * rng.uniform(2.0, 12.0)
    blist = []
    for i, (v, f) in enumerate(bodies):
        if mode == "full_both" or (i == 1 and mode == "full"):
            blist.append(Body(v, f, None, full_space=True))
        elif i == 1 and mode in ("static", "tet"):
            blist.append(Body(v, f, None))
        elif i == 0 and mode == "tet":
            blist.append(Body(v, f, SingleTet(v)))
        else:
            dims = tuple(int(d) for d in rng.integers(2, 4, size=3))
            blist.append(Body(v, f, padded_grid(v, dims)))
    asm = _assemble(blist)
    q0 = asm[5]
    # small perturbation of the nodes, far below the gap
    q = q0 + rng.normal(0.0, gap * 0.02, q0.shape)
    dq = rng_for(seed, 1).normal(0.0, 5e-3, q0.shape)
    return _make(f"tiny{seed}_{mode}", blist, q, dq, dhat_v, 1e3, seed, assembled=asm,
                 meta={"gap": gap, "normal": nrm.tolist(), "mode": mode,
                       "n_vert_a": len(bodies[0][0])})


def full_space_scene(seed: int = 0) -> Scene:
    """The paper's full-space special case: every vertex is its own node."""
    return tiny_scene(seed, mode="full_both")


def single_tet_scene(seed: int = 0) -> Scene:
    """The paper's affine-body special case: body A in one tetrahedron."""
    return tiny_scene(seed, mode="tet")


def _grid_sheet(n: int, lo: float, hi: float, z: float) -> tuple[np.ndarray, np.ndarray]:
    """(n+1) x (n+1) vertices on [lo, hi]^2 at height z, two triangles per
    quad (alternating diagonals)."""
    t = np.linspace(lo, hi, n + 1)
    gx, gy = np.meshgrid(t, t, indexing="ij")
    v = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, z)], 1)
    f = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, (i + 1) * (n + 1) + j, (i + 1) * (n + 1) + j + 1, i * (n + 1) + j + 1
            f += [(a, b, c), (a, c, d)] if (i + j) % 2 == 0 else [(a, b, d), (b, c, d)]
    return v, np.array(f, dtype=np.int64)


def mixed_scale_scene(seed: int = 0, n: int = 80, size: float = 0.1, dhat: float = 2e-4,
                      plates_first: bool = False) -> Scene:
    """A deformable n x n sheet (edge size/n, embedded in a 4x4x2 grid)
    hovering 0.2-0.8 dhat above two static coplanar plates: a 2-triangle
    plate twice the sheet's width (triangles spanning about a hundred broad-
    phase cells per axis) and a 3x3-quad plate under the middle (tens of
    cells per axis).  dq moves the sheet down by up to about 2 dhat.
    ``plates_first`` numbers the plates' vertices (and so their edges)
    before the sheet's: every plate edge is then the lower index of its
    edge-edge pairs, so one plate edge queries thousands of sheet edges."""
    rng = rng_for(seed, 0)
    sv, sf = _grid_sheet(n, 0.0, size, 0.5 * dhat)
    sv[:, 2] += rng.uniform(-0.3, 0.3, len(sv)) * dhat
    pv, pf = _grid_sheet(1, -0.5 * size, 1.5 * size, 0.0)
    mv, mf = _grid_sheet(3, 0.2 * size, 0.8 * size, 0.0)
    bodies = [Body(sv, sf, padded_grid(sv, (4, 4, 2))), Body(pv, pf, None), Body(mv, mf, None)]
    if plates_first:
        bodies = bodies[1:] + bodies[:1]
    asm = _assemble(bodies)
    q = asm[5].copy()
    dq = np.zeros_like(q).reshape(-1, 3)
    dq[:, 2] = -rng.uniform(0.0, 2.0, len(dq)) * dhat
    dq[:, :2] = rng.normal(0.0, 0.2 * dhat, (len(dq), 2))
    return _make(f"mixed{seed}" + ("_pf" if plates_first else ""), bodies, q, dq.reshape(-1), dhat, 1e3, seed,
                 assembled=asm,
                 meta={"sheet_n": n, "size": size})


def long_row_scene(seed: int = 0, n: int = 80, size: float = 0.1, dhat: float = 2e-4) -> Scene:
    """The mixed-scale sheet with other embeddings: the n x n sheet is
    full-space (W = I, one node per vertex) over the 3x3-quad middle plate
    alone, now a dynamic affine body (one enclosing tetrahedron, 4 nodes).
    Every sheet vertex over the plate couples with its 4 nodes, so those
    reduced-Hessian rows hold thousands of blocks."""
    rng = rng_for(seed, 0)
    sv, sf = _grid_sheet(n, 0.0, size, 0.5 * dhat)
    sv[:, 2] += rng.uniform(-0.3, 0.3, len(sv)) * dhat
    mv, mf = _grid_sheet(3, 0.2 * size, 0.8 * size, 0.0)
    bodies = [Body(sv, sf, None, full_space=True), Body(mv, mf, SingleTet(mv))]
    asm = _assemble(bodies)
    q = asm[5].copy()
    dq = rng.normal(0.0, 0.2 * dhat, q.shape)
    return _make(f"longrow{seed}", bodies, q, dq, dhat, 1e3, seed, assembled=asm,
                 meta={"sheet_n": n, "size": size})


# ---------------------------------------------------------------------------
# Config 3: plate over a rack of cylinders
# ---------------------------------------------------------------------------

def config3(seed: int = 0, n_cyl: int = 40, spacing: float = 1.75e-3) -> Scene:
    """Disc plate (R = 0.12 m, 4 mm thick, about 60k triangles) in a
    ~300-node grid, face down over 40 static cylinders (r = 3 mm, L = 0.15 m,
    32 x 77 facets + fan caps = 4,992 triangles each) whose axes run along x
    with an 8 mm pitch in y and whose tops are at z = 0.  Seeded pose: yaw
    U(-1, 1) degrees, tilt giving a height change across the plate of
    U(0, 2 mm), lowest point at a gap dhat U(0.1, 0.9) above z = 0.
    dhat = 2e-4 m, kappa = 1e3."""
    rng = rng_for(seed, 0)
    dhat = 2e-4
    pv, pf = disc_plate_mesh(0.12, 4e-3, spacing)
    yaw = math.radians(rng.uniform(-1.0, 1.0))
    drop = rng.uniform(0.0, 2e-3)
    tilt = math.atan2(drop, 0.24)
    tdir = rng.uniform(0, 2 * math.pi)
    ax = np.array([math.cos(tdir), math.sin(tdir), 0.0])
    # Rodrigues rotation about a horizontal axis, then yaw about z
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Rt = np.eye(3) + math.sin(tilt) * K + (1 - math.cos(tilt)) * K @ K
    Rz = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]])
    pv = pv @ (Rz @ Rt).T
    gap = dhat * rng.uniform(0.1, 0.9)
    pv[:, 2] += gap - pv[:, 2].min()
    grid = padded_grid(pv, near_cubic_dims(pv.max(0) - pv.min(0), 300))
    bodies = [Body(pv, pf, grid)]
    cv, cf = cylinder_mesh(3e-3, 0.15, 32, 77)
    for i in range(n_cyl):
        y = (i - (n_cyl - 1) / 2.0) * 8e-3
        v = cv + np.array([-0.075, y, -3e-3])
        bodies.append(Body(v, cf, None))
    asm = _assemble(bodies)
    q0 = asm[5]
    dq = rng_for(seed, 1).normal(0.0, 2e-4, q0.shape)
    return _make("config3", bodies, q0.copy(), dq, dhat, 1e3, seed, assembled=asm,
                 meta={"yaw_deg": math.degrees(yaw), "drop": drop, "gap": gap,
                       "grid_dims": grid.dims})


# ---------------------------------------------------------------------------
# Config 2 / batch: conformed bubble grasp
# ---------------------------------------------------------------------------

def _real_sh_sum(lmax: int, theta: np.ndarray, phi: np.ndarray, coef: np.ndarray) -> np.ndarray:
    """sum over 1 <= l <= lmax, -l <= m <= l of coef[(l, m)] Y_lm(theta, phi)
    for real spherical harmonics (coefficients in (l, m) order).  Associated
    Legendre functions by the standard three-term recurrence in l."""
    x = np.cos(theta)
    sx = np.sqrt(np.maximum(1.0 - x * x, 0.0))
    P = {}
    pmm = np.ones_like(x)
    for m in range(lmax + 1):
        if m > 0:
            pmm = -pmm * (2 * m - 1) * sx
        P[m, m] = pmm
        if m + 1 <= lmax:
            P[m + 1, m] = x * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[l, m] = ((2 * l - 1) * x * P[l - 1, m] - (l + m - 1) * P[l - 2, m]) / (l - m)
    cosm = [np.cos(m * phi) for m in range(lmax + 1)]
    sinm = [np.sin(m * phi) for m in range(lmax + 1)]
    out = np.zeros_like(x)
    k = 0
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m < 0:
                out += (coef[k] * math.sqrt(2) * norm) * P[l, am] * sinm[am]
            elif m == 0:
                out += (coef[k] * norm) * P[l, 0]
            else:
                out += (coef[k] * math.sqrt(2) * norm) * P[l, am] * cosm[am]
            k += 1
    return out


class Blob:
    """Star-shaped body r(dir) = R0 (1 + sum a_lm Y_lm(dir)), perturbation
    rescaled to a maximum magnitude ``amp`` over a dense direction sample."""

    def __init__(self, rng, r0=0.04, lmax=8, amp=0.10):
        self.r0 = r0
        self.lmax = lmax
        n = sum(2 * l + 1 for l in range(1, lmax + 1))
        self.a = rng.normal(size=n)
        d, _ = geodesic_sphere(24)
        p = self._pert(d)
        self.a *= amp / np.abs(p).max()

    def _pert(self, d):
        th = np.arccos(np.clip(d[:, 2], -1, 1))
        ph = np.arctan2(d[:, 1], d[:, 0])
        return _real_sh_sum(self.lmax, th, ph, self.a)

    def radius(self, d):
        return self.r0 * (1.0 + self._pert(d))

    def inside(self, p: np.ndarray) -> np.ndarray:
        r = np.linalg.norm(p, axis=-1)
        d = p / np.maximum(r, 1e-300)[..., None]
        return r < self.radius(d.reshape(-1, 3)).reshape(r.shape)

    def first_hit(self, origin: np.ndarray, direction: np.ndarray, t_hi: float, n_march: int = 96,
                  n_bisect: int = 60):
        """Smallest t in [0, t_hi] where origin + t dir enters the body:
        a march over all rays at once, then a joint bisection on the first
        bracketing interval (nan where a ray misses)."""
        n = len(origin)
        if n == 0:
            return np.zeros(0)
        ts = np.linspace(0.0, t_hi, n_march)
        P = origin[:, None, :] + ts[None, :, None] * direction[None, None, :]
        ins = self.inside(P)
        first = np.argmax(ins, axis=1)
        hit = ins[np.arange(n), first]
        hit &= first > 0
        lo = np.where(hit, ts[np.maximum(first - 1, 0)], 0.0)
        hi = np.where(hit, ts[first], 0.0)
        for _ in range(n_bisect):
            mid = 0.5 * (lo + hi)
            pm = origin + mid[:, None] * direction
            ins_m = self.inside(pm)
            hi = np.where(ins_m, mid, hi)
            lo = np.where(ins_m, lo, mid)
        return np.where(hit, lo, np.nan)


# barycentric sample points of a triangle (centroid, edge midpoints, inner points)
_FACE_SAMPLES = np.array([[1 / 3, 1 / 3, 1 / 3], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5],
                          [2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])


def mesh_bulge(blob: Blob, v: np.ndarray, f: np.ndarray) -> float:
    """Largest radial distance by which the flat faces of the object mesh
    stand outside the smooth surface (where the surface is concave)."""
    P = np.einsum("sk,fkc->fsc", _FACE_SAMPLES, v[f]).reshape(-1, 3)
    r = np.linalg.norm(P, axis=1)
    return max(0.0, float((r - blob.radius(P / r[:, None])).max()))


def _conformed_finger(blob: Blob, obj_v: np.ndarray, nu: int, semi, side: float,
                      frac: float, dhat: float, rng, clearance: float = 0.0) -> np.ndarray:
    """Ellipsoidal membrane (semi-axes semi = (a_x, a_y, a_z), x the grasp
    axis) on the ``side`` (-1 or +1) of the object along x.  Vertices on the
    object-facing half whose (y, z) lie within ``frac`` of the semi-axes are
    pressed onto the object: moved along x to the object's first-hit surface
    minus a gap dhat U(0.1, 0.9).  Then, so that the flat finger faces do
    not dip into the object, sample points of every facing face must keep
    ``clearance`` above the smooth surface along x: faces short of it push
    their vertices out (repeated until none is).  Returns the conformed
    vertex positions."""
    v_unit, ff = geodesic_sphere(nu)
    v = v_unit * np.asarray(semi)
    facing = (v[:, 0] * -side) > 0  # half pointing at the object
    ell = (v[:, 1] / semi[1]) ** 2 + (v[:, 2] / semi[2]) ** 2
    sel = facing & (ell < frac ** 2)
    # place the finger so its facing apex touches the object's extreme
    ext = obj_v[:, 0].max() if side > 0 else -obj_v[:, 0].min()
    v[:, 0] += side * (ext + semi[0])
    # pressed region: cast rays from the finger toward the object
    o = v[sel].copy()
    o[:, 0] = side * (ext + 0.02)
    direction = np.array([-side, 0.0, 0.0])
    t = blob.first_hit(o, direction, ext + 0.02)
    ok = ~np.isnan(t)
    gap = dhat * rng.uniform(0.1, 0.9, size=ok.sum())
    surf_x = o[ok, 0] - side * t[ok]
    idx = np.nonzero(sel)[0][ok]
    v[idx, 0] = surf_x + side * gap
    # smooth the transition: vertices on the facing half but outside the
    # pressed set must stay outside; push any that crossed back out
    rest = np.nonzero(facing & ~np.isin(np.arange(len(v)), idx))[0]
    if len(rest):
        o2 = v[rest].copy()
        o2[:, 0] = side * (ext + 0.02)
        t2 = blob.first_hit(o2, direction, ext + 0.02)
        hit = ~np.isnan(t2)
        lim = o2[hit, 0] - side * t2[hit] + side * dhat * 2.0
        cur = v[rest[hit], 0]
        bad = (cur - lim) * side < 0
        v[rest[hit][bad], 0] = lim[bad]
    # keep the flat faces outside the object (chords of the conformed
    # surface sag toward it)
    # faces with a pressed vertex (the others stay >= 2 dhat away)
    fsel = ff[np.isin(ff, idx).any(axis=1)]
    need = clearance + 0.05 * dhat
    for _ in range(6):
        if len(fsel) == 0:
            break
        P = np.einsum("sk,fkc->fsc", _FACE_SAMPLES, v[fsel])
        # short rays through each sample point: from 2 mm outside, 6 mm long
        o = P.reshape(-1, 3).copy()
        o[:, 0] += side * 2e-3
        t = blob.first_hit(o, direction, 6e-3, n_march=25, n_bisect=34)
        surf = o[:, 0] - side * t
        clear = ((P.reshape(-1, 3)[:, 0] - surf) * side).reshape(len(fsel), -1)
        short = np.nan_to_num(need - clear, nan=-1.0).max(axis=1)
        if short.max() <= 0.0:
            break
        push = np.zeros(len(v))
        for k in range(3):
            np.maximum.at(push, fsel[:, k], np.maximum(short, 0.0) * 1.05)
        v[:, 0] += side * push
        # only faces touching a moved vertex can have changed
        fsel = ff[(push[ff] > 0).any(axis=1)]
    return v


def grasp_scene(seed: int, obj_nu: int, obj_nodes: int, finger_nu: int,
                finger_semi=(0.015, 0.04, 0.06), finger_dims=(5, 10, 10),
                frac: float = 0.8, dhat: float = 5e-4, kappa: float = 1e3,
                rotate: bool = False, dq_sigma: float = 1e-3, name="grasp",
                r0: float = 0.04) -> Scene:
    rng = rng_for(seed, 0)
    blob = Blob(rng, r0=r0)
    v_unit, of = geodesic_sphere(obj_nu)
    ov = v_unit * blob.radius(v_unit)[:, None]
    clr = 2.0 * mesh_bulge(blob, ov, of)
    f1 = _conformed_finger(blob, ov, finger_nu, finger_semi, -1.0, frac, dhat, rng, clr)
    f2 = _conformed_finger(blob, ov, finger_nu, finger_semi, +1.0, frac, dhat, rng, clr)
    _, ff = geodesic_sphere(finger_nu)
    if rotate:
        R = _random_rotation(rng)
        ov, f1, f2 = ov @ R.T, f1 @ R.T, f2 @ R.T
    og = padded_grid(ov, near_cubic_dims(ov.max(0) - ov.min(0), obj_nodes))
    g1 = padded_grid(f1, finger_dims)
    g2 = padded_grid(f2, finger_dims)
    bodies = [Body(ov, of, og), Body(f1, ff, g1), Body(f2, ff, g2)]
    asm = _assemble(bodies)
    q0 = asm[5]
    dq = rng_for(seed, 1).normal(0.0, dq_sigma, q0.shape)
    return _make(name, bodies, q0.copy(), dq, dhat, kappa, seed, assembled=asm,
                 meta={"obj_nu": obj_nu, "finger_nu": finger_nu, "frac": frac,
                       "obj_grid": og.dims, "finger_grid": finger_dims})


def config2(seed: int = 0, frac: float = 0.75) -> Scene:
    """Bubble-gripper grasp: blob of frequency 71 (100,820 f, r0 = 0.04 m,
    SH order 8, 10 % amplitude) in a ~2,000-node grid, two ellipsoidal
    membranes (semi-axes 0.015 x 0.04 x 0.06 m, x the grasp axis, frequency
    32, 20,480 f each) in 5x10x10-node grids, pressed onto the object over
    ``frac`` of their semi-axes with gaps dhat U(0.1, 0.9).  dhat = 5e-4 m,
    kappa = 1e3, dq ~ N(0, 1e-3 m).  The default closure puts 483,655 pairs
    within dhat at seed 0 (2,453,031 candidates), inside the 1e5 - 5e5 band
    the workload asks for; 0.8 would give 520,384."""
    return grasp_scene(seed, 71, 2000, 32, frac=frac, name="config2")


def batch_scenes(n: int = 256, seed0: int = 0) -> list[Scene]:
    """Ragged grasp batch: object triangle count log-uniform in [2e3, 5e4]
    (frequency round(sqrt(F / 20))), object nodes log-uniform in
    [100, 2000], fingers of frequency 16, random SE(3) orientation, pressed
    fraction log-uniform in [0.1, 0.8] so contact counts spread over orders
    of magnitude."""
    out = []
    for i in range(n):
        rng = rng_for(seed0 + i, 7)
        F = math.exp(rng.uniform(math.log(2e3), math.log(5e4)))
        nu = max(2, int(round(math.sqrt(F / 20.0))))
        nodes = int(round(math.exp(rng.uniform(math.log(100), math.log(2000)))))
        frac = math.exp(rng.uniform(math.log(0.1), math.log(0.8)))
        out.append(grasp_scene(seed0 + i, nu, nodes, 16, frac=frac, rotate=True,
                               name=f"batch{seed0 + i}"))
    return out


# ---------------------------------------------------------------------------
# Inputs of one implicit step on config 1 (the differentiable form)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class StepInputs:
    """Inputs of one implicit time step of the sphere-on-ground scene: the
    contact scene, the coarse grid (rest nodes, tets), seeded interior
    samples of the body with their tet and barycentric weights (each sample
    carries volume V / n_samples: the aggregation of Eq. 15), material and
    time-step parameters, the previous state and a seeded target for the
    loss 1/2 |q* - q_target|^2.  The ground is the kinematic body (empty W
    rows); its rest positions define the pose theta = 0."""
    scene: Scene
    grid_nodes: np.ndarray   # [n_node, 3] rest positions of the coarse nodes
    tets: np.ndarray         # [n_tet, 4] node indices
    sample_tet: np.ndarray   # [n_s] tet of each interior sample
    sample_w: np.ndarray     # [n_s, 4] barycentric weights in that tet
    sample_vol: float        # volume carried by one sample
    young: float
    poisson: float
    rho: float
    g: float
    h: float
    q_n: np.ndarray
    v_n: np.ndarray
    kin_rows: np.ndarray     # vertex indices of the kinematic body
    kin_rest: np.ndarray     # [k, 3]
    q_target: np.ndarray


def step_inputs(seed: int = 0, grid_dims=(5, 5, 5), n_samples: int = 20000, h: float = 0.01,
                young: float = 5e4, poisson: float = 0.45, rho: float = 1e3, g: float = 9.81,
                target_sigma: float = 1e-3) -> StepInputs:
    """Config 1's sphere (r = 0.05 m) in a grid of grid_dims nodes over the
    ground, E = 5e4 Pa, nu = 0.45, rho = 1e3 kg/m^3 (the paper's teddy
    material, Sec. IV-A), h = 0.01 s, gravity along -z, at rest (v_n = 0)."""
    sc = config1(seed, grid_dims=grid_dims)
    v_unit, _ = geodesic_sphere(16)
    r = 0.05
    grid = padded_grid(r * v_unit, grid_dims)
    rng = np.random.Generator(np.random.PCG64([seed, 11]))
    u = rng.normal(size=(n_samples, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    pts = u * (r * rng.uniform(size=(n_samples, 1)) ** (1.0 / 3.0))
    _, w, tet = grid.embed(pts, with_tet=True)
    vol = 4.0 / 3.0 * math.pi * r ** 3
    kin = np.nonzero(np.diff(sc.W_rowptr) == 0)[0]
    q_target = sc.q + np.random.Generator(np.random.PCG64([seed, 12])).normal(0, target_sigma, sc.q.shape)
    return StepInputs(scene=sc, grid_nodes=grid.nodes.copy(), tets=grid.tets.copy(), sample_tet=tet, sample_w=w,
                      sample_vol=vol / n_samples, young=young, poisson=poisson, rho=rho, g=g, h=h,
                      q_n=sc.q.copy(), v_n=np.zeros_like(sc.q), kin_rows=kin, kin_rest=sc.x_off[kin].copy(),
                      q_target=q_target)
