"""Pins for the oracle's large-scene tools and for its swept candidate
predicate (the pair set B of Sec. III-B, widened to the motion of a Newton
step for the CCD bound of Sec. III-C).

* The uniform-grid broad phase must give exactly the brute-force pairs, in
  the same order, at positions and over swept boxes.
* The swept predicate must catch a pair only because of where it ends up
  (hand-listed), and every pair whose linear motion over the step comes
  within dhat (sampled) must be a swept candidate.
* The block-sparse reduction must equal the dense reduction (Eq. 17) bit
  for bit when run as one call, and be symmetric with sorted columns.
"""
import numpy as np
import pytest

import oracle as O
from scenes import config1, tiny_scene
from scenes.meshes import unique_edges
from scenes.scene import Scene
from tests import _geom as G

MODES = ["grid", "static", "full", "full_both", "tet"]


def _swept_end(sc, scale=1.0):
    x = O.embed(sc, sc.q)
    p = O.embed(sc, scale * sc.dq, off=sc.dx_off)
    return x, x + p, p


@pytest.mark.parametrize("seed", range(40))
def test_grid_equals_brute_force_tiny(seed):
    sc = tiny_scene(seed, mode=MODES[seed % 5])
    x, x1, _ = _swept_end(sc, scale=0.2)
    for end in (None, x1):
        pt, ee = O.candidates(sc, x, sc.dhat, x1=end)
        for cell in (0.0, 0.5 * sc.dhat, 50 * sc.dhat):
            gpt, gee = O.candidates_grid(sc, x, sc.dhat, x1=end, cell=cell, nthreads=3)
            assert np.array_equal(pt, gpt) and np.array_equal(ee, gee), (seed, cell, end is None)


def test_grid_equals_brute_force_config1(c1):
    x, x1, _ = _swept_end(c1)
    for end in (None, x1):
        pt, ee = O.candidates(c1, x, c1.dhat, x1=end)
        gpt, gee = O.candidates_grid(c1, x, c1.dhat, x1=end)
        assert len(pt) > 100 and len(ee) > 1000
        assert np.array_equal(pt, gpt) and np.array_equal(ee, gee)


def _swept_hand_scene():
    """A static triangle in z = 0 and a free triangle (full-space rows)
    far above it; dhat = 0.125.  At rest no box overlaps; the step moves the
    free triangle down through the static one."""
    v = np.array([
        [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0],     # static
        [0.2, 0.2, 2.0], [0.6, 0.2, 2.0], [0.2, 0.6, 2.0],     # free, 2 m above
    ])
    faces = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    edges = unique_edges(faces)
    rowptr = np.array([0, 0, 0, 0, 1, 2, 3], dtype=np.int32)
    col = np.arange(3, dtype=np.int32)
    val = np.ones(3)
    x_off = np.zeros((6, 3))
    x_off[:3] = v[:3]
    q = v[3:].reshape(-1).copy()
    return Scene("swept_hand", 3, faces, edges, rowptr, col, val, x_off, v.copy(), q,
                 np.zeros_like(q), None, 0.125, 1.0)


def test_swept_candidates_hand_listed():
    """Boxes by hand (h = dhat/2 = 0.0625; every number below is exact in
    binary).  At q the free triangle's boxes sit at z in [1.9375, 2.0625]:
    nothing overlaps the static boxes (z in [-0.0625, 0.0625]).  With a
    step of -2.0 in z every free box spans z in [-0.0625, 2.0625] (start
    and end), so the swept set holds the pairs whose xy boxes meet:
    PT: the free vertices 3, 4, 5 over face 0 (xy [-0.0625, 1.0625]^2);
    the static vertices 0, 1, 2 miss face 1's xy box [0.1375, 0.6625]^2.
    EE: static edge (1,2) (the hypotenuse, x, y in [-0.0625, 1.0625])
    meets every free edge; edge (0,1) (y in [-0.0625, 0.0625]) and edge
    (0,2) (x in [-0.0625, 0.0625]) miss them (free edges have x, y >=
    0.1375).  Edges are numbered (0,1)=0, (0,2)=1, (1,2)=2, (3,4)=3,
    (3,5)=4, (4,5)=5.  A step of -1.875 ends the free boxes at z = 0.0625,
    touching the static ones (closed intervals keep the set); -1.75 ends
    them at z = 0.1875 and leaves nothing."""
    sc = _swept_hand_scene()
    assert sc.edges.tolist() == [[0, 1], [0, 2], [1, 2], [3, 4], [3, 5], [4, 5]]
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    assert len(pt) == 0 and len(ee) == 0
    for dz, expect in ((-2.0, True), (-1.875, True), (-1.75, False)):
        p = np.zeros((6, 3))
        p[3:, 2] = dz
        pt, ee = O.candidates(sc, x, sc.dhat, x1=x + p)
        gpt, gee = O.candidates_grid(sc, x, sc.dhat, x1=x + p)
        assert np.array_equal(pt, gpt) and np.array_equal(ee, gee)
        if expect:
            assert pt.tolist() == [[3, 0], [4, 0], [5, 0]], dz
            assert ee.tolist() == [[2, 3], [2, 4], [2, 5]], dz
        else:
            assert len(pt) == 0 and len(ee) == 0, dz
        # the per-query forms agree with the whole-set form
        for v in range(6):
            assert O.pt_query(sc, x, sc.dhat, v, x1=x + p).tolist() == [f for vv, f in pt if vv == v]


def _ball_gap(x, x1, vid_a, vid_b):
    """Lower bound of the distance between two primitives at every t in
    [0, 1] under linear motion: each primitive stays inside the ball around
    the mean of its start and end vertices that holds them all, so the
    distance is at least the gap between the two balls."""
    def ball(vid):
        pts = np.concatenate([x[vid], x1[vid]], axis=1)  # [n, 2k, 3]
        c = pts.mean(axis=1)
        r = np.linalg.norm(pts - c[:, None, :], axis=2).max(axis=1)
        return c, r
    ca, ra = ball(vid_a)
    cb, rb = ball(vid_b)
    return np.linalg.norm(ca - cb, axis=1) - ra - rb


@pytest.mark.parametrize("seed", range(8))
def test_swept_superset_of_sampled_motion(seed):
    """Every pair whose linear motion x + t p, t in [0, 1], comes within
    dhat at a sampled t is a swept candidate (its boxes at t, widened by
    dhat/2, overlap and lie inside the swept boxes); and the swept set
    contains the candidate sets at the start and at the end.  Pairs whose
    bounding balls stay dhat apart cannot come within dhat and are not
    sampled."""
    sc = tiny_scene(seed, mode=MODES[seed % 5])
    x, x1, p = _swept_end(sc, scale=0.05)
    spt, see = O.candidates(sc, x, sc.dhat, x1=x1)
    sp = {tuple(r) for r in spt.tolist()}
    se = {tuple(r) for r in see.tolist()}
    for pos in (x, x1):
        pt, ee = O.candidates(sc, pos, sc.dhat)
        assert {tuple(r) for r in pt.tolist()} <= sp
        assert {tuple(r) for r in ee.tolist()} <= se
    dof = np.diff(sc.W_rowptr) > 0
    ts = np.linspace(0.0, 1.0, 33)
    # all PT and EE pairs of the rules, then the ball filter
    V, F = np.meshgrid(np.arange(sc.n_vert), np.arange(sc.n_face), indexing="ij")
    V, F = V.ravel(), F.ravel()
    fv = sc.faces[F]
    keep = ~(fv == V[:, None]).any(axis=1) & (dof[V] | dof[fv].any(axis=1))
    V, F = V[keep], F[keep]
    near = _ball_gap(x, x1, V[:, None], sc.faces[F]) < sc.dhat
    hits = 0
    for v, f in zip(V[near], F[near]):
        vid = [v, *sc.faces[f]]
        if min(G.pair_distance(0, (x[vid] + t * p[vid]).reshape(12)) for t in ts) < sc.dhat:
            hits += 1
            assert (v, f) in sp
    A, B = np.triu_indices(sc.n_edge, 1)
    ea, eb = sc.edges[A], sc.edges[B]
    keep = ~((ea[:, :, None] == eb[:, None, :]).any(axis=(1, 2))) & (dof[ea].any(axis=1) | dof[eb].any(axis=1))
    A, B = A[keep], B[keep]
    near = _ball_gap(x, x1, sc.edges[A], sc.edges[B]) < sc.dhat
    for a, b in zip(A[near], B[near]):
        vid = [*sc.edges[a], *sc.edges[b]]
        if min(G.pair_distance(1, (x[vid] + t * p[vid]).reshape(12)) for t in ts) < sc.dhat:
            hits += 1
            assert (a, b) in se
    assert hits > 0


def _dense(b, n_node):
    H = np.zeros((3 * n_node, 3 * n_node))
    for I in range(n_node):
        for k in range(b["rowptr"][I], b["rowptr"][I + 1]):
            J = b["col"][k]
            H[3 * I:3 * I + 3, 3 * J:3 * J + 3] = b["blocks"][k]
    return H


@pytest.mark.parametrize("seed", range(10))
def test_bsr_reduction_equals_dense_tiny(seed):
    sc = tiny_scene(seed, mode=MODES[seed % 5])
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    for flags in (O.ENERGY | O.GRAD | O.HESS | O.PROJECT, O.ENERGY | O.GRAD | O.HESS):
        ref = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags)
        b = O.barrier_reduce_bsr(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags, nthreads=1)
        assert b["status"] == ref["status"] == O.OK and b["n_active"] == ref["n_active"]
        assert b["energy"] == ref["energy"]
        assert np.array_equal(b["grad"], ref["grad"])
        H = _dense(b, sc.n_node)
        assert np.array_equal(H, ref["hess"])
        # pattern: every nonzero block of the dense result is listed once,
        # columns sorted, both triangles
        for I in range(sc.n_node):
            cols = b["col"][b["rowptr"][I]:b["rowptr"][I + 1]]
            assert np.all(np.diff(cols) > 0)
        nz = np.abs(ref["hess"]).reshape(sc.n_node, 3, sc.n_node, 3).sum(axis=(1, 3)) > 0
        listed = np.zeros_like(nz)
        for I in range(sc.n_node):
            listed[I, b["col"][b["rowptr"][I]:b["rowptr"][I + 1]]] = True
        assert np.all(listed[nz]) and np.array_equal(listed, listed.T)


def test_bsr_reduction_config1_threads(c1):
    """Sliced over threads the sums change only by rounding."""
    x = O.embed(c1, c1.q)
    pt, ee = O.candidates_grid(c1, x, c1.dhat)
    flags = O.ENERGY | O.GRAD | O.HESS | O.PROJECT
    ref = O.barrier_reduce(c1, c1.q, pt, ee, c1.dhat, c1.kappa, flags)
    one = O.barrier_reduce_bsr(c1, c1.q, pt, ee, c1.dhat, c1.kappa, flags, nthreads=1)
    many = O.barrier_reduce_bsr(c1, c1.q, pt, ee, c1.dhat, c1.kappa, flags, nthreads=4)
    assert np.array_equal(_dense(one, c1.n_node), ref["hess"])
    Hm = _dense(many, c1.n_node)
    assert np.linalg.norm(Hm - ref["hess"]) <= 1e-14 * np.linalg.norm(ref["hess"])
    assert np.linalg.norm(many["grad"] - ref["grad"]) <= 1e-14 * np.linalg.norm(ref["grad"])
    assert abs(many["energy"] - ref["energy"]) <= 1e-14 * abs(ref["energy"])
    assert many["n_active"] == ref["n_active"]
