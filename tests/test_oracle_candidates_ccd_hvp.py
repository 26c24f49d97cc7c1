"""Pins for the oracle's candidate set (pair set B of Sec. III-B), its
conservative CCD step bound (Sec. III-C) and its Hessian-vector product."""
import numpy as np
import pytest

import oracle as O
from scenes import tiny_scene
from scenes.scene import Scene
from tests import _geom as G


def _hand_scene():
    """Two triangles over a third; dhat = 0.1.  Hand-listed candidates."""
    v = np.array([
        [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0],      # T0 (static)
        [0.2, 0.2, 0.05], [0.6, 0.2, 0.05], [0.2, 0.6, 0.05],   # T1 just above T0
        [5.0, 5.0, 5.0], [6.0, 5.0, 5.0], [5.0, 6.0, 5.0],      # T2 far away
    ])
    faces = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], dtype=np.int32)
    from scenes.meshes import unique_edges
    edges = unique_edges(faces)
    rowptr = np.array([0, 0, 0, 0, 1, 2, 3, 4, 5, 6], dtype=np.int32)
    col = np.arange(6, dtype=np.int32)
    val = np.ones(6)
    x_off = np.zeros((9, 3))
    x_off[:3] = v[:3]
    q = v[3:].reshape(-1)
    return Scene("hand", 6, faces, edges, rowptr, col, val, x_off, v.copy(), q.copy(),
                 np.zeros_like(q), None, 0.1, 1.0)


def test_hand_listed_candidates():
    """Boxes by hand (h = dhat/2 = 0.05):
    T0 edges (z in [-.05,.05]): e0=(0,1) y in [-.05,.05]; e1=(0,2) x in
    [-.05,.05]; e2=(1,2) x,y in [-.05,1.05].  T1 edges (z in [0,.1]):
    e3=(3,4) x [.15,.65] y [.15,.25]; e4=(3,5) x [.15,.25] y [.15,.65];
    e5=(4,5) x,y [.15,.65].  Only e2 reaches T1's edges; edges of one
    triangle share vertices; T2 is far.  PT: the three T1 vertices over
    face 0; T0's corner boxes miss face 1's box [.15,.65]^2."""
    sc = _hand_scene()
    assert sc.edges.tolist() == [[0, 1], [0, 2], [1, 2], [3, 4], [3, 5], [4, 5],
                                 [6, 7], [6, 8], [7, 8]]
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    assert pt.tolist() == [[3, 0], [4, 0], [5, 0]]
    assert ee.tolist() == [[2, 3], [2, 4], [2, 5]]
    # the same scene with T1 lifted by 0.11 leaves no candidate at all
    sc.q = sc.q + np.tile([0.0, 0.0, 0.11], 6)
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    assert len(pt) == 0 and len(ee) == 0


@pytest.mark.parametrize("seed", range(6))
def test_candidates_rules_and_superset(seed):
    sc = tiny_scene(seed, mode=["grid", "static", "full"][seed % 3])
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    dof = np.diff(sc.W_rowptr) > 0
    # ordering and exclusion rules
    assert np.all(np.diff(pt[:, 0].astype(np.int64) * 2 ** 32 + pt[:, 1]) > 0)
    assert np.all(np.diff(ee[:, 0].astype(np.int64) * 2 ** 32 + ee[:, 1]) > 0)
    assert np.all(ee[:, 0] < ee[:, 1])
    for v, f in pt:
        assert v not in sc.faces[f]
        assert dof[[v, *sc.faces[f]]].any()
    for a, b in ee:
        assert not set(sc.edges[a]) & set(sc.edges[b])
    # superset: every pair closer than dhat is a candidate
    ptset = {tuple(r) for r in pt.tolist()}
    eeset = {tuple(r) for r in ee.tolist()}
    for v in range(sc.n_vert):
        for f in range(sc.n_face):
            if v in sc.faces[f] or not dof[[v, *sc.faces[f]]].any():
                continue
            if G.pair_distance(0, x[[v, *sc.faces[f]]].reshape(12)) < sc.dhat:
                assert (v, f) in ptset
    for a in range(sc.n_edge):
        for b in range(a + 1, sc.n_edge):
            vs = [*sc.edges[a], *sc.edges[b]]
            if len(set(vs)) < 4 or not dof[vs].any():
                continue
            if G.pair_distance(1, x[vs].reshape(12)) < sc.dhat:
                assert (a, b) in eeset


def test_ccd_closed_form_normal_approach():
    """A point above the triangle (0,0,0),(1,0,0),(0,1,0) falling straight
    down at speed v: the bound is exactly (1 - s) d0 / v."""
    s = 0.1
    for d0, v in [(0.5, 1.0), (1e-3, 0.37), (2.0, 5.0)]:
        x12 = np.array([0.25, 0.25, d0, 0, 0, 0, 1, 0, 0, 0, 1, 0], dtype=float)
        p12 = np.zeros(12)
        p12[2] = -v
        t, it = O.accd_pair(0, x12, p12, s=s, t_c=10.0)
        assert t == pytest.approx((1 - s) * d0 / v, rel=1e-15)
        assert it == 2


def test_ccd_zero_motion_and_cap():
    x12 = np.array([0.25, 0.25, 0.1, 0, 0, 0, 1, 0, 0, 0, 1, 0], dtype=float)
    assert O.accd_pair(0, x12, np.zeros(12))[0] == 1.0
    # a translation of everything is no relative motion
    assert O.accd_pair(0, x12, np.tile([0.3, -2.0, 1.0], 4))[0] == 1.0
    p12 = np.zeros(12)
    p12[2] = -1.0
    t, it = O.accd_pair(0, x12, p12, max_iter=1)
    assert it == 1 and 0 < t <= 0.09 + 1e-15


def _first_contact(kind, x12, p12, t_hi, n=2000):
    """Brute-force first time of contact on [0, t_hi]: dense scan of the
    type-free distance d(t); every local minimum is refined by golden-section
    search and counts as contact when it reaches 1e-10 of the scale."""
    ts = np.linspace(0.0, t_hi, n + 1)
    d = np.array([G.pair_distance(kind, x12 + t * p12) for t in ts])
    scale = np.abs(x12).max() + np.abs(p12).max()
    gr = (5 ** 0.5 - 1) / 2
    for i in range(1, n):
        if d[i] <= d[i - 1] and d[i] <= d[i + 1]:
            a, b = ts[i - 1], ts[i + 1]
            for _ in range(80):
                c1 = b - gr * (b - a)
                c2 = a + gr * (b - a)
                if G.pair_distance(kind, x12 + c1 * p12) < G.pair_distance(kind, x12 + c2 * p12):
                    b = c2
                else:
                    a = c1
            tm = 0.5 * (a + b)
            if G.pair_distance(kind, x12 + tm * p12) <= 1e-10 * scale:
                return tm
    if d[-1] <= 1e-10 * scale:
        return t_hi
    return np.inf


@pytest.mark.parametrize("kind", [0, 1])
def test_ccd_is_conservative_on_random_pairs(kind):
    rng = np.random.default_rng(30 + kind)
    hits = 0
    for _ in range(60):
        x12 = rng.normal(size=12)
        p12 = rng.normal(size=12) * 0.1
        # aim the first primitive at the second so many cases collide
        if kind == 0:
            tgt = x12[3:].reshape(3, 3).mean(axis=0)
            p12[:3] = (tgt - x12[:3]) * rng.uniform(0.5, 2.0) + rng.normal(size=3) * 0.05
        else:
            tgt = x12[6:].reshape(2, 3).mean(axis=0)
            m = x12[:6].reshape(2, 3).mean(axis=0)
            p12[:6] = np.tile((tgt - m) * rng.uniform(0.5, 2.0), 2) + rng.normal(size=6) * 0.05
        t, it = O.accd_pair(kind, x12, p12, t_c=1.0)
        toi = _first_contact(kind, x12, p12, 1.0)
        assert t <= toi
        if toi < np.inf:
            hits += 1
            assert t > 0
        # sampled motion over [0, t] never touches
        for tau in np.linspace(0, t, 200):
            assert G.pair_distance(kind, x12 + tau * p12) > 0
    assert hits > 10


def test_ccd_scene_bound_properties():
    sc = tiny_scene(1, mode="grid")
    a, nc, ncap = O.ccd_max_step(sc, sc.q, sc.dq, sc.dhat)
    assert nc > 0 and 0 < a <= 1.0 and ncap == 0
    assert O.ccd_max_step(sc, sc.q, np.zeros_like(sc.dq), sc.dhat)[0] == 1.0
    # rigid translation of the whole scene (nodes and the static offsets)
    shift = np.array([0.01, -0.02, 0.005])
    sc2 = tiny_scene(1, mode="grid")
    sc2.q = (sc.q.reshape(-1, 3) + shift).reshape(-1)
    a2 = O.ccd_max_step(sc2, sc2.q, sc2.dq, sc2.dhat)[0]
    assert a2 == pytest.approx(a, rel=1e-9)


@pytest.mark.parametrize("seed", [0, 3])
def test_hvp_matches_dense_and_differences(seed):
    sc = tiny_scene(seed, mode="grid")
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3 * sc.n_node)
    w = rng.normal(size=3 * sc.n_node)
    rP = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, O.ENERGY | O.GRAD | O.HESS | O.PROJECT)
    st, hv, _ = O.barrier_hvp(sc, sc.q, pt, ee, sc.dhat, sc.kappa, O.PROJECT, v)
    assert st == O.OK
    assert np.linalg.norm(hv - rP["hess"] @ v) <= 1e-12 * np.linalg.norm(hv)
    # true Hessian: symmetric and equal to differences of the gradient
    st, hv, _ = O.barrier_hvp(sc, sc.q, pt, ee, sc.dhat, sc.kappa, 0, v)
    st, hw, _ = O.barrier_hvp(sc, sc.q, pt, ee, sc.dhat, sc.kappa, 0, w)
    assert w @ hv == pytest.approx(v @ hw, rel=1e-10)
    eps = 1e-7 * sc.dhat / np.abs(v).max()
    gp = O.barrier_reduce(sc, sc.q + eps * v, pt, ee, sc.dhat, sc.kappa, O.GRAD, hess=False)["grad"]
    gm = O.barrier_reduce(sc, sc.q - eps * v, pt, ee, sc.dhat, sc.kappa, O.GRAD, hess=False)["grad"]
    assert np.linalg.norm((gp - gm) / (2 * eps) - hv) <= 1e-5 * np.linalg.norm(hv)


def test_hvp_kinematic_rows():
    """out_off collects the unreduced per-vertex H z; its DoF rows reduce
    through W to the reduced product."""
    sc = tiny_scene(2, mode="static")
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    rng = np.random.default_rng(9)
    v = rng.normal(size=3 * sc.n_node)
    v_off = rng.normal(size=(sc.n_vert, 3))
    st, hv, off = O.barrier_hvp(sc, sc.q, pt, ee, sc.dhat, sc.kappa, 0, v, v_off, want_off=True)
    red = np.zeros_like(hv).reshape(-1, 3)
    rows = np.repeat(np.arange(sc.n_vert), np.diff(sc.W_rowptr))
    np.add.at(red, sc.W_col, sc.W_val[:, None] * off[rows])
    assert np.abs(red.reshape(-1) - hv).max() <= 1e-12 * np.abs(hv).max()
