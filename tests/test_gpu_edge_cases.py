"""Edge cases on the GPU against the oracle: pairs at d / dhat from 1e-2
down to 1e-8 of every family of distance type (energy, gradient, true and
projected Hessian within 1e-10, types and squared distances bit for bit),
and a scene with degenerate primitives (zero-area triangles, zero-length
edges), whose candidates, barrier terms and step bound match the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from scenes.meshes import unique_edges  # noqa: E402
from scenes.scene import Scene, _random_rotation, _grid_sheet  # noqa: E402

TOL = 1e-10
DHAT = 1e-3
L = 1e-2


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (n if n > 0 else 1.0)


def _full_space(name, verts, faces, dhat=DHAT):
    n = len(verts)
    faces = np.asarray(faces, dtype=np.int32)
    return Scene(name, n, faces, unique_edges(faces), np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                 np.ones(n), None, verts.copy(), verts.reshape(-1).copy(), np.zeros(3 * n), None, dhat, 1e3)


def _tiny_distance_scene(r, seed):
    """Per case two triangles A and B (full-space), B's first vertex or
    first edge at distance r * dhat from A's interior, an edge or a vertex;
    returns the scene and the (kind, pair) list of the cases."""
    rng = np.random.default_rng(seed)
    d = r * DHAT
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=float) * L
    cases = [
        (0, np.array([0.2 * L, 0.3 * L, d])),                       # point over the interior
        (0, np.array([0.5 * L, -d / np.sqrt(2), d / np.sqrt(2)])),  # point off edge t0t1
        (0, -d / np.sqrt(3) * np.ones(3)),                          # point off vertex t0
        (1, np.array([[0.5 * L, -0.5 * L, d], [0.5 * L, 0.5 * L, d]])),       # crossing edges
        (1, np.array([[1.0 * L + d, 0.0, 0.0], [2.0 * L, 0.3 * L, 0.2 * L]])),  # end to end
        (1, np.array([[0.5 * L, 0.0, d], [0.5 * L, 0.7 * L, 0.6 * L]])),      # end onto the interior
    ]
    verts, faces, pairs = [], [], []
    for k, (kind, geo) in enumerate(cases):
        R = _random_rotation(rng)
        c = np.array([3 * L * k, 0.0, 0.0]) + rng.normal(size=3) * L
        base = len(verts)
        A = tri @ R.T + c
        if kind == 0:
            p = geo @ R.T + c
            B = np.array([p, p + R @ np.array([-0.5, -0.5, 1.0]) * L, p + R @ np.array([-0.6, 0.4, 1.2]) * L])
        else:
            a0, a1 = geo[0] @ R.T + c, geo[1] @ R.T + c
            B = np.array([a0, a1, a1 + R @ np.array([0.1, 0.0, 1.0]) * L])
        verts += list(A) + list(B)
        faces += [[base, base + 1, base + 2], [base + 3, base + 4, base + 5]]
        pairs.append((kind, (base + 3, len(faces) - 2) if kind == 0 else None, (base, base + 1, base + 3, base + 4)))
    sc = _full_space(f"tiny_d_{r:g}", np.array(verts), faces)
    out = []
    for kind, pt, ev in pairs:
        if kind == 0:
            out.append((0, np.array(pt, dtype=np.int32)))
        else:
            ea = [i for i, e in enumerate(sc.edges.tolist()) if e == sorted(ev[:2])][0]
            eb = [i for i, e in enumerate(sc.edges.tolist()) if e == sorted(ev[2:])][0]
            out.append((1, np.array(sorted((ea, eb)), dtype=np.int32)))
    return sc, out


@pytest.mark.parametrize("r", [1e-2, 1e-4, 1e-6, 1e-8])
@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_distances_per_pair(ctx, r, seed):
    sc, cases = _tiny_distance_scene(r, seed)
    dsc = E.Scene.from_host(ctx, sc)
    q = _dev(sc.q)
    x = O.embed(sc, sc.q)
    for kind in (0, 1):
        lst = np.array([p for k, p in cases if k == kind], dtype=np.int32)
        for flags in (0, E.PROJECT):
            ty, s2, e, g, H = (t.cpu().numpy() for t in E.pair_eval(ctx, dsc, q, kind, _dev(lst), DHAT, sc.kappa,
                                                                     flags))
            for i, pr in enumerate(lst):
                vid = [pr[0], *sc.faces[pr[1]]] if kind == 0 else [*sc.edges[pr[0]], *sc.edges[pr[1]]]
                st, t, s, er, gr, Hr = O.pair_eval(kind, x[vid].reshape(12), DHAT, sc.kappa)
                assert st == O.OK and ty[i] == t and s2[i] == s
                assert np.sqrt(s) == pytest.approx(r * DHAT, rel=1e-6)
                if flags:
                    Hr, _ = O.project_psd(Hr)
                assert abs(e[i] - er) <= TOL * abs(er)
                assert _rel(g[i], gr) <= TOL
                assert _rel(H[i], Hr) <= TOL, (kind, t, r)


def _degenerate_scene():
    """Isolated degenerate triangles hovering 0.3 dhat over a sheet: three
    with two coincident vertices (a zero-length edge, zero area) and three
    with collinear vertices (zero area), all full-space.  A degenerate
    primitive inside a mesh would touch its neighbours at distance 0, so
    each one is its own body."""
    vb, fb = _grid_sheet(4, 0.0, 4 * L, 0.0)
    rng = np.random.default_rng(2)
    verts, faces = list(vb), [list(f) for f in fb]
    for k in range(6):
        c = np.array([rng.uniform(0.5, 3.5) * L, rng.uniform(0.5, 3.5) * L, 0.3 * DHAT])
        a = rng.normal(size=3) * L * 0.4
        a[2] = 0.0
        p0, p1 = c, c + a
        p2 = p1.copy() if k < 3 else c + rng.uniform(0.2, 0.8) * a
        base = len(verts)
        verts += [p0, p1, p2]
        faces.append([base, base + 1, base + 2])
    sc = _full_space("degenerate", np.array(verts), faces)
    sc.dq = np.random.default_rng(1).normal(0.0, 0.2 * DHAT, sc.q.shape)
    return sc


def test_degenerate_primitives_scene(ctx):
    sc = _degenerate_scene()
    assert np.abs(np.linalg.norm(sc.x_rest[sc.edges[:, 0]] - sc.x_rest[sc.edges[:, 1]], axis=1)).min() == 0.0
    dsc = E.Scene.from_host(ctx, sc)
    q = _dev(sc.q)
    x = O.embed(sc, sc.q)
    opt, oee = O.candidates(sc, x, DHAT)
    pt, ee = E.build_candidates(ctx, dsc, q, DHAT)
    assert np.array_equal(pt.cpu().numpy(), opt) and np.array_equal(ee.cpu().numpy(), oee)
    flags = E.ENERGY | E.GRAD | E.HESS | E.PROJECT
    ref = O.barrier_reduce(sc, sc.q, opt, oee, DHAT, sc.kappa, flags)
    assert ref["status"] == O.OK and ref["n_active"] > 0
    r = E.barrier_reduce(ctx, dsc, q, pt, ee, DHAT, sc.kappa, flags, hess="dense")
    assert r["n_active"] == ref["n_active"]
    assert abs(r["energy"].item() - ref["energy"]) <= TOL * abs(ref["energy"])
    assert _rel(r["grad"].cpu().numpy(), ref["grad"]) <= TOL
    assert _rel(r["hess"].cpu().numpy(), ref["hess"]) <= TOL
    a, n, _ = E.ccd_max_step(ctx, dsc, q, _dev(sc.dq), DHAT)
    a_ref, n_ref, _ = O.ccd_max_step(sc, sc.q, sc.dq, DHAT)
    assert n == n_ref and a == a_ref
