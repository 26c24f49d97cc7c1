"""Pins for the oracle's embedding (Eq. 13-14) and its reduction through
the embedding (Eq. 17), including the paper's two special cases: full-space
IPC (W = I) and the single-tetrahedron affine body."""
import numpy as np
import pytest

import oracle as O
from scenes import config1, tiny_scene
from tests import _geom as G


def test_rest_reproduction_and_partition_of_unity(c1):
    rp, val = c1.W_rowptr, c1.W_val
    rows = np.repeat(np.arange(c1.n_vert), np.diff(rp))
    sums = np.bincount(rows, weights=val, minlength=c1.n_vert)
    dof = np.diff(rp) > 0
    assert np.abs(sums[dof] - 1.0).max() <= 1e-15
    # with the undeformed grid the embedding gives back the rest surface
    from scenes.meshes import geodesic_sphere, padded_grid
    v, _ = geodesic_sphere(16)
    v = 0.05 * v
    grid = padded_grid(v, (5, 5, 5))
    x = O.embed(c1, grid.nodes.reshape(-1), off=None)
    assert np.abs(x[:len(v)] - v).max() <= 4 * np.finfo(float).eps * 0.05


def test_affine_precision(c1):
    rng = np.random.default_rng(0)
    A = np.eye(3) + 0.1 * rng.normal(size=(3, 3))
    t = rng.normal(size=3) * 0.01
    q0 = c1.q.reshape(-1, 3)
    x0 = O.embed(c1, c1.q, off=None)
    x = O.embed(c1, (q0 @ A.T + t).reshape(-1), off=None)
    dof = np.diff(c1.W_rowptr) > 0
    ref = x0 @ A.T + t
    assert np.abs(x[dof] - ref[dof]).max() <= 1e-14 * np.abs(ref).max()


def test_embedding_identity_special_case():
    sc = tiny_scene(5, mode="full_both")
    x = O.embed(sc, sc.q)
    assert np.array_equal(x, sc.q.reshape(-1, 3) + 0.0)


def _dense_reduce(sc, flags=O.ENERGY | O.GRAD | O.HESS | O.PROJECT, q=None):
    q = sc.q if q is None else q
    x = O.embed(sc, q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    return pt, ee, O.barrier_reduce(sc, q, pt, ee, sc.dhat, sc.kappa, flags)


def test_full_space_reduction_equals_per_vertex_sums():
    """W = I: grad_q and hess_q are the full-space per-vertex sums."""
    sc = tiny_scene(2, mode="full_both")
    pt, ee, r = _dense_reduce(sc, O.ENERGY | O.GRAD | O.HESS)
    assert r["n_active"] > 0
    x = O.embed(sc, sc.q)
    g = np.zeros_like(x)
    H = np.zeros((x.size, x.size))
    for kind, lst in ((0, pt), (1, ee)):
        for pr in lst:
            if kind == 0:
                vid = [pr[0], *sc.faces[pr[1]]]
            else:
                vid = [*sc.edges[pr[0]], *sc.edges[pr[1]]]
            st, t, s, e, gk, Hk = O.pair_eval(kind, x[vid].reshape(12), sc.dhat, sc.kappa)
            if st != O.OK:
                continue
            g[vid] += gk.reshape(4, 3)
            idx = np.concatenate([[3 * v, 3 * v + 1, 3 * v + 2] for v in vid])
            H[np.ix_(idx, idx)] += Hk
    assert np.abs(r["grad"] - g.reshape(-1)).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(r["hess"] - H).max() <= 1e-12 * np.abs(H).max()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_momentum_and_translation_invariance(seed):
    sc = tiny_scene(seed, mode="grid")
    pt, ee, r = _dense_reduce(sc)
    assert r["status"] == O.OK and r["n_active"] > 0
    g = r["grad"].reshape(-1, 3)
    gs = np.abs(g).max()
    assert np.abs(g.sum(axis=0)).max() <= 1e-11 * gs
    torque = np.cross(sc.q.reshape(-1, 3), g).sum(axis=0)
    assert np.abs(torque).max() <= 1e-11 * gs * np.abs(sc.q).max()
    H = r["hess"]
    t = np.tile(np.array([0.3, -1.2, 0.7]), sc.n_node)
    assert np.abs(H @ t).max() <= 1e-11 * np.abs(H).max()
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.abs(H).max()


@pytest.mark.parametrize("mode", ["grid", "tet", "static", "full"])
def test_chain_rule_against_energy_differences(mode):
    """grad_q = J^T grad_x and hess_q = J^T hess_x J (Eq. 17) against
    central differences of the total barrier energy in q."""
    sc = tiny_scene(4, mode=mode)
    pt, ee, r = _dense_reduce(sc, O.ENERGY | O.GRAD | O.HESS)
    assert r["n_active"] > 0
    q = sc.q
    h = 1e-7 * sc.dhat
    g = r["grad"]
    H = r["hess"]
    for i in range(len(q)):
        e = np.zeros_like(q)
        e[i] = h
        rp = O.barrier_reduce(sc, q + e, pt, ee, sc.dhat, sc.kappa, O.ENERGY | O.GRAD, hess=False)
        rm = O.barrier_reduce(sc, q - e, pt, ee, sc.dhat, sc.kappa, O.ENERGY | O.GRAD, hess=False)
        assert (rp["energy"] - rm["energy"]) / (2 * h) == pytest.approx(g[i], rel=1e-5, abs=1e-6 * np.abs(g).max())
        assert np.abs((rp["grad"] - rm["grad"]) / (2 * h) - H[i]).max() <= 1e-5 * np.abs(H).max()


def test_single_tet_is_affine_body():
    """One enclosing tetrahedron: 4 nodes, 12 reduced DoF, and every
    surface vertex moves affinely with the nodes."""
    sc = tiny_scene(6, mode="tet")
    nA = sc.meta["n_vert_a"]
    assert sc.n_node == 4
    pt, ee, r = _dense_reduce(sc)
    assert r["hess"].shape == (12, 12)
    rng = np.random.default_rng(0)
    A = np.eye(3) + 0.05 * rng.normal(size=(3, 3))
    q2 = (sc.q.reshape(-1, 3) @ A.T).reshape(-1)
    x = O.embed(sc, sc.q, off=None)[:nA]
    x2 = O.embed(sc, q2, off=None)[:nA]
    assert np.abs(x2 - x @ A.T).max() <= 1e-14


def test_energy_matches_sum_of_barriers(c1):
    x = O.embed(c1, c1.q)
    pt, ee = O.candidates(c1, x, c1.dhat)
    r = O.barrier_reduce(c1, c1.q, pt, ee, c1.dhat, c1.kappa, O.ENERGY, hess=False)
    tot = 0.0
    n = 0
    for kind, lst in ((0, pt), (1, ee)):
        for pr in lst:
            vid = [pr[0], *c1.faces[pr[1]]] if kind == 0 else [*c1.edges[pr[0]], *c1.edges[pr[1]]]
            d = G.pair_distance(kind, x[vid].reshape(12))
            if d < c1.dhat:
                n += 1
                tot += c1.kappa * -((d - c1.dhat) ** 2) * np.log(d / c1.dhat)
    assert r["n_active"] == n
    assert r["energy"] == pytest.approx(tot, rel=1e-9)
