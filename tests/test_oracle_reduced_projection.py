"""Pins for the oracle's alternative projection (PROJECT_REDUCED): each
pair's reduced local block W_k^T H_k W_k (over the pair's distinct nodes)
is projected onto the PSD cone instead of its 12x12 Hessian H_k.

Pinned by the full-space special case (W = I: the reduced block is the
12x12 Hessian, so the result is the per-pair projection), by a single pair
against numpy's symmetric eigendecomposition of its true reduced Hessian
(V max(L, 0) V^T), positive semidefiniteness of the summed result, the
unchanged gradient, and a difference from the per-pair projection under a
coarse embedding (config 1)."""
import numpy as np
import pytest

import oracle as O
from scenes import tiny_scene

F = O.ENERGY | O.GRAD | O.HESS


def _lists(sc):
    return O.candidates(sc, O.embed(sc, sc.q), sc.dhat)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("seed", range(4))
def test_full_space_equals_per_pair_projection(seed):
    sc = tiny_scene(seed, mode="full_both")
    pt, ee = _lists(sc)
    red = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, F | O.PROJECT_REDUCED)
    per = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, F | O.PROJECT)
    assert red["n_active"] == per["n_active"] > 0
    assert _rel(red["hess"], per["hess"]) <= 1e-12
    assert _rel(red["grad"], per["grad"]) <= 1e-15


@pytest.mark.parametrize("kind", [0, 1])
def test_single_pair_is_the_clamped_eigendecomposition(c1, kind):
    # config 1's active pairs cover the point-line and interior types (the
    # tiny scenes' active pairs are all point-point)
    x = O.embed(c1, c1.q)
    lst = _lists(c1)[kind]
    ty, _, act = O.narrow(c1, x, kind, lst, c1.dhat)
    done = {}
    empty = np.zeros((0, 2), np.int32)
    for k in np.nonzero(act)[0]:
        if done.get(ty[k], 0) >= 2:
            continue
        one = lst[k:k + 1]
        args = (one, empty) if kind == 0 else (empty, one)
        true = O.barrier_reduce(c1, c1.q, *args, c1.dhat, c1.kappa, O.HESS)
        red = O.barrier_reduce(c1, c1.q, *args, c1.dhat, c1.kappa, O.HESS | O.PROJECT_REDUCED)
        K = true["hess"]
        lam, V = np.linalg.eigh(0.5 * (K + K.T))
        ref = (V * np.maximum(lam, 0.0)) @ V.T
        assert np.linalg.norm(red["hess"] - ref) <= 1e-11 * np.abs(lam).max()
        done[ty[k]] = done.get(ty[k], 0) + 1
    assert len(done) >= 2


@pytest.mark.parametrize("seed,mode", [(0, "grid"), (1, "tet"), (2, "static")])
def test_sum_is_psd_and_gradient_unchanged(seed, mode):
    sc = tiny_scene(seed, mode=mode)
    pt, ee = _lists(sc)
    red = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, F | O.PROJECT_REDUCED)
    per = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, F | O.PROJECT)
    H = red["hess"]
    lam = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert lam.min() >= -1e-12 * np.abs(lam).max()
    assert np.array_equal(red["grad"], per["grad"]) and red["energy"] == per["energy"]


def test_differs_from_the_per_pair_projection(c1):
    # Point-point pairs (X = e e^T (x) H3) project the same either way; the
    # tiny scenes' active pairs are of that kind.  On config 1 the point-line
    # and interior pairs make the two projections differ.
    pt, ee = _lists(c1)
    red = O.barrier_reduce(c1, c1.q, pt, ee, c1.dhat, c1.kappa, F | O.PROJECT_REDUCED)
    per = O.barrier_reduce(c1, c1.q, pt, ee, c1.dhat, c1.kappa, F | O.PROJECT)
    assert _rel(red["hess"], per["hess"]) > 1e-4
    lam = np.linalg.eigvalsh(red["hess"])
    assert lam.min() >= -1e-12 * np.abs(lam).max()
