"""Pins for the oracle's pair distances (the d_k of the paper's Sec. III-B,
Eq. 7; the distance itself follows IPC, which the paper defers to)."""
import os

import numpy as np
import pytest

import oracle as O
from tests import _geom as G

HERE = os.path.dirname(__file__)


def _golden_cases():
    rows = []
    with open(os.path.join(HERE, "golden", "distance_cases.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            rows.append((tok[0], np.array([float(t) for t in tok[1:13]]), float(tok[13]), tok[14]))
    return rows


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: f"{c[0]}-{c[3]}")
def test_hand_closed_forms(case):
    kind_s, x12, expected, expected_type = case
    kind = 0 if kind_s == "PT" else 1
    x = x12.reshape(4, 3)
    t = O.pt_type(*x) if kind == 0 else O.ee_type(*x)
    names = O.PT_TYPES if kind == 0 else O.EE_TYPES
    assert names[t] == expected_type
    d = np.sqrt(O.pair_dist2(kind, t, x12))
    assert d == pytest.approx(expected, rel=1e-15)


def _random_pair(rng, kind):
    x = rng.normal(size=(4, 3))
    # mix of scales and near-degenerate layouts
    mode = rng.integers(0, 4)
    if mode == 1:
        x[0] = x[1] + rng.normal(size=3) * 1e-3
    elif mode == 2 and kind == 1:
        d = rng.normal(size=3)
        x[1] = x[0] + d
        x[3] = x[2] + d * rng.uniform(0.5, 2) + rng.normal(size=3) * 1e-7
    elif mode == 3:
        x *= 1e-3
    return x.reshape(12)


@pytest.mark.parametrize("kind", [0, 1])
def test_typed_distance_matches_type_free_definition(kind):
    rng = np.random.default_rng(11 + kind)
    seen = set()
    for _ in range(4000):
        x12 = _random_pair(rng, kind)
        x = x12.reshape(4, 3)
        t = O.pt_type(*x) if kind == 0 else O.ee_type(*x)
        seen.add(t)
        d = np.sqrt(O.pair_dist2(kind, t, x12))
        ref = G.pair_distance(kind, x12)
        scale = np.abs(x12).max()
        assert abs(d - ref) <= 1e-12 * scale + 1e-12 * ref, (t, d, ref)
    assert seen == set(range(7 if kind == 0 else 9))


@pytest.mark.parametrize("kind", [0, 1])
def test_typed_distance_against_dense_sampling(kind):
    rng = np.random.default_rng(5 + kind)
    for _ in range(60):
        x12 = rng.normal(size=12)
        x = x12.reshape(4, 3)
        t = O.pt_type(*x) if kind == 0 else O.ee_type(*x)
        d = np.sqrt(O.pair_dist2(kind, t, x12))
        samp = G.sampled_distance(kind, x12, n=150)
        # the grid minimum is an upper bound within the grid spacing
        assert d <= samp + 1e-12
        assert samp - d <= 0.05 * np.abs(x12).max()


@pytest.mark.parametrize("kind", [0, 1])
def test_distance_rigid_invariance(kind):
    rng = np.random.default_rng(21 + kind)
    for _ in range(500):
        x12 = rng.normal(size=12)
        x = x12.reshape(4, 3)
        t = O.pt_type(*x) if kind == 0 else O.ee_type(*x)
        d = np.sqrt(O.pair_dist2(kind, t, x12))
        R = G.random_rotation(rng)
        y = x @ R.T + rng.normal(size=3)
        ty = O.pt_type(*y) if kind == 0 else O.ee_type(*y)
        dy = np.sqrt(O.pair_dist2(kind, ty, y.reshape(12)))
        assert dy == pytest.approx(d, rel=1e-12, abs=1e-12)


def test_ee_argument_swap():
    rng = np.random.default_rng(3)
    for _ in range(500):
        a0, a1, b0, b1 = rng.normal(size=(4, 3))
        t = O.ee_type(a0, a1, b0, b1)
        d = np.sqrt(O.pair_dist2(1, t, np.concatenate([a0, a1, b0, b1])))
        t2 = O.ee_type(b0, b1, a0, a1)
        d2 = np.sqrt(O.pair_dist2(1, t2, np.concatenate([b0, b1, a0, a1])))
        assert d2 == pytest.approx(d, rel=1e-12)


def test_near_parallel_edges_use_endpoint_types():
    a0, a1 = np.zeros(3), np.array([1.0, 0, 0])
    for ang in [0.0, 1e-12, 1e-11]:
        b0 = np.array([0.3, 0.2, 0.1])
        b1 = b0 + np.array([np.cos(ang), np.sin(ang), 0.0])
        t = O.ee_type(a0, a1, b0, b1)
        assert O.EE_TYPES[t] != "EA-EB"
        d = np.sqrt(O.pair_dist2(1, t, np.concatenate([a0, a1, b0, b1])))
        assert d == pytest.approx(G.segment_segment(a0, a1, b0, b1), rel=1e-12)


@pytest.mark.parametrize("kind,type_", [(0, t) for t in range(7)] + [(1, t) for t in range(9)])
def test_dist2_derivatives_central_differences(kind, type_):
    """Gradient and Hessian of each type's closed form s = d^2 against
    central differences of the value formula."""
    rng = np.random.default_rng(100 + 10 * kind + type_)
    for _ in range(5):
        x12 = rng.normal(size=12)
        s, g, H = O.pair_dist2_derivs(kind, type_, x12)
        assert s == O.pair_dist2(kind, type_, x12)
        h = 1e-6
        gf = np.zeros(12)
        Hf = np.zeros((12, 12))
        for i in range(12):
            e = np.zeros(12)
            e[i] = h
            gf[i] = (O.pair_dist2(kind, type_, x12 + e) - O.pair_dist2(kind, type_, x12 - e)) / (2 * h)
            Hf[i] = (O.pair_dist2_derivs(kind, type_, x12 + e)[1] - O.pair_dist2_derivs(kind, type_, x12 - e)[1]) / (2 * h)
        assert np.abs(g - gf).max() <= 1e-6 * max(1.0, np.abs(g).max())
        assert np.abs(H - Hf).max() <= 1e-6 * max(1.0, np.abs(H).max())
        assert np.abs(H - H.T).max() <= 1e-12 * max(1.0, np.abs(H).max())
        # translation invariance: gradient sums to zero per axis, H kills translations
        assert np.abs(g.reshape(4, 3).sum(axis=0)).max() <= 1e-12 * max(1.0, np.abs(g).max())
        t = np.tile(rng.normal(size=3), 4)
        assert np.abs(H @ t).max() <= 1e-11 * max(1.0, np.abs(H).max())
