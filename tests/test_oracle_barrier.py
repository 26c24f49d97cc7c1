"""Pins for the log barrier (Eq. 7), the pair energy kappa*b(d) of the
barrier potential (Eq. 10-11) and the EE mollifier."""
import math
import os

import numpy as np
import pytest

import oracle as O
from tests import _geom as G

HERE = os.path.dirname(__file__)


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "barrier_half.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                vals[k] = float(v)
    return vals


@pytest.mark.parametrize("dhat", [1e-3, 5e-4, 2e-4, 1.0])
def test_midpoint_closed_forms(dhat):
    g = _golden()
    b, b1, b2 = O.barrier(0.5 * dhat, dhat)
    assert b / dhat ** 2 == pytest.approx(g["b_over_dhat2"], rel=1e-14)
    assert b1 / dhat == pytest.approx(g["b1_over_dhat"], rel=1e-14)
    assert b2 == pytest.approx(g["b2"], rel=1e-14)


def test_support_and_c2_at_dhat():
    dhat = 1e-3
    for d in [dhat, 1.5 * dhat, 0.0, -1e-4]:
        assert O.barrier(d, dhat) == (0.0, 0.0, 0.0)
    b, b1, b2 = O.barrier(dhat * (1 - 1e-7), dhat)
    assert abs(b) < 1e-19 and abs(b1) < 1e-12 and abs(b2) < 1e-5


def test_sign_and_convexity_on_open_interval():
    dhat = 1e-3
    for r in np.linspace(1e-6, 1 - 1e-6, 2001):
        b, b1, b2 = O.barrier(r * dhat, dhat)
        assert b > 0 and b1 < 0 and b2 > 0


def test_barrier_derivatives_by_differences():
    dhat = 1e-3
    for r in [0.01, 0.2, 0.5, 0.9]:
        d = r * dhat
        h = 1e-7 * dhat
        _, b1, b2 = O.barrier(d, dhat)
        bp = O.barrier(d + h, dhat)
        bm = O.barrier(d - h, dhat)
        assert (bp[0] - bm[0]) / (2 * h) == pytest.approx(b1, rel=1e-6)
        assert (bp[1] - bm[1]) / (2 * h) == pytest.approx(b2, rel=1e-6)


def test_barrier_against_definition():
    dhat = 2e-4
    for d in np.linspace(1e-6, dhat * 0.999, 50):
        b = O.barrier(d, dhat)[0]
        assert b == pytest.approx(-((d - dhat) ** 2) * math.log(d / dhat), rel=1e-13)


def test_mollifier_c1_at_eps():
    eps = 3e-7
    m, m1, m2 = O.mollifier(eps * (1 - 1e-12), eps)
    assert m == pytest.approx(1.0, abs=1e-12) and abs(m1) < 1e-6 / eps
    assert O.mollifier(eps, eps) == (1.0, 0.0, 0.0)
    assert O.mollifier(0.0, eps)[0] == 0.0
    for c in np.linspace(0, eps, 20)[1:-1]:
        m, m1, _ = O.mollifier(c, eps)
        h = 1e-6 * eps
        assert (O.mollifier(c + h, eps)[0] - O.mollifier(c - h, eps)[0]) / (2 * h) == pytest.approx(m1, rel=1e-6)


def _close_pair(rng, kind, dhat):
    """A random pair at distance ~U(0.1, 0.9) dhat."""
    for _ in range(1000):
        x = rng.normal(size=(4, 3)) * 1e-2
        d = G.pair_distance(kind, x.reshape(12))
        target = dhat * rng.uniform(0.1, 0.9)
        # move the first primitive toward the second along the closest direction
        # by scaling the configuration about the second primitive's centroid
        if kind == 0:
            c = x[1:].mean(axis=0)
            for _ in range(60):
                dd = G.pair_distance(kind, x.reshape(12))
                if abs(dd - target) < 0.05 * dhat:
                    break
                x[0] = c + (x[0] - c) * (1 - (dd - target) / max(np.linalg.norm(x[0] - c), 1e-30))
        else:
            c = x[2:].mean(axis=0)
            for _ in range(60):
                dd = G.pair_distance(kind, x.reshape(12))
                if abs(dd - target) < 0.05 * dhat:
                    break
                m = x[:2].mean(axis=0)
                shift = (c - m) / np.linalg.norm(c - m) * (dd - target) * 0.9
                x[:2] += shift
        d = G.pair_distance(kind, x.reshape(12))
        if 0.05 * dhat < d < 0.95 * dhat:
            return x.reshape(12)
    raise RuntimeError("could not place pair")


@pytest.mark.parametrize("kind,moll", [(0, False), (1, False), (1, True)])
def test_pair_energy_gradient_and_hessian_by_differences(kind, moll):
    rng = np.random.default_rng(7 + kind + 3 * moll)
    dhat, kappa = 1e-3, 1e3
    for _ in range(8):
        x12 = _close_pair(rng, kind, dhat)
        rest = None
        if moll:
            # rest edges nearly as they are now but the current edges
            # made close to parallel so c < eps_x
            x = x12.reshape(4, 3).copy()
            u = x[1] - x[0]
            v = x[3] - x[2]
            x[3] = x[2] + u / np.linalg.norm(u) * np.linalg.norm(v) + rng.normal(size=3) * 1e-4 * np.linalg.norm(v)
            x12 = x.reshape(12)
            if not (0 < G.pair_distance(1, x12) < dhat):
                continue
            rest = x12 * 1.0 + rng.normal(size=12) * 1e-3
        st, t, s, e, g, H = O.pair_eval(kind, x12, dhat, kappa, rest12=rest)
        assert st == O.OK
        assert np.sqrt(s) == pytest.approx(G.pair_distance(kind, x12), rel=1e-10)
        b = O.barrier(np.sqrt(s), dhat)[0]
        if not moll:
            assert e == pytest.approx(kappa * b, rel=1e-14)
        h = 1e-7 * dhat
        gf = np.zeros(12)
        Hf = np.zeros((12, 12))
        for i in range(12):
            d = np.zeros(12)
            d[i] = h
            ep = O.pair_eval(kind, x12 + d, dhat, kappa, rest12=rest)
            em = O.pair_eval(kind, x12 - d, dhat, kappa, rest12=rest)
            if ep[1] != t or em[1] != t:
                continue  # crossed a type boundary: skip this coordinate
            gf[i] = (ep[3] - em[3]) / (2 * h)
            Hf[i] = (ep[4] - em[4]) / (2 * h)
            assert gf[i] == pytest.approx(g[i], rel=1e-5, abs=1e-6 * np.abs(g).max())
            assert np.abs(Hf[i] - H[i]).max() <= 1e-5 * np.abs(H).max()
        assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()


def test_mollified_energy_is_product():
    rng = np.random.default_rng(2)
    dhat, kappa = 1e-3, 1e3
    a0 = np.zeros(3)
    a1 = np.array([1e-2, 0, 0])
    b0 = np.array([2e-3, 1e-4, 4e-4])
    b1 = b0 + np.array([1e-2, 2e-5, 0])
    x12 = np.concatenate([a0, a1, b0, b1])
    rest = x12 + rng.normal(size=12) * 1e-5
    st, t, s, e, g, H = O.pair_eval(1, x12, dhat, kappa, rest12=rest)
    u, v = a1 - a0, b1 - b0
    c = np.linalg.norm(np.cross(u, v)) ** 2
    ru, rv = rest[3:6] - rest[0:3], rest[9:12] - rest[6:9]
    eps = 1e-3 * (ru @ ru) * (rv @ rv)
    assert c < eps
    m = (2 - c / eps) * (c / eps)
    b = O.barrier(G.pair_distance(1, x12), dhat)[0]
    assert e == pytest.approx(kappa * m * b, rel=1e-9)
