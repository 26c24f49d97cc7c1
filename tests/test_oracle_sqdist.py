"""Pins for the oracle's alternative barrier formulation (SQDIST): the log
barrier of Eq. 7 written in the squared distance, b(s) = -(s - shat)^2
ln(s / shat) with s = d^2 and shat = dhat^2.

Pinned by its closed-form values at s = shat / 2, its vanishing with its
first two derivatives at shat, convexity and monotonicity on (0, shat),
differences of b and of its derivatives, a pair's energy at a distance
fixed by construction, pair gradients and Hessians against central
differences, the reduced gradient against differences of the total
energy in q, and the lagged friction normal force against differences of
the energy along the contact normal."""
import numpy as np
import pytest

import oracle as O
from scenes import tiny_scene

LN2 = np.log(2.0)


@pytest.mark.parametrize("shat", [1.0, 2.5e-7, 1e-6, 4e-10])
def test_closed_form_at_half(shat):
    b, b1, b2 = O.barrier_sq(shat / 2, shat)
    assert b == pytest.approx(shat * shat * LN2 / 4, rel=1e-14)
    assert b1 == pytest.approx(-shat * (LN2 + 0.5), rel=1e-14)
    assert b2 == pytest.approx(5.0 + 2.0 * LN2, rel=1e-14)


@pytest.mark.parametrize("shat", [1.0, 1e-6])
def test_vanishes_smoothly_at_shat(shat):
    assert O.barrier_sq(shat, shat) == (0.0, 0.0, 0.0)
    assert O.barrier_sq(1.5 * shat, shat) == (0.0, 0.0, 0.0)
    assert O.barrier_sq(0.0, shat) == (0.0, 0.0, 0.0)
    e = 1e-6
    b, b1, b2 = O.barrier_sq(shat * (1 - e), shat)
    # b ~ e^3 shat^2, b' ~ -3 e^2 shat, b'' ~ 6 e
    assert 0 < b <= 2 * (e * shat) ** 3 / shat
    assert -4 * e * e * shat <= b1 < 0
    assert 0 < b2 <= 10 * e


def test_convex_and_decreasing():
    shat = 1e-6
    for s in np.linspace(1e-3, 1 - 1e-3, 199) * shat:
        _, b1, b2 = O.barrier_sq(s, shat)
        assert b1 < 0 and b2 > 0


@pytest.mark.parametrize("r", [0.01, 0.2, 0.5, 0.9, 0.999])
def test_derivatives_by_differences(r):
    shat = 1e-6
    s = r * shat
    h = 1e-6 * s
    b, b1, b2 = O.barrier_sq(s, shat)
    fb = (O.barrier_sq(s + h, shat)[0] - O.barrier_sq(s - h, shat)[0]) / (2 * h)
    fb1 = (O.barrier_sq(s + h, shat)[1] - O.barrier_sq(s - h, shat)[1]) / (2 * h)
    assert fb == pytest.approx(b1, rel=1e-7, abs=1e-9 * shat)
    assert fb1 == pytest.approx(b2, rel=1e-6, abs=1e-6)


def _pt_above(h):
    # point h above the interior of a triangle in the z = 0 plane
    return np.array([0.2e-3, 0.25e-3, h, 0, 0, 0, 1e-3, 0, 0, 0, 1e-3, 0])


def _ee_crossing(h):
    # edge a along x at height h over edge b along y
    return np.array([-1e-3, 0, h, 1e-3, 0, h, 0, -1e-3, 0, 0, 1e-3, 0])


@pytest.mark.parametrize("kind,make", [(0, _pt_above), (1, _ee_crossing)])
@pytest.mark.parametrize("h", [1e-5, 2e-4, 7e-4])
def test_energy_at_a_known_distance(kind, make, h):
    dhat, kappa = 1e-3, 3e2
    st, _, s, e, _, _ = O.pair_eval(kind, make(h), dhat, kappa, flags=O.SQDIST)
    assert st == O.OK and s == pytest.approx(h * h, rel=1e-14)
    shat = dhat * dhat
    assert e == pytest.approx(-kappa * (h * h - shat) ** 2 * np.log(h * h / shat), rel=1e-12)
    # the distance form differs but has the same active set
    st_d, _, _, e_d, _, _ = O.pair_eval(kind, make(h), dhat, kappa)
    assert st_d == O.OK and e_d != e
    assert O.pair_eval(kind, make(1.01 * dhat), dhat, kappa, flags=O.SQDIST)[0] == O.INACTIVE


@pytest.mark.parametrize("kind", [0, 1])
def test_pair_derivatives_by_differences(kind):
    rng = np.random.default_rng(70 + kind)
    dhat, kappa = 1e-3, 1e2
    n_done = 0
    for _ in range(400):
        x12 = rng.normal(size=12) * 1.5e-3
        st, _, s, e, g, H = O.pair_eval(kind, x12, dhat, kappa, flags=O.SQDIST)
        if st != O.OK or s < 1e-2 * dhat * dhat:
            continue
        # fourth-order central differences
        h = 1e-7
        fg = np.zeros(12)
        fH = np.zeros((12, 12))
        for i in range(12):
            r = []
            for k in (2, 1, -1, -2):
                xk = x12.copy()
                xk[i] += k * h
                r.append(O.pair_eval(kind, xk, dhat, kappa, flags=O.SQDIST))
            if len({t[1] for t in r}) > 1:  # crossed a type boundary
                break
            fg[i] = (-r[0][3] + 8 * r[1][3] - 8 * r[2][3] + r[3][3]) / (12 * h)
            fH[i] = (-r[0][4] + 8 * r[1][4] - 8 * r[2][4] + r[3][4]) / (12 * h)
        else:
            assert np.linalg.norm(fg - g) <= 1e-6 * np.linalg.norm(g)
            assert np.linalg.norm(fH - H) <= 1e-6 * np.linalg.norm(H)
            n_done += 1
        if n_done >= 12:
            break
    assert n_done >= 6


def test_reduced_gradient_by_differences():
    sc = tiny_scene(3)
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    flags = O.ENERGY | O.GRAD | O.SQDIST
    r = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags, hess=False)
    assert r["n_active"] > 0
    g = r["grad"]
    rng = np.random.default_rng(5)
    idx = rng.choice(len(sc.q), size=12, replace=False)
    h = 1e-9
    for i in idx:
        qp, qm = sc.q.copy(), sc.q.copy()
        qp[i] += h
        qm[i] -= h
        ep = O.barrier_reduce(sc, qp, pt, ee, sc.dhat, sc.kappa, O.ENERGY | O.SQDIST, hess=False)["energy"]
        em = O.barrier_reduce(sc, qm, pt, ee, sc.dhat, sc.kappa, O.ENERGY | O.SQDIST, hess=False)["energy"]
        assert (ep - em) / (2 * h) == pytest.approx(g[i], rel=1e-5, abs=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("h", [5e-5, 4e-4])
def test_friction_normal_force_is_the_energy_slope(h):
    dhat, kappa = 1e-3, 3e2
    st, lag = O.friction_lag(0, _pt_above(h), dhat, kappa, flags=O.SQDIST)
    assert st == O.OK
    eps = 1e-9
    ep = O.pair_eval(0, _pt_above(h + eps), dhat, kappa, flags=O.SQDIST)[3]
    em = O.pair_eval(0, _pt_above(h - eps), dhat, kappa, flags=O.SQDIST)[3]
    assert lag[0] == pytest.approx(abs(ep - em) / (2 * eps), rel=1e-6)
    # the distance form's force differs
    assert O.friction_lag(0, _pt_above(h), dhat, kappa)[1][0] != pytest.approx(lag[0], rel=1e-3)
