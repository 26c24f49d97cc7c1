"""Pins for the oracle's lagged friction (Sec. III-B): D_k = mu lambda_k^n
f0(|u_k|) with f0 the integral of the paper's f1.

Pinned against the definitions: f0 against numerical quadrature of f1, the
smoothness of f0 at eps_v h, the lagged normal force against differences
of the barrier, the closest-point weights against the type-free distance,
the friction energy's gradient and Hessian against central differences,
positive semidefiniteness, Coulomb's bound (the sliding force on the point
of a point-triangle pair has magnitude mu lambda), invariance under
translation, and the reduction through W against differences of the total
friction energy in q."""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O
from scenes import tiny_scene
from tests import _geom as G

EPSVH = 1e-3 * 0.01  # eps_v h: 1e-3 m/s at h = 0.01 s


def _f1(y, e):
    return -(y * y) / (e * e) + 2.0 * y / e if y < e else 1.0


@pytest.mark.parametrize("y", [0.0, 1e-7, 3e-6, 9.99e-6, 1e-5, 1.7e-5, 5e-5])
def test_f0_is_the_integral_of_f1(y):
    f0, f1, f1p = O.friction_f(y, EPSVH)
    ref = quad(lambda t: _f1(t, EPSVH), EPSVH, y, epsabs=1e-16, epsrel=1e-13, points=[EPSVH])[0] + EPSVH
    assert f0 == pytest.approx(ref, rel=1e-12, abs=1e-18)
    assert f1 == pytest.approx(_f1(y, EPSVH), rel=1e-14, abs=1e-18)
    h = 1e-5 * EPSVH
    if y >= h:
        fd = (O.friction_f(y + h, EPSVH)[0] - O.friction_f(y - h, EPSVH)[0]) / (2 * h)
        assert fd == pytest.approx(f1, rel=1e-6, abs=1e-9)
        fd1 = (O.friction_f(y + h, EPSVH)[1] - O.friction_f(y - h, EPSVH)[1]) / (2 * h)
        assert fd1 == pytest.approx(f1p, rel=1e-6, abs=1e-3 / EPSVH)


def test_f0_smooth_at_the_transition():
    lo = O.friction_f(EPSVH * (1 - 1e-12), EPSVH)
    hi = O.friction_f(EPSVH, EPSVH)
    assert lo[0] == pytest.approx(EPSVH, rel=1e-11) and hi[0] == EPSVH
    assert lo[1] == pytest.approx(1.0, abs=1e-11) and hi[1] == 1.0
    assert abs(lo[2]) <= 1e-6 / EPSVH and hi[2] == 0.0  # f0 is C^2
    f0, f1, _ = O.friction_f(0.0, EPSVH)
    assert f0 == pytest.approx(EPSVH / 3, rel=1e-15) and f1 == 0.0
    ys = np.linspace(0, EPSVH, 101)
    f1s = [O.friction_f(y, EPSVH)[1] for y in ys]
    assert np.all(np.diff(f1s) >= 0) and max(f1s) <= 1.0


@pytest.mark.parametrize("kind", [0, 1])
def test_lag_record_against_definitions(kind):
    rng = np.random.default_rng(20 + kind)
    dhat, kappa = 1e-3, 1e3
    n_done = 0
    for _ in range(200):
        x12 = rng.normal(size=12) * 2e-3
        d = G.pair_distance(kind, x12)
        if not (0 < d < dhat):
            continue
        st, lag = O.friction_lag(kind, x12, dhat, kappa)
        assert st == O.OK
        lam, beta, nrm, gx = lag[0], lag[1:5], lag[5:8], lag[8:11]
        # lambda = kappa |b'(d)| with b(d) = -(d - dhat)^2 ln(d / dhat)
        b = lambda t: -((t - dhat) ** 2) * np.log(t / dhat)
        hh = 1e-6 * d
        assert lam == pytest.approx(kappa * abs((b(d + hh) - b(d - hh)) / (2 * hh)), rel=1e-6)
        # closest points: G x = sum beta_a x_a has length d, the normal is
        # its direction, the weights are translation-free with the first
        # primitive's weights summing to 1 and each side's in [0, 1]
        xa = x12.reshape(4, 3)
        assert np.allclose(beta @ xa, gx, rtol=0, atol=1e-15)
        assert np.linalg.norm(gx) == pytest.approx(d, rel=1e-10)
        assert np.allclose(nrm, gx / np.linalg.norm(gx), atol=1e-12)
        assert abs(beta.sum()) <= 1e-15
        side1 = beta[:1] if kind == 0 else beta[:2]
        side2 = -beta[1:] if kind == 0 else -beta[2:]
        assert side1.sum() == pytest.approx(1.0, abs=1e-14) and side2.sum() == pytest.approx(1.0, abs=1e-14)
        assert np.all(side1 >= -1e-14) and np.all(side2 >= -1e-14)
        n_done += 1
    assert n_done > 30


def _lagged(rng, kind, dhat=1e-3, kappa=1e3):
    while True:
        xn = rng.normal(size=12) * 2e-3
        d = G.pair_distance(kind, xn)
        if 0 < d < dhat:
            st, lag = O.friction_lag(kind, xn, dhat, kappa)
            assert st == O.OK
            return xn, lag


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("scale", [0.3, 3.0])
def test_friction_energy_derivatives_by_differences(kind, scale):
    """Static (|u| < eps_v h) and sliding (|u| > eps_v h) displacements."""
    rng = np.random.default_rng(100 + kind + int(10 * scale))
    mu = 0.7
    for _ in range(6):
        xn, lag = _lagged(rng, kind)
        x = xn + rng.normal(size=12) * EPSVH * scale
        e, g, H = O.friction_pair(x, lag, mu, EPSVH)
        h = 1e-4 * EPSVH
        fd_g = np.array([(O.friction_pair(x + h * ei, lag, mu, EPSVH)[0]
                          - O.friction_pair(x - h * ei, lag, mu, EPSVH)[0]) / (2 * h) for ei in np.eye(12)])
        assert np.linalg.norm(fd_g - g) <= 1e-6 * np.linalg.norm(g)
        fd_H = np.array([(O.friction_pair(x + h * ei, lag, mu, EPSVH)[1]
                          - O.friction_pair(x - h * ei, lag, mu, EPSVH)[1]) / (2 * h) for ei in np.eye(12)])
        assert np.linalg.norm(fd_H - H) <= 1e-5 * np.linalg.norm(H)
        assert np.allclose(H, H.T, rtol=0, atol=1e-12 * np.abs(H).max())
        assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.linalg.norm(H)


def test_coulomb_bound_and_rest():
    rng = np.random.default_rng(7)
    mu = 0.5
    for _ in range(10):
        xn, lag = _lagged(rng, 0)
        lam, nrm = lag[0], lag[5:8]
        # at x = x^n: no tangential displacement, no force, energy mu lam eps h / 3
        e, g, H = O.friction_pair(xn, lag, mu, EPSVH)
        assert not g.any() and e == pytest.approx(mu * lam * EPSVH / 3, rel=1e-14)
        assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.linalg.norm(H)
        # slide the point tangentially: the force on it has magnitude mu lam
        t = np.cross(nrm, rng.normal(size=3))
        t /= np.linalg.norm(t)
        for amount, sliding in ((5 * EPSVH, True), (0.4 * EPSVH, False)):
            x = xn.copy()
            x[:3] += amount * t
            _, g, _ = O.friction_pair(x, lag, mu, EPSVH)
            f = np.linalg.norm(g[:3])
            if sliding:
                assert f == pytest.approx(mu * lam, rel=1e-12)
            else:
                assert f == pytest.approx(mu * lam * _f1(amount, EPSVH), rel=1e-10)
            assert abs(g[:3] @ nrm) <= 1e-12 * mu * lam  # tangential
        # a normal displacement adds no friction
        x = xn.copy()
        x[:3] += 0.3 * EPSVH * nrm
        _, g, _ = O.friction_pair(x, lag, mu, EPSVH)
        assert np.linalg.norm(g) <= 1e-12 * mu * lam
        # translating all four vertices changes nothing
        shift = np.tile(rng.normal(size=3) * 1e-3, 4)
        x = xn + rng.normal(size=12) * EPSVH
        e1, g1, _ = O.friction_pair(x, lag, mu, EPSVH)
        e2, g2, _ = O.friction_pair(x + shift, lag, mu, EPSVH)
        assert e2 == pytest.approx(e1, rel=1e-9) and np.allclose(g2, g1, rtol=1e-6, atol=1e-12 * mu * lam)


@pytest.mark.parametrize("mode", ["grid", "full", "tet"])
def test_friction_reduction_is_the_chain_rule(mode):
    """Lag at q^n, evaluate at q = q^n + small step: the reduced gradient is
    the central difference of the total friction energy in q, the reduced
    Hessian the difference of the reduced gradient."""
    sc = tiny_scene(4, mode=mode)
    xn = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, xn, sc.dhat)
    st1, lpt = O.friction_lag_list(sc, sc.q, 0, pt, sc.dhat, sc.kappa)
    st2, lee = O.friction_lag_list(sc, sc.q, 1, ee, sc.dhat, sc.kappa)
    assert st1 == O.OK and st2 == O.OK and (lpt[:, 0] > 0).sum() + (lee[:, 0] > 0).sum() > 0
    epsvh = 0.05 * sc.dhat
    rng = np.random.default_rng(3)
    q = sc.q + rng.normal(size=sc.q.shape) * 0.3 * epsvh
    r = O.friction_reduce(sc, q, pt, lpt, ee, lee, 0.8, epsvh)
    h = 1e-3 * epsvh
    for i in rng.choice(len(q), size=min(12, len(q)), replace=False):
        ei = np.zeros_like(q)
        ei[i] = h
        ep = O.friction_reduce(sc, q + ei, pt, lpt, ee, lee, 0.8, epsvh, hess=False)
        em = O.friction_reduce(sc, q - ei, pt, lpt, ee, lee, 0.8, epsvh, hess=False)
        assert (ep["energy"] - em["energy"]) / (2 * h) == pytest.approx(r["grad"][i], rel=1e-5,
                                                                        abs=1e-7 * np.abs(r["grad"]).max())
        fd = (ep["grad"] - em["grad"]) / (2 * h)
        assert np.linalg.norm(fd - r["hess"][:, i]) <= 1e-4 * np.linalg.norm(r["hess"]) + 1e-12
    assert np.linalg.eigvalsh(r["hess"]).min() >= -1e-10 * np.linalg.norm(r["hess"])
