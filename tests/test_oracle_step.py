"""Pins for the oracle of one implicit step and its adjoint (Sec. III-A
Eq. 5-6, III-B Eq. 10-12, III-C): the assembled mass, stiffness and
gravity against their definitions (total mass, partition of unity, rigid
null space of the elastic energy, the energy of a constant strain), the
linear model as the rest linearization of the paper's corotational one,
the corotational term (rigid invariance, differences, warped stiffness),
the converged step under either model, and the adjoint gradients against
central differences of the loss with the step solved again."""
import numpy as np
import pytest

from oracle import step as OS
from scenes.scene import step_inputs


@pytest.fixture(scope="module")
def st():
    return OS.Step(step_inputs())


def test_mass_and_gravity(st):
    si = st.si
    n = len(si.grid_nodes)
    Mn = st.M[0::3, 0::3]
    assert np.allclose(st.M, st.M.T, rtol=0, atol=1e-18)
    assert np.linalg.eigvalsh(st.M).min() > 0
    vol = si.sample_vol * len(si.sample_tet)
    reached = np.zeros(n, dtype=bool)
    reached[np.unique(si.tets[si.sample_tet])] = True
    # partition of unity: the sampled mass sums to rho V (lumped masses of
    # unreached nodes aside)
    assert Mn[np.ix_(reached, reached)].sum() == pytest.approx(si.rho * vol, rel=1e-12)
    assert st.f.reshape(-1, 3)[:, 2].sum() == pytest.approx(-si.rho * vol * si.g, rel=1e-12)
    assert not st.f.reshape(-1, 3)[:, :2].any()


def test_stiffness_null_space_and_constant_strain(st):
    si = st.si
    X = si.grid_nodes
    K = st.K
    assert np.allclose(K, K.T, rtol=0, atol=1e-9 * np.abs(K).max())
    scale = np.abs(K).max()
    for k in range(3):
        t = np.zeros_like(X)
        t[:, k] = 1.0
        assert np.abs(K @ t.reshape(-1)).max() <= 1e-10 * scale
        e = np.zeros(3)
        e[k] = 1.0
        assert np.abs(K @ np.cross(e, X).reshape(-1)).max() <= 1e-10 * scale * np.abs(X).max()
    # a constant strain eps = sym(A): energy V_sampled (mu eps:eps + lam/2 tr(eps)^2)
    rng = np.random.default_rng(2)
    A = rng.normal(size=(3, 3)) * 1e-3
    u = X @ A.T
    eps = 0.5 * (A + A.T)
    lam = si.young * si.poisson / ((1 + si.poisson) * (1 - 2 * si.poisson))
    mu = si.young / (2 * (1 + si.poisson))
    vol = si.sample_vol * len(si.sample_tet)
    psi = mu * np.sum(eps * eps) + 0.5 * lam * np.trace(eps) ** 2
    assert 0.5 * u.reshape(-1) @ (K @ u.reshape(-1)) == pytest.approx(vol * psi, rel=1e-10)


def _corotational_energy(si, x):
    """Linear corotational elastic energy of the coarse tets at node
    positions x (Sec. IV-A's model): sum_T V_T (mu |F - R|^2 + lam/2
    tr(R^T F - I)^2), F = Ds Dm^-1, R the rotation of F's polar
    decomposition, V_T the aggregated sample volumes (Eq. 15)."""
    lam = si.young * si.poisson / ((1 + si.poisson) * (1 - 2 * si.poisson))
    mu = si.young / (2 * (1 + si.poisson))
    VT = np.zeros(len(si.tets))
    np.add.at(VT, si.sample_tet, si.sample_vol)
    X = si.grid_nodes
    e = 0.0
    for t in np.nonzero(VT)[0]:
        a, b, c, d = si.tets[t]
        Dm = np.column_stack([X[b] - X[a], X[c] - X[a], X[d] - X[a]])
        Ds = np.column_stack([x[b] - x[a], x[c] - x[a], x[d] - x[a]])
        F = Ds @ np.linalg.inv(Dm)
        U, _, Vt = np.linalg.svd(F)
        R = U @ Vt
        if np.linalg.det(R) < 0:
            U[:, -1] *= -1
            R = U @ Vt
        S = R.T @ F - np.eye(3)
        e += VT[t] * (mu * np.sum((F - R) ** 2) + 0.5 * lam * np.trace(S) ** 2)
    return e


def test_linear_model_is_the_rest_linearization_of_corotational(st):
    """The step's elastic model (small-strain linear elasticity) stands in
    for the paper's linear corotational model: the two agree to second
    order about the rest shape (equal energy, gradient and Hessian there),
    so for a displacement of scale s their energies differ by O(s^3); a
    finite rotation shows they are different models (corotational energy
    zero, linear energy not)."""
    si = st.si
    X = si.grid_nodes
    rng = np.random.default_rng(5)
    u = rng.normal(size=X.shape) * np.ptp(X, axis=0).max()
    rel = []
    for s in (1e-3, 1e-4):
        us = s * u
        e_lin = 0.5 * us.reshape(-1) @ (st.K @ us.reshape(-1))
        e_cor = _corotational_energy(si, X + us)
        rel.append(abs(e_cor - e_lin) / e_lin)
    assert rel[0] < 1e-2 and rel[1] < 0.2 * rel[0]
    th = 0.3
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    xr = (X - X.mean(0)) @ Rz.T + X.mean(0)
    ur = (xr - X).reshape(-1)
    assert _corotational_energy(si, xr) <= 1e-20 * (0.5 * ur @ (st.K @ ur))
    assert 0.5 * ur @ (st.K @ ur) > 0


def _rigid(X, th, t):
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(0.7 * th), -np.sin(0.7 * th)], [0, np.sin(0.7 * th), np.cos(0.7 * th)]])
    return (X - X.mean(0)) @ (Rz @ Rx).T + X.mean(0) + t


def test_corotational_oracle_definition(st):
    """The oracle's corotational term: its energy equals the definition
    evaluated separately above; rigid motions (finite rotations) give zero
    energy and zero gradient; the gradient matches central differences of
    the energy; the warped stiffness equals the linear stiffness at the rest
    shape and stays positive semidefinite when deformed."""
    from oracle.step import corotational
    si = st.si
    X = si.grid_nodes
    rng = np.random.default_rng(8)
    xd = X + 0.02 * np.ptp(X, axis=0).max() * rng.normal(size=X.shape)
    e, g, H = corotational(si, xd.reshape(-1))
    assert e == pytest.approx(_corotational_energy(si, xd), rel=1e-12)
    xr = _rigid(X, 0.9, np.array([0.01, -0.02, 0.03]))
    er, gr, _ = corotational(si, xr.reshape(-1), want_hess=False)
    assert abs(er) <= 1e-20 * e and np.abs(gr).max() <= 1e-10 * np.abs(g).max()
    for _ in range(3):
        v = rng.normal(size=g.shape)
        eps = 1e-6 * np.ptp(X, axis=0).max()
        ep, _, _ = corotational(si, xd.reshape(-1) + eps * v, want_hess=False)
        em, _, _ = corotational(si, xd.reshape(-1) - eps * v, want_hess=False)
        assert (ep - em) / (2 * eps) == pytest.approx(g @ v, rel=1e-6)
    _, g0, H0 = corotational(si, X.reshape(-1))
    assert np.abs(g0).max() <= 1e-10 * np.abs(g).max()
    assert np.allclose(H0, st.K, rtol=0, atol=1e-12 * np.abs(st.K).max())
    lam = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert lam.min() >= -1e-10 * lam.max()


def test_corotational_step_converges(st):
    """One step under the corotational model converges (its Newton matrix
    carries the warped stiffness, not the exact Hessian, so it stops on the
    energy's rounding level with a gradient a little above the linear
    model's) and lands near the linear model's step."""
    stc = OS.Step(st.si, elastic="corotational")
    q, it = stc.solve()
    assert it < 60
    g, _, _ = stc.grad_hess(q, project=False)
    qt = stc.q_n + stc.h * stc.v_n
    assert np.linalg.norm(g) <= 1e-7 * np.linalg.norm(stc.M @ qt)
    ql, _ = st.solve()
    rel = np.linalg.norm(q - ql) / np.linalg.norm(ql - st.q_n)
    assert 0 < rel < 0.1


@pytest.fixture(scope="module")
def solved(st):
    q, it = st.solve()
    return q, it


def test_step_converges(st, solved):
    q, it = solved
    assert it < 60
    g, H, _ = st.grad_hess(q, project=False)
    qt = st.q_n + st.h * st.v_n
    assert np.linalg.norm(g) <= 1e-9 * np.linalg.norm(st.M @ qt)
    assert np.linalg.eigvalsh(H).min() > 0  # a strict minimum


def test_adjoint_against_central_differences(st, solved):
    """Perturb q_n and the ground's pose, solve the step again each time."""
    q, _ = solved
    target = st.si.q_target
    dq_n, dv_n, dth, res = st.adjoint(q, q - target)
    assert res <= 1e-12
    assert np.array_equal(dv_n, st.h * dq_n)

    def loss():
        qs, _ = st.solve()
        return 0.5 * np.sum((qs - target) ** 2)

    rng = np.random.default_rng(4)
    q_n0 = st.q_n.copy()
    eps = 1e-6
    d = rng.normal(size=q_n0.shape)
    d /= np.abs(d).max()
    st.q_n = q_n0 + eps * d
    lp = loss()
    st.q_n = q_n0 - eps * d
    lm = loss()
    st.q_n = q_n0
    assert (lp - lm) / (2 * eps) == pytest.approx(dq_n @ d, rel=2e-4, abs=1e-9)
    for k in (2, 3):
        th = np.zeros(6)
        th[k] = eps
        st.set_pose(th)
        lp = loss()
        th[k] = -eps
        st.set_pose(th)
        lm = loss()
        st.set_pose(np.zeros(6))
        assert (lp - lm) / (2 * eps) == pytest.approx(dth[k], rel=2e-4, abs=1e-9)
