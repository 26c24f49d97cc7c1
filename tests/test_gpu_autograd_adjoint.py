"""Differentiable form on config 1: autograd barrier energy (backward =
reduced gradient, double backward = Hessian-vector product), the dense
Cholesky kernels, and the adjoint of one converged implicit step, checked
against the oracle and central differences."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import adjoint as A  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


@pytest.fixture(scope="module")
def state(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    q = torch.as_tensor(c1.q, device="cuda:0")
    pt, ee = E.build_candidates(ctx, dsc, q, c1.dhat)
    return E.BarrierState(ctx, dsc, pt, ee, c1.dhat, c1.kappa)


def test_backward_is_the_oracle_gradient(state, c1):
    q = torch.as_tensor(c1.q, device="cuda:0").requires_grad_(True)
    e = E.barrier_energy(q, state)
    (g,) = torch.autograd.grad(e, q)
    ref = O.barrier_reduce(c1, c1.q, state.pt.cpu().numpy(), state.ee.cpu().numpy(), c1.dhat, c1.kappa,
                           O.ENERGY | O.GRAD, hess=False)
    assert e.item() == pytest.approx(ref["energy"], rel=1e-10)
    assert np.linalg.norm(g.cpu().numpy() - ref["grad"]) <= 1e-10 * np.linalg.norm(ref["grad"])


def test_backward_against_central_differences(state, c1):
    rng = np.random.default_rng(0)
    q0 = torch.as_tensor(c1.q, device="cuda:0")
    q = q0.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(E.barrier_energy(q, state), q)
    for _ in range(4):
        d = torch.as_tensor(rng.normal(size=q0.shape), device="cuda:0")
        d /= d.abs().max()
        eps = 1e-7
        fd = (E.barrier_energy(q0 + eps * d, state) - E.barrier_energy(q0 - eps * d, state)).item() / (2 * eps)
        assert fd == pytest.approx(float(g @ d), rel=1e-5)


def test_double_backward_is_the_hvp(state, c1):
    """32 seeded directions: d/dq (g . v) by autograd equals the library HVP
    with the true Hessian, the oracle's HVP, and differences of g."""
    q0 = torch.as_tensor(c1.q, device="cuda:0")
    q = q0.clone().requires_grad_(True)
    (g,) = torch.autograd.grad(E.barrier_energy(q, state), q, create_graph=True)
    rng = np.random.default_rng(1)
    pt, ee = state.pt.cpu().numpy(), state.ee.cpu().numpy()
    for k in range(32):
        v = torch.as_tensor(rng.normal(size=q0.shape), device="cuda:0")
        (hv,) = torch.autograd.grad(g, q, grad_outputs=v, retain_graph=True)
        st, ref, _ = O.barrier_hvp(c1, c1.q, pt, ee, c1.dhat, c1.kappa, 0, v.cpu().numpy())
        assert np.linalg.norm(hv.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
        if k < 4:
            eps = 1e-7 * c1.dhat / float(v.abs().max())
            gp = E.barrier_grad(q0 + eps * v, state)
            gm = E.barrier_grad(q0 - eps * v, state)
            fd = ((gp - gm) / (2 * eps)).cpu().numpy()
            assert np.linalg.norm(fd - ref) <= 1e-5 * np.linalg.norm(ref)


def test_backward_forward_time_ratio(state, c1):
    q = torch.as_tensor(c1.q, device="cuda:0").requires_grad_(True)
    for _ in range(3):
        torch.autograd.grad(E.barrier_energy(q, state), q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        e = E.barrier_energy(q, state)
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / 20
    t0 = time.perf_counter()
    for _ in range(20):
        e = E.barrier_energy(q, state)
        torch.autograd.grad(e, q)
    torch.cuda.synchronize()
    tfb = (time.perf_counter() - t0) / 20
    print(f"\nconfig1 barrier energy: forward {tf * 1e6:.1f} us, forward+backward {tfb * 1e6:.1f} us, "
          f"backward/forward = {(tfb - tf) / tf:.2f}")
    assert tfb > 0


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 130, 700])
def test_cholesky_factor_and_solve(ctx, n):
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, n))
    Aref = X @ X.T + n * np.eye(n)
    A_ = torch.as_tensor(Aref.copy(), device="cuda:0")
    info = E.cholesky(ctx, A_)
    assert info == 0
    L = np.tril(A_.cpu().numpy())
    Lref = np.linalg.cholesky(Aref)
    assert np.abs(L - Lref).max() <= 1e-12 * np.abs(Lref).max()
    Bm = rng.normal(size=(n, 3))
    Xs = torch.as_tensor(Bm.copy(), device="cuda:0")
    E.cholesky_solve(ctx, A_, Xs)
    res = np.linalg.norm(Aref @ Xs.cpu().numpy() - Bm) / np.linalg.norm(Bm)
    assert res <= 1e-12


def test_cholesky_reports_indefinite(ctx):
    A_ = torch.eye(100, dtype=torch.float64, device="cuda:0")
    A_[70, 70] = -1.0
    assert E.cholesky(ctx, A_) == 71


@pytest.fixture(scope="module")
def step(ctx):
    prob, target = A.build_config1_step(ctx)
    q_star, info = A.solve_step(prob)
    return prob, target, q_star, info


def _loss(prob, target):
    q, _ = A.solve_step(prob)
    d = q - target
    return 0.5 * float(d @ d)


def test_step_converges_without_intersection(step, c1):
    prob, target, q_star, info = step
    assert info["iters"] < 60
    x = O.embed(prob.host, q_star.cpu().numpy())
    pt, ee = O.candidates(prob.host, x, prob.dhat)
    r = O.barrier_reduce(prob.host, q_star.cpu().numpy(), pt, ee, prob.dhat, prob.kappa, O.ENERGY, hess=False)
    assert r["status"] == O.OK and r["n_active"] > 0


def test_adjoint_against_central_differences(step):
    prob, target, q_star, info = step
    dq_n, dv_n, dth, used_true = A.adjoint(prob, q_star, q_star - target)
    assert used_true
    rng = np.random.default_rng(7)
    q_n0 = prob.q_n.clone()
    for _ in range(2):
        d = torch.as_tensor(rng.normal(size=q_n0.shape), device="cuda:0")
        d /= d.abs().max()
        eps = 1e-6
        prob.q_n = q_n0 + eps * d
        lp = _loss(prob, target)
        prob.q_n = q_n0 - eps * d
        lm = _loss(prob, target)
        prob.q_n = q_n0
        fd = (lp - lm) / (2 * eps)
        assert fd == pytest.approx(float(dq_n @ d), rel=2e-4, abs=1e-9)
    for k in (2, 3):  # vertical translation and a tilt of the ground
        eps = 1e-6
        th = np.zeros(6)
        th[k] = eps
        prob.set_pose(th)
        lp = _loss(prob, target)
        th[k] = -eps
        prob.set_pose(th)
        lm = _loss(prob, target)
        prob.set_pose(np.zeros(6))
        fd = (lp - lm) / (2 * eps)
        assert fd == pytest.approx(dth[k], rel=2e-4, abs=1e-9)


def test_step_and_adjoint_match_the_oracle(step):
    """The oracle's own step (numpy Newton around the contact oracle, its
    own mass, stiffness and gravity assembly, CPU Cholesky) and adjoint at
    375 reduced DoF: the converged q, dL/dq_n, dL/dv_n and dL/dtheta."""
    from oracle import step as OS
    from scenes.scene import step_inputs
    prob, target, q_star, info = step
    st = OS.Step(step_inputs())
    q_ref, _ = st.solve()
    q = q_star.cpu().numpy()
    assert np.linalg.norm(q - q_ref) <= 1e-9 * np.linalg.norm(q_ref - st.q_n)
    dq_n, dv_n, dth, used_true = A.adjoint(prob, q_star, q_star - target)
    r_qn, r_vn, r_th, res = st.adjoint(q_ref, q_ref - st.si.q_target)
    assert used_true and res <= 1e-12
    assert np.linalg.norm(dq_n.cpu().numpy() - r_qn) <= 1e-6 * np.linalg.norm(r_qn)
    assert np.linalg.norm(dv_n.cpu().numpy() - r_vn) <= 1e-6 * np.linalg.norm(r_vn)
    assert np.linalg.norm(dth - r_th) <= 1e-6 * np.linalg.norm(r_th)


def test_large_reduced_system_step_and_adjoint(ctx):
    """About 7.6k reduced DoF (14x14x13 grid): one converged step and its
    adjoint through the library's dense Cholesky, whose solve has a
    residual |H lambda - dL/dq| / |dL/dq| <= 1e-12."""
    prob, target = A.build_config1_step(ctx, grid_dims=(14, 14, 13), n_samples=60000)
    assert prob.n == 3 * 14 * 14 * 13
    t0 = time.perf_counter()
    q_star, info = A.solve_step(prob, tol=1e-10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dq_n, dv_n, dth, used_true = A.adjoint(prob, q_star, q_star - target)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"\n{prob.n} DoF: step {info['iters']} Newton iterations in {t1 - t0:.2f} s, adjoint {t2 - t1:.3f} s")
    assert np.isfinite(dq_n.cpu().numpy()).all() and np.isfinite(dth).all()
    # residual of the adjoint solve: lambda = M^-1 dL/dq_n (dL/dq_n = M lambda)
    g, H, _ = A.gradient_hessian(prob, q_star, project=not used_true)
    b = q_star - target
    L = H.clone()
    assert E.cholesky(ctx, L) == 0
    lam = b.clone()
    E.cholesky_solve(ctx, L, lam)
    res = float(torch.linalg.vector_norm(H @ lam - b) / torch.linalg.vector_norm(b))
    assert res <= 1e-12, res
    assert torch.allclose(prob.M @ lam, dq_n, rtol=1e-12, atol=1e-12 * float(dq_n.abs().max()))


@pytest.mark.parametrize("variant", ["sqdist", "reduced", "closest_direction"])
def test_step_converges_under_each_formulation(ctx, variant):
    """The implicit step under the alternative formulations converges to a
    position near the distance-barrier step's (the same problem up to the
    barrier's form inside dhat)."""
    prob, _ = A.build_config1_step(ctx)
    q0, info0 = A.solve_step(prob)
    if variant == "sqdist":
        prob.barrier_flags = E.SQDIST
        prob.kappa *= A.SQDIST_KAPPA_FACTOR / prob.dhat ** 2
    elif variant == "reduced":
        prob.reduced_projection = True
    else:
        E.set_ccd_method(ctx, E.CCD_CLOSEST_DIRECTION)
    try:
        q1, info1 = A.solve_step(prob)
    finally:
        E.set_ccd_method(ctx, E.CCD_ADDITIVE)
    assert info0["converged"] and info1["converged"] and len(info1["alpha_ccd"]) > 0
    dn = float(torch.linalg.vector_norm(q0 - prob.q_n))
    rel = float(torch.linalg.vector_norm(q1 - q0)) / dn
    if variant == "sqdist":
        assert rel < 0.5  # another barrier: close, not equal
    else:
        assert rel < 1e-6  # the same minimizer
