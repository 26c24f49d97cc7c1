"""The step's inertial and elastic terms in the library (eipc_reduced_mass,
eipc_elastic) against the oracle of the step: the reduced mass and gravity
from interior samples (Eq. 1, 15, 16; nodes that no sample reaches get the
lumped mass), the elastic energy, gradient and Newton matrix of the coarse
tets in the linear model and in the paper's linear corotational model
(Sec. IV-A), within 1e-10 at a deformed position; an inverted element is
reported; one implicit step under the corotational model converges to the
oracle's; the adjoint refuses the corotational model (it needs the exact
Hessian)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import adjoint as A  # noqa: E402
from oracle import step as OS  # noqa: E402
from scenes.scene import step_inputs  # noqa: E402

TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


@pytest.fixture(scope="module")
def si():
    return step_inputs()


@pytest.fixture(scope="module")
def st(si):
    return OS.Step(si)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def test_mass_and_gravity(ctx, si, st):
    M, f = E.reduced_mass(ctx, len(si.grid_nodes), torch.as_tensor(si.tets[si.sample_tet], dtype=torch.int32),
                          torch.as_tensor(si.sample_w), si.rho * si.sample_vol, si.g)
    assert _rel(M.cpu().numpy(), st.M) <= 1e-12
    assert _rel(f.cpu().numpy(), st.f) <= 1e-12
    # the grid has nodes that no sample reaches: they carry the lumped mass
    assert (np.diag(st.M) < 1e-2 * np.diag(st.M).max()).any()


def _terms(ctx, si, model, x):
    n = len(si.grid_nodes)
    VT = np.bincount(si.sample_tet, minlength=len(si.tets)) * si.sample_vol
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    g = torch.zeros(3 * n, dtype=torch.float64, device="cuda:0")
    H = torch.zeros((3 * n, 3 * n), dtype=torch.float64, device="cuda:0")
    E.elastic(ctx, n, _dev(si.tets, torch.int32), _dev(si.grid_nodes.reshape(-1)), _dev(VT), si.young, si.poisson,
              model, _dev(x.reshape(-1)), 1.0, energy=e, grad=g, hess=H)
    assert ctx.sync_status() == E.binding.OK
    return e.item(), g.cpu().numpy(), H.cpu().numpy()


@pytest.mark.parametrize("amp", [1e-3, 3e-2])
def test_linear_terms(ctx, si, st, amp):
    X = si.grid_nodes
    x = X + amp * np.ptp(X, axis=0).max() * np.random.default_rng(3).normal(size=X.shape)
    e, g, H = _terms(ctx, si, E.ELASTIC_LINEAR, x)
    u = (x - X).reshape(-1)
    assert e == pytest.approx(0.5 * u @ (st.K @ u), rel=TOL)
    assert _rel(g, st.K @ u) <= TOL
    assert _rel(H, st.K) <= TOL


@pytest.mark.parametrize("amp", [1e-3, 3e-2])
def test_corotational_terms(ctx, si, amp):
    X = si.grid_nodes
    rng = np.random.default_rng(4)
    x = X + amp * np.ptp(X, axis=0).max() * rng.normal(size=X.shape)
    # plus a finite rotation of the whole grid: the model factors it out
    th = 0.6
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    x = (x - X.mean(0)) @ Rz.T + X.mean(0)
    e, g, H = _terms(ctx, si, E.ELASTIC_COROTATIONAL, x)
    er, gr, Hr = OS.corotational(si, x.reshape(-1))
    assert e == pytest.approx(er, rel=TOL)
    assert _rel(g, gr) <= TOL
    assert _rel(H, Hr) <= TOL


def test_inverted_element_is_reported(ctx, si):
    X = si.grid_nodes.copy()
    t = si.tets[si.sample_tet[0]]
    # mirror one node of a sampled tet through the opposite face's plane
    a, b, c, d = X[t]
    nrm = np.cross(b - d, c - d)
    nrm /= np.linalg.norm(nrm)
    X[t[0]] = a - 2.0 * ((a - d) @ nrm) * nrm
    n = len(X)
    VT = np.bincount(si.sample_tet, minlength=len(si.tets)) * si.sample_vol
    e = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    E.elastic(ctx, n, _dev(si.tets, torch.int32), _dev(si.grid_nodes.reshape(-1)), _dev(VT), si.young, si.poisson,
              E.ELASTIC_COROTATIONAL, _dev(X.reshape(-1)), 1.0, energy=e)
    assert ctx.sync_status() == E.binding.ERR_DEGENERATE
    assert ctx.sync_status() == E.binding.OK  # reading the status clears it


def test_corotational_step_matches_the_oracle(ctx, si):
    prob, _ = A.build_config1_step(ctx)
    prob.elastic_model = E.ELASTIC_COROTATIONAL
    q, info = A.solve_step(prob)
    assert info["converged"]
    stc = OS.Step(si, elastic="corotational")
    q_ref, _ = stc.solve()
    assert np.linalg.norm(q.cpu().numpy() - q_ref) <= 1e-7 * np.linalg.norm(q_ref - stc.q_n)
    with pytest.raises(NotImplementedError):
        A.adjoint(prob, q, q)
