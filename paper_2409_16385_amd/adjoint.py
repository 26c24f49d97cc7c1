"""One implicit step of Embedded IPC and its adjoint.

The step minimizes the incremental potential with contact (Eq. 5-6, 10-12)
over the reduced coordinates q:

    E(q) = 1/2 (q - qt)^T M (q - qt) + h^2 [ Phi(q) - f^T q + kappa B(q) ],
    qt = q_n + h v_n,

with M = J^T M_x J the reduced mass (Eq. 1), Phi the elastic energy on the
coarse tetrahedra with aggregated volumes V_T (Eq. 15), f = J^T f_ext
(Eq. 16) and B the barrier potential of the contact stage.  Projected
Newton (Sec. III-C) with a CCD-clamped backtracking line search solves it;
the adjoint of the converged step gives dL/dq_n, dL/dv_n and dL/dtheta for
the pose theta of a kinematic body (its vertices' x_off).

Elastic model: linear (small-strain) isotropic elasticity, whose Hessian
is exact and constant; the paper's experiments use linear corotational
elasticity.  Volumes and masses come from seeded uniform samples of the
body's interior, each carrying V/N, assigned to their coarse tetrahedron
(the aggregation of Eq. 15).  Grid nodes that no sample reaches get a
lumped mass of 1e-3 of the mean node mass.

Dense linear algebra runs in the library (eipc_cholesky / _solve); the
contact terms come from the library's contact stage.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import binding as B


def _rodrigues(r):
    th = float(np.linalg.norm(r))
    if th == 0.0:
        return np.eye(3)
    k = np.asarray(r) / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def _tet_stiffness(X: np.ndarray, V: float, lam: float, mu: float) -> np.ndarray:
    """12x12 linear-elastic stiffness of one tetrahedron with rest corners X
    (4x3) and volume weight V:  Psi = mu |eps|^2 + lam/2 tr(eps)^2."""
    Dm = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    Bm = np.linalg.inv(Dm)
    # gradients of the 4 barycentric shape functions
    G = np.zeros((4, 3))
    G[1:] = Bm
    G[0] = -Bm.sum(axis=0)
    K = np.zeros((12, 12))
    for a in range(4):
        for b in range(4):
            ga, gb = G[a], G[b]
            blk = mu * (np.outer(gb, ga) + (ga @ gb) * np.eye(3)) + lam * np.outer(ga, gb)
            K[3 * a:3 * a + 3, 3 * b:3 * b + 3] = V * blk
    return K


@dataclasses.dataclass
class StepProblem:
    ctx: B.Context
    scene: B.Scene
    host: object
    M: torch.Tensor          # reduced mass [n, n]
    K: torch.Tensor          # reduced elastic stiffness [n, n]
    q_rest: torch.Tensor     # elastic rest nodes [n]
    f: torch.Tensor          # reduced external force [n]
    q_n: torch.Tensor
    v_n: torch.Tensor
    h: float
    kappa: float
    dhat: float
    kin_rows: np.ndarray     # vertex indices of the kinematic body
    kin_rest: np.ndarray     # their rest positions [k, 3]
    theta: np.ndarray        # pose (tx, ty, tz, rx, ry, rz)
    # barrier formulation: B.SQDIST for the squared-distance form, and
    # reduced_projection for the projection of each pair's reduced block
    # (B.PROJECT_REDUCED) in place of the per-pair B.PROJECT
    barrier_flags: int = 0
    reduced_projection: bool = False

    @property
    def n(self) -> int:
        return self.M.shape[0]

    def set_pose(self, theta):
        """Move the kinematic body to pose theta (rotation about its centroid)."""
        self.theta = np.asarray(theta, dtype=np.float64)
        c = self.kin_rest.mean(axis=0)
        R = _rodrigues(self.theta[3:])
        x = (self.kin_rest - c) @ R.T + c + self.theta[:3]
        off = self.scene.x_off
        off[torch.as_tensor(self.kin_rows, device=off.device)] = torch.as_tensor(x, device=off.device)

    def pose_tangents(self) -> torch.Tensor:
        """d x_off / d theta at theta = 0, [6, n_vert, 3]."""
        c = self.kin_rest.mean(axis=0)
        T = np.zeros((6, self.scene.n_vert, 3))
        for k in range(3):
            T[k, self.kin_rows, k] = 1.0
            e = np.zeros(3)
            e[k] = 1.0
            T[3 + k, self.kin_rows] = np.cross(e, self.kin_rest - c)
        return torch.as_tensor(T, device=self.ctx.torch_device)


def build_step(ctx: B.Context, si) -> tuple[StepProblem, torch.Tensor]:
    """The step problem of the given inputs (scenes.step_inputs): reduced
    mass M = sum_s rho V_s (w_s w_s^T) (x) I3 over the interior samples,
    linear elasticity on each coarse tet with the aggregated volume V_T of
    its samples (Eq. 15), gravity f = J^T f_ext (Eq. 16).  Returns the
    problem and the loss target."""
    sc = si.scene
    dev = ctx.torch_device
    nodes, tets = si.grid_nodes, si.tets
    n_node = len(nodes)
    tet_nodes = tets[si.sample_tet]
    w = si.sample_w
    Vs = si.sample_vol
    Mn = np.zeros((n_node, n_node))
    for a in range(4):
        for b in range(4):
            np.add.at(Mn, (tet_nodes[:, a], tet_nodes[:, b]), si.rho * Vs * w[:, a] * w[:, b])
    # nodes no interior sample reaches carry no mass and no stiffness; give
    # them a small lumped mass so the step's Newton matrix stays definite
    d = np.diag(Mn).copy()
    empty = d <= 0.0
    if empty.any():
        Mn[empty, empty] = 1e-3 * d[~empty].mean()
    M = np.kron(Mn, np.eye(3))
    VT = np.bincount(si.sample_tet, minlength=len(tets)) * Vs
    lam = si.young * si.poisson / ((1 + si.poisson) * (1 - 2 * si.poisson))
    mu = si.young / (2 * (1 + si.poisson))
    Kd = np.zeros((3 * n_node, 3 * n_node))
    for t in np.nonzero(VT)[0]:
        tn = tets[t]
        Ke = _tet_stiffness(nodes[tn], VT[t], lam, mu)
        idx = np.concatenate([[3 * i, 3 * i + 1, 3 * i + 2] for i in tn])
        Kd[np.ix_(idx, idx)] += Ke
    fn = np.zeros((n_node, 3))
    for a in range(4):
        np.add.at(fn[:, 2], tet_nodes[:, a], -si.rho * Vs * si.g * w[:, a])
    scene = B.Scene.from_host(ctx, sc)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    prob = StepProblem(ctx=ctx, scene=scene, host=sc, M=T(M), K=T(Kd), q_rest=T(nodes.reshape(-1)),
                       f=T(fn.reshape(-1)), q_n=T(si.q_n), v_n=T(si.v_n), h=si.h, kappa=sc.kappa,
                       dhat=sc.dhat, kin_rows=si.kin_rows, kin_rest=si.kin_rest.copy(), theta=np.zeros(6))
    return prob, T(si.q_target)


def build_config1_step(ctx: B.Context, grid_dims=(5, 5, 5), seed: int = 0, n_samples: int = 20000,
                       **kw) -> tuple[StepProblem, torch.Tensor]:
    """The step problem on the sphere-on-ground scene (body = the sphere,
    kinematic body = the ground) and the seeded target of the loss
    L = 1/2 |q* - q_target|^2."""
    from scenes.scene import step_inputs
    return build_step(ctx, step_inputs(seed, grid_dims=grid_dims, n_samples=n_samples, **kw))


# kappa for the squared-distance barrier with the distance form's energy at
# d = dhat / sqrt(2): kappa_sq = kappa * SQDIST_KAPPA_FACTOR / dhat^2
# (b(d) = dhat^2 (1 - 1/sqrt2)^2 ln2 / 2 there, b(s) = dhat^4 ln2 / 4)
SQDIST_KAPPA_FACTOR = 2.0 * (1.0 - 0.5 ** 0.5) ** 2


def _contact(prob: StepProblem, q, flags, hess):
    pt, ee = B.build_candidates(prob.ctx, prob.scene, q, prob.dhat)
    r = B.barrier_reduce(prob.ctx, prob.scene, q, pt, ee, prob.dhat, prob.h ** 2 * prob.kappa,
                         flags | prob.barrier_flags, hess=hess, count=False)
    return r, pt, ee


def energy(prob: StepProblem, q) -> float:
    qt = prob.q_n + prob.h * prob.v_n
    d = q - qt
    e = 0.5 * d @ (prob.M @ d)
    dr = q - prob.q_rest
    e = e + prob.h ** 2 * (0.5 * dr @ (prob.K @ dr) - prob.f @ q)
    r, _, _ = _contact(prob, q, B.ENERGY, None)
    return float(e + r["energy"][0])


def gradient_hessian(prob: StepProblem, q, project: bool):
    qt = prob.q_n + prob.h * prob.v_n
    proj = B.PROJECT_REDUCED if prob.reduced_projection else B.PROJECT
    flags = B.ENERGY | B.GRAD | B.HESS | (proj if project else 0)
    r, pt, ee = _contact(prob, q, flags, "dense")
    g = prob.M @ (q - qt) + prob.h ** 2 * (prob.K @ (q - prob.q_rest) - prob.f) + r["grad"]
    H = prob.M + prob.h ** 2 * prob.K + r["hess"]
    return g, H, (pt, ee)


def solve_step(prob: StepProblem, tol: float = 1e-12, max_iter: int = 100, verbose: bool = False):
    """Projected Newton with CCD-clamped backtracking (Armijo); switches to
    the true Hessian when it is positive definite.  Converged when
    |grad E| <= tol |M qt|, when the Newton decrement falls below the
    energy's rounding level, or when the step no longer changes q."""
    q = prob.q_n.clone()
    qt = prob.q_n + prob.h * prob.v_n
    scale = float(torch.linalg.vector_norm(prob.M @ qt))
    it = 0
    info = {"iters": 0, "true_hessian_steps": 0, "alpha_ccd": [], "alpha": [], "converged": False}
    for it in range(max_iter):
        g, H, _ = gradient_hessian(prob, q, project=False)
        gn = float(torch.linalg.vector_norm(g))
        if verbose:
            print(f"newton {it}: |g| = {gn:.3e} (rel {gn / scale:.3e})")
        if gn <= tol * scale:
            info["converged"] = True
            break
        L = H.clone()
        used_true = B.cholesky(prob.ctx, L) == 0
        if not used_true:
            _, L, _ = gradient_hessian(prob, q, project=True)
            if B.cholesky(prob.ctx, L) != 0:
                raise RuntimeError("projected Newton matrix is not positive definite")
        info["true_hessian_steps"] += int(used_true)
        dq = -g.clone()
        B.cholesky_solve(prob.ctx, L, dq)
        e0 = energy(prob, q)
        slope = float(g @ dq)
        # the predicted decrease (half the Newton decrement) is below the
        # rounding level of the energy: nothing left to gain
        if -0.5 * slope <= 1e-15 * abs(e0):
            info["converged"] = True
            break
        alpha, _, _ = B.ccd_max_step(prob.ctx, prob.scene, q, dq, prob.dhat)
        alpha = min(1.0, alpha)
        info["alpha_ccd"].append(alpha)
        while True:
            q1 = q + alpha * dq
            if energy(prob, q1) <= e0 + 1e-4 * alpha * slope or alpha < 1e-12:
                break
            alpha *= 0.5
        info["alpha"].append(alpha)
        if float(torch.linalg.vector_norm(q1 - q)) == 0.0:
            info["converged"] = True
            break
        q = q1
    info["iters"] = it
    return q, info


def adjoint(prob: StepProblem, q_star, dLdq):
    """Adjoint of the converged step.  Returns (dL/dq_n, dL/dv_n,
    dL/dtheta[6], used_true_hessian)."""
    g, H, (pt, ee) = gradient_hessian(prob, q_star, project=False)
    L = H.clone()
    used_true = B.cholesky(prob.ctx, L) == 0
    if not used_true:
        _, L, _ = gradient_hessian(prob, q_star, project=True)
        if B.cholesky(prob.ctx, L) != 0:
            raise RuntimeError("adjoint matrix is not positive definite")
    lam = dLdq.clone()
    B.cholesky_solve(prob.ctx, L, lam)
    dq_n = prob.M @ lam
    dv_n = prob.h * dq_n
    # cross term: d(grad_q E)/d theta_k = W^T H_x (dx_off/dtheta_k) (times h^2 kappa)
    T = prob.pose_tangents()
    zero = torch.zeros(prob.n, dtype=torch.float64, device=prob.ctx.torch_device)
    dth = np.zeros(6)
    for k in range(6):
        cross = B.barrier_hvp(prob.ctx, prob.scene, q_star, pt, ee, prob.dhat, prob.h ** 2 * prob.kappa,
                              prob.barrier_flags & B.SQDIST, zero, T[k].contiguous())
        dth[k] = -float(lam @ cross)
    return dq_n, dv_n, dth, used_true
