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

Elastic model (StepProblem.elastic_model): linear (small-strain) isotropic
elasticity, whose Hessian is exact and constant, or the paper's linear
corotational elasticity (Sec. IV-A), whose Newton matrix takes the warped
stiffness R K0 R^T; the adjoint needs the exact Hessian and is taken with
the linear model.  Volumes and masses come from seeded uniform samples of
the body's interior, each carrying V/N, assigned to their coarse
tetrahedron (the aggregation of Eq. 15).  Grid nodes that no sample
reaches get a lumped mass of 1e-3 of the mean node mass.

The mass, gravity and elastic terms (eipc_reduced_mass, eipc_elastic), the
dense Cholesky factorization and solves (eipc_cholesky / _solve) and the
contact terms run in the library; the Newton loop and the dense
matrix-vector products with M are driven from here.
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
    tets: torch.Tensor       # coarse tets (int32 [n_tet, 4])
    vol: torch.Tensor        # their aggregated volumes V_T (Eq. 15)
    young: float
    poisson: float
    # B.ELASTIC_LINEAR or B.ELASTIC_COROTATIONAL
    elastic_model: int = B.ELASTIC_LINEAR
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
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    # mass and gravity from the samples, in the library (with the lumped
    # mass of nodes that no sample reaches)
    M, f = B.reduced_mass(ctx, n_node, torch.as_tensor(tets[si.sample_tet], dtype=torch.int32),
                          torch.as_tensor(si.sample_w), si.rho * si.sample_vol, si.g)
    VT = np.bincount(si.sample_tet, minlength=len(tets)) * si.sample_vol
    tets_d = torch.as_tensor(np.ascontiguousarray(tets, dtype=np.int32), device=dev)
    vol_d = T(VT)
    q_rest = T(nodes.reshape(-1))
    # the linear model's constant stiffness: its Newton matrix at rest
    K = torch.zeros((3 * n_node, 3 * n_node), dtype=torch.float64, device=dev)
    B.elastic(ctx, n_node, tets_d, q_rest, vol_d, si.young, si.poisson, B.ELASTIC_LINEAR, q_rest, hess=K)
    scene = B.Scene.from_host(ctx, sc)
    prob = StepProblem(ctx=ctx, scene=scene, host=sc, M=M, K=K, q_rest=q_rest, f=f, q_n=T(si.q_n),
                       v_n=T(si.v_n), h=si.h, kappa=sc.kappa, dhat=sc.dhat, kin_rows=si.kin_rows,
                       kin_rest=si.kin_rest.copy(), theta=np.zeros(6), tets=tets_d, vol=vol_d, young=si.young,
                       poisson=si.poisson)
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


def _elastic(prob: StepProblem, q, scale, energy=None, grad=None, hess=None):
    B.elastic(prob.ctx, prob.n // 3, prob.tets, prob.q_rest, prob.vol, prob.young, prob.poisson,
              prob.elastic_model, q, scale, energy=energy, grad=grad, hess=hess)


def energy(prob: StepProblem, q) -> float:
    qt = prob.q_n + prob.h * prob.v_n
    d = q - qt
    e_el = torch.zeros(1, dtype=torch.float64, device=q.device)
    _elastic(prob, q.contiguous(), 1.0, energy=e_el)
    e = 0.5 * d @ (prob.M @ d) + prob.h ** 2 * (e_el[0] - prob.f @ q)
    r, _, _ = _contact(prob, q, B.ENERGY, None)
    return float(e + r["energy"][0])


def gradient_hessian(prob: StepProblem, q, project: bool):
    qt = prob.q_n + prob.h * prob.v_n
    proj = B.PROJECT_REDUCED if prob.reduced_projection else B.PROJECT
    flags = B.ENERGY | B.GRAD | B.HESS | (proj if project else 0)
    r, pt, ee = _contact(prob, q, flags, "dense")
    g = prob.M @ (q - qt) - prob.h ** 2 * prob.f + r["grad"]
    H = prob.M + r["hess"]
    # elastic terms (times h^2) added in the library
    _elastic(prob, q.contiguous(), prob.h ** 2, grad=g, hess=H)
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
    dL/dtheta[6], used_true_hessian).  Needs the exact Hessian: linear
    elastic model only (the corotational Newton matrix is the warped
    stiffness)."""
    if prob.elastic_model != B.ELASTIC_LINEAR:
        raise NotImplementedError("the adjoint takes the exact Hessian: use the linear elastic model")
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
