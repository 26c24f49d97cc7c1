"""Oracle of one implicit time step and its adjoint (TEST INFRASTRUCTURE
ONLY): plain numpy around the contact oracle of eipc_oracle.c.

The step (Sec. III-A, Eq. 5-6; contact terms Sec. III-B, Eq. 10-12):

    E(q) = 1/2 (q - qt)^T M (q - qt) + h^2 (Phi(q) - f^T q) + kappa h^2 sum_k b(d_k(W q + x_off)),
    qt = q_n + h v_n,

with the reduced mass M = J^T M_x J (Eq. 1) built from interior samples of
the body, each of volume V_s and density rho, at barycentric weights w_s in
its coarse tet: M = sum_s rho V_s (w_s w_s^T) (x) I3 (nodes that no sample
reaches get a lumped mass of 1e-3 of the mean diagonal, so the Newton
matrix stays definite); Phi the elastic energy of the coarse tets with the
aggregated volumes V_T of their samples (Eq. 15), here linear elasticity
written through the strain-displacement matrix B (Voigt) and the isotropic
elasticity matrix C, K_T = V_T B^T C B (the rest-pose linearization of the
paper's corotational model: the two share energy, gradient and Hessian at
the rest shape); gravity f = J^T f_ext (Eq. 16).

The paper's linear corotational model is available as the elastic term
of the step (Step(si, "corotational"), function corotational): the same
energy with the rotation of each tet's deformation gradient factored out,
its Newton matrix taking the warped stiffness R K0 R^T; the adjoint is
taken with the linear model, whose Hessian is exact.

Solved by projected Newton (Sec. III-C): the true Hessian when Cholesky
accepts it, else the per-pair PSD-projected one; the step length clamped
by the oracle's conservative CCD bound over the swept candidates, then
halved until the Armijo condition (1e-4) holds.  Stops when |grad E| <= tol
|M qt|, when half the Newton decrement is below 1e-15 |E|, or when a step
leaves q unchanged.

Adjoint of L(q*) at the converged q* (grad E(q*, q_n, theta) = 0):
lambda = H(q*)^-1 dL/dq*, dL/dq_n = M lambda, dL/dv_n = h M lambda and
dL/dtheta_k = -lambda^T d(grad_q E)/d theta_k, where theta moves the
kinematic body's vertices (their x_off) and the cross term is the
barrier's Hessian applied to the pose tangent of x_off (the HVP's v_off).
"""
from __future__ import annotations

import math

import numpy as np

from . import barrier_reduce, barrier_hvp, candidates_grid, ccd_toi_threads, embed, scene as _oscene
from . import ENERGY, GRAD, HESS, PROJECT, OK


def _voigt_B(X: np.ndarray) -> np.ndarray:
    """6 x 12 strain-displacement matrix of a linear tet with rest corners X
    (engineering shear strains: exx, eyy, ezz, 2eyz, 2exz, 2exy)."""
    Dm = np.column_stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]])
    Dinv = np.linalg.inv(Dm)
    grads = np.vstack([-Dinv.sum(axis=0), Dinv])  # d N_a / d X (rows)
    B = np.zeros((6, 12))
    for a in range(4):
        gx, gy, gz = grads[a]
        c = 3 * a
        B[0, c] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1], B[3, c + 2] = gz, gy
        B[4, c], B[4, c + 2] = gz, gx
        B[5, c], B[5, c + 1] = gy, gx
    return B


def _voigt_C(young: float, poisson: float) -> np.ndarray:
    lam = young * poisson / ((1 + poisson) * (1 - 2 * poisson))
    mu = young / (2 * (1 + poisson))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[[0, 1, 2], [0, 1, 2]] += 2 * mu
    C[[3, 4, 5], [3, 4, 5]] = mu
    return C


def assemble(si):
    """(M, K, f) of the step inputs (scenes.step_inputs)."""
    n_node = len(si.grid_nodes)
    M = np.zeros((n_node, n_node))
    f = np.zeros((n_node, 3))
    for s in range(len(si.sample_tet)):
        tn = si.tets[si.sample_tet[s]]
        w = si.sample_w[s]
        m = si.rho * si.sample_vol
        for a in range(4):
            f[tn[a], 2] -= m * si.g * w[a]
            for b in range(4):
                M[tn[a], tn[b]] += m * w[a] * w[b]
    d = np.diag(M).copy()
    empty = d <= 0.0
    if empty.any():
        M[empty, empty] = 1e-3 * d[~empty].mean()
    VT = np.zeros(len(si.tets))
    np.add.at(VT, si.sample_tet, si.sample_vol)
    C = _voigt_C(si.young, si.poisson)
    K = np.zeros((3 * n_node, 3 * n_node))
    for t in np.nonzero(VT)[0]:
        tn = si.tets[t]
        B = _voigt_B(si.grid_nodes[tn])
        idx = (3 * tn[:, None] + np.arange(3)[None, :]).reshape(-1)
        K[np.ix_(idx, idx)] += VT[t] * (B.T @ C @ B)
    return np.kron(M, np.eye(3)), K, f.reshape(-1)


def elastic_tets(si):
    """(node indices [4], rest shape-function gradients g_a as rows [4, 3],
    aggregated volume V_T) of each coarse tet that holds samples."""
    VT = np.zeros(len(si.tets))
    np.add.at(VT, si.sample_tet, si.sample_vol)
    out = []
    for t in np.nonzero(VT)[0]:
        tn = si.tets[t]
        X = si.grid_nodes[tn]
        Dinv = np.linalg.inv(np.column_stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]]))
        out.append((tn, np.vstack([-Dinv.sum(axis=0), Dinv]), VT[t]))
    return out


def corotational(si, q, tets=None, want_hess=True):
    """Linear corotational elasticity on the coarse tets (the paper's model,
    Sec. IV-A), per tet with deformation gradient F = sum_a x_a g_a^T and R
    the rotation of its polar decomposition (from the SVD, F = U S V^T,
    R = U V^T):

        energy   V (mu |F - R|^2 + lam/2 tr(R^T F - I)^2),
        gradient V P g_a at node a, P = 2 mu (F - R) + lam tr(R^T F - I) R,
        Hessian  the warped stiffness R K0 R^T: K0 the tet's linear
                 stiffness, its (a, b) block V (mu (g_b g_a^T + (g_a.g_b) I)
                 + lam g_a g_b^T), each block rotated by R on both sides
                 (positive semidefinite; at the rest shape it is the linear
                 stiffness).

    Returns (energy, gradient [3 n], Hessian [3 n, 3 n] or None)."""
    lam = si.young * si.poisson / ((1 + si.poisson) * (1 - 2 * si.poisson))
    mu = si.young / (2 * (1 + si.poisson))
    tets = elastic_tets(si) if tets is None else tets
    n = len(si.grid_nodes)
    x = np.asarray(q).reshape(-1, 3)
    e = 0.0
    g = np.zeros(3 * n)
    H = np.zeros((3 * n, 3 * n)) if want_hess else None
    I3 = np.eye(3)
    for tn, G, V in tets:
        F = sum(np.outer(x[tn[a]], G[a]) for a in range(4))
        U, _, Vt = np.linalg.svd(F)
        R = U @ Vt
        if np.linalg.det(R) < 0:
            U[:, -1] *= -1
            R = U @ Vt
        tr = np.trace(R.T @ F) - 3.0
        e += V * (mu * np.sum((F - R) ** 2) + 0.5 * lam * tr * tr)
        P = 2 * mu * (F - R) + lam * tr * R
        for a in range(4):
            g[3 * tn[a]:3 * tn[a] + 3] += V * (P @ G[a])
        if want_hess:
            for a in range(4):
                for b in range(4):
                    ga, gb = G[a], G[b]
                    blk = V * (mu * (np.outer(gb, ga) + (ga @ gb) * I3) + lam * np.outer(ga, gb))
                    H[3 * tn[a]:3 * tn[a] + 3, 3 * tn[b]:3 * tn[b] + 3] += R @ blk @ R.T
    return e, g, H


class Step:
    """The oracle step of the given inputs; pose theta (tx, ty, tz, rx, ry,
    rz) places the kinematic body, rotated about its rest centroid.
    elastic: "linear" (the constant stiffness K) or "corotational" (the
    paper's model, Newton matrix with the warped stiffness)."""

    def __init__(self, si, elastic="linear"):
        self.si = si
        self.sc = si.scene
        self.elastic = elastic
        self._tets = elastic_tets(si)
        self.M, self.K, self.f = assemble(si)
        self.q_rest = si.grid_nodes.reshape(-1).copy()
        self.q_n = si.q_n.copy()
        self.v_n = si.v_n.copy()
        self.h, self.kappa, self.dhat = si.h, self.sc.kappa, self.sc.dhat
        self.x_off0 = self.sc.x_off.copy()
        self.set_pose(np.zeros(6))

    def set_pose(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        rest = self.si.kin_rest
        c = rest.mean(axis=0)
        r = theta[3:]
        th = float(np.linalg.norm(r))
        R = np.eye(3)
        if th > 0:
            k = r / th
            Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
            R = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * (Kx @ Kx)
        x_off = self.x_off0.copy()
        x_off[self.si.kin_rows] = (rest - c) @ R.T + c + theta[:3]
        self.sc.x_off = x_off
        self._osc = _oscene(self.sc)

    def pose_tangents(self):
        """d x_off / d theta at theta = 0: [6, n_vert, 3]."""
        rest = self.si.kin_rest
        c = rest.mean(axis=0)
        T = np.zeros((6, self.sc.n_vert, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1.0
            T[k, self.si.kin_rows] = e
            T[3 + k, self.si.kin_rows] = np.cross(e, rest - c)
        return T

    def _contact(self, q, flags, hess):
        x = embed(self._osc, q)
        pt, ee = candidates_grid(self._osc, x, self.dhat)
        r = barrier_reduce(self._osc, q, pt, ee, self.dhat, self.h ** 2 * self.kappa, flags, hess=hess)
        if r["status"] != OK:
            raise RuntimeError(f"contact oracle status {r['status']}")
        return r, pt, ee

    def _elastic(self, q, want_hess):
        if self.elastic == "corotational":
            return corotational(self.si, q, self._tets, want_hess)
        dr = q - self.q_rest
        Kd = self.K @ dr
        return 0.5 * dr @ Kd, Kd, self.K

    def energy(self, q):
        qt = self.q_n + self.h * self.v_n
        d = q - qt
        r, _, _ = self._contact(q, ENERGY, False)
        e_el, _, _ = self._elastic(q, False)
        return 0.5 * d @ (self.M @ d) + self.h ** 2 * (e_el - self.f @ q) + r["energy"]

    def grad_hess(self, q, project):
        qt = self.q_n + self.h * self.v_n
        r, pt, ee = self._contact(q, ENERGY | GRAD | HESS | (PROJECT if project else 0), True)
        _, g_el, K_el = self._elastic(q, True)
        g = self.M @ (q - qt) + self.h ** 2 * (g_el - self.f) + r["grad"]
        H = self.M + self.h ** 2 * K_el + r["hess"]
        return g, H, (pt, ee)

    def step_bound(self, q, dq):
        x = embed(self._osc, q)
        p = embed(self._osc, dq, off=None)
        spt, see = candidates_grid(self._osc, x, self.dhat, x1=x + p)
        tp, _ = ccd_toi_threads(self._osc, x, p, 0, spt)
        te, _ = ccd_toi_threads(self._osc, x, p, 1, see)
        return min(1.0, tp.min(initial=1.0), te.min(initial=1.0))

    def solve(self, tol=1e-12, max_iter=100):
        q = self.q_n.copy()
        qt = self.q_n + self.h * self.v_n
        scale = np.linalg.norm(self.M @ qt)
        it = 0
        for it in range(max_iter):
            g, H, _ = self.grad_hess(q, project=False)
            if np.linalg.norm(g) <= tol * scale:
                break
            try:
                L = np.linalg.cholesky(H)
            except np.linalg.LinAlgError:
                _, Hp, _ = self.grad_hess(q, project=True)
                L = np.linalg.cholesky(Hp)
            dq = -np.linalg.solve(L.T, np.linalg.solve(L, g))
            e0 = self.energy(q)
            slope = g @ dq
            if -0.5 * slope <= 1e-15 * abs(e0):
                break
            alpha = self.step_bound(q, dq)
            while True:
                q1 = q + alpha * dq
                if self.energy(q1) <= e0 + 1e-4 * alpha * slope or alpha < 1e-12:
                    break
                alpha *= 0.5
            if np.linalg.norm(q1 - q) == 0.0:
                break
            q = q1
        return q, it

    def adjoint(self, q_star, dLdq):
        """(dL/dq_n, dL/dv_n, dL/dtheta[6], the Cholesky residual of the
        adjoint solve |H lambda - dL/dq| / |dL/dq|)."""
        _, H, (pt, ee) = self.grad_hess(q_star, project=False)
        L = np.linalg.cholesky(H)
        lam = np.linalg.solve(L.T, np.linalg.solve(L, dLdq))
        res = np.linalg.norm(H @ lam - dLdq) / np.linalg.norm(dLdq)
        dq_n = self.M @ lam
        T = self.pose_tangents()
        dth = np.zeros(6)
        zero = np.zeros_like(q_star)
        for k in range(6):
            st, cross, _ = barrier_hvp(self._osc, q_star, pt, ee, self.dhat, self.h ** 2 * self.kappa, 0, zero,
                                       v_off=T[k])
            dth[k] = -lam @ cross
        return dq_n, self.h * dq_n, dth, res
