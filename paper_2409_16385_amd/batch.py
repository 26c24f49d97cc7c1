"""Batched contact stage: many independent scenes in one planned step,
captured once in a HIP graph and replayed per Newton iteration.

A batch is one library scene whose arrays are the concatenation of the
scenes' arrays with global vertex / node numbering and a scene id per
vertex; the ragged layout is described by int64 offsets per scene
(``vert_off``, ``node_off``, ``face_off``, ``edge_off``).  All kernels run
over the whole batch at once: broad-phase cells are keyed by (scene, cell),
so pairs never join two scenes, and energies and step bounds are reduced
per scene.  The autotuner picks the broad-phase cell size and the
workgroups per compute unit of the grid-stride kernels by timing the
batch itself.

This module only marshals arguments and drives the library; every step of
the contact stage runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import binding as B


@dataclasses.dataclass
class HostBatch:
    """Concatenated host arrays of a list of scenes (numpy)."""
    n_scene: int
    n_node: int
    faces: np.ndarray
    edges: np.ndarray
    W_rowptr: np.ndarray
    W_col: np.ndarray
    W_val: np.ndarray
    x_off: np.ndarray | None
    x_rest: np.ndarray | None
    q: np.ndarray
    dq: np.ndarray
    dx_off: np.ndarray | None
    vert_scene: np.ndarray
    vert_off: np.ndarray   # int64 [n_scene + 1]
    node_off: np.ndarray
    face_off: np.ndarray
    edge_off: np.ndarray
    dhat: float
    kappa: float


def concat(scenes) -> HostBatch:
    """Concatenate scenes (objects with the fields of scenes.Scene) into one
    batch.  All scenes must share dhat and kappa."""
    if not scenes:
        raise ValueError("empty batch")
    dhat, kappa = scenes[0].dhat, scenes[0].kappa
    if any(s.dhat != dhat or s.kappa != kappa for s in scenes):
        raise ValueError("scenes of one batch must share dhat and kappa")
    nv = np.array([s.n_vert for s in scenes], dtype=np.int64)
    nn = np.array([s.n_node for s in scenes], dtype=np.int64)
    nf = np.array([s.n_face for s in scenes], dtype=np.int64)
    ne = np.array([s.n_edge for s in scenes], dtype=np.int64)
    vo = np.concatenate([[0], np.cumsum(nv)])
    no = np.concatenate([[0], np.cumsum(nn)])
    fo = np.concatenate([[0], np.cumsum(nf)])
    eo = np.concatenate([[0], np.cumsum(ne)])
    if vo[-1] >= 2**31 or no[-1] * 3 >= 2**31:
        raise ValueError("batch too large for int32 indices")
    nnz = np.array([len(s.W_col) for s in scenes], dtype=np.int64)
    zo = np.concatenate([[0], np.cumsum(nnz)])
    faces = np.concatenate([s.faces.astype(np.int64) + vo[i] for i, s in enumerate(scenes)]).astype(np.int32)
    edges = np.concatenate([s.edges.astype(np.int64) + vo[i] for i, s in enumerate(scenes)]).astype(np.int32)
    rowptr = np.concatenate([[0]] + [s.W_rowptr[1:].astype(np.int64) + zo[i] for i, s in enumerate(scenes)])
    col = np.concatenate([s.W_col.astype(np.int64) + no[i] for i, s in enumerate(scenes)])
    val = np.concatenate([s.W_val for s in scenes])

    def cat_opt(name):
        parts = [getattr(s, name) for s in scenes]
        if all(p is None for p in parts):
            return None
        return np.concatenate([np.zeros((s.n_vert, 3)) if p is None else np.asarray(p).reshape(-1, 3)
                               for s, p in zip(scenes, parts)])

    return HostBatch(
        n_scene=len(scenes), n_node=int(no[-1]), faces=faces, edges=edges,
        W_rowptr=rowptr.astype(np.int32), W_col=col.astype(np.int32), W_val=val,
        x_off=cat_opt("x_off"), x_rest=cat_opt("x_rest"),
        q=np.concatenate([s.q for s in scenes]), dq=np.concatenate([s.dq for s in scenes]),
        dx_off=cat_opt("dx_off"),
        vert_scene=np.repeat(np.arange(len(scenes), dtype=np.int32), nv),
        vert_off=vo, node_off=no, face_off=fo, edge_off=eo, dhat=float(dhat), kappa=float(kappa))


DEFAULT_FLAGS = B.ENERGY | B.GRAD | B.HESS | B.PROJECT
# workgroups per CU of the pair-terms, expansion, narrow and CCD kernels: the
# library context's defaults
DEFAULT_WG_PER_CU = (1, 2, 4, 4)


class Batch:
    """Device batch with a planned, graph-captured contact step.

    ``q``, ``dq`` (and ``dx_off``) are device tensors with fixed storage:
    write new values into them (``copy_``) and call ``replay()``.  The batch
    owns a library context of its own on the device of ``ctx``: a captured
    graph holds that context's scratch addresses, which stay fixed as long
    as only planned steps run on it.
    """

    def __init__(self, ctx: B.Context, hb: HostBatch, flags: int = DEFAULT_FLAGS, s: float = 0.1,
                 t_max: float = 1.0, max_iter: int = 100000):
        dev = ctx.torch_device
        self.ctx, self.hb = B.Context(ctx.device), hb
        self.scene = B.Scene(ctx, hb.faces, hb.edges, hb.W_rowptr, hb.W_col, hb.W_val, hb.n_node, hb.x_off,
                             hb.x_rest, n_scene=hb.n_scene, vert_scene=hb.vert_scene)
        self.q = torch.as_tensor(hb.q, dtype=torch.float64, device=dev).clone()
        self.dq = torch.as_tensor(hb.dq, dtype=torch.float64, device=dev).clone()
        self.dx_off = None if hb.dx_off is None else torch.as_tensor(hb.dx_off, device=dev).reshape(-1).clone()
        self.flags, self.s, self.t_max, self.max_iter = flags, s, t_max, max_iter
        self.plan: B.Plan | None = None
        self.out: B.StepOut | None = None
        self.graph: torch.cuda.CUDAGraph | None = None
        self.tuning = {"cell_scale": 2.0, "wg_per_cu": [8, 2, 4, 4], "query_cells": 1}

    # -- planning ---------------------------------------------------------
    def make_plan(self, margin: float = 1.5):
        """Measure capacities at the current q, dq and reserve scratch."""
        self.graph = None
        self.plan = B.plan_step(self.ctx, self.scene, self.q, self.hb.dhat, self.dq, self.dx_off, margin,
                                with_hess=bool(self.flags & B.HESS))
        self.out = B.StepOut(self.ctx, self.scene, self.plan, self.flags, with_alpha=True)
        return self.plan

    def step(self):
        """Enqueue one step eagerly (no synchronization)."""
        if self.plan is None:
            self.make_plan()
        B.contact_step(self.ctx, self.scene, self.plan, self.q, self.hb.dhat, self.hb.kappa, self.out, self.dq,
                       self.dx_off, self.flags, self.s, self.t_max, self.max_iter)

    def status(self) -> int:
        """Synchronize and read the step's status (a capacity overflow means
        the plan must be remade and the graph captured again)."""
        return self.ctx.sync_status()

    # -- graph ------------------------------------------------------------
    def capture(self):
        """Capture one step in a graph (the plan's scratch is already
        reserved, so nothing is allocated while capturing)."""
        if self.plan is None:
            self.make_plan()
        self.step()  # warm: every buffer at its planned size
        torch.cuda.synchronize(self.ctx.torch_device)
        if self.status() not in (B.OK, B.WARN_CCD_CAPPED):
            raise B.EipcError(B.ERR_CAPACITY, "step failed before capture")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def run_checked(self, margin: float = 1.5, use_graph: bool = True) -> int:
        """One step; on a capacity overflow re-plan (larger margin) and run
        again.  Synchronizes."""
        for _ in range(3):
            self.replay() if use_graph else self.step()
            st = self.status()
            if st != B.ERR_CAPACITY:
                return st
            margin *= 2.0
            self.make_plan(margin)
        raise B.EipcError(B.ERR_CAPACITY, "re-planning did not converge")

    # -- results ----------------------------------------------------------
    def counts(self) -> dict:
        c = self.out.counts.cpu().numpy()
        return {"cand_pt": int(c[0]), "cand_ee": int(c[1]), "active": int(c[2]), "swept_pt": int(c[3]),
                "swept_ee": int(c[4])}

    def per_scene_grad(self, i: int) -> torch.Tensor:
        no = self.hb.node_off
        return self.out.grad[3 * no[i]:3 * no[i + 1]]

    # -- autotuning -------------------------------------------------------
    def _time_steps(self, reps: int) -> float:
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        self.step()
        ev0.record()
        for _ in range(reps):
            self.step()
        ev1.record()
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / reps

    def _device_ms(self, reps: int) -> float:
        """Summed kernel time of one step, each kernel timed alone (the two
        chains one after the other), averaged over reps eager steps."""
        self.step()
        torch.cuda.synchronize(self.ctx.torch_device)
        self.ctx.profile(True, serial=True)
        try:
            self.ctx.profile_read(reset=True)
            for _ in range(reps):
                self.step()
            prof = self.ctx.profile_read(reset=True)
        finally:
            self.ctx.profile(False)
        return sum(ms for ms, _ in prof.values()) / reps

    def autotune(self, cell_scales=(2.0, 3.0, 4.0, 6.0), query_modes=(0, 5, 12, 15), wg_values=(1, 2, 4, 8, 16),
                 reps: int = 3, margin: float = 1.5, verbose: bool = False) -> dict:
        """Pick the broad-phase cell scale and work split per query kind
        (whole-step time, re-planning for each pair of values; among pairs
        within 1% of the fastest, the one with the least device time summed
        over the step's kernels, each timed alone), then for each
        grid-stride kernel family in turn the workgroups per CU (values
        from wg_values, starting from the library's defaults; whole-step
        time; a change is kept when it saves more than 2%)."""
        # start from the library's defaults (where offered): a family keeps
        # its start unless a value beats it by the noise margin below, and
        # the expansion (one workgroup per CU by its LDS) is slow at 4
        wg = [v if v in wg_values else wg_values[len(wg_values) // 2] for v in DEFAULT_WG_PER_CU]
        trace, timed = [], []
        for cs in cell_scales:
            for qm in query_modes:
                B.set_tuning(self.ctx, cs, wg, qm)
                self.make_plan(margin)
                ms = self._time_steps(reps)
                if self.status() not in (B.OK, B.WARN_CCD_CAPPED):
                    continue
                trace.append((f"cell_scale/query_cells {qm}", cs, ms))
                timed.append((ms, cs, qm))
        fastest = min(timed)[0]
        ties = [(cs, qm) for ms, cs, qm in timed if ms <= 1.01 * fastest]
        if len(ties) > 1:
            # the two chains run side by side, so pairs can tie on step time
            # while one of them keeps the device busier
            scored = []
            for cs, qm in ties:
                B.set_tuning(self.ctx, cs, wg, qm)
                self.make_plan(margin)
                dev_ms = self._device_ms(reps)
                trace.append((f"device ms, query_cells {qm}", cs, dev_ms))
                scored.append((dev_ms, cs, qm))
            _, cs, qm = min(scored)
        else:
            cs, qm = ties[0]
        B.set_tuning(self.ctx, cs, wg, qm)
        self.make_plan(margin)
        # workgroups per CU of each grid-stride family (pair terms,
        # expansion, narrow phase, CCD) by coordinate descent on the whole
        # step time: the two kinds' chains run concurrently, so a kernel's
        # own time is not the step's
        best_ms = self._time_steps(reps)
        for k in range(4):
            for v in wg_values:
                if v == wg[k]:
                    continue
                trial = list(wg)
                trial[k] = v
                B.set_tuning(self.ctx, cs, trial, qm)
                ms = self._time_steps(reps)
                trace.append((f"wg_per_cu[{k}]", v, ms))
                if ms < 0.98 * best_ms:  # a change must beat timing noise
                    best_ms, wg = ms, trial
            B.set_tuning(self.ctx, cs, wg, qm)
        self.tuning = {"cell_scale": cs, "wg_per_cu": wg, "query_cells": qm, "trace": trace}
        self.make_plan(margin)
        if verbose:
            print("autotune:", {k: v for k, v in self.tuning.items() if k != "trace"})
        return self.tuning


def sequential_reference(ctx: B.Context, scenes, dev_scenes=None, flags: int = DEFAULT_FLAGS, s: float = 0.1,
                         t_max: float = 1.0, max_iter: int = 100000):
    """The plain single-scene calls for every scene in turn (candidates,
    barrier + reduction with BSR Hessian, step bound).  Returns per-scene
    results and the wall time of the loop."""
    dev = ctx.torch_device
    if dev_scenes is None:
        dev_scenes = [B.Scene.from_host(ctx, sc) for sc in scenes]
    qs = [torch.as_tensor(sc.q, device=dev) for sc in scenes]
    dqs = [torch.as_tensor(sc.dq, device=dev) for sc in scenes]
    res = []
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for sc, dsc, q, dq in zip(scenes, dev_scenes, qs, dqs):
        pt, ee = B.build_candidates(ctx, dsc, q, sc.dhat)
        r = B.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags, hess="bsr", count=True)
        a, nc, _ = B.ccd_max_step(ctx, dsc, q, dq, sc.dhat, sc.dx_off, s, t_max, max_iter)
        res.append({"n_pt": pt.shape[0], "n_ee": ee.shape[0], "n_active": r["n_active"], "energy": r["energy"],
                    "grad": r["grad"], "hess": r["hess"], "alpha": a, "n_swept": nc})
    torch.cuda.synchronize(dev)
    return res, time.perf_counter() - t0
