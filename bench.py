"""Benchmark of the contact stage on one MI355X.

One step = one full pass of the contact stage over a resident scene:
candidate pairs (broad phase), barrier energy + reduced gradient + reduced
PSD-projected Hessian (BSR) over all candidates (narrow phase inside), and
the CCD step bound for a displacement dq.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "contact pairs/s (barrier+reduce) & CCD pairs/s, FP64, % HBM roofline"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 flops per active pair (ENERGY|GRAD|HESS|PROJECT), by the
# feature function of its distance type (point-point / point-line /
# triple-product), in the 9-dimensional translation-free basis:
#   distance derivatives          30 / 350 / 700
#   barrier chain rule            220
#   basis change G^T H G          200
#   9x9 eigen-projection          9 n^3 + 2 n^2 (n+1)/2 = 6561 + 810
#   12x12 blocks Q X Q^T          810
#   W expansion (16 weights)      136 block pairs x 19 = 2584
#   gradient expansion            132
FLOPS_COMMON = 220 + 200 + 6561 + 810 + 810 + 2584 + 132
FLOPS_DIST = {"PP": 30, "PL": 350, "TRI": 700}
PT_FN = ["PP", "PP", "PP", "PL", "PL", "PL", "TRI"]
EE_FN = ["PP", "PP", "PP", "PP", "PL", "PL", "PL", "PL", "TRI"]


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="config2", choices=["config1", "config2", "config3"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-queries", type=int, default=2000,
                    help="oracle CPU baseline: number of sampled query primitives per kind")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB (reference for HBM counters)")
    return ap.parse_args()


def make_scene(name, seed):
    import scenes
    return {"config1": scenes.config1, "config2": scenes.config2, "config3": scenes.config3}[name](seed)


def cpu_baseline(sc, n_queries, log):
    """Oracle (single thread) on a bounded sample: brute-force candidate
    queries for a sample of vertices and edges (untimed), then the oracle's
    barrier + reduction timed on the pairs they produce."""
    import numpy as np

    import oracle as O
    dof = np.diff(sc.W_rowptr) > 0
    x = O.embed(sc, sc.q)
    rng = np.random.default_rng(sc.seed + 99)
    # sample queries among vertices/edges that have a DoF and lie near the
    # other bodies' boxes: use every vertex/edge whose own dhat box meets
    # another body's vertex within 2 dhat (cheap numpy filter on a grid)
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    e = sc.edges.astype(np.int64)
    adj = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(sc.n_vert, sc.n_vert))
    _, body = connected_components(adj, directed=False)
    # vertices within 2 dhat (grid cells) of a vertex of another body
    h = 2 * sc.dhat
    keys = np.floor(x / h).astype(np.int64)
    keys -= keys.min(axis=0)
    span = keys.max(axis=0) + 3
    near = np.zeros(sc.n_vert, dtype=bool)
    code = lambda k: (k[:, 0] * span[1] + k[:, 1]) * span[2] + k[:, 2]
    base = code(keys + 1)
    order = np.argsort(base)
    sb = base[order]
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                c = code(keys + 1 + np.array([dx, dy, dz]))
                lo = np.searchsorted(sb, c, side="left")
                hi = np.searchsorted(sb, c, side="right")
                has = hi > lo
                # another body present in that cell?  compare with min/max body label in the cell
                idx = np.nonzero(has)[0]
                if len(idx) == 0:
                    continue
                bl = body[order]
                mn = np.minimum.reduceat(bl, lo[idx]) if len(idx) else None
                mx = np.maximum.reduceat(bl, lo[idx])
                other = (mn != body[idx]) | (mx != body[idx])
                near[idx[other]] = True
    vq = np.nonzero(near & dof)[0]
    eq = np.nonzero(near[sc.edges[:, 0]] & near[sc.edges[:, 1]])[0]
    vq = rng.choice(vq, size=min(n_queries, len(vq)), replace=False) if len(vq) else vq
    eq = rng.choice(eq, size=min(n_queries, len(eq)), replace=False) if len(eq) else eq
    t0 = time.perf_counter()
    pt = [(v, f) for v in sorted(vq) for f in O.pt_query(sc, x, sc.dhat, v)]
    ee = [(a, b) for a in sorted(eq) for b in O.ee_query(sc, x, sc.dhat, a)]
    t_query = time.perf_counter() - t0
    pt = np.array(pt, dtype=np.int32).reshape(-1, 2)
    ee = np.array(ee, dtype=np.int32).reshape(-1, 2)
    flags = O.ENERGY | O.GRAD | O.HESS | O.PROJECT | (O.MOLLIFY if sc.name == "config3" else 0)
    t0 = time.perf_counter()
    r = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags)
    t_red = time.perf_counter() - t0
    log(f"cpu baseline: {len(vq)} PT + {len(eq)} EE queries ({t_query:.1f} s untimed) -> "
        f"{len(pt)} + {len(ee)} candidates, {r['n_active']} active, barrier+reduce {t_red:.2f} s")
    return {"value": r["n_active"] / t_red if t_red > 0 else None, "unit": "contact pairs/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{sc.name}: oracle brute-force candidates of {len(vq)} vertices and {len(eq)} edges "
                       f"sampled near contact ({len(pt) + len(ee)} candidates, {r['n_active']} active); timed: "
                       f"or_barrier_reduce energy+grad+projected dense Hessian, 1 thread, {t_red:.2f} s")}


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    import numpy as np
    import torch

    import paper_2409_16385_amd as E

    t0 = time.perf_counter()
    sc = make_scene(a.config, a.seed)
    log(f"{sc.summary()} (generated in {time.perf_counter() - t0:.1f} s)")
    ctx = E.Context(0)
    dev = ctx.torch_device
    dsc = E.Scene.from_host(ctx, sc)
    q = torch.as_tensor(sc.q, device=dev)
    dq = torch.as_tensor(sc.dq, device=dev)
    flags = E.ENERGY | E.GRAD | E.HESS | E.PROJECT | (E.MOLLIFY if a.config == "config3" else 0)

    info = {}

    def step():
        pt, ee = E.build_candidates(ctx, dsc, q, sc.dhat)
        r = E.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags, hess="bsr", count=False)
        alpha, ncand, capped = E.ccd_max_step(ctx, dsc, q, dq, sc.dhat)
        info.update(pt=pt, ee=ee, r=r, alpha=alpha, ncand=ncand, capped=capped)

    if a.copy_calibration_mib:
        src = torch.ones(a.copy_calibration_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # workload counts (outside the timed region)
    pt, ee = info["pt"], info["ee"]
    ap, tp, ae, te = E.narrow_phase(ctx, dsc, q, pt, ee, sc.dhat)
    n_act_pt, n_act_ee = int(ap.numel()), int(ae.numel())
    n_active = n_act_pt + n_act_ee
    tpc = np.bincount(tp.cpu().numpy(), minlength=7)
    tec = np.bincount(te.cpu().numpy(), minlength=9)
    flops_pt = sum(int(tpc[i]) * (FLOPS_COMMON + FLOPS_DIST[PT_FN[i]]) for i in range(7))
    flops_ee = sum(int(tec[i]) * (FLOPS_COMMON + FLOPS_DIST[EE_FN[i]]) for i in range(9))
    log(f"candidates pt={pt.shape[0]} ee={ee.shape[0]} active pt={n_act_pt} ee={n_act_ee} "
        f"ccd candidates={info['ncand']} alpha={info['alpha']:.6g} nnzb={info['r']['hess'][1].numel()}")
    log(f"PT types {tpc.tolist()} EE types {tec.tolist()}")

    if not a.no_profile:
        ctx.profile(True)
        ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / a.steps
    prof = ctx.profile_read(reset=True) if not a.no_profile else {}
    ctx.profile(False)
    for k, (ms, n) in prof.items():
        if n:
            log(f"kernel {k:16s} {ms / n * 1e3:10.1f} us/launch x {n}")

    # call-level breakdown with events (separate short run)
    ev = {}
    for name, fn in (("candidates", lambda: E.build_candidates(ctx, dsc, q, sc.dhat)),
                     ("barrier_reduce", lambda: E.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags,
                                                                 hess="bsr", count=False)),
                     ("ccd", lambda: E.ccd_max_step(ctx, dsc, q, dq, sc.dhat))):
        fn()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ev[name] = 1e3 * (time.perf_counter() - t1) / 5

    # dominant kernel and its roofline
    roofline = None
    if prof:
        dom = max(prof, key=lambda k: prof[k][0])
        ms, n = prof[dom]
        avg_s = ms / n / 1e3
        if dom in ("barrier_pt", "barrier_ee"):
            fl = flops_pt if dom == "barrier_pt" else flops_ee
            ach = fl / avg_s / 1e12
            roofline = {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / PEAK_FP64_TFLOPS, "traffic": None, "kernel": dom,
                        "avg_launch_us": avg_s * 1e6,
                        "per_unit": f"{FLOPS_COMMON}+dist flop per active pair"}
        else:
            roofline = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": None, "traffic": None, "kernel": dom, "avg_launch_us": avg_s * 1e6}
        roofline["kernels_us"] = {k: round(v[0] / v[1] * 1e3, 2) for k, v in prof.items() if v[1]}
        # the barrier kernels' own roofline is reported too
        for k, fl in (("barrier_pt", flops_pt), ("barrier_ee", flops_ee)):
            if prof.get(k, (0, 0))[1]:
                s_ = prof[k][0] / prof[k][1] / 1e3
                roofline[f"{k}_tflops"] = fl / s_ / 1e12

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(sc, a.cpu_queries, log)

    value = n_active / (ms_per_step / 1e3)
    out = {
        "metric": METRIC, "value": value, "unit": "contact pairs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{a.config} ({sc.name}): n_vert={sc.n_vert} n_face={sc.n_face} "
                               f"n_edge={sc.n_edge} n_node={sc.n_node} dhat={sc.dhat:g}",
                   "active_pairs": n_active, "candidates": int(pt.shape[0] + ee.shape[0]),
                   "ccd_candidates": info["ncand"], "seed": a.seed},
        "barrier_reduce_pairs_per_s": n_active / (ev["barrier_reduce"] / 1e3),
        "ccd_pairs_per_s": info["ncand"] / (ev["ccd"] / 1e3),
        "call_ms": ev, "alpha": info["alpha"],
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
