"""Benchmark of the contact stage on one MI355X.

One step = one full pass of the contact stage over resident inputs:
candidate pairs (broad phase), narrow phase, barrier energy + reduced
gradient + reduced PSD-projected Hessian (BSR), and the conservative step
bound for the search direction dq (swept broad phase + CCD).  The timed
step is the planned, synchronization-free entry point replayed from a
captured HIP graph; the plain per-call entry points are timed beside it.
``--config batch`` runs 256 ragged grasp scenes as one batch and compares
with 256 sequential single-scene calls.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
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

# Algorithmic FP64 flops per active pair, split by kernel.  Pair terms
# (distance type fixed): derivatives of the feature function in the
# 9-dimensional translation-free basis (point-point / point-line /
# triple-product) + barrier chain rule + basis change + 9x9 Jacobi
# eigen-projection (9 n^3) + reconstruction (2 n^2 (n+1) / 2).  Expansion:
# blocks z_I^T X z_J over the merged nodes of the pair (16 weights, 136
# block pairs) and the gradient expansion.
FLOPS_TERMS = 220 + 200 + 6561 + 810
FLOPS_DIST = {"PP": 30, "PL": 350, "TRI": 700}
FLOPS_EXPAND = 810 + 2584 + 132
PT_FN = ["PP", "PP", "PP", "PL", "PL", "PL", "TRI"]
EE_FN = ["PP", "PP", "PP", "PP", "PL", "PL", "PL", "PL", "TRI"]
FAMILIES = {
    "query": ("query_count_pt", "query_count_ee", "query_write_pt", "query_write_ee"),
    "pair_terms": ("barrier_pt", "barrier_ee"), "expand": ("expand_pt", "expand_ee"),
    "narrow": ("narrow_pt", "narrow_ee"), "ccd": ("ccd_pt", "ccd_ee", "ccd_long_pt", "ccd_long_ee"),
    "embed": ("embed",),
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="config2", choices=["config1", "config2", "config3", "batch", "resolution"],
                    help="resolution: config 2's surface meshes with object grids from 250 to 32,000 nodes")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n-scene", type=int, default=256, help="scenes in the batch config")
    ap.add_argument("--cpu-queries", type=int, default=2000,
                    help="oracle CPU baseline: number of sampled query primitives per kind")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--no-graph", action="store_true", help="time eager planned steps instead of graph replays")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip timing the per-call entry points (batch: the sequential single-scene calls)")
    ap.add_argument("--tuning", default=None,
                    help="fixed tuning 'cell_scale,wg_terms,wg_expand,wg_narrow,wg_ccd,query_cells' "
                         "(skips the autotuner)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB (reference for HBM counters)")
    return ap.parse_args()


def make_scene(name, seed):
    import scenes
    return {"config1": scenes.config1, "config2": scenes.config2, "config3": scenes.config3}[name](seed)


def _batch_one(i):
    from scenes import scene as S
    return S.batch_scenes(1, seed0=i)[0]


def make_batch(n, seed0, log):
    """The ragged grasp batch, generated in worker processes (spawned
    before the GPU is touched)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        out = list(ex.map(_batch_one, range(seed0, seed0 + n), chunksize=4))
    log(f"generated {n} batch scenes with {workers} processes in {time.perf_counter() - t0:.1f} s")
    return out


def source_digest():
    """Digest of the library sources (traffic counters are valid only for
    the sources they were taken with)."""
    h = hashlib.sha256()
    for d in ("paper_2409_16385_amd/csrc", "include"):
        for f in sorted(os.listdir(os.path.join(ROOT, d))):
            with open(os.path.join(ROOT, d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, tuning=None):
    """HBM bytes per launch from committed counter summaries, when taken
    with the current sources and the same broad-phase tuning (cell scale
    and work split; workgroups per CU barely move the bytes)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if tuning is None:
        return None
    e = t.get(f"{workload}:{kernel}@{float(tuning['cell_scale']):g},{int(tuning['query_cells'])}")
    if not e or e.get("sources") != source_digest():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(sc, n_queries, log):
    """Oracle (single thread) on a bounded sample: brute-force candidate
    queries for a sample of vertices and edges (untimed), then the oracle's
    barrier + reduction timed on the pairs they produce."""
    import numpy as np

    import oracle as O
    dof = np.diff(sc.W_rowptr) > 0
    x = O.embed(sc, sc.q)
    rng = np.random.default_rng(sc.seed + 99)
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
    bl = body[order]
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                c = code(keys + 1 + np.array([dx, dy, dz]))
                lo = np.searchsorted(sb, c, side="left")
                hi = np.searchsorted(sb, c, side="right")
                idx = np.nonzero(hi > lo)[0]
                if len(idx) == 0:
                    continue
                mn = np.minimum.reduceat(bl, lo[idx])
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


def _timed(fn, reps, sync):
    fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    sync()
    return 1e3 * (time.perf_counter() - t0) / reps


def _rooflines(prof, n_steps, work, workload, tuning=None):
    """Per-family averages and the roofline entry of the dominant family.
    work: active pairs per type, candidate and query counts of one step."""
    fam_ms = {f: sum(prof.get(k, (0.0, 0))[0] for k in ks) / n_steps for f, ks in FAMILIES.items()}
    launches = {k: v[1] for k, v in prof.items() if v[1]}
    dom = max(fam_ms, key=fam_ms.get)
    kernels = [k for k in FAMILIES[dom] if prof.get(k, (0, 0))[1]]
    # dominant single kernel of that family
    kdom = max(kernels, key=lambda k: prof[k][0])
    ms, n = prof[kdom]
    avg_s = ms / n / 1e3
    ent = {"kernel": kdom, "family": dom, "avg_launch_us": avg_s * 1e6, "traffic": None,
           "timing": "HIP events on the launch stream over eager planned steps that run the PT and EE chains one "
                     "after the other (each kernel alone on the device)"}
    if dom in ("pair_terms", "expand"):
        kind = 0 if kdom.endswith("_pt") else 1
        per = work["terms_flops"][kind] if dom == "pair_terms" else FLOPS_EXPAND * work["active"][kind]
        ach = per / avg_s / 1e12
        ent.update(bound="alu", achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s", frac=ach / PEAK_FP64_TFLOPS,
                   per_unit=(f"{FLOPS_TERMS}+distance flop per active pair" if dom == "pair_terms"
                             else f"{FLOPS_EXPAND} flop per active pair"))
    else:
        # algorithmic bytes: query = query records + item table + pairs out;
        # narrow = pair ids + 4 gathered vertices + type/index out; ccd
        # (fused with the narrow phase) = pair ids + vertex records once +
        # active pairs out
        kind = 0 if kdom.endswith("_pt") else 1
        if dom == "query":
            swept = kdom.startswith("query_write") and work.get("swept_query", False)
            nq, ni = work["n_query"][kind], work["n_item"][kind]
            qb = (24 if kind == 0 else 64)
            ncand = work["cand"][kind]
            nbytes = nq * qb + ni * 64 + 8 * ncand
            per_unit = f"{qb} B per query + 64 B per item + 8 B per candidate"
        elif dom == "narrow":
            nbytes = work["cand"][kind] * (8 + 4 * 24) + 8 * work["active"][kind]
            per_unit = "104 B per candidate + 8 B per active pair"
        elif dom == "ccd":
            # planned step, narrow phase fused in: the swept list read, the
            # active pairs written, each vertex's position and displacement
            # records (32 B each) read once (the per-pair gathers of them
            # are cache traffic, not compulsory)
            nbytes = work["swept"][kind] * 8 + 8 * work["active"][kind] + 64 * work["n_vert"]
            per_unit = "8 B per swept candidate + 8 B per active pair + 64 B per vertex"
        else:
            nbytes = work["n_vert"] * (24 + 24 + 16 * 4)
            per_unit = "112 B per vertex"
        ach = nbytes / avg_s / 1e9
        ent.update(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS,
                   per_unit=per_unit)
    tb = load_traffic(kdom, workload, tuning)
    if tb is not None:
        ent["traffic"] = tb
    ent["family_ms_per_step"] = {f: round(v, 4) for f, v in fam_ms.items()}
    ent["kernels_us"] = {k: round(v[0] / v[1] * 1e3, 2) for k, v in prof.items() if v[1]}
    for k, kind in (("barrier_pt", 0), ("barrier_ee", 1)):
        if prof.get(k, (0, 0))[1]:
            s_ = prof[k][0] / prof[k][1] / 1e3
            ent[f"{k}_tflops"] = work["terms_flops"][kind] / s_ / 1e12
    ent["launches"] = launches
    return ent


RESOLUTION_NODES = (250, 1000, 2000, 8000, 32000)


def resolution_sweep(a, log):
    """Contact-stage throughput against the embedding's resolution: config
    2's surface meshes (object frequency 71, fingers 32, seed a.seed) with
    the object's coarse grid at each size of RESOLUTION_NODES (the fingers
    keep their grids).  The contact work depends on the surface alone; only
    the embedding and the reduction through W see the grid.  Each scene is
    autotuned, then timed as in the single-scene bench (graph replays)."""
    import torch
    from scenes import scene as S
    import paper_2409_16385_amd as E
    from paper_2409_16385_amd import batch as BT
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    flags = E.ENERGY | E.GRAD | E.HESS | E.PROJECT
    rows = []
    for nodes in RESOLUTION_NODES:
        t0 = time.perf_counter()
        sc = S.grasp_scene(a.seed, 71, nodes, 32, name=f"config2_grid{nodes}")
        bt = BT.Batch(ctx, BT.concat([sc]), flags=flags)
        tuning = bt.autotune(reps=2)
        bt.capture()
        for _ in range(a.warmup):
            bt.replay()
        torch.cuda.synchronize(dev)
        t1 = time.perf_counter()
        for _ in range(a.steps):
            bt.replay()
        torch.cuda.synchronize(dev)
        ms = 1e3 * (time.perf_counter() - t1) / a.steps
        st = bt.status()
        if st not in (E.binding.OK, E.binding.WARN_CCD_CAPPED):
            raise RuntimeError(f"resolution {nodes}: status {st}")
        cnt = bt.counts()
        bt.ctx.profile(True, serial=True)
        bt.ctx.profile_read(reset=True)
        for _ in range(3):
            bt.step()
        prof = bt.ctx.profile_read(reset=True)
        bt.ctx.profile(False)
        fam = {f: round(sum(prof.get(k, (0.0, 0))[0] for k in ks) / 3, 4) for f, ks in FAMILIES.items()}
        row = {"object_grid_nodes": nodes, "n_node": int(sc.n_node), "n_vert": int(sc.n_vert),
               "active_pairs": cnt["active"], "swept": cnt["swept_pt"] + cnt["swept_ee"], "ms_per_step": ms,
               "pairs_per_s": cnt["active"] / (ms * 1e-3), "family_ms_alone": fam,
               "tuning": {k: v for k, v in tuning.items() if k != "trace"}}
        log(f"resolution {nodes}: n_node={sc.n_node} active={cnt['active']} {ms:.3f} ms/step "
            f"({time.perf_counter() - t0:.1f} s)")
        rows.append(row)
        del bt
    ref = next(r for r in rows if r["object_grid_nodes"] == 2000)
    out = {"metric": "contact pairs/s against embedding resolution", "value": ref["pairs_per_s"],
           "unit": "contact pairs/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": ref["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "config 2 surfaces, object grid of 2,000 nodes (value); sweep over "
                                  + ", ".join(str(n) for n in RESOLUTION_NODES) + " nodes", "seed": a.seed},
           "sweep": rows, "sources": source_digest()}
    print(json.dumps(out), flush=True)


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                                   "(a multi-GPU run would shard scenes or pairs, see the design notes)",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if a.config == "resolution":
        resolution_sweep(a, log)
        return
    batch_scenes = make_batch(a.n_scene, a.seed, log) if a.config == "batch" else None

    import numpy as np
    import torch

    import paper_2409_16385_amd as E
    from paper_2409_16385_amd import batch as BT

    dev = torch.device("cuda", 0)
    sync = lambda: torch.cuda.synchronize(dev)  # noqa: E731
    t0 = time.perf_counter()
    if batch_scenes is None:
        sc = make_scene(a.config, a.seed)
        log(f"{sc.summary()} (generated in {time.perf_counter() - t0:.1f} s)")
        scenes_list = [sc]
    else:
        scenes_list = batch_scenes
    ctx = E.Context(0)
    flags = E.ENERGY | E.GRAD | E.HESS | E.PROJECT | (E.MOLLIFY if a.config == "config3" else 0)
    hb = BT.concat(scenes_list)
    bt = BT.Batch(ctx, hb, flags=flags)
    if a.copy_calibration_mib:
        src = torch.ones(a.copy_calibration_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        sync()
        del src, dst
    tuning = None
    if a.tuning:
        v = [float(t) for t in a.tuning.split(",")]
        tuning = {"cell_scale": v[0], "wg_per_cu": [int(t) for t in v[1:5]],
                  "query_cells": int(v[5]) if len(v) > 5 else -1}
        E.set_tuning(bt.ctx, tuning["cell_scale"], tuning["wg_per_cu"], tuning["query_cells"])
        bt.make_plan(1.5)
    elif not a.no_autotune:
        t1 = time.perf_counter()
        tuning = bt.autotune(reps=2)
        log(f"autotune: cell_scale={tuning['cell_scale']} wg_per_cu={tuning['wg_per_cu']} "
            f"({time.perf_counter() - t1:.1f} s)")
        log("autotune trace (what, value, ms): " + " ".join(f"{w}={v}:{t:.3f}" for w, v, t in tuning["trace"]))
    else:
        bt.make_plan(1.5)
    plan = bt.plan.as_dict()
    log(f"plan: {plan}")

    # workload (outside the timed region): counts and active pairs per type
    bt.step()
    st = bt.status()
    if st not in (E.binding.OK, E.binding.WARN_CCD_CAPPED):
        raise RuntimeError(f"planned step failed with status {st}")
    cnt = bt.counts()
    n_active = cnt["active"]
    swept = cnt["swept_pt"] + cnt["swept_ee"]
    tpc = np.zeros(7, dtype=np.int64)
    tec = np.zeros(9, dtype=np.int64)
    dsc = bt.scene
    q = bt.q
    pt, ee = E.build_candidates(ctx, dsc, q, hb.dhat)
    ap, tp, ae, te = E.narrow_phase(ctx, dsc, q, pt, ee, hb.dhat)
    tpc += np.bincount(tp.cpu().numpy(), minlength=7)
    tec += np.bincount(te.cpu().numpy(), minlength=9)
    assert int(ap.numel() + ae.numel()) == n_active and pt.shape[0] == cnt["cand_pt"] and ee.shape[0] == cnt["cand_ee"]
    terms_pt = sum(int(tpc[i]) * (FLOPS_TERMS + FLOPS_DIST[PT_FN[i]]) for i in range(7))
    terms_ee = sum(int(tec[i]) * (FLOPS_TERMS + FLOPS_DIST[EE_FN[i]]) for i in range(9))
    work = {"active": (int(ap.numel()), int(ae.numel())), "cand": (cnt["cand_pt"], cnt["cand_ee"]),
            "swept": (cnt["swept_pt"], cnt["swept_ee"]), "terms_flops": (terms_pt, terms_ee),
            "n_query": (hb.W_rowptr.size - 1, hb.edges.shape[0]), "n_item": (hb.faces.shape[0], hb.edges.shape[0]),
            "n_vert": hb.W_rowptr.size - 1}
    log(f"candidates pt={cnt['cand_pt']} ee={cnt['cand_ee']} active pt={work['active'][0]} "
        f"ee={work['active'][1]} swept={swept} PT types {tpc.tolist()} EE types {tec.tolist()}")
    del pt, ee, ap, tp, ae, te

    # timed region: graph replays (or eager planned steps)
    use_graph = not a.no_graph
    if use_graph:
        bt.capture()
    run = bt.replay if use_graph else bt.step
    for _ in range(a.warmup):
        run()
    sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        run()
    sync()
    elapsed = time.perf_counter() - t0
    st = bt.status()
    if st not in (E.binding.OK, E.binding.WARN_CCD_CAPPED):
        raise RuntimeError(f"timed steps reported status {st}")
    ms_per_step = 1e3 * elapsed / a.steps

    # per-kernel event profile of eager planned steps (same kernels)
    prof = {}
    if not a.no_profile:
        bt.ctx.profile(True, serial=True)  # each kernel timed alone on the device
        bt.ctx.profile_read(reset=True)
        n_prof = max(3, min(a.steps, 10))
        for _ in range(n_prof):
            bt.step()
        prof = bt.ctx.profile_read(reset=True)
        bt.ctx.profile(False)
        for k, (ms, n) in prof.items():
            if n:
                log(f"kernel {k:16s} {ms / n * 1e3:10.1f} us/launch x {n}")
    workload = a.config
    roofline = _rooflines(prof, max(3, min(a.steps, 10)), work, workload, tuning) if prof else None

    out = {
        "metric": METRIC, "value": n_active / (ms_per_step / 1e3), "unit": "contact pairs/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
    }
    if a.config == "batch":
        # 256 sequential single-scene calls on the same scenes
        t_seq = float("nan")
        if not a.no_plain:
            dscs = [E.Scene.from_host(ctx, s) for s in scenes_list]
            BT.sequential_reference(ctx, scenes_list[:4], dscs[:4])
            _, t_seq = BT.sequential_reference(ctx, scenes_list, dscs)
        nv = np.diff(hb.vert_off)
        out["config"] = {"workload": (f"batch of {hb.n_scene} ragged grasp scenes (objects 2e3-5e4 triangles, "
                                      f"100-2000 coarse nodes, fingers 2x5120 triangles, random SE(3)): "
                                      f"n_vert={int(hb.vert_off[-1])} n_face={hb.faces.shape[0]} "
                                      f"n_node={hb.n_node} dhat={hb.dhat:g}"),
                         "n_scene": hb.n_scene, "active_pairs": n_active,
                         "candidates": cnt["cand_pt"] + cnt["cand_ee"], "ccd_candidates": swept,
                         "verts_per_scene_min_max": [int(nv.min()), int(nv.max())], "seed0": a.seed}
        out["scenes_per_s"] = hb.n_scene / (ms_per_step / 1e3)
        if not a.no_plain:
            out["sequential_ms"] = 1e3 * t_seq
            out["sequential_scenes_per_s"] = hb.n_scene / t_seq
            out["sequential_pairs_per_s"] = n_active / t_seq
            out["batch_speedup"] = (t_seq * 1e3) / ms_per_step
    elif not a.no_plain:
        sc = scenes_list[0]
        out["config"] = {"workload": f"{a.config} ({sc.name}): n_vert={sc.n_vert} n_face={sc.n_face} "
                                     f"n_edge={sc.n_edge} n_node={sc.n_node} dhat={sc.dhat:g}",
                         "active_pairs": n_active, "candidates": cnt["cand_pt"] + cnt["cand_ee"],
                         "ccd_candidates": swept, "seed": a.seed}
        # plain per-call entry points, for comparison
        q0 = torch.as_tensor(sc.q, device=dev)
        dq0 = torch.as_tensor(sc.dq, device=dev)
        dsc0 = E.Scene.from_host(ctx, sc)
        pt, ee = E.build_candidates(ctx, dsc0, q0, sc.dhat)
        ev = {"candidates": _timed(lambda: E.build_candidates(ctx, dsc0, q0, sc.dhat), 5, sync),
              "barrier_reduce": _timed(lambda: E.barrier_reduce(ctx, dsc0, q0, pt, ee, sc.dhat, sc.kappa, flags,
                                                                hess="bsr", count=False), 5, sync),
              "ccd": _timed(lambda: E.ccd_max_step(ctx, dsc0, q0, dq0, sc.dhat), 5, sync)}
        out["call_ms"] = ev
        out["plain_calls_ms_per_step"] = sum(ev.values())
        out["barrier_reduce_pairs_per_s"] = n_active / (ev["barrier_reduce"] / 1e3)
        out["ccd_pairs_per_s"] = swept / (ev["ccd"] / 1e3)
    if "config" not in out:
        sc = scenes_list[0]
        out["config"] = {"workload": f"{a.config} ({sc.name}): n_vert={sc.n_vert} n_face={sc.n_face} "
                                     f"n_edge={sc.n_edge} n_node={sc.n_node} dhat={sc.dhat:g}",
                         "active_pairs": n_active, "candidates": cnt["cand_pt"] + cnt["cand_ee"],
                         "ccd_candidates": swept, "seed": a.seed}
    out["timed"] = "graph replay of the planned step" if use_graph else "eager planned step"
    out["alpha_min"] = float(bt.out.alpha.min().item())
    out["tuning"] = None if tuning is None else {"cell_scale": tuning["cell_scale"],
                                                 "wg_per_cu": tuning["wg_per_cu"],
                                                 "query_cells": tuning.get("query_cells", -1)}
    out["roofline"] = roofline
    out["cpu_baseline"] = None
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scenes_list[0] if a.config != "batch" else _largest(scenes_list),
                                           a.cpu_queries, log)
    out["sources"] = source_digest()
    print(json.dumps(out), flush=True)


def _largest(scenes_list):
    return max(scenes_list, key=lambda s: s.n_face)


if __name__ == "__main__":
    main()
