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

# Algorithmic FP64 flops per active pair (counts of the operations the
# method needs, not of what a kernel executes).  Pair terms: distance, its
# gradient and Hessian ~1e3, barrier chain rule and assembly ~0.3e3, the
# symmetric eigendecomposition of the 9x9 translation-free Hessian
# 9 n^3 = 6,561 and the reconstruction V max(L, 0) V^T ~2e3.  Expansion
# through W (16 weights, merged nodes, blocks and gradient): ~4.6e3.  The
# pair-terms kernel ("barrier" scope) does the first for every active pair
# (its class-specialised projections execute fewer flops than the nominal
# 9x9 count for point-point and point-line pairs), the expansion kernel the
# second.  Algorithmic bytes per active pair for the whole barrier +
# reduction: the pair record, its share of the gathered geometry and of the
# outputs, ~85 B at config 2's reuse.
FLOPS_TERMS = 1000 + 300 + 6561 + 2000
FLOPS_EXPAND = 4600
BYTES_BARRIER_PAIR = 85
FAMILIES = {
    "query": ("query_count_pt", "query_count_ee", "query_write_pt", "query_write_ee"),
    "barrier": ("barrier_pt", "barrier_ee"), "expand": ("expand_pt", "expand_ee"),
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
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the main workload (skip configs 1, 3, 4 and the batch beside it)")
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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, log, slice_frac=1.0 / 16):
    """The oracle on the host cores: its uniform-grid candidates of the
    whole scene (untimed), then its barrier + reduction (energy, gradient,
    PSD-projected block-sparse Hessian) over all candidates, timed on every
    host thread (the pair lists cut into slices, one oracle call per slice),
    and on one thread over the first slice_frac of each list."""
    import numpy as np

    import oracle as O
    x = O.embed(sc, sc.q)
    t0 = time.perf_counter()
    pt, ee = O.candidates_grid(sc, x, sc.dhat)
    t_cand = time.perf_counter() - t0
    flags = O.ENERGY | O.GRAD | O.HESS | O.PROJECT | (O.MOLLIFY if sc.name == "config3" else 0)
    nth = O.threads()
    t0 = time.perf_counter()
    r = O.barrier_reduce_bsr(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags, nthreads=nth)
    t_all = time.perf_counter() - t0
    k_pt, k_ee = max(1, int(len(pt) * slice_frac)), max(1, int(len(ee) * slice_frac))
    t0 = time.perf_counter()
    r1 = O.barrier_reduce_bsr(sc, sc.q, pt[:k_pt], ee[:k_ee], sc.dhat, sc.kappa, flags, nthreads=1)
    t_one = time.perf_counter() - t0
    log(f"cpu baseline: {len(pt)} + {len(ee)} candidates ({t_cand:.1f} s untimed), {r['n_active']} active, "
        f"barrier+reduce {t_all:.2f} s on {nth} threads; one thread {r1['n_active']} active in {t_one:.2f} s")
    return {"value": r["n_active"] / t_all if t_all > 0 else None, "unit": "contact pairs/s", "cores": nth,
            "kind": "oracle", "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_thread_value": r1["n_active"] / t_one if t_one > 0 else None,
            "sample": (f"{sc.name}, whole workload: oracle uniform-grid candidates ({len(pt) + len(ee)}, untimed), "
                       f"then or_barrier_reduce_bsr (energy, gradient, projected block-sparse Hessian) over all "
                       f"{r['n_active']} active pairs on {nth} threads, slices merged in order ({t_all:.2f} s); "
                       f"single_thread_value: the first {slice_frac:g} of each list on one thread "
                       f"({r1['n_active']} active, {t_one:.2f} s)")}


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
    if dom in ("barrier", "expand"):
        # FP64-bound: ~1.5e4 algorithmic flop against ~85 B per pair is far
        # above the ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B)
        kind = 0 if kdom.endswith("_pt") else 1
        per_pair = FLOPS_TERMS if dom == "barrier" else FLOPS_EXPAND
        per = per_pair * work["active"][kind]
        ach = per / avg_s / 1e12
        ent.update(bound="alu", achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                   frac=ach / PEAK_FP64_TFLOPS, per_unit=f"{per_pair} flop per active pair",
                   hbm_algorithmic_GBs=BYTES_BARRIER_PAIR * work["active"][kind] / avg_s / 1e9)
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
        ent["hbm_measured_GBs"] = tb / avg_s / 1e9
        ent["hbm_measured_frac"] = tb / avg_s / 1e9 / PEAK_HBM_GBS
    ent["family_ms_per_step"] = {f: round(v, 4) for f, v in fam_ms.items()}
    ent["kernels_us"] = {k: round(v[0] / v[1] * 1e3, 2) for k, v in prof.items() if v[1]}
    for k, kind in (("barrier_pt", 0), ("barrier_ee", 1)):
        if prof.get(k, (0, 0))[1]:
            s_ = prof[k][0] / prof[k][1] / 1e3
            ent[f"{k}_tflops"] = FLOPS_TERMS * work["active"][kind] / s_ / 1e12
    for k, kind in (("expand_pt", 0), ("expand_ee", 1)):
        if prof.get(k, (0, 0))[1]:
            s_ = prof[k][0] / prof[k][1] / 1e3
            ent[f"{k}_tflops"] = FLOPS_EXPAND * work["active"][kind] / s_ / 1e12
    ent["launches"] = launches
    return ent


def _median_us(fn, reps, sync, warm=5):
    """Median wall time of fn() in microseconds, each call synchronized."""
    import statistics
    for _ in range(warm):
        fn()
    sync()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        sync()
        ts.append(1e6 * (time.perf_counter() - t0))
    return statistics.median(ts)


def _replay_ms(bt, steps, warmup, sync):
    bt.capture()
    for _ in range(warmup):
        bt.replay()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        bt.replay()
    sync()
    return 1e3 * (time.perf_counter() - t0) / steps


def extra_config1(sc, log):
    """Config 1 is latency-bound: microseconds per call of each entry point
    (median of 200 synchronized calls) and per planned step (graph
    replay)."""
    import torch
    import paper_2409_16385_amd as E
    from paper_2409_16385_amd import batch as BT
    dev = torch.device("cuda", 0)
    sync = lambda: torch.cuda.synchronize(dev)  # noqa: E731
    ctx = E.Context(0)
    dsc = E.Scene.from_host(ctx, sc)
    q, dq = torch.as_tensor(sc.q, device=dev), torch.as_tensor(sc.dq, device=dev)
    v = torch.as_tensor(sc.dq, device=dev)
    flags = E.ENERGY | E.GRAD | E.HESS | E.PROJECT
    pt, ee = E.build_candidates(ctx, dsc, q, sc.dhat)
    r = E.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags, hess="bsr")
    a, n_swept, _ = E.ccd_max_step(ctx, dsc, q, dq, sc.dhat)
    us = {"build_candidates": _median_us(lambda: E.build_candidates(ctx, dsc, q, sc.dhat), 200, sync),
          "barrier_reduce": _median_us(lambda: E.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags,
                                                                hess="bsr", count=False), 200, sync),
          "ccd_max_step": _median_us(lambda: E.ccd_max_step(ctx, dsc, q, dq, sc.dhat), 200, sync),
          "barrier_hvp": _median_us(lambda: E.barrier_hvp(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, E.PROJECT, v),
                                    200, sync)}
    bt = BT.Batch(ctx, BT.concat([sc]), flags=flags)
    bt.make_plan(1.5)
    step_ms = _replay_ms(bt, 200, 10, sync)
    log(f"config1: per call {us}, planned step {1e3 * step_ms:.1f} us")
    return {"workload": f"config1 ({sc.name}): n_vert={sc.n_vert} n_node={sc.n_node} dhat={sc.dhat:g}",
            "active_pairs": int(r["n_active"]), "candidates": int(pt.shape[0] + ee.shape[0]),
            "ccd_candidates": int(n_swept), "call_us": us, "planned_step_us": 1e3 * step_ms,
            "timing": "median of 200 synchronized calls; planned step: graph replays"}


def extra_single(sc, log, flags_extra=0, steps=20):
    """A single-scene workload timed like the main one (autotuned planned
    step, graph replays) plus its per-call barrier + reduction and CCD."""
    import torch
    import paper_2409_16385_amd as E
    from paper_2409_16385_amd import batch as BT
    dev = torch.device("cuda", 0)
    sync = lambda: torch.cuda.synchronize(dev)  # noqa: E731
    ctx = E.Context(0)
    flags = E.ENERGY | E.GRAD | E.HESS | E.PROJECT | flags_extra
    bt = BT.Batch(ctx, BT.concat([sc]), flags=flags)
    tuning = bt.autotune(reps=3)
    ms = _replay_ms(bt, steps, 3, sync)
    st = bt.status()
    if st not in (E.binding.OK, E.binding.WARN_CCD_CAPPED):
        raise RuntimeError(f"{sc.name}: status {st}")
    cnt = bt.counts()
    dsc = E.Scene.from_host(ctx, sc)
    q, dq = torch.as_tensor(sc.q, device=dev), torch.as_tensor(sc.dq, device=dev)
    pt, ee = E.build_candidates(ctx, dsc, q, sc.dhat)
    t_red = _median_us(lambda: E.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags, hess="bsr",
                                                count=False), 10, sync, warm=2)
    t_ccd = _median_us(lambda: E.ccd_max_step(ctx, dsc, q, dq, sc.dhat), 10, sync, warm=2)
    swept = cnt["swept_pt"] + cnt["swept_ee"]
    log(f"{sc.name}: {ms:.3f} ms/step, {cnt['active']} active, barrier+reduce {t_red:.0f} us, ccd {t_ccd:.0f} us")
    return {"workload": f"{sc.name}: n_vert={sc.n_vert} n_face={sc.n_face} n_node={sc.n_node} dhat={sc.dhat:g}",
            "ms_per_step": ms, "pairs_per_s": cnt["active"] / (ms * 1e-3), "active_pairs": cnt["active"],
            "candidates": cnt["cand_pt"] + cnt["cand_ee"], "ccd_candidates": swept,
            "barrier_reduce_ms": t_red / 1e3, "barrier_reduce_pairs_per_s": cnt["active"] / (t_red * 1e-6),
            "ccd_ms": t_ccd / 1e3, "ccd_pairs_per_s": swept / (t_ccd * 1e-6),
            "tuning": {k: v for k, v in tuning.items() if k != "trace"}}


def extra_config4(sc, log):
    """Differentiable form on config 1: the autograd barrier energy, its
    backward (the reduced gradient) and double backward (HVP with the true
    pair Hessians, recomputed), backward / forward time ratio."""
    import statistics
    import torch
    import paper_2409_16385_amd as E
    dev = torch.device("cuda", 0)
    sync = lambda: torch.cuda.synchronize(dev)  # noqa: E731
    ctx = E.Context(0)
    dsc = E.Scene.from_host(ctx, sc)
    q0 = torch.as_tensor(sc.q, device=dev)
    pt, ee = E.build_candidates(ctx, dsc, q0, sc.dhat)
    state = E.BarrierState(ctx, dsc, pt, ee, sc.dhat, sc.kappa)
    q = q0.clone().requires_grad_(True)
    v = torch.as_tensor(sc.dq, device=dev)

    def fwd():
        return E.barrier_energy(q, state)

    def fwd_bwd():
        torch.autograd.grad(E.barrier_energy(q, state), q)

    def hvp():
        (g,) = torch.autograd.grad(E.barrier_energy(q, state), q, create_graph=True)
        torch.autograd.grad(g, q, grad_outputs=v)

    t_f = _median_us(fwd, 100, sync)
    t_fb = _median_us(fwd_bwd, 100, sync)
    t_h = _median_us(hvp, 100, sync)
    log(f"config4: forward {t_f:.1f} us, forward+backward {t_fb:.1f} us, with HVP {t_h:.1f} us")
    return {"workload": f"differentiable form on config1 ({pt.shape[0] + ee.shape[0]} candidate pairs)",
            "forward_us": t_f, "forward_backward_us": t_fb, "backward_over_forward": (t_fb - t_f) / t_f,
            "energy_grad_hvp_us": t_h, "timing": "median of 100 synchronized calls"}


def extra_formulations(log):
    """The alternative formulations on one implicit step of config 1's
    step problem (projected Newton with CCD-clamped backtracking): Newton
    iterations, the CCD step bounds along the way and the converged
    position, per barrier form, projection, CCD and elastic model."""
    import time
    import torch
    import paper_2409_16385_amd as E
    from paper_2409_16385_amd import adjoint as A
    dev = torch.device("cuda", 0)
    ctx = E.Context(0)
    prob, _ = A.build_config1_step(ctx)
    lin, cor = E.ELASTIC_LINEAR, E.ELASTIC_COROTATIONAL
    variants = [("distance barrier, per-pair projection, additive CCD", 0, False, E.CCD_ADDITIVE, lin),
                ("squared-distance barrier", E.SQDIST, False, E.CCD_ADDITIVE, lin),
                ("reduced-block projection", 0, True, E.CCD_ADDITIVE, lin),
                ("closest-direction CCD", 0, False, E.CCD_CLOSEST_DIRECTION, lin),
                ("linear corotational elasticity", 0, False, E.CCD_ADDITIVE, cor)]
    out, q_base = [], None
    kappa0 = prob.kappa
    for name, bf, red, ccd, model in variants:
        prob.barrier_flags, prob.reduced_projection, prob.elastic_model = bf, red, model
        # the squared-distance barrier is about dhat^2 smaller at equal
        # kappa: its stiffness is rescaled so that both forms give the same
        # energy at d = dhat / sqrt(2)
        prob.kappa = kappa0 * (A.SQDIST_KAPPA_FACTOR / prob.dhat ** 2 if bf & E.SQDIST else 1.0)
        E.set_ccd_method(ctx, ccd)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        q, info = A.solve_step(prob)
        torch.cuda.synchronize(dev)
        ms = (time.perf_counter() - t0) * 1e3
        if q_base is None:
            q_base = q
        dn = float(torch.linalg.vector_norm(q_base - prob.q_n))
        ent = {"formulation": name, "kappa": prob.kappa, "converged": info["converged"],
               "newton_iters": info["iters"], "true_hessian_steps": info["true_hessian_steps"],
               "alpha_ccd": [round(a, 6) for a in info["alpha_ccd"]], "alpha_taken": [round(a, 6) for a in info["alpha"]],
               "solve_ms": ms, "q_vs_first_rel": float(torch.linalg.vector_norm(q - q_base)) / dn if dn > 0 else 0.0}
        log(f"formulation {name}: {info['iters']} Newton iterations, CCD alphas {ent['alpha_ccd'][:4]}, {ms:.1f} ms")
        out.append(ent)
    E.set_ccd_method(ctx, E.CCD_ADDITIVE)
    prob.kappa, prob.elastic_model = kappa0, lin
    return {"workload": f"one implicit step of config 1's step problem ({prob.n} reduced DoF)", "variants": out}


def extra_batch(scenes_list, log, steps=10):
    """The batched form: one planned step over the ragged batch, graph
    replays, against the same scenes as sequential single-scene steps."""
    import numpy as np
    import torch
    import paper_2409_16385_amd as E
    from paper_2409_16385_amd import batch as BT
    dev = torch.device("cuda", 0)
    sync = lambda: torch.cuda.synchronize(dev)  # noqa: E731
    ctx = E.Context(0)
    hb = BT.concat(scenes_list)
    bt = BT.Batch(ctx, hb)
    tuning = bt.autotune(reps=4)
    ms = _replay_ms(bt, steps, 2, sync)
    st = bt.status()
    if st not in (E.binding.OK, E.binding.WARN_CCD_CAPPED):
        raise RuntimeError(f"batch: status {st}")
    cnt = bt.counts()
    dscs = [E.Scene.from_host(ctx, s) for s in scenes_list]
    BT.sequential_reference(ctx, scenes_list[:4], dscs[:4])
    _, t_seq = BT.sequential_reference(ctx, scenes_list, dscs)
    nv = np.diff(hb.vert_off)
    log(f"batch: {ms:.2f} ms/step ({hb.n_scene / (ms * 1e-3):.0f} scenes/s), sequential {1e3 * t_seq:.1f} ms")
    return {"workload": (f"batch of {hb.n_scene} ragged grasp scenes: n_vert={int(hb.vert_off[-1])} "
                         f"n_face={hb.faces.shape[0]} n_node={hb.n_node}"),
            "ms_per_step": ms, "scenes_per_s": hb.n_scene / (ms * 1e-3),
            "pairs_per_s": cnt["active"] / (ms * 1e-3), "active_pairs": cnt["active"],
            "ccd_candidates": cnt["swept_pt"] + cnt["swept_ee"],
            "sequential_ms": 1e3 * t_seq, "sequential_scenes_per_s": hb.n_scene / t_seq,
            "batch_speedup": 1e3 * t_seq / ms, "verts_per_scene_min_max": [int(nv.min()), int(nv.max())],
            "tuning": {k: v for k, v in tuning.items() if k != "trace"}}


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
        sc = S.grasp_scene(a.seed, 71, nodes, 32, frac=0.75, name=f"config2_grid{nodes}")
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
    extras = a.config == "config2" and not a.no_extras
    batch_scenes = make_batch(a.n_scene, a.seed, log) if (a.config == "batch" or extras) else None
    extra_scenes = {}
    if extras:
        extra_scenes = {"config1": make_scene("config1", a.seed), "config3": make_scene("config3", a.seed)}
        extra_batch_scenes, batch_scenes = batch_scenes, None

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
        tuning = bt.autotune(reps=5)  # timed over eager steps: with fewer, timing noise decides the pick
        # the autotuner times eager steps, the timed region replays a graph:
        # its pick against the library's default shapes at cell scales 2
        # and 3, each timed as the timed region is, and the fastest kept
        cands = [(tuning["cell_scale"], list(tuning["wg_per_cu"]), tuning["query_cells"])]
        for cs in (2.0, 3.0):
            if (cs, list(BT.DEFAULT_WG_PER_CU), 15) not in cands:
                cands.append((cs, list(BT.DEFAULT_WG_PER_CU), 15))
        checked = []
        for cs, wg, qc in cands:
            E.set_tuning(bt.ctx, cs, wg, qc)
            bt.make_plan(1.5)
            ms = _replay_ms(bt, 20, 3, sync)
            tuning["trace"].append((f"replayed {wg} {qc}", cs, ms))
            checked.append((ms, cs, wg, qc))
        _, cs, wg, qc = min(checked, key=lambda c: c[0])
        E.set_tuning(bt.ctx, cs, wg, qc)
        bt.make_plan(1.5)
        tuning.update(cell_scale=cs, wg_per_cu=wg, query_cells=qc)
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
    work = {"active": (int(ap.numel()), int(ae.numel())), "cand": (cnt["cand_pt"], cnt["cand_ee"]),
            "swept": (cnt["swept_pt"], cnt["swept_ee"]),
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
        out["cpu_baseline"] = cpu_baseline(scenes_list[0] if a.config != "batch" else _largest(scenes_list), log)
    if extras:
        import paper_2409_16385_amd as E
        jobs = (("config1", lambda: extra_config1(extra_scenes["config1"], log)),
                ("config3", lambda: extra_single(extra_scenes["config3"], log, E.MOLLIFY)),
                ("config4", lambda: extra_config4(extra_scenes["config1"], log)),
                ("formulations", lambda: extra_formulations(log)),
                ("batch", lambda: extra_batch(extra_batch_scenes, log)))
        for key, job in jobs:
            t0 = time.perf_counter()
            try:
                out[key] = job()
            except Exception as e:  # recorded, never fatal to the main line
                out[key] = {"error": f"{type(e).__name__}: {e}"}
            log(f"extra {key}: {time.perf_counter() - t0:.1f} s")
    out["sources"] = source_digest()
    print(json.dumps(out), flush=True)


def _largest(scenes_list):
    return max(scenes_list, key=lambda s: s.n_face)


if __name__ == "__main__":
    main()
