"""The planned step (the launch configuration bench.py times, eager and
replayed from a captured graph) at full size, against the per-call entry
points on the same inputs: identical candidate, active and swept counts,
identical BSR structure, energy / gradient / Hessian blocks to rounding, the
step bound bit for bit.  The per-call path is checked against the oracle on
sampled outputs in test_gpu_fullsize.py."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import batch as BT  # noqa: E402
from scenes import config2, config3  # noqa: E402

_CACHE = {}


def _scene(name):
    if name not in _CACHE:
        _CACHE[name] = config2() if name == "config2" else config3()
    return _CACHE[name]


def _flags(sc):
    return E.ENERGY | E.GRAD | E.HESS | E.PROJECT | (E.MOLLIFY if sc.name == "config3" else 0)


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


_PLAIN = {}


def _plain(ctx, name):
    if name not in _PLAIN:
        sc = _scene(name)
        dsc = E.Scene.from_host(ctx, sc)
        q = torch.as_tensor(sc.q, device="cuda:0")
        dq = torch.as_tensor(sc.dq, device="cuda:0")
        pt, ee = E.build_candidates(ctx, dsc, q, sc.dhat)
        r = E.barrier_reduce(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, _flags(sc), hess="bsr")
        a, nc, _ = E.ccd_max_step(ctx, dsc, q, dq, sc.dhat, sc.dx_off)
        _PLAIN[name] = {"n_pt": pt.shape[0], "n_ee": ee.shape[0], "r": r, "alpha": a, "n_swept": nc}
    return _PLAIN[name]


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a - b)


def _compare(b, ref):
    cnt = b.counts()
    assert cnt["cand_pt"] == ref["n_pt"] and cnt["cand_ee"] == ref["n_ee"]
    assert cnt["active"] == ref["r"]["n_active"]
    assert cnt["swept_pt"] + cnt["swept_ee"] == ref["n_swept"]
    assert b.out.energy[0].item() == pytest.approx(ref["r"]["energy"][0].item(), rel=1e-12)
    assert _rel(b.out.grad.cpu().numpy(), ref["r"]["grad"].cpu().numpy()) <= 1e-12
    rp, col, blk = (t.cpu().numpy() for t in b.out.hess(b.ctx))
    rp0, col0, blk0 = (t.cpu().numpy() for t in ref["r"]["hess"])
    assert np.array_equal(rp, rp0) and np.array_equal(col, col0)
    assert _rel(blk, blk0) <= 1e-12
    assert b.out.alpha[0].item() == ref["alpha"]


def test_profiling_mode_2_gives_the_same_step(ctx):
    # timing mode 2 runs the PT chain on the caller's stream before the EE
    # chain (bench.py times kernels that way); results must not change
    sc = _scene("config2")
    b = BT.Batch(ctx, BT.concat([sc]), flags=_flags(sc))
    b.make_plan(1.5)
    b.ctx.profile(True, serial=True)  # the batch owns a context of its own
    try:
        b.step()
        prof = b.ctx.profile_read(reset=True)
    finally:
        b.ctx.profile(False)
    assert b.status() in (E.binding.OK, E.binding.WARN_CCD_CAPPED)
    assert prof["ccd_pt"][1] == 1 and prof["ccd_ee"][1] == 1 and prof["barrier_ee"][1] == 1
    _compare(b, _plain(ctx, "config2"))
    assert E.binding._load().eipc_profile(b.ctx._h, 3) == E.binding.ERR_ARG


@pytest.mark.parametrize("name", ["config2", "config3"])
def test_planned_step_matches_per_call_path(ctx, name):
    sc = _scene(name)
    b = BT.Batch(ctx, BT.concat([sc]), flags=_flags(sc))
    b.make_plan(1.5)
    b.step()
    assert b.status() in (E.binding.OK, E.binding.WARN_CCD_CAPPED)
    _compare(b, _plain(ctx, name))


def test_graph_replay_at_full_size(ctx):
    sc = _scene("config2")
    b = BT.Batch(ctx, BT.concat([sc]), flags=_flags(sc))
    b.make_plan(1.5)
    b.capture()
    for _ in range(3):
        b.replay()
        assert b.status() == E.binding.OK
        _compare(b, _plain(ctx, "config2"))


@pytest.mark.parametrize("mode,cs", [(0, 1.5), (5, 3.0), (10, 3.0), (15, 3.0), (15, 1.0)])
def test_tuning_does_not_change_results(ctx, mode, cs):
    """Work splits and cell sizes (at cell_scale 1 several hundred edges and
    faces span more than 64 cells and take the large-item path)."""
    sc = _scene("config2")
    b = BT.Batch(ctx, BT.concat([sc]), flags=_flags(sc))
    E.set_tuning(b.ctx, cs, [1, 16, 1, 16], mode)
    b.make_plan(1.5)
    b.step()
    assert b.status() == E.binding.OK
    _compare(b, _plain(ctx, "config2"))


def test_proximity_only_planned_step(ctx):
    """Without the step bound the planned step runs the proximity broad
    phase; counts, energy and gradient are those of the per-call path."""
    sc = _scene("config2")
    ref = _plain(ctx, "config2")
    b = BT.Batch(ctx, BT.concat([sc]), flags=_flags(sc))
    plan = E.plan_step(b.ctx, b.scene, b.q, sc.dhat, None, None, 1.5, with_hess=True)
    out = E.StepOut(b.ctx, b.scene, plan, _flags(sc), with_alpha=False)
    E.contact_step(b.ctx, b.scene, plan, b.q, sc.dhat, sc.kappa, out, None, None, _flags(sc))
    assert b.ctx.sync_status() == E.binding.OK
    c = out.counts.cpu().numpy()
    assert c[0] == ref["n_pt"] and c[1] == ref["n_ee"] and c[2] == ref["r"]["n_active"]
    assert out.energy[0].item() == pytest.approx(ref["r"]["energy"][0].item(), rel=1e-12)
    assert _rel(out.grad.cpu().numpy(), ref["r"]["grad"].cpu().numpy()) <= 1e-12
