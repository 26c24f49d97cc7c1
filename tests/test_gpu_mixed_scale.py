"""Primitives of very different sizes (a fine sheet over coarse plates, so
that the broad-phase hash holds one-thread, one-wavefront and unhashed
primitives): sorted candidates bit-exact against the oracle at several cell
sizes; the step bound and swept-candidate count of every broad-phase work
split equal the oracle's; the planned step (every split) reproduces the
oracle's counts, energy and step bound.  With the plates numbered first, a
plate edge is the lower index of some 19,000 edge-edge candidates: queries
spanning many cells run one wavefront each, and that query's sorted list is
put in order by rank through LDS tiles."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import batch as BT  # noqa: E402
from scenes import mixed_scale_scene  # noqa: E402

SPLITS = [0, 5, 10, 15]
FLAGS = E.ENERGY | E.GRAD | E.HESS | E.PROJECT


@pytest.fixture(scope="module", params=[False, True], ids=["sheet_first", "plates_first"])
def sc(request):
    return mixed_scale_scene(plates_first=request.param)


@pytest.fixture(scope="module")
def ref(sc):
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    spt, see = O.candidates(sc, x, sc.dhat, x1=O.embed(sc, sc.q + sc.dq))
    alpha, _, _ = O.ccd_max_step(sc, sc.q, sc.dq, sc.dhat)
    r = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, O.ENERGY)
    return {"pt": pt, "ee": ee, "spt": spt, "see": see, "n_swept": len(spt) + len(see), "alpha": alpha,
            "energy": r["energy"], "n_active": r["n_active"]}


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


@pytest.mark.parametrize("cs", [0.3, 1.0, 2.0, 4.0])
def test_candidates_bit_exact(ctx, sc, ref, cs):
    """At cell scale 0.3 each sheet primitive covers tens of cells, so a
    workgroup's entries reach more distinct buckets than its LDS bucket
    table holds and part of them take the global counters directly."""
    E.set_tuning(ctx, cs)
    dsc = E.Scene.from_host(ctx, sc)
    pt, ee = E.build_candidates(ctx, dsc, _dev(sc.q), sc.dhat)
    assert np.array_equal(pt.cpu().numpy(), ref["pt"])
    assert np.array_equal(ee.cpu().numpy(), ref["ee"])
    E.set_tuning(ctx, 2.0)


@pytest.mark.parametrize("cs", [0.3, 1.0, 2.0])
@pytest.mark.parametrize("mode", SPLITS)
def test_step_bound_every_split(ctx, sc, ref, mode, cs):
    E.set_tuning(ctx, cs, (0, 0, 0, 0), mode)
    dsc = E.Scene.from_host(ctx, sc)
    a, n, _ = E.ccd_max_step(ctx, dsc, _dev(sc.q), _dev(sc.dq), sc.dhat)
    E.set_tuning(ctx, 2.0, (0, 0, 0, 0), 15)
    assert n == ref["n_swept"]
    assert a == ref["alpha"]


@pytest.mark.parametrize("cs", [1.0, 2.0])
@pytest.mark.parametrize("mode", SPLITS)
def test_planned_step_every_split(ctx, sc, ref, mode, cs):
    b = BT.Batch(ctx, BT.concat([sc]), flags=FLAGS)
    E.set_tuning(b.ctx, cs, (0, 0, 0, 0), mode)
    b.make_plan(1.5)
    b.step()
    assert b.status() == E.binding.OK
    cnt = b.counts()
    assert cnt["cand_pt"] == len(ref["pt"]) and cnt["cand_ee"] == len(ref["ee"])
    assert cnt["swept_pt"] + cnt["swept_ee"] == ref["n_swept"]
    assert cnt["active"] == ref["n_active"]
    assert b.out.energy[0].item() == pytest.approx(ref["energy"], rel=1e-10)
    assert b.out.alpha[0].item() == ref["alpha"]
    for which, key in ((0, "spt"), (1, "see")):
        got = E.step_pairs(b.ctx, which).cpu().numpy().astype(np.int64)
        got = got[np.lexsort((got[:, 1], got[:, 0]))]
        assert np.array_equal(got, ref[key]), which


@pytest.mark.parametrize("mode", SPLITS)
def test_swept_candidates_sorted_every_split(ctx, sc, ref, mode):
    E.set_tuning(ctx, 2.0, (0, 0, 0, 0), mode)
    dsc = E.Scene.from_host(ctx, sc)
    spt, see = E.ccd_candidates(ctx, dsc, _dev(sc.q), _dev(sc.dq), sc.dhat)
    E.set_tuning(ctx, 2.0, (0, 0, 0, 0), 15)
    assert np.array_equal(spt.cpu().numpy(), ref["spt"]) and np.array_equal(see.cpu().numpy(), ref["see"])
