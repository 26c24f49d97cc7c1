"""The reduced-block projection (EIPC_PROJECT_REDUCED: each pair's reduced
local block W^T H W projected instead of its 12x12 Hessian) on the GPU
against the oracle, which builds that block over the pair's nodes and
projects it by Jacobi: reduced energy, gradient and Hessian within 1e-10
on tiny scenes and config 1 (dense and BSR, per call and in the planned
step, with either barrier form); per-pair entry points refuse the flag."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import batch as BT  # noqa: E402
from scenes import tiny_scene  # noqa: E402

TOL = 1e-10
FLAGS = E.ENERGY | E.GRAD | E.HESS | E.PROJECT_REDUCED
TINY = [(s, m) for s in range(3) for m in ("grid", "tet", "full_both")]


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (n if n > 0 else 1.0)


def _both(ctx, sc, flags, hess):
    dsc = E.Scene.from_host(ctx, sc)
    pt, ee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    r = E.barrier_reduce(ctx, dsc, _dev(sc.q), _dev(pt), _dev(ee), sc.dhat, sc.kappa, flags, hess=hess)
    ref = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags)
    H = r["hess"].cpu().numpy() if hess == "dense" else E.bsr_to_dense(*r["hess"], sc.n_node)
    assert r["n_active"] == ref["n_active"] > 0
    assert abs(r["energy"].item() - ref["energy"]) <= TOL * abs(ref["energy"])
    assert _rel(r["grad"].cpu().numpy(), ref["grad"]) <= TOL
    assert _rel(H, ref["hess"]) <= TOL
    return H, ref


@pytest.mark.parametrize("seed,mode", TINY)
def test_tiny(ctx, seed, mode):
    _both(ctx, tiny_scene(seed, mode=mode), FLAGS, "dense")


@pytest.mark.parametrize("hess", ["dense", "bsr"])
@pytest.mark.parametrize("sq", [False, True])
def test_config1(ctx, c1, hess, sq):
    H, ref = _both(ctx, c1, FLAGS | (E.SQDIST if sq else 0), hess)
    lam = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert lam.min() >= -1e-10 * np.abs(lam).max()


def test_planned_step(ctx, c1):
    b = BT.Batch(ctx, BT.concat([c1]), flags=FLAGS)
    b.make_plan(1.5)
    b.step()
    assert b.status() in (E.binding.OK, E.binding.WARN_CCD_CAPPED)
    pt, ee = O.candidates(c1, O.embed(c1, c1.q), c1.dhat)
    ref = O.barrier_reduce(c1, c1.q, pt, ee, c1.dhat, c1.kappa, FLAGS)
    rp, col, blk = b.out.hess(b.ctx)
    assert _rel(E.bsr_to_dense(rp, col, blk, c1.n_node), ref["hess"]) <= TOL
    assert _rel(b.out.grad.cpu().numpy(), ref["grad"]) <= TOL


def test_per_pair_entry_points_refuse_it(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    pt, ee = O.candidates(c1, O.embed(c1, c1.q), c1.dhat)
    with pytest.raises(E.EipcError):
        E.barrier_hvp(ctx, dsc, _dev(c1.q), _dev(pt), _dev(ee), c1.dhat, c1.kappa, E.PROJECT_REDUCED,
                      _dev(np.ones_like(c1.q)))
    with pytest.raises(E.EipcError):
        E.pair_eval(ctx, dsc, _dev(c1.q), 0, _dev(pt), c1.dhat, c1.kappa, E.PROJECT_REDUCED)
