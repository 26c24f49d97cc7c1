"""The planned step on one grasp geometry embedded at several coarse-grid
resolutions (the same surface meshes, only W changes), against the oracle:
candidate and active counts exact, energy, reduced gradient and reduced
Hessian to 1e-10, the step bound bit for bit.  The contact terms depend on
the surface alone, so the energy and the active set must also agree across
the resolutions (to the rounding of x = W q + x_off)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import batch as BT  # noqa: E402
from scenes import scene as S  # noqa: E402

TOL = 1e-10
FLAGS = E.ENERGY | E.GRAD | E.HESS | E.PROJECT
NODES = (40, 300, 1500)
_RES = {}


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


def _scene(nodes):
    # object frequency 20 (8,000 triangles), fingers frequency 8 in 3x4x4 grids
    return S.grasp_scene(0, 20, nodes, 8, finger_dims=(3, 4, 4), name=f"grasp_grid{nodes}")


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a - b)


@pytest.mark.parametrize("nodes", NODES)
def test_planned_step_matches_oracle_at_resolution(ctx, nodes):
    sc = _scene(nodes)
    b = BT.Batch(ctx, BT.concat([sc]), flags=FLAGS)
    b.make_plan(1.5)
    b.step()
    assert b.status() in (E.binding.OK, E.binding.WARN_CCD_CAPPED)
    cnt = b.counts()
    x = O.embed(sc, sc.q)
    opt, oee = O.candidates(sc, x, sc.dhat)
    assert cnt["cand_pt"] == len(opt) and cnt["cand_ee"] == len(oee)
    ref = O.barrier_reduce(sc, sc.q, opt, oee, sc.dhat, sc.kappa, FLAGS)
    assert cnt["active"] == ref["n_active"] > 0
    assert abs(b.out.energy[0].item() - ref["energy"]) <= TOL * abs(ref["energy"])
    assert _rel(b.out.grad.cpu().numpy(), ref["grad"]) <= TOL
    H = E.bsr_to_dense(*b.out.hess(b.ctx), sc.n_node)
    assert _rel(H, ref["hess"]) <= TOL
    a_ref, n_ref, _ = O.ccd_max_step(sc, sc.q, sc.dq, sc.dhat)
    assert cnt["swept_pt"] + cnt["swept_ee"] == n_ref
    assert b.out.alpha[0].item() == a_ref
    _RES[nodes] = (cnt["active"], ref["energy"])


def test_contact_terms_do_not_depend_on_resolution():
    if len(_RES) < len(NODES):
        pytest.skip("needs the per-resolution cases of this module")
    act = {v[0] for v in _RES.values()}
    en = [v[1] for v in _RES.values()]
    assert len(act) == 1
    assert max(en) - min(en) <= 1e-9 * max(abs(e) for e in en)
