"""The squared-distance barrier (EIPC_SQDIST, an alternative formulation of
Eq. 7: b(s) = -(s - dhat^2)^2 ln(s / dhat^2), s = d^2) on the GPU against
the oracle: per-pair energy, gradient and (projected) Hessian through the
per-class paths, the reduced energy, gradient and Hessian (per call and in
the planned step), Hessian-vector products and the lagged friction normal
force, within 1e-10 (relative, global norms); the active set is the one
of the distance form."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import batch as BT  # noqa: E402
from scenes import tiny_scene  # noqa: E402

TOL = 1e-10
FLAGS = E.ENERGY | E.GRAD | E.HESS | E.PROJECT | E.SQDIST
TINY = [(s, m) for s in range(4) for m in ("grid", "static", "full", "tet")]


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (n if n > 0 else 1.0)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("project", [False, True])
def test_pair_eval(ctx, c1, kind, project):
    sc = c1
    dsc = E.Scene.from_host(ctx, sc)
    x = O.embed(sc, sc.q)
    pairs = O.candidates(sc, x, sc.dhat)[kind]
    flags = E.SQDIST | (E.PROJECT if project else 0)
    ty, s2, e, g, H = (t.cpu().numpy() for t in E.pair_eval(ctx, dsc, _dev(sc.q), kind, _dev(pairs), sc.dhat,
                                                             sc.kappa, flags))
    n_act = 0
    for i, pr in enumerate(pairs):
        vid = [pr[0], *sc.faces[pr[1]]] if kind == 0 else [*sc.edges[pr[0]], *sc.edges[pr[1]]]
        st, t, s, er, gr, Hr = O.pair_eval(kind, x[vid].reshape(12), sc.dhat, sc.kappa, flags=O.SQDIST)
        assert ty[i] == t and s2[i] == s
        if st != O.OK:
            assert e[i] == 0 and not g[i].any()
            continue
        n_act += 1
        if project:
            Hr, _ = O.project_psd(Hr)
        assert abs(e[i] - er) <= TOL * abs(er)
        assert _rel(g[i], gr) <= TOL
        assert _rel(H[i], Hr) <= TOL
    assert n_act > 0


def _reduce(ctx, sc, hess):
    dsc = E.Scene.from_host(ctx, sc)
    pt, ee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    flags = FLAGS | (E.MOLLIFY if sc.x_rest is not None else 0)
    r = E.barrier_reduce(ctx, dsc, _dev(sc.q), _dev(pt), _dev(ee), sc.dhat, sc.kappa, flags, hess=hess)
    ref = O.barrier_reduce(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags)
    return r, ref


def _check(r, ref, H=None):
    assert r["n_active"] == ref["n_active"] > 0
    assert abs(r["energy"].item() - ref["energy"]) <= TOL * abs(ref["energy"])
    assert _rel(r["grad"].cpu().numpy(), ref["grad"]) <= TOL
    assert _rel(r["hess"].cpu().numpy() if H is None else H, ref["hess"]) <= TOL


@pytest.mark.parametrize("seed,mode", TINY)
def test_reduce_tiny(ctx, seed, mode):
    r, ref = _reduce(ctx, tiny_scene(seed, mode=mode), "dense")
    _check(r, ref)


def test_reduce_config1_bsr(ctx, c1):
    r, ref = _reduce(ctx, c1, "bsr")
    _check(r, ref, E.bsr_to_dense(*r["hess"], c1.n_node))
    # the distance form gives another energy on the same active set
    d = O.barrier_reduce(c1, c1.q, *O.candidates(c1, O.embed(c1, c1.q), c1.dhat), c1.dhat, c1.kappa,
                         FLAGS & ~E.SQDIST, hess=False)
    assert d["n_active"] == ref["n_active"] and abs(d["energy"] - ref["energy"]) > 1e-3 * abs(ref["energy"])


def test_planned_step_config1(ctx, c1):
    b = BT.Batch(ctx, BT.concat([c1]), flags=FLAGS)
    b.make_plan(1.5)
    b.step()
    assert b.status() in (E.binding.OK, E.binding.WARN_CCD_CAPPED)
    pt, ee = O.candidates(c1, O.embed(c1, c1.q), c1.dhat)
    ref = O.barrier_reduce(c1, c1.q, pt, ee, c1.dhat, c1.kappa, FLAGS)
    assert b.out.energy[0].item() == pytest.approx(ref["energy"], rel=TOL)
    assert _rel(b.out.grad.cpu().numpy(), ref["grad"]) <= TOL
    rp, col, blk = b.out.hess(b.ctx)
    assert _rel(E.bsr_to_dense(rp, col, blk, c1.n_node), ref["hess"]) <= TOL


@pytest.mark.parametrize("seed,mode", TINY[:6])
def test_hvp(ctx, seed, mode):
    sc = tiny_scene(seed, mode=mode)
    dsc = E.Scene.from_host(ctx, sc)
    pt, ee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3 * sc.n_node)
    flags = E.PROJECT | E.SQDIST
    out = E.barrier_hvp(ctx, dsc, _dev(sc.q), _dev(pt), _dev(ee), sc.dhat, sc.kappa, flags, _dev(v), None)
    out = out[0] if isinstance(out, tuple) else out
    st, ref, _ = O.barrier_hvp(sc, sc.q, pt, ee, sc.dhat, sc.kappa, flags, v, None)
    assert st == O.OK
    assert _rel(out.cpu().numpy(), ref) <= TOL


def test_friction_normal_force(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    pt, ee = O.candidates_grid(c1, O.embed(c1, c1.q), c1.dhat)
    st1, rpt = O.friction_lag_list(c1, c1.q, 0, pt, c1.dhat, c1.kappa, O.SQDIST)
    st2, ree = O.friction_lag_list(c1, c1.q, 1, ee, c1.dhat, c1.kappa, O.SQDIST)
    assert st1 == O.OK and st2 == O.OK
    lpt, lee = E.friction_lag(ctx, dsc, _dev(c1.q), _dev(pt), _dev(ee), c1.dhat, c1.kappa, E.SQDIST)
    for got, ref in ((lpt, rpt), (lee, ree)):
        got = got.cpu().numpy()
        act = ref[:, 0] > 0
        assert act.any() and np.array_equal(got[:, 0] > 0, act)
        assert _rel(got[act], ref[act]) <= TOL
