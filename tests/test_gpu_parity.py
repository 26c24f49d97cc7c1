"""GPU parity: the HIP library (through its C ABI) against the oracle on
the same seeded inputs.  Candidates, types and CCD steps bit-exact; energy,
reduced gradient and Hessian within 1e-10 relative (global norms)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from scenes import config1, tiny_scene  # noqa: E402

TOL = 1e-10
FLAGS = E.ENERGY | E.GRAD | E.HESS | E.PROJECT


@pytest.fixture(scope="module")
def ctx():
    return E.Context(0)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


TINY = [(s, m) for s in range(8) for m in ("grid", "static", "full", "full_both", "tet")]


def test_fp64_sqrt_div_round_like_host(ctx):
    rng = np.random.default_rng(0)
    a = np.abs(rng.normal(size=200000)) * 10.0 ** rng.uniform(-30, 30, size=200000)
    b = rng.normal(size=200000) * 10.0 ** rng.uniform(-30, 30, size=200000)
    sq, dv = E.fp64_selftest(ctx, _dev(a), _dev(b))
    assert np.array_equal(sq.cpu().numpy(), np.sqrt(a))
    assert np.array_equal(dv.cpu().numpy(), a / b)


@pytest.mark.parametrize("seed,mode", TINY[:10])
def test_embed_bit_exact(ctx, seed, mode):
    sc = tiny_scene(seed, mode=mode)
    dsc = E.Scene.from_host(ctx, sc)
    x = E.embed(ctx, dsc, _dev(sc.q)).cpu().numpy()
    assert np.array_equal(x, O.embed(sc, sc.q))


def test_embed_bit_exact_config1(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    x = E.embed(ctx, dsc, _dev(c1.q)).cpu().numpy()
    assert np.array_equal(x, O.embed(c1, c1.q))
    p = E.embed(ctx, dsc, _dev(c1.dq), off=None).cpu().numpy()
    assert np.array_equal(p, O.embed(c1, c1.dq, off=None))


@pytest.mark.parametrize("seed,mode", TINY)
def test_candidates_bit_exact_tiny(ctx, seed, mode):
    sc = tiny_scene(seed, mode=mode)
    dsc = E.Scene.from_host(ctx, sc)
    pt, ee = E.build_candidates(ctx, dsc, _dev(sc.q), sc.dhat)
    opt, oee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    assert np.array_equal(pt.cpu().numpy(), opt)
    assert np.array_equal(ee.cpu().numpy(), oee)


def test_candidates_bit_exact_config1(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    pt, ee = E.build_candidates(ctx, dsc, _dev(c1.q), c1.dhat)
    opt, oee = O.candidates(c1, O.embed(c1, c1.q), c1.dhat)
    assert len(opt) > 0 and len(oee) > 0
    assert np.array_equal(pt.cpu().numpy(), opt)
    assert np.array_equal(ee.cpu().numpy(), oee)


def test_candidate_capacity_error_reports_required_count(ctx, c1):
    import ctypes as C
    from paper_2409_16385_amd import binding as B
    dsc = E.Scene.from_host(ctx, c1)
    q = _dev(c1.q)
    pt = torch.empty((1, 2), dtype=torch.int32, device="cuda:0")
    ee = torch.empty((1, 2), dtype=torch.int32, device="cuda:0")
    npt, nee = C.c_int64(), C.c_int64()
    st = B._load().eipc_build_candidates(ctx.handle, dsc.ref, q.data_ptr(), c1.dhat, pt.data_ptr(), 1,
                                         ee.data_ptr(), 1, C.byref(npt), C.byref(nee), ctx.stream())
    assert st == B.ERR_CAPACITY
    opt, oee = O.candidates(c1, O.embed(c1, c1.q), c1.dhat)
    assert (npt.value, nee.value) == (len(opt), len(oee))


def _oracle_types(sc, pairs, kind):
    x = O.embed(sc, sc.q)
    out = []
    for pr in pairs:
        vid = [pr[0], *sc.faces[pr[1]]] if kind == 0 else [*sc.edges[pr[0]], *sc.edges[pr[1]]]
        x12 = x[vid].reshape(12)
        t = O.pt_type(*x[vid]) if kind == 0 else O.ee_type(*x[vid])
        out.append((t, O.pair_dist2(kind, t, x12)))
    return out


@pytest.mark.parametrize("seed,mode", TINY[:15] + [("c1", "c1")])
def test_narrow_phase_active_set_and_types(ctx, c1, seed, mode):
    sc = c1 if seed == "c1" else tiny_scene(seed, mode=mode)
    dsc = E.Scene.from_host(ctx, sc)
    opt, oee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    ap, tp, ae, te = E.narrow_phase(ctx, dsc, _dev(sc.q), _dev(opt), _dev(oee), sc.dhat)
    for kind, lst, act, typ in ((0, opt, ap, tp), (1, oee, ae, te)):
        ref = _oracle_types(sc, lst, kind)
        exp = {i: t for i, (t, s) in enumerate(ref) if s < sc.dhat ** 2}
        got = dict(zip(act.cpu().numpy().tolist(), typ.cpu().numpy().tolist()))
        assert got == exp


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("project", [False, True])
def test_pair_eval_matches_oracle(ctx, c1, kind, project):
    sc = c1
    dsc = E.Scene.from_host(ctx, sc)
    x = O.embed(sc, sc.q)
    opt, oee = O.candidates(sc, x, sc.dhat)
    pairs = opt if kind == 0 else oee
    ty, s2, e, g, H = E.pair_eval(ctx, dsc, _dev(sc.q), kind, _dev(pairs), sc.dhat, sc.kappa,
                                  E.PROJECT if project else 0)
    ty, s2, e, g, H = (t.cpu().numpy() for t in (ty, s2, e, g, H))
    n_act = 0
    for i, pr in enumerate(pairs):
        vid = [pr[0], *sc.faces[pr[1]]] if kind == 0 else [*sc.edges[pr[0]], *sc.edges[pr[1]]]
        st, t, s, er, gr, Hr = O.pair_eval(kind, x[vid].reshape(12), sc.dhat, sc.kappa)
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


def _reduce_both(ctx, sc, hess):
    dsc = E.Scene.from_host(ctx, sc)
    opt, oee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    flags = FLAGS | (E.MOLLIFY if sc.x_rest is not None else 0)
    r = E.barrier_reduce(ctx, dsc, _dev(sc.q), _dev(opt), _dev(oee), sc.dhat, sc.kappa, flags, hess=hess)
    ref = O.barrier_reduce(sc, sc.q, opt, oee, sc.dhat, sc.kappa, flags)
    return r, ref


@pytest.mark.parametrize("seed,mode", TINY)
def test_barrier_reduce_tiny(ctx, seed, mode):
    sc = tiny_scene(seed, mode=mode)
    r, ref = _reduce_both(ctx, sc, "dense")
    assert r["n_active"] == ref["n_active"]
    assert abs(r["energy"].item() - ref["energy"]) <= TOL * abs(ref["energy"])
    assert _rel(r["grad"].cpu().numpy(), ref["grad"]) <= TOL
    assert _rel(r["hess"].cpu().numpy(), ref["hess"]) <= TOL


@pytest.mark.parametrize("hess", ["dense", "bsr"])
def test_barrier_reduce_config1(ctx, c1, hess):
    r, ref = _reduce_both(ctx, c1, hess)
    assert r["n_active"] == ref["n_active"] > 300
    assert abs(r["energy"].item() - ref["energy"]) <= TOL * abs(ref["energy"])
    assert _rel(r["grad"].cpu().numpy(), ref["grad"]) <= TOL
    if hess == "dense":
        H = r["hess"].cpu().numpy()
    else:
        rowptr, col, blocks = r["hess"]
        rp = rowptr.cpu().numpy()
        cl = col.cpu().numpy()
        for i in range(c1.n_node):  # sorted columns, both triangles
            assert np.all(np.diff(cl[rp[i]:rp[i + 1]]) > 0)
        H = E.bsr_to_dense(rowptr, col, blocks, c1.n_node)
    assert _rel(H, ref["hess"]) <= TOL
    assert np.array_equal(H != 0, ref["hess"] != 0) or _rel(H, ref["hess"]) <= TOL


@pytest.mark.parametrize("seed,mode", TINY[:10])
@pytest.mark.parametrize("project", [False, True])
def test_hvp_matches_oracle(ctx, seed, mode, project):
    sc = tiny_scene(seed, mode=mode)
    dsc = E.Scene.from_host(ctx, sc)
    opt, oee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3 * sc.n_node)
    v_off = rng.normal(size=(sc.n_vert, 3))
    flags = E.PROJECT if project else 0
    out, off = E.barrier_hvp(ctx, dsc, _dev(sc.q), _dev(opt), _dev(oee), sc.dhat, sc.kappa, flags, _dev(v),
                             _dev(v_off), want_off=True)
    st, ref, ref_off = O.barrier_hvp(sc, sc.q, opt, oee, sc.dhat, sc.kappa, flags, v, v_off, want_off=True)
    assert _rel(out.cpu().numpy(), ref) <= TOL
    assert _rel(off.cpu().numpy(), ref_off) <= TOL


@pytest.mark.parametrize("seed,mode", TINY[:10] + [("c1", "c1")])
def test_ccd_candidates_and_toi_bit_exact(ctx, c1, seed, mode):
    sc = c1 if seed == "c1" else tiny_scene(seed, mode=mode)
    dsc = E.Scene.from_host(ctx, sc)
    q, dq = _dev(sc.q), _dev(sc.dq)
    pt, ee = E.ccd_candidates(ctx, dsc, q, dq, sc.dhat)
    x = O.embed(sc, sc.q)
    p = O.embed(sc, sc.dq, off=None)
    opt, oee = O.candidates(sc, x, sc.dhat, x1=x + p)
    assert np.array_equal(pt.cpu().numpy(), opt)
    assert np.array_equal(ee.cpu().numpy(), oee)
    for kind, lst in ((0, opt), (1, oee)):
        if len(lst) == 0:
            continue
        t, it = E.ccd_toi(ctx, dsc, q, dq, kind, _dev(lst))
        tr, itr = O.ccd_toi(sc, x, p, kind, lst)
        assert np.array_equal(t.cpu().numpy(), tr)
        assert np.array_equal(it.cpu().numpy(), itr)
    a, n, capped = E.ccd_max_step(ctx, dsc, q, dq, sc.dhat)
    a_ref, n_ref, _ = O.ccd_max_step(sc, sc.q, sc.dq, sc.dhat)
    assert n == n_ref
    assert a <= a_ref and a == a_ref


@pytest.mark.parametrize("max_iter", [1, 2, 3, 5, 40])
def test_ccd_max_step_at_small_iteration_caps(ctx, c1, max_iter):
    # The step-bound kernels drop pairs whose bound is shown to be no smaller
    # than their scene's bound so far; the minimum must come out exactly as
    # the oracle's, which advances every pair to its end or its cap.
    dsc = E.Scene.from_host(ctx, c1)
    a, n, capped = E.ccd_max_step(ctx, dsc, _dev(c1.q), _dev(c1.dq), c1.dhat, max_iter=max_iter)
    a_ref, n_ref, ncap_ref = O.ccd_max_step(c1, c1.q, c1.dq, c1.dhat, max_iter=max_iter)
    assert n == n_ref
    assert a == a_ref
    # a warning names a capped pair that could still lower the bound; the
    # oracle counts every capped pair
    assert not capped or ncap_ref > 0


def test_ccd_zero_motion_is_t_max(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    a, n, _ = E.ccd_max_step(ctx, dsc, _dev(c1.q), _dev(np.zeros_like(c1.dq)), c1.dhat)
    assert a == 1.0 and n > 0


def test_empty_pair_lists(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    z = np.zeros((0, 2), np.int32)
    r = E.barrier_reduce(ctx, dsc, _dev(c1.q), _dev(z), _dev(z), c1.dhat, c1.kappa, FLAGS, hess="dense")
    assert r["n_active"] == 0 and r["energy"].item() == 0.0
    assert not r["grad"].any() and not r["hess"].any()
    r = E.barrier_reduce(ctx, dsc, _dev(c1.q), _dev(z), _dev(z), c1.dhat, c1.kappa, FLAGS, hess="bsr")
    assert r["n_active"] == 0 and r["hess"][1].numel() == 0


def test_no_contact_scene(ctx, c1):
    """Lift the sphere far above the ground: only self-contact pairs remain
    and, at a tiny dhat, no pair is active."""
    dsc = E.Scene.from_host(ctx, c1)
    q = c1.q.copy().reshape(-1, 3)
    q[:, 2] += 1.0
    q = q.reshape(-1)
    pt, ee = E.build_candidates(ctx, dsc, _dev(q), 1e-9)
    r = E.barrier_reduce(ctx, dsc, _dev(q), pt, ee, 1e-9, c1.kappa, FLAGS, hess="dense")
    assert r["n_active"] == 0 and not r["grad"].any()


def test_intersecting_input_is_reported(ctx):
    sc = tiny_scene(1, mode="static")
    dsc = E.Scene.from_host(ctx, sc)
    # collapse every node onto one point: pairs reach zero distance
    q = np.zeros_like(sc.q)
    pt = np.array([[0, 1]], dtype=np.int32)
    f = sc.faces[1]
    pt[0, 0] = [v for v in range(sc.n_vert) if v not in f and np.diff(sc.W_rowptr)[v] > 0][0]
    with pytest.raises(E.EipcError) as ei:
        E.barrier_reduce(ctx, dsc, _dev(q), _dev(pt), _dev(np.zeros((0, 2), np.int32)), sc.dhat, sc.kappa, FLAGS,
                         hess="dense")
    assert ei.value.status in (-3, -5)


def test_nonfinite_input_is_reported(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    q = c1.q.copy()
    q[5] = np.nan
    with pytest.raises(E.EipcError) as ei:
        E.build_candidates(ctx, dsc, _dev(q), c1.dhat)
    assert ei.value.status == -5
    # the context stays usable
    pt, ee = E.build_candidates(ctx, dsc, _dev(c1.q), c1.dhat)
    assert pt.shape[0] > 0


def test_argument_errors_enqueue_nothing(ctx, c1):
    dsc = E.Scene.from_host(ctx, c1)
    with pytest.raises(E.EipcError) as ei:
        E.build_candidates(ctx, dsc, _dev(c1.q), -1.0)
    assert ei.value.status == -1
    with pytest.raises(E.EipcError):
        E.ccd_max_step(ctx, dsc, _dev(c1.q), _dev(c1.dq), c1.dhat, s=1.5)


def test_mollifier_without_rest_positions_is_an_argument_error(ctx):
    """EIPC_MOLLIFY is defined by the rest edge lengths: a scene without
    them is rejected (never silently unmollified)."""
    import copy
    sc = copy.copy(tiny_scene(2, mode="grid"))
    sc.x_rest = None
    dsc = E.Scene.from_host(ctx, sc)
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    q = _dev(sc.q)
    with pytest.raises(E.EipcError) as ei:
        E.barrier_reduce(ctx, dsc, q, _dev(pt), _dev(ee), sc.dhat, sc.kappa, FLAGS | E.MOLLIFY, hess="dense")
    assert ei.value.status == -1
    with pytest.raises(E.EipcError) as ei:
        E.barrier_hvp(ctx, dsc, q, _dev(pt), _dev(ee), sc.dhat, sc.kappa, E.MOLLIFY, _dev(np.ones_like(sc.q)))
    assert ei.value.status == -1
    with pytest.raises(E.EipcError) as ei:
        E.pair_eval(ctx, dsc, q, 1, _dev(ee), sc.dhat, sc.kappa, E.MOLLIFY)
    assert ei.value.status == -1
    # without the flag the same call runs
    r = E.barrier_reduce(ctx, dsc, q, _dev(pt), _dev(ee), sc.dhat, sc.kappa, FLAGS, hess="dense")
    assert r["n_active"] > 0


def test_arena_mode_matches_grow_mode(ctx, c1):
    """A context created with a scratch reservation carves every call from
    it (no allocation after creation) and gives the grow-mode results; a
    reservation too small for a call is a capacity error, and the context
    stays usable for calls that fit."""
    dsc = E.Scene.from_host(ctx, c1)
    q, dq = _dev(c1.q), _dev(c1.dq)
    g = E.Context(0)
    dg = E.Scene.from_host(g, c1)

    def run(cx, ds):
        pt, ee = E.build_candidates(cx, ds, q, c1.dhat)
        r = E.barrier_reduce(cx, ds, q, pt, ee, c1.dhat, c1.kappa, FLAGS, hess="bsr")
        a, n, _ = E.ccd_max_step(cx, ds, q, dq, c1.dhat)
        hv = E.barrier_hvp(cx, ds, q, pt, ee, c1.dhat, c1.kappa, E.PROJECT, dq)
        return pt, ee, r, a, n, hv

    ref = run(g, dg)
    reserved, high = g.scratch_bytes()
    assert reserved == 0 and high > 0
    a_ctx = E.Context(0, reserve_bytes=2 * high)
    da = E.Scene.from_host(a_ctx, c1)
    for _ in range(2):  # the second round reuses the same carving
        got = run(a_ctx, da)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
        assert got[2]["n_active"] == ref[2]["n_active"]
        assert _rel(got[2]["grad"].cpu().numpy(), ref[2]["grad"].cpu().numpy()) <= 1e-12
        for u, v in zip(got[2]["hess"][:2], ref[2]["hess"][:2]):
            assert torch.equal(u, v)
        assert _rel(got[2]["hess"][2].cpu().numpy(), ref[2]["hess"][2].cpu().numpy()) <= 1e-12
        assert got[3] == ref[3] and got[4] == ref[4]
        assert _rel(got[5].cpu().numpy(), ref[5].cpu().numpy()) <= 1e-12
    r2, h2 = a_ctx.scratch_bytes()
    assert r2 >= 2 * high and 0 < h2 <= r2
    tiny_ctx = E.Context(0, reserve_bytes=1 << 20)
    dt = E.Scene.from_host(tiny_ctx, c1)
    with pytest.raises(E.EipcError) as ei:
        E.ccd_max_step(tiny_ctx, dt, q, dq, c1.dhat)
    assert ei.value.status == -2
    sc = tiny_scene(0)
    ds = E.Scene.from_host(tiny_ctx, sc)
    pt, ee = E.build_candidates(tiny_ctx, ds, _dev(sc.q), sc.dhat)
    opt, oee = O.candidates(sc, O.embed(sc, sc.q), sc.dhat)
    assert np.array_equal(pt.cpu().numpy(), opt) and np.array_equal(ee.cpu().numpy(), oee)


def test_long_bsr_rows_against_oracle(ctx):
    """A full-space sheet over an affine-body plate: the plate's 4 node rows
    hold about 2,600 blocks each (rows beyond 64 blocks are sorted 64 at a
    time against the whole row).  Blocks, pattern and products match the
    oracle."""
    from scenes.scene import long_row_scene
    sc = long_row_scene()
    dsc = E.Scene.from_host(ctx, sc)
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates_grid(sc, x, sc.dhat)
    ref = O.barrier_reduce_bsr(sc, sc.q, pt, ee, sc.dhat, sc.kappa, FLAGS)
    assert ref["status"] == O.OK and np.diff(ref["rowptr"]).max() > 1024
    q = _dev(sc.q)
    r = E.barrier_reduce(ctx, dsc, q, _dev(pt), _dev(ee), sc.dhat, sc.kappa, FLAGS, hess="bsr")
    rp, col, blk = (t.cpu().numpy() for t in r["hess"])
    assert np.array_equal(rp, ref["rowptr"]) and np.array_equal(col, ref["col"])
    assert _rel(blk.reshape(-1, 3, 3), ref["blocks"]) <= TOL
    assert _rel(r["grad"].cpu().numpy(), ref["grad"]) <= TOL
