"""The no-allocation entry point (eipc_barrier_hvp_noalloc, for callers
that cannot allocate device memory): its products equal those of
eipc_barrier_hvp to 1e-10 (relative, global norm) on two calls in a row,
the second with a smaller input, so the fixed scratch array's leftovers
from a larger call must not leak into a smaller one; inputs beyond the
array's size are refused before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
import paper_2409_16385_amd as E  # noqa: E402
from paper_2409_16385_amd import binding as B  # noqa: E402
from scenes import config1, tiny_scene  # noqa: E402

TOL = 1e-10


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda:0")


def _rel(a, b):
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (n if n > 0 else 1.0)


def _case(ctx, sc, seed):
    dsc = E.Scene.from_host(ctx, sc)
    x = O.embed(sc, sc.q)
    pt, ee = O.candidates(sc, x, sc.dhat)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3 * sc.n_node)
    off = rng.normal(size=(sc.n_vert, 3)) if sc.x_off is not None else None
    return dsc, _dev(sc.q), _dev(pt), _dev(ee), _dev(v), None if off is None else _dev(off)


def test_noalloc_hvp_matches_allocating_entry_point():
    ctx = E.Context(0)
    big, small = config1(), tiny_scene(3, mode="static")
    for sc, seed in ((big, 1), (small, 2), (big, 3)):
        dsc, q, pt, ee, v, voff = _case(ctx, sc, seed)
        for flags in (E.PROJECT, 0):
            ref, ref_off = E.barrier_hvp(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags, v, voff, want_off=True)
            got, got_off = E.barrier_hvp(ctx, dsc, q, pt, ee, sc.dhat, sc.kappa, flags, v, voff, want_off=True,
                                         noalloc=True)
            assert ctx.sync_status() == E.binding.OK
            r = ref.cpu().numpy()
            assert np.linalg.norm(r) > 0, sc.name
            assert _rel(got.cpu().numpy(), r) <= TOL, (sc.name, flags)
            assert _rel(got_off.cpu().numpy(), ref_off.cpu().numpy()) <= TOL, (sc.name, flags)


def test_noalloc_hvp_refuses_inputs_beyond_its_array():
    """8 M PT pairs need 64 MB of active lists on top of the positions:
    more than the 64 MiB array.  The lists are real device memory (zeros:
    vertex 0 against face 0), so nothing would read out of bounds even
    if the check were missing."""
    ctx = E.Context(0)
    sc = config1()
    dsc = E.Scene.from_host(ctx, sc)
    pt = torch.zeros((8 << 20, 2), dtype=torch.int32, device="cuda:0")
    ee = torch.zeros((0, 2), dtype=torch.int32, device="cuda:0")
    out = torch.zeros(3 * sc.n_node, dtype=torch.float64, device="cuda:0")
    q = _dev(sc.q)
    st = B._load().eipc_barrier_hvp_noalloc(ctx.handle, dsc.ref, q.data_ptr(), pt.data_ptr(), pt.shape[0],
                                            ee.data_ptr(), 0, sc.dhat, sc.kappa, E.PROJECT, q.data_ptr(), None,
                                            out.data_ptr(), None, ctx.stream())
    assert st == E.binding.ERR_CAPACITY
    assert b"fixed array" in B._load().eipc_last_error(ctx.handle)
    torch.cuda.synchronize()
    assert not out.any()  # nothing was enqueued
