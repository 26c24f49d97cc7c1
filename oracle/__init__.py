"""Oracle for the Embedded IPC contact stage: TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation (``eipc_oracle.c``) of what the contact
stage computes, written from the paper's definitions, plus this ctypes
wrapper.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may use it; the product path never does.  It shares no code with
the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ENERGY, GRAD, HESS, PROJECT, MOLLIFY, SQDIST, PROJECT_REDUCED = 1, 2, 4, 8, 16, 32, 64
OK, INACTIVE, ERR_CAPACITY, ERR_INTERSECTING, ERR_NONFINITE = 0, 1, -2, -3, -5
PT_TYPES = ["P-T0", "P-T1", "P-T2", "P-E0", "P-E1", "P-E2", "P-T"]
EE_TYPES = ["EA0-EB0", "EA0-EB1", "EA1-EB0", "EA1-EB1", "EA-EB0", "EA-EB1",
            "EA0-EB", "EA1-EB", "EA-EB"]

_P = C.c_void_p
_D = C.c_double
_I64 = C.c_int64
_I32 = C.c_int32


class OrScene(C.Structure):
    _fields_ = [("n_vert", _I32), ("n_node", _I32), ("n_face", _I32), ("n_edge", _I32),
                ("faces", _P), ("edges", _P), ("rowptr", _P), ("col", _P), ("val", _P),
                ("x_off", _P), ("x_rest", _P)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        sig = {
            "or_embed": (None, [_P, _P, _P, _P]),
            "or_pt_query": (_I64, [_P, _P, _P, _D, _I32, _P, _I64]),
            "or_ee_query": (_I64, [_P, _P, _P, _D, _I32, _P, _I64]),
            "or_candidates": (C.c_int, [_P, _P, _P, _D, _P, _I64, _P, _P, _I64, _P]),
            "or_pt_type": (C.c_int, [_P, _P, _P, _P]),
            "or_ee_type": (C.c_int, [_P, _P, _P, _P]),
            "or_pair_dist2": (_D, [C.c_int, C.c_int, _P]),
            "or_pair_dist2_derivs": (None, [C.c_int, C.c_int, _P, _P, _P, _P]),
            "or_barrier": (None, [_D, _D, _P, _P, _P]),
            "or_mollifier": (None, [_D, _D, _P, _P, _P]),
            "or_pair_eval": (C.c_int, [C.c_int, _P, _P, _D, _D, _P, _P, _P, _P, _P]),
            "or_pair_eval_f": (C.c_int, [C.c_int, _P, _P, _D, _D, C.c_uint32, _P, _P, _P, _P, _P]),
            "or_barrier_sq": (None, [_D, _D, _P, _P, _P]),
            "or_project_psd": (C.c_int, [C.c_int, _P, _P]),
            "or_barrier_reduce": (C.c_int, [_P, _P, _P, _I64, _P, _I64, _D, _D, C.c_uint32,
                                            _P, _P, _P, _P]),
            "or_barrier_hvp": (C.c_int, [_P, _P, _P, _I64, _P, _I64, _D, _D, C.c_uint32,
                                         _P, _P, _P, _P]),
            "or_accd_pair": (_D, [C.c_int, _P, _P, _D, _D, _I64, _P]),
            "or_ccd_toi": (C.c_int, [_P, _P, _P, C.c_int, _P, _I64, _D, _D, _I64, _P, _P]),
            "or_ccd_toi_m": (C.c_int, [_P, _P, _P, C.c_int, _P, _I64, _D, _D, _I64, C.c_int, _P, _P]),
            "or_c2a_pair": (_D, [C.c_int, _P, _P, _D, _D, _I64, _P]),
            "or_ccd_max_step": (C.c_int, [_P, _P, _P, _P, _D, _D, _D, _I64, _P, _P, _P]),
            "or_narrow": (None, [_P, _P, C.c_int, _P, _I64, _D, _P, _P, _P]),
            "or_friction_f": (None, [_D, _D, _P, _P, _P]),
            "or_friction_lag": (C.c_int, [C.c_int, _P, _P, _D, _D, _P]),
            "or_friction_lag_f": (C.c_int, [C.c_int, _P, _P, _D, _D, C.c_uint32, _P]),
            "or_friction_pair": (None, [_P, _P, _D, _D, _P, _P, _P]),
            "or_friction_lag_list": (C.c_int, [_P, _P, C.c_int, _P, _I64, _D, _D, C.c_uint32, _P]),
            "or_friction_reduce": (C.c_int, [_P, _P, _P, _I64, _P, _P, _I64, _P, _D, _D, _P, _P, _P]),
            "or_grid_build": (_P, [_P, _P, _P, _D, _D]),
            "or_grid_pairs": (_I64, [_P, C.c_int, _I32, _I32, _P, _I64]),
            "or_grid_cell": (_D, [_P]),
            "or_grid_free": (None, [_P]),
            "or_barrier_reduce_bsr": (_P, [_P, _P, _P, _I64, _P, _I64, _D, _D, C.c_uint32, _P, _P, _P, _P]),
            "or_bsr_nnzb": (_I64, [_P]),
            "or_bsr_copy": (None, [_P, _P, _P, _P]),
            "or_bsr_free": (None, [_P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


class _Sc:
    """ctypes view of a scenes.Scene (keeps the arrays alive)."""

    def __init__(self, sc):
        self.keep = [_i32(sc.faces), _i32(sc.edges), _i32(sc.W_rowptr), _i32(sc.W_col),
                     _f64(sc.W_val), _f64(sc.x_off), _f64(sc.x_rest)]
        f, e, rp, col, val, xo, xr = self.keep
        self.s = OrScene(sc.n_vert, sc.n_node, sc.n_face, sc.n_edge, _ptr(f), _ptr(e),
                         _ptr(rp), _ptr(col), _ptr(val), _ptr(xo), _ptr(xr))
        self.n_vert, self.n_node = sc.n_vert, sc.n_node
        self.n_face, self.n_edge = sc.n_face, sc.n_edge

    @property
    def ref(self):
        return C.byref(self.s)


def scene(sc) -> _Sc:
    return sc if isinstance(sc, _Sc) else _Sc(sc)


def embed(sc, q, off="scene"):
    """x = W q + off (AoS [n_vert, 3]); off defaults to the scene's x_off."""
    s = scene(sc)
    q = _f64(q)
    if isinstance(off, str):
        off = s.keep[5]
    off = _f64(off)
    x = np.empty((s.n_vert, 3))
    lib().or_embed(s.ref, _ptr(q), _ptr(off), _ptr(x))
    return x


def candidates(sc, x, dhat, x1=None):
    s = scene(sc)
    x = _f64(x)
    x1 = _f64(x1)
    npt, nee = _I64(), _I64()
    lib().or_candidates(s.ref, _ptr(x), _ptr(x1), dhat, None, 0, C.byref(npt), None, 0, C.byref(nee))
    pt = np.empty((max(npt.value, 1), 2), dtype=np.int32)
    ee = np.empty((max(nee.value, 1), 2), dtype=np.int32)
    st = lib().or_candidates(s.ref, _ptr(x), _ptr(x1), dhat, _ptr(pt), npt.value, C.byref(npt),
                             _ptr(ee), nee.value, C.byref(nee))
    assert st == OK
    return pt[:npt.value].copy(), ee[:nee.value].copy()


def pt_query(sc, x, dhat, v, x1=None):
    s = scene(sc)
    x, x1 = _f64(x), _f64(x1)
    out = np.empty(max(s.n_face, 1), dtype=np.int32)
    n = lib().or_pt_query(s.ref, _ptr(x), _ptr(x1), dhat, int(v), _ptr(out), len(out))
    return out[:n].copy()


def ee_query(sc, x, dhat, ea, x1=None):
    s = scene(sc)
    x, x1 = _f64(x), _f64(x1)
    out = np.empty(max(s.n_edge, 1), dtype=np.int32)
    n = lib().or_ee_query(s.ref, _ptr(x), _ptr(x1), dhat, int(ea), _ptr(out), len(out))
    return out[:n].copy()


def pt_type(p, t0, t1, t2) -> int:
    a = [_f64(v) for v in (p, t0, t1, t2)]
    return lib().or_pt_type(*[_ptr(v) for v in a])


def ee_type(a0, a1, b0, b1) -> int:
    a = [_f64(v) for v in (a0, a1, b0, b1)]
    return lib().or_ee_type(*[_ptr(v) for v in a])


def pair_dist2(kind: int, type_: int, x12) -> float:
    x12 = _f64(x12).reshape(12)
    return lib().or_pair_dist2(kind, type_, _ptr(x12))


def pair_dist2_derivs(kind: int, type_: int, x12):
    x12 = _f64(x12).reshape(12)
    s = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros((12, 12))
    lib().or_pair_dist2_derivs(kind, type_, _ptr(x12), _ptr(s), _ptr(g), _ptr(H))
    return s[0], g, H


def barrier(d, dhat):
    out = np.zeros(3)
    lib().or_barrier(d, dhat, _ptr(out[0:]), _ptr(out[1:]), _ptr(out[2:]))
    return out[0], out[1], out[2]


def mollifier(c, eps):
    out = np.zeros(3)
    lib().or_mollifier(c, eps, _ptr(out[0:]), _ptr(out[1:]), _ptr(out[2:]))
    return out[0], out[1], out[2]


def barrier_sq(s, shat):
    """(b, db/ds, d2b/ds2) of the squared-distance barrier at s."""
    out = np.zeros(3)
    lib().or_barrier_sq(float(s), float(shat), _ptr(out[0:]), _ptr(out[1:]), _ptr(out[2:]))
    return out[0], out[1], out[2]


def pair_eval(kind, x12, dhat, kappa, rest12=None, flags=0):
    """Returns (status, type, s, e, g[12], H[12,12]) with the true Hessian
    (flags: SQDIST for the squared-distance barrier)."""
    x12 = _f64(x12).reshape(12)
    r12 = None if rest12 is None else _f64(rest12).reshape(12)
    t = C.c_int()
    s = np.zeros(1)
    e = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros((12, 12))
    st = lib().or_pair_eval_f(kind, _ptr(x12), _ptr(r12), dhat, kappa, flags, C.byref(t), _ptr(s),
                              _ptr(e), _ptr(g), _ptr(H))
    return st, t.value, s[0], e[0], g, H


def project_psd(A):
    A = _f64(A)
    n = A.shape[0]
    P = np.zeros((n, n))
    sweeps = lib().or_project_psd(n, _ptr(A), _ptr(P))
    return P, sweeps


def barrier_reduce(sc, q, pt, ee, dhat, kappa, flags, hess=True):
    """Returns dict(status, energy, grad, hess (dense or None), n_active)."""
    s = scene(sc)
    q = _f64(q)
    pt = _i32(pt).reshape(-1, 2) if pt is not None else np.zeros((0, 2), np.int32)
    ee = _i32(ee).reshape(-1, 2) if ee is not None else np.zeros((0, 2), np.int32)
    nd = 3 * s.n_node
    e = np.zeros(1)
    g = np.zeros(nd)
    H = np.zeros((nd, nd)) if hess else None
    na = _I64()
    st = lib().or_barrier_reduce(s.ref, _ptr(q), _ptr(pt), len(pt), _ptr(ee), len(ee), dhat, kappa,
                                 int(flags), _ptr(e), _ptr(g), _ptr(H), C.byref(na))
    return {"status": st, "energy": e[0], "grad": g, "hess": H, "n_active": na.value}


def barrier_hvp(sc, q, pt, ee, dhat, kappa, flags, v, v_off=None, want_off=False):
    s = scene(sc)
    q, v, v_off = _f64(q), _f64(v), _f64(v_off)
    pt = _i32(pt).reshape(-1, 2)
    ee = _i32(ee).reshape(-1, 2)
    out = np.zeros(3 * s.n_node)
    out_off = np.zeros((s.n_vert, 3)) if want_off else None
    st = lib().or_barrier_hvp(s.ref, _ptr(q), _ptr(pt), len(pt), _ptr(ee), len(ee), dhat, kappa,
                              int(flags), _ptr(v), _ptr(v_off), _ptr(out), _ptr(out_off))
    return st, out, out_off


def accd_pair(kind, x12, p12, s=0.1, t_c=1.0, max_iter=100000):
    x12 = _f64(x12).reshape(12)
    p12 = _f64(p12).reshape(12)
    it = _I64()
    t = lib().or_accd_pair(kind, _ptr(x12), _ptr(p12), s, t_c, max_iter, C.byref(it))
    return t, it.value


def c2a_pair(kind, x12, p12, s=0.1, t_c=1.0, max_iter=100000):
    """Conservative advancement along the closest direction (method 1)."""
    x12 = _f64(x12).reshape(12)
    p12 = _f64(p12).reshape(12)
    it = _I64()
    t = lib().or_c2a_pair(kind, _ptr(x12), _ptr(p12), s, t_c, max_iter, C.byref(it))
    return t, it.value


def ccd_toi(sc, x, p, kind, pairs, s=0.1, t_c=1.0, max_iter=100000, method=0):
    """Per-pair step bounds; method 0 additive CCD, 1 closest-direction advancement."""
    sc_ = scene(sc)
    x, p = _f64(x), _f64(p)
    pairs = _i32(pairs).reshape(-1, 2)
    t = np.zeros(len(pairs))
    it = np.zeros(len(pairs), dtype=np.int64)
    lib().or_ccd_toi_m(sc_.ref, _ptr(x), _ptr(p), kind, _ptr(pairs), len(pairs), s, t_c, max_iter, int(method),
                       _ptr(t), _ptr(it))
    return t, it


def ccd_max_step(sc, q, dq, dhat, dx_off=None, s=0.1, t_max=1.0, max_iter=100000):
    sc_ = scene(sc)
    q, dq, dx_off = _f64(q), _f64(dq), _f64(dx_off)
    a = np.zeros(1)
    nc, ncap = _I64(), _I64()
    lib().or_ccd_max_step(sc_.ref, _ptr(q), _ptr(dq), _ptr(dx_off), dhat, s, t_max, max_iter,
                          _ptr(a), C.byref(nc), C.byref(ncap))
    return a[0], nc.value, ncap.value


# ---------------------------------------------------------------------------
# Workloads too large for the brute-force loops: the uniform-grid broad phase
# and the block-sparse reduction, run over contiguous slices of the queries
# or pairs on several host threads (ctypes releases the GIL during a call).
# Slices are merged in order, so the lists come out exactly as from one call.
# ---------------------------------------------------------------------------

def threads() -> int:
    """Host threads for the sliced oracle calls: the OMP_NUM_THREADS share
    if set, else every core."""
    n = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, n if n > 0 else (os.cpu_count() or 1))


def _slices(n: int, parts: int):
    parts = max(1, min(parts, n)) if n > 0 else 1
    b = np.linspace(0, n, parts + 1).astype(np.int64)
    return [(int(b[i]), int(b[i + 1])) for i in range(parts)]


def _pmap(fn, items, nthreads):
    if nthreads <= 1 or len(items) <= 1:
        return [fn(it) for it in items]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(nthreads) as ex:
        return list(ex.map(fn, items))


def candidates_grid(sc, x, dhat, x1=None, cell=0.0, nthreads=None):
    """The candidate set of candidates() (same pairs, same order), found
    through a uniform grid of the given cell edge (<= 0: twice the mean
    primitive box extent)."""
    s = scene(sc)
    x, x1 = _f64(x), _f64(x1)
    L = lib()
    g = L.or_grid_build(s.ref, _ptr(x), _ptr(x1), dhat, cell)
    nthreads = nthreads or threads()
    try:
        out = []
        for kind, nq in ((0, s.n_vert), (1, s.n_edge)):
            def run(r, kind=kind):
                a, b = r
                n = L.or_grid_pairs(g, kind, a, b, None, 0)
                buf = np.empty((max(n, 1), 2), dtype=np.int32)
                m = L.or_grid_pairs(g, kind, a, b, _ptr(buf), n)
                assert m == n
                return buf[:n]
            parts = _pmap(run, _slices(nq, 8 * nthreads), nthreads)
            out.append(np.concatenate(parts).astype(np.int32) if parts else np.zeros((0, 2), np.int32))
        return out[0], out[1]
    finally:
        L.or_grid_free(g)


def barrier_reduce_bsr(sc, q, pt, ee, dhat, kappa, flags, nthreads=None):
    """or_barrier_reduce with the reduced Hessian (flags HESS) as BSR.
    Returns dict(status, energy, grad, n_active, rowptr, col, blocks[nnzb,3,3])
    for one call; with several threads the pair lists are cut into slices,
    each reduced by one call, and the slices' energies, gradients and
    blocks are added in slice order."""
    s = scene(sc)
    q = _f64(q)
    pt = _i32(pt).reshape(-1, 2) if pt is not None else np.zeros((0, 2), np.int32)
    ee = _i32(ee).reshape(-1, 2) if ee is not None else np.zeros((0, 2), np.int32)
    nthreads = nthreads or threads()
    L = lib()
    nd = 3 * s.n_node
    if nthreads == 1:
        jobs = [(-1, 0, 0)]  # one call over both lists: the oracle's own order
    else:
        jobs = [(0, a, b) for a, b in _slices(len(pt), 4 * nthreads)] + \
               [(1, a, b) for a, b in _slices(len(ee), 4 * nthreads)]

    def run(job):
        kind, a, b = job
        lp = pt if kind == -1 else (pt[a:b] if kind == 0 else np.zeros((0, 2), np.int32))
        le = ee if kind == -1 else (ee[a:b] if kind == 1 else np.zeros((0, 2), np.int32))
        e = np.zeros(1)
        g = np.zeros(nd)
        na = _I64()
        st = C.c_int()
        h = L.or_barrier_reduce_bsr(s.ref, _ptr(q), _ptr(lp), len(lp), _ptr(le), len(le), dhat, kappa,
                                    int(flags), _ptr(e), _ptr(g), C.byref(na), C.byref(st))
        try:
            nnzb = L.or_bsr_nnzb(h)
            rp = np.zeros(s.n_node + 1, dtype=np.int32)
            col = np.zeros(max(nnzb, 1), dtype=np.int32)
            blk = np.zeros((max(nnzb, 1), 3, 3))
            L.or_bsr_copy(h, _ptr(rp), _ptr(col), _ptr(blk))
        finally:
            L.or_bsr_free(h)
        return st.value, e[0], g, na.value, rp, col[:nnzb], blk[:nnzb]

    parts = _pmap(run, jobs, nthreads)
    status = next((p[0] for p in parts if p[0] != OK), OK)
    energy = 0.0
    grad = np.zeros(nd)
    n_active = 0
    for p in parts:
        energy += p[1]
        grad += p[2]
        n_active += p[3]
    rowptr, col, blocks = _bsr_sum(s.n_node, [(p[4], p[5], p[6]) for p in parts])
    return {"status": status, "energy": energy, "grad": grad, "n_active": n_active,
            "rowptr": rowptr, "col": col, "blocks": blocks}


def _bsr_sum(n_rows, parts):
    """Sum of block-sparse matrices with sorted columns (union pattern)."""
    if len(parts) == 1:
        return parts[0]
    rows = np.concatenate([np.repeat(np.arange(n_rows), np.diff(rp)) for rp, _, _ in parts])
    cols = np.concatenate([c for _, c, _ in parts])
    blks = np.concatenate([b for _, _, b in parts]) if rows.size else np.zeros((0, 3, 3))
    key = rows.astype(np.int64) * max(n_rows, 1) + cols
    order = np.argsort(key, kind="stable")
    key, blks = key[order], blks[order]
    uk, start = np.unique(key, return_index=True)
    out = np.add.reduceat(blks, start, axis=0) if uk.size else np.zeros((0, 3, 3))
    ur = (uk // max(n_rows, 1)).astype(np.int64)
    rowptr = np.zeros(n_rows + 1, dtype=np.int32)
    np.add.at(rowptr, ur + 1, 1)
    return np.cumsum(rowptr).astype(np.int32), (uk % max(n_rows, 1)).astype(np.int32), out


def ccd_toi_threads(sc, x, p, kind, pairs, s=0.1, t_c=1.0, max_iter=100000, nthreads=None, method=0):
    """ccd_toi over slices of the pairs on several threads (same values)."""
    pairs = _i32(pairs).reshape(-1, 2)
    nthreads = nthreads or threads()
    parts = _pmap(lambda r: ccd_toi(sc, x, p, kind, pairs[r[0]:r[1]], s=s, t_c=t_c, max_iter=max_iter,
                                    method=method),
                  _slices(len(pairs), 8 * nthreads), nthreads)
    if not parts:
        return np.zeros(0), np.zeros(0, dtype=np.int64)
    return np.concatenate([a for a, _ in parts]), np.concatenate([b for _, b in parts])


def narrow(sc, x, kind, pairs, dhat, nthreads=None):
    """(type int32[n], d^2 f64[n], active bool[n]) of a pair list."""
    s = scene(sc)
    x = _f64(x)
    pairs = _i32(pairs).reshape(-1, 2)
    n = len(pairs)
    ty = np.zeros(n, dtype=np.int32)
    s2 = np.zeros(n)
    act = np.zeros(n, dtype=np.uint8)
    L = lib()

    def run(r):
        a, b = r
        L.or_narrow(s.ref, _ptr(x), kind, _ptr(pairs[a:b]), b - a, dhat, _ptr(ty[a:]), _ptr(s2[a:]),
                    _ptr(act[a:]))
    _pmap(run, _slices(n, 8 * (nthreads or threads())), nthreads or threads())
    return ty, s2, act.astype(bool)


# ---------------------------------------------------------------------------
# Lagged friction (lag record: lambda, beta[4], normal[3], G x^n[3])
# ---------------------------------------------------------------------------
LAG = 11


def friction_f(y, epsvh):
    """(f0, f1, f1') at y."""
    out = np.zeros(3)
    lib().or_friction_f(float(y), float(epsvh), _ptr(out[0:]), _ptr(out[1:]), _ptr(out[2:]))
    return out[0], out[1], out[2]


def friction_lag(kind, x12, dhat, kappa, rest12=None, flags=0):
    x12 = _f64(x12).reshape(12)
    r12 = None if rest12 is None else _f64(rest12).reshape(12)
    lag = np.zeros(LAG)
    st = lib().or_friction_lag_f(kind, _ptr(x12), _ptr(r12), dhat, kappa, flags, _ptr(lag))
    return st, lag


def friction_pair(x12, lag, mu, epsvh):
    """(energy, g[12], H[12, 12]) of one lagged pair."""
    x12 = _f64(x12).reshape(12)
    lag = _f64(lag).reshape(LAG)
    e = np.zeros(1)
    g = np.zeros(12)
    H = np.zeros((12, 12))
    lib().or_friction_pair(_ptr(x12), _ptr(lag), mu, epsvh, _ptr(e), _ptr(g), _ptr(H))
    return e[0], g, H


def friction_lag_list(sc, q_n, kind, pairs, dhat, kappa, flags=0):
    s = scene(sc)
    q_n = _f64(q_n)
    pairs = _i32(pairs).reshape(-1, 2)
    lag = np.zeros((len(pairs), LAG))
    st = lib().or_friction_lag_list(s.ref, _ptr(q_n), kind, _ptr(pairs), len(pairs), dhat, kappa, int(flags),
                                    _ptr(lag))
    return st, lag


def friction_reduce(sc, q, pt, lag_pt, ee, lag_ee, mu, epsvh, hess=True):
    """dict(energy, grad, hess (dense or None)) of the lagged friction."""
    s = scene(sc)
    q = _f64(q)
    pt = _i32(pt).reshape(-1, 2)
    ee = _i32(ee).reshape(-1, 2)
    lag_pt = _f64(lag_pt).reshape(-1, LAG)
    lag_ee = _f64(lag_ee).reshape(-1, LAG)
    nd = 3 * s.n_node
    e = np.zeros(1)
    g = np.zeros(nd)
    H = np.zeros((nd, nd)) if hess else None
    lib().or_friction_reduce(s.ref, _ptr(q), _ptr(pt), len(pt), _ptr(lag_pt), _ptr(ee), len(ee), _ptr(lag_ee),
                             mu, epsvh, _ptr(e), _ptr(g), _ptr(H))
    return {"energy": e[0], "grad": g, "hess": H}
