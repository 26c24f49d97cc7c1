"""ctypes binding of libeipc.so with torch tensors for device memory.

Names follow the C ABI (``eipc_<name>`` -> ``<name>``).  All tensors passed
in must live on the context's device; they are made contiguous and cast to
the ABI's types (float64 / int32) before the call.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

ENERGY, GRAD, HESS, PROJECT, MOLLIFY, SQDIST, PROJECT_REDUCED = 1, 2, 4, 8, 16, 32, 64
OK, ERR_ARG, ERR_CAPACITY, ERR_INTERSECTING, ERR_DEGENERATE, ERR_NONFINITE, ERR_HIP = 0, -1, -2, -3, -4, -5, -6
WARN_CCD_CAPPED = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("EIPC_LIBRARY", os.path.join(_HERE, "libeipc.so"))
_P, _D, _I32, _I64, _U32 = C.c_void_p, C.c_double, C.c_int32, C.c_int64, C.c_uint32


def lib_path() -> str:
    return _LIB_PATH


class EipcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"eipc status {status}: {msg}")
        self.status = status


class _Scene(C.Structure):
    _fields_ = [("n_vert", _I32), ("n_node", _I32), ("n_face", _I32), ("n_edge", _I32),
                ("faces", _P), ("edges", _P), ("W_rowptr", _P), ("W_col", _P), ("W_val", _P),
                ("x_off", _P), ("x_rest", _P), ("n_scene", _I32), ("vert_scene", _P)]


class _Bsr(C.Structure):
    _fields_ = [("n_rows", _I32), ("nnzb", _I64), ("rowptr", _P), ("col", _P), ("blocks", _P)]


class Plan(C.Structure):
    """Capacities of a planned contact step (eipc_plan)."""
    _fields_ = [("cand_pt", _I64), ("cand_ee", _I64), ("swept_pt", _I64), ("swept_ee", _I64),
                ("act_pt", _I64), ("act_ee", _I64),
                ("ent", _I64 * 4), ("qent", _I64 * 4), ("buckets", _I64 * 4), ("hess_blocks", _I64),
                ("nnzb", _I64)]

    def as_dict(self) -> dict:
        return {"cand_pt": self.cand_pt, "cand_ee": self.cand_ee, "swept_pt": self.swept_pt,
                "swept_ee": self.swept_ee, "act_pt": self.act_pt, "act_ee": self.act_ee,
                "ent": list(self.ent), "qent": list(self.qent), "buckets": list(self.buckets),
                "hess_blocks": self.hess_blocks, "nnzb": self.nnzb}


_lib = None
_hip = None


def _load():
    global _lib, _hip
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() "
                          "or python paper_2409_16385_amd/_build.py")
    L = C.CDLL(_LIB_PATH)
    sig = {
        "eipc_create": (_I32, [C.POINTER(_P), _I32, C.c_size_t]),
        "eipc_scratch_bytes": (_I32, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
        "eipc_destroy": (None, [_P]),
        "eipc_last_error": (C.c_char_p, [_P]),
        "eipc_status_string": (C.c_char_p, [_I32]),
        "eipc_sync_status": (_I32, [_P, _P]),
        "eipc_embed": (_I32, [_P, _P, _P, _P, _P, _P]),
        "eipc_build_candidates": (_I32, [_P, _P, _P, _D, _P, _I64, _P, _I64, _P, _P, _P]),
        "eipc_barrier_reduce": (_I32, [_P, _P, _P, _P, _I64, _P, _I64, _D, _D, _U32, _P, _P, _P, _P, _P, _P]),
        "eipc_ccd_max_step": (_I32, [_P, _P, _P, _P, _P, _D, _D, _D, _I64, _P, _P, _P]),
        "eipc_barrier_hvp": (_I32, [_P, _P, _P, _P, _I64, _P, _I64, _D, _D, _U32, _P, _P, _P, _P, _P]),
        "eipc_narrow_phase": (_I32, [_P, _P, _P, _P, _I64, _P, _I64, _D, _P, _P, _P, _P, _P, _P, _P]),
        "eipc_pair_eval": (_I32, [_P, _P, _P, _I32, _P, _I64, _D, _D, _U32, _P, _P, _P, _P, _P, _P]),
        "eipc_ccd_candidates": (_I32, [_P, _P, _P, _P, _P, _D, _P, _I64, _P, _I64, _P, _P, _P]),
        "eipc_ccd_toi": (_I32, [_P, _P, _P, _P, _P, _I32, _P, _I64, _D, _D, _I64, _P, _P, _P]),
        "eipc_fp64_selftest": (_I32, [_P, _P, _P, _P, _P, _I64, _P]),
        "eipc_profile": (_I32, [_P, _I32]),
        "eipc_cholesky": (_I32, [_P, _P, _I64, _I64, _P, _P]),
        "eipc_cholesky_solve": (_I32, [_P, _P, _I64, _I64, _P, _I64, _P]),
        "eipc_profile_read": (_I32, [_P, C.c_char_p, _P, _P, _I32]),
        "eipc_plan_step": (_I32, [_P, _P, _P, _P, _P, _D, _D, _I32, _P, _P]),
        "eipc_contact_step": (_I32, [_P, _P, _P, _P, _P, _P, _D, _D, _U32, _D, _D, _I64, _P, _P, _P, _P, _P, _P]),
        "eipc_set_tuning": (_I32, [_P, _D, _P, _I32]),
        "eipc_set_ccd_method": (_I32, [_P, _I32]),
        "eipc_step_pairs": (_I32, [_P, _I32, _P, _I64, _P, _P]),
        "eipc_friction_lag": (_I32, [_P, _P, _P, _P, _I64, _P, _I64, _D, _D, _U32, _P, _P, _P]),
        "eipc_friction_reduce": (_I32, [_P, _P, _P, _P, _I64, _P, _P, _I64, _P, _D, _D, _U32, _P, _P, _P, _P, _P]),
        "eipc_barrier_hvp_noalloc": (_I32, [_P, _P, _P, _P, _I64, _P, _I64, _D, _D, _U32, _P, _P, _P, _P, _P]),
        "eipc_reduced_mass": (_I32, [_P, _I32, _I64, _P, _P, _D, _D, _P, _I64, _P, _P]),
        "eipc_elastic": (_I32, [_P, _I32, _I32, _P, _P, _P, _D, _D, _I32, _P, _D, _P, _P, _P, _I64, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _hiprt():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.restype = C.c_int
        _hip.hipMemcpyAsync.argtypes = [_P, _P, C.c_size_t, C.c_int, _P]
    return _hip


def _ptr(t):
    return None if t is None else t.data_ptr()


class Context:
    """One eipc context on one GPU (owns the library's scratch memory).
    reserve_bytes > 0 reserves all scratch at creation (no allocation in
    any later call; a call that needs more reports ERR_CAPACITY)."""

    def __init__(self, device: int | torch.device | None = None, reserve_bytes: int = 0):
        L = _load()
        if not torch.cuda.is_available():
            raise RuntimeError("the contact stage needs a ROCm GPU (torch.cuda.is_available() is False)")
        if device is None:
            device = torch.cuda.current_device()
        if isinstance(device, torch.device):
            device = device.index if device.index is not None else torch.cuda.current_device()
        self.device = int(device)
        self.torch_device = torch.device("cuda", self.device)
        h = _P()
        st = L.eipc_create(C.byref(h), self.device, int(reserve_bytes))
        if st != OK:
            raise EipcError(st, "eipc_create failed")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _load().eipc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.torch_device).cuda_stream)

    def check(self, st: int, allow=(OK,)):
        if st in allow:
            return st
        msg = _load().eipc_last_error(self._h).decode(errors="replace")
        raise EipcError(st, msg or _load().eipc_status_string(st).decode())

    def scratch_bytes(self) -> tuple[int, int]:
        """(reserved, high water): the arena size (0 in grow mode) and the
        most scratch one call has used (grow mode: all buffers held)."""
        r, h = C.c_size_t(), C.c_size_t()
        self.check(_load().eipc_scratch_bytes(self._h, C.byref(r), C.byref(h)))
        return r.value, h.value

    def sync_status(self) -> int:
        return _load().eipc_sync_status(self._h, self.stream())

    KERNELS = ("embed", "query_count_pt", "query_count_ee", "query_write_pt", "query_write_ee", "narrow_pt",
               "narrow_ee", "barrier_pt", "barrier_ee", "ccd_pt", "ccd_ee", "hvp_pt", "hvp_ee", "expand_pt",
               "expand_ee", "ccd_long_pt", "ccd_long_ee")

    def profile(self, enable: bool = True, serial: bool = False):
        """Per-kernel HIP-event timing inside the library (on the launch stream);
        serial: the planned step runs its two chains one after the other on
        the caller's stream while timing, so each kernel is timed alone."""
        self.check(_load().eipc_profile(self._h, (2 if serial else 1) if enable else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """{kernel: (total_ms, launches)} since the last reset."""
        out = {}
        for i, k in enumerate(self.KERNELS):
            ms, n = _D(), _I64()
            last = reset and i == len(self.KERNELS) - 1
            self.check(_load().eipc_profile_read(self._h, k.encode(), C.byref(ms), C.byref(n), 1 if last else 0))
            out[k] = (ms.value, n.value)
        return out


def _f64(t, dev):
    return None if t is None else torch.as_tensor(t, dtype=torch.float64, device=dev).contiguous()


def _i32(t, dev):
    return None if t is None else torch.as_tensor(t, dtype=torch.int32, device=dev).contiguous()


class Scene:
    """Device copy of a scene: faces, edges, W (CSR), x_off, x_rest; for a
    batch also n_scene and the scene id of every vertex."""

    def __init__(self, ctx: Context, faces, edges, W_rowptr, W_col, W_val, n_node, x_off=None, x_rest=None,
                 n_scene: int = 1, vert_scene=None):
        dev = ctx.torch_device
        self.ctx = ctx
        self.faces = _i32(faces, dev).reshape(-1, 3)
        self.edges = _i32(edges, dev).reshape(-1, 2)
        self.W_rowptr = _i32(W_rowptr, dev)
        self.W_col = _i32(W_col, dev)
        self.W_val = _f64(W_val, dev)
        self.x_off = None if x_off is None else _f64(x_off, dev).reshape(-1, 3)
        self.x_rest = None if x_rest is None else _f64(x_rest, dev).reshape(-1, 3)
        self.n_vert = self.W_rowptr.numel() - 1
        self.n_node = int(n_node)
        self.n_face = self.faces.shape[0]
        self.n_edge = self.edges.shape[0]
        self.n_scene = int(n_scene)
        self.vert_scene = None if vert_scene is None else _i32(vert_scene, dev)
        self._s = _Scene(self.n_vert, self.n_node, self.n_face, self.n_edge, _ptr(self.faces), _ptr(self.edges),
                         _ptr(self.W_rowptr), _ptr(self.W_col), _ptr(self.W_val), _ptr(self.x_off),
                         _ptr(self.x_rest), self.n_scene, _ptr(self.vert_scene))

    @classmethod
    def from_host(cls, ctx: Context, sc):
        """From a scenes.Scene (numpy arrays)."""
        return cls(ctx, sc.faces, sc.edges, sc.W_rowptr, sc.W_col, sc.W_val, sc.n_node, sc.x_off, sc.x_rest)

    @property
    def ref(self):
        return C.byref(self._s)


def embed(ctx: Context, sc: Scene, q, off="scene"):
    """x = W q + off, AoS [n_vert, 3] (off defaults to the scene's x_off)."""
    dev = ctx.torch_device
    q = _f64(q, dev)
    off = sc.x_off if isinstance(off, str) else (None if off is None else _f64(off, dev))
    x = torch.empty((sc.n_vert, 3), dtype=torch.float64, device=dev)
    ctx.check(_load().eipc_embed(ctx.handle, sc.ref, _ptr(q), _ptr(off), _ptr(x), ctx.stream()))
    return x


def build_candidates(ctx: Context, sc: Scene, q, dhat: float, cap: tuple[int, int] | None = None):
    """Candidate PT and EE pairs as int32 [n, 2] tensors (sorted)."""
    dev = ctx.torch_device
    q = _f64(q, dev)
    cpt, cee = cap if cap is not None else getattr(sc, "_cand_cap", (1024, 1024))
    L = _load()
    for _ in range(3):
        pt = torch.empty((max(cpt, 1), 2), dtype=torch.int32, device=dev)
        ee = torch.empty((max(cee, 1), 2), dtype=torch.int32, device=dev)
        npt, nee = _I64(), _I64()
        st = L.eipc_build_candidates(ctx.handle, sc.ref, _ptr(q), float(dhat), _ptr(pt), cpt, _ptr(ee), cee,
                                     C.byref(npt), C.byref(nee), ctx.stream())
        if st == ERR_CAPACITY:
            cpt, cee = max(cpt, int(npt.value * 1.25) + 16), max(cee, int(nee.value * 1.25) + 16)
            continue
        ctx.check(st)
        sc._cand_cap = (max(cpt, npt.value), max(cee, nee.value))
        return pt[:npt.value], ee[:nee.value]
    raise EipcError(ERR_CAPACITY, "candidate capacity retries exhausted")


def bsr_to_dense(rowptr, col, blocks, n_node):
    """Dense [3n, 3n] from a BSR triple (host-side helper for checks)."""
    rowptr = torch.as_tensor(rowptr).cpu().numpy()
    col = torch.as_tensor(col).cpu().numpy()
    blocks = torch.as_tensor(blocks).cpu().numpy().reshape(-1, 3, 3)
    H = np.zeros((3 * n_node, 3 * n_node))
    for i in range(n_node):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = col[p]
            H[3 * i:3 * i + 3, 3 * j:3 * j + 3] = blocks[p]
    return H


def barrier_reduce(ctx: Context, sc: Scene, q, pt, ee, dhat: float, kappa: float,
                   flags: int = ENERGY | GRAD | HESS | PROJECT, hess: str | None = "bsr",
                   count: bool = True):
    """Energy, reduced gradient and reduced Hessian ('bsr', 'dense' or None).

    Returns a dict: energy (tensor [n_scene]), grad (tensor [3 n_node] or None),
    hess (dense tensor, or (rowptr, col, blocks) tensors for BSR, or None),
    n_active (int or None)."""
    dev = ctx.torch_device
    q = _f64(q, dev)
    pt = _i32(pt, dev).reshape(-1, 2)
    ee = _i32(ee, dev).reshape(-1, 2)
    energy = torch.empty(max(sc.n_scene, 1), dtype=torch.float64, device=dev) if flags & ENERGY else None
    grad = torch.empty(3 * sc.n_node, dtype=torch.float64, device=dev) if flags & GRAD else None
    dense = None
    bsr = None
    if flags & HESS and hess == "dense":
        dense = torch.empty((3 * sc.n_node, 3 * sc.n_node), dtype=torch.float64, device=dev)
    elif flags & HESS and hess == "bsr":
        bsr = _Bsr()
    na = _I64()
    st = _load().eipc_barrier_reduce(ctx.handle, sc.ref, _ptr(q), _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0],
                                     float(dhat), float(kappa), int(flags), _ptr(energy), _ptr(grad), _ptr(dense),
                                     None if bsr is None else C.byref(bsr), C.byref(na) if count else None,
                                     ctx.stream())
    ctx.check(st)
    H = dense
    if bsr is not None:
        H = _copy_bsr(ctx, bsr)
    return {"energy": energy, "grad": grad, "hess": H, "n_active": na.value if count else None}


def _copy_bsr(ctx: Context, b: _Bsr):
    dev = ctx.torch_device
    rowptr = torch.empty(b.n_rows + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(b.nnzb, 1), dtype=torch.int32, device=dev)
    blocks = torch.empty((max(b.nnzb, 1), 3, 3), dtype=torch.float64, device=dev)
    hip = _hiprt()
    s = ctx.stream()
    for dst, src, nbytes in ((rowptr, b.rowptr, 4 * (b.n_rows + 1)), (col, b.col, 4 * b.nnzb),
                             (blocks, b.blocks, 72 * b.nnzb)):
        if nbytes:
            err = hip.hipMemcpyAsync(_P(dst.data_ptr()), _P(src), nbytes, 3, s)
            if err != 0:
                raise EipcError(ERR_HIP, f"hipMemcpyAsync failed ({err})")
    return rowptr, col[:b.nnzb], blocks[:b.nnzb]


def ccd_max_step(ctx: Context, sc: Scene, q, dq, dhat: float, dx_off=None, s: float = 0.1, t_max: float = 1.0,
                 max_iter: int = 100000):
    """Returns (alpha, n_candidates, capped); alpha is a float for one
    scene and a float64 array of n_scene values for a batch."""
    dev = ctx.torch_device
    q, dq, dx_off = _f64(q, dev), _f64(dq, dev), _f64(dx_off, dev)
    a = (_D * max(sc.n_scene, 1))()
    nc = _I64()
    st = _load().eipc_ccd_max_step(ctx.handle, sc.ref, _ptr(q), _ptr(dq), _ptr(dx_off), float(dhat), float(s),
                                   float(t_max), int(max_iter), a, C.byref(nc), ctx.stream())
    ctx.check(st, allow=(OK, WARN_CCD_CAPPED))
    alpha = a[0] if sc.n_scene <= 1 else np.array(a[:], dtype=np.float64)
    return alpha, nc.value, st == WARN_CCD_CAPPED


def barrier_hvp(ctx: Context, sc: Scene, q, pt, ee, dhat: float, kappa: float, flags: int, v, v_off=None,
                want_off: bool = False, noalloc: bool = False):
    """Hessian-vector product; noalloc: the library's no-allocation entry
    point (fixed scratch array; inputs and outputs still come from torch)."""
    dev = ctx.torch_device
    q, v, v_off = _f64(q, dev), _f64(v, dev), _f64(v_off, dev)
    pt = _i32(pt, dev).reshape(-1, 2)
    ee = _i32(ee, dev).reshape(-1, 2)
    out = torch.empty(3 * sc.n_node, dtype=torch.float64, device=dev)
    out_off = torch.empty((sc.n_vert, 3), dtype=torch.float64, device=dev) if want_off else None
    fn = _load().eipc_barrier_hvp_noalloc if noalloc else _load().eipc_barrier_hvp
    st = fn(ctx.handle, sc.ref, _ptr(q), _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0],
                                  float(dhat), float(kappa), int(flags), _ptr(v), _ptr(v_off), _ptr(out),
                                  _ptr(out_off), ctx.stream())
    ctx.check(st)
    return (out, out_off) if want_off else out


def narrow_phase(ctx: Context, sc: Scene, q, pt, ee, dhat: float):
    """Active pairs: (act_pt, type_pt, act_ee, type_ee) index/type tensors."""
    dev = ctx.torch_device
    q = _f64(q, dev)
    pt = _i32(pt, dev).reshape(-1, 2)
    ee = _i32(ee, dev).reshape(-1, 2)
    ap = torch.empty(max(pt.shape[0], 1), dtype=torch.int32, device=dev)
    tp = torch.empty_like(ap)
    ae = torch.empty(max(ee.shape[0], 1), dtype=torch.int32, device=dev)
    te = torch.empty_like(ae)
    npt, nee = _I64(), _I64()
    st = _load().eipc_narrow_phase(ctx.handle, sc.ref, _ptr(q), _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0],
                                   float(dhat), _ptr(ap), _ptr(tp), C.byref(npt), _ptr(ae), _ptr(te), C.byref(nee),
                                   ctx.stream())
    ctx.check(st)
    return ap[:npt.value], tp[:npt.value], ae[:nee.value], te[:nee.value]


def pair_eval(ctx: Context, sc: Scene, q, kind: int, pairs, dhat: float, kappa: float, flags: int = 0):
    """Per-pair (type, s, e, g[n,12], H[n,12,12])."""
    dev = ctx.torch_device
    q = _f64(q, dev)
    pairs = _i32(pairs, dev).reshape(-1, 2)
    n = pairs.shape[0]
    ty = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    s2 = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    e = torch.empty_like(s2)
    g = torch.empty((max(n, 1), 12), dtype=torch.float64, device=dev)
    H = torch.empty((max(n, 1), 12, 12), dtype=torch.float64, device=dev)
    st = _load().eipc_pair_eval(ctx.handle, sc.ref, _ptr(q), int(kind), _ptr(pairs), n, float(dhat), float(kappa),
                                int(flags), _ptr(ty), _ptr(s2), _ptr(e), _ptr(g), _ptr(H), ctx.stream())
    ctx.check(st)
    return ty[:n], s2[:n], e[:n], g[:n], H[:n]


def ccd_candidates(ctx: Context, sc: Scene, q, dq, dhat: float, dx_off=None):
    dev = ctx.torch_device
    q, dq, dx_off = _f64(q, dev), _f64(dq, dev), _f64(dx_off, dev)
    cpt, cee = getattr(sc, "_ccd_cap", (4096, 4096))
    L = _load()
    for _ in range(3):
        pt = torch.empty((max(cpt, 1), 2), dtype=torch.int32, device=dev)
        ee = torch.empty((max(cee, 1), 2), dtype=torch.int32, device=dev)
        npt, nee = _I64(), _I64()
        st = L.eipc_ccd_candidates(ctx.handle, sc.ref, _ptr(q), _ptr(dq), _ptr(dx_off), float(dhat), _ptr(pt), cpt,
                                   _ptr(ee), cee, C.byref(npt), C.byref(nee), ctx.stream())
        if st == ERR_CAPACITY:
            cpt, cee = max(cpt, int(npt.value * 1.25) + 16), max(cee, int(nee.value * 1.25) + 16)
            continue
        ctx.check(st)
        sc._ccd_cap = (max(cpt, npt.value), max(cee, nee.value))
        return pt[:npt.value], ee[:nee.value]
    raise EipcError(ERR_CAPACITY, "swept candidate capacity retries exhausted")


def ccd_toi(ctx: Context, sc: Scene, q, dq, kind: int, pairs, dx_off=None, s: float = 0.1, t_max: float = 1.0,
            max_iter: int = 100000):
    dev = ctx.torch_device
    q, dq, dx_off = _f64(q, dev), _f64(dq, dev), _f64(dx_off, dev)
    pairs = _i32(pairs, dev).reshape(-1, 2)
    n = pairs.shape[0]
    t = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    it = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    st = _load().eipc_ccd_toi(ctx.handle, sc.ref, _ptr(q), _ptr(dq), _ptr(dx_off), int(kind), _ptr(pairs), n,
                              float(s), float(t_max), int(max_iter), _ptr(t), _ptr(it), ctx.stream())
    ctx.check(st)
    return t[:n], it[:n]


def cholesky(ctx: Context, A: torch.Tensor):
    """In-place Cholesky of a square float64 device matrix (lower factor
    overwrites the lower triangle).  Returns info (0 = success)."""
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("A must be a contiguous square float64 tensor")
    info = _I64()
    ctx.check(_load().eipc_cholesky(ctx.handle, _ptr(A), A.shape[0], A.shape[1], C.byref(info), ctx.stream()))
    return info.value


def cholesky_solve(ctx: Context, L: torch.Tensor, B: torch.Tensor):
    """Solve (L L^T) X = B in place; B is [n] or [n, nrhs] float64 (contiguous)."""
    n = L.shape[0]
    Bm = B.reshape(n, -1)
    if not Bm.is_contiguous():
        raise ValueError("B must be contiguous")
    ctx.check(_load().eipc_cholesky_solve(ctx.handle, _ptr(L), n, L.shape[1], _ptr(Bm), Bm.shape[1], ctx.stream()))
    return B


ELASTIC_LINEAR = 0
ELASTIC_COROTATIONAL = 1


def reduced_mass(ctx: Context, n_node: int, sample_nodes: torch.Tensor, sample_w: torch.Tensor,
                 sample_mass: float, gravity: float):
    """Reduced mass M [3 n_node, 3 n_node] and gravity f [3 n_node] from
    interior samples (int32 [n_s, 4] tet nodes, float64 [n_s, 4] weights)."""
    dev = ctx.torch_device
    n3 = 3 * n_node
    M = torch.zeros((n3, n3), dtype=torch.float64, device=dev)
    f = torch.zeros(n3, dtype=torch.float64, device=dev)
    sn = sample_nodes.to(device=dev, dtype=torch.int32).contiguous()
    sw = sample_w.to(device=dev, dtype=torch.float64).contiguous()
    ctx.check(_load().eipc_reduced_mass(ctx.handle, n_node, sn.shape[0], _ptr(sn), _ptr(sw), float(sample_mass),
                                        float(gravity), _ptr(M), n3, _ptr(f), ctx.stream()))
    return M, f


def elastic(ctx: Context, n_node: int, tets: torch.Tensor, rest: torch.Tensor, vol: torch.Tensor, young: float,
            poisson: float, model: int, q: torch.Tensor, scale: float = 1.0, energy: torch.Tensor | None = None,
            grad: torch.Tensor | None = None, hess: torch.Tensor | None = None):
    """Adds scale * (elastic energy, gradient, Newton matrix) of the coarse
    tets at q into the given float64 device tensors (each optional)."""
    lda = hess.shape[1] if hess is not None else 3 * n_node
    for t in (energy, grad, hess):
        if t is not None and (t.dtype != torch.float64 or not t.is_contiguous()):
            raise ValueError("outputs must be contiguous float64 tensors")
    ctx.check(_load().eipc_elastic(ctx.handle, n_node, tets.shape[0], _ptr(tets), _ptr(rest), _ptr(vol),
                                   float(young), float(poisson), int(model), _ptr(q), float(scale),
                                   _ptr(energy) if energy is not None else None,
                                   _ptr(grad) if grad is not None else None,
                                   _ptr(hess) if hess is not None else None, lda, ctx.stream()))


def fp64_selftest(ctx: Context, a, b):
    dev = ctx.torch_device
    a, b = _f64(a, dev), _f64(b, dev)
    sq = torch.empty_like(a)
    dv = torch.empty_like(a)
    ctx.check(_load().eipc_fp64_selftest(ctx.handle, _ptr(a), _ptr(b), _ptr(sq), _ptr(dv), a.numel(), ctx.stream()))
    return sq, dv


def set_tuning(ctx: Context, cell_scale: float, wg_per_cu=(0, 0, 0, 0), query_cells: int = -1):
    """Broad-phase cell scale, workgroups per CU of the grid-stride kernels
    (pair terms, expansion, narrow phase, CCD; 0 keeps a value) and the
    unsorted broad phase's work split, mode_PT + 4 * mode_EE with modes 0
    (thread per query), 1 (thread per query cell), 2 (wavefront per query
    cell), 3 (bucket join); -1 keeps it."""
    w = (_I32 * 4)(*[int(v) for v in wg_per_cu])
    ctx.check(_load().eipc_set_tuning(ctx.handle, float(cell_scale), w, int(query_cells)))


CCD_ADDITIVE, CCD_CLOSEST_DIRECTION = 0, 1


def set_ccd_method(ctx: Context, method: int):
    """The context's per-pair CCD step bound: CCD_ADDITIVE (default) or
    CCD_CLOSEST_DIRECTION (advancement along the closest direction)."""
    ctx.check(_load().eipc_set_ccd_method(ctx.handle, int(method)))


def plan_step(ctx: Context, sc: Scene, q, dhat: float, dq=None, dx_off=None, margin: float = 1.5,
              with_hess: bool = True) -> Plan:
    """Capacities for contact_step measured at (q, dq) times `margin`;
    reserves the context's scratch (synchronizes)."""
    dev = ctx.torch_device
    q, dq, dx_off = _f64(q, dev), _f64(dq, dev), _f64(dx_off, dev)
    p = Plan()
    ctx.check(_load().eipc_plan_step(ctx.handle, sc.ref, _ptr(q), _ptr(dq), _ptr(dx_off), float(dhat),
                                     float(margin), 1 if with_hess else 0, C.byref(p), ctx.stream()))
    return p


class StepOut:
    """Output tensors of contact_step (allocated once, reused by replays)."""

    def __init__(self, ctx: Context, sc: Scene, plan: Plan, flags: int, with_alpha: bool = True):
        dev = ctx.torch_device
        ns = max(sc.n_scene, 1)
        self.energy = torch.zeros(ns, dtype=torch.float64, device=dev) if flags & ENERGY else None
        self.grad = torch.zeros(3 * sc.n_node, dtype=torch.float64, device=dev) if flags & GRAD else None
        self.alpha = torch.zeros(ns, dtype=torch.float64, device=dev) if with_alpha else None
        self.counts = torch.zeros(5, dtype=torch.int64, device=dev)
        self.bsr = _Bsr() if (flags & HESS and plan.hess_blocks > 0) else None

    def hess(self, ctx: Context):
        """BSR of the last step as (rowptr, col, blocks) copies (synchronizes)."""
        if self.bsr is None or not self.bsr.rowptr:
            return None
        b = _Bsr(self.bsr.n_rows, 0, self.bsr.rowptr, self.bsr.col, self.bsr.blocks)
        rp = torch.empty(b.n_rows + 1, dtype=torch.int32, device=ctx.torch_device)
        err = _hiprt().hipMemcpyAsync(_P(rp.data_ptr()), _P(b.rowptr), 4 * (b.n_rows + 1), 3, ctx.stream())
        if err != 0:
            raise EipcError(ERR_HIP, f"hipMemcpyAsync failed ({err})")
        b.nnzb = int(rp[-1].item())
        return _copy_bsr(ctx, b)


def contact_step(ctx: Context, sc: Scene, plan: Plan, q, dhat: float, kappa: float, out: StepOut, dq=None,
                 dx_off=None, flags: int = ENERGY | GRAD | HESS | PROJECT, s: float = 0.1, t_max: float = 1.0,
                 max_iter: int = 100000):
    """Enqueue one planned contact step (no synchronization, no allocation:
    capturable in a graph).  q, dq, dx_off must be float64 device tensors
    whose storage stays fixed across replays.  Errors are read later with
    ctx.sync_status()."""
    st = _load().eipc_contact_step(ctx.handle, sc.ref, C.byref(plan), _ptr(q), _ptr(dq), _ptr(dx_off),
                                   float(dhat), float(kappa), int(flags), float(s), float(t_max), int(max_iter),
                                   _ptr(out.energy), _ptr(out.grad),
                                   None if out.bsr is None else C.byref(out.bsr), _ptr(out.alpha),
                                   _ptr(out.counts), ctx.stream())
    ctx.check(st)


def step_pairs(ctx: Context, which: int):
    """Pair list of the last contact_step as an int32 [n, 2] device tensor:
    which = 0 / 1 the PT / EE pairs it tested (swept candidates when it
    computed alpha), 2 / 3 its active PT / EE pairs (synchronizes)."""
    L = _load()
    n = _I64()
    ctx.check(L.eipc_step_pairs(ctx.handle, int(which), None, 0, C.byref(n), ctx.stream()),
              allow=(OK, ERR_CAPACITY))
    out = torch.empty((max(n.value, 1), 2), dtype=torch.int32, device=ctx.torch_device)
    ctx.check(L.eipc_step_pairs(ctx.handle, int(which), _ptr(out), n.value, C.byref(n), ctx.stream()))
    return out[:n.value]


FRICTION_LAG = 11


def friction_lag(ctx: Context, sc: Scene, q_n, pt, ee, dhat: float, kappa: float, flags: int = 0):
    """Lag records (device [n, 11] tensors for the PT and EE pairs) of the
    friction potential at the previous step's q_n (asynchronous)."""
    dev = ctx.torch_device
    q_n = _f64(q_n, dev)
    pt = _i32(pt, dev).reshape(-1, 2)
    ee = _i32(ee, dev).reshape(-1, 2)
    lpt = torch.empty((pt.shape[0], FRICTION_LAG), dtype=torch.float64, device=dev)
    lee = torch.empty((ee.shape[0], FRICTION_LAG), dtype=torch.float64, device=dev)
    ctx.check(_load().eipc_friction_lag(ctx.handle, sc.ref, _ptr(q_n), _ptr(pt), pt.shape[0], _ptr(ee), ee.shape[0],
                                        float(dhat), float(kappa), int(flags), _ptr(lpt), _ptr(lee), ctx.stream()))
    return lpt, lee


def friction_reduce(ctx: Context, sc: Scene, q, pt, lag_pt, ee, lag_ee, mu: float, eps_h: float,
                    flags: int = ENERGY | GRAD | HESS, hess: str | None = "bsr"):
    """Lagged friction energy, reduced gradient and reduced Hessian ('bsr',
    'dense' or None) at q; returns dict(energy, grad, hess)."""
    dev = ctx.torch_device
    q = _f64(q, dev)
    pt = _i32(pt, dev).reshape(-1, 2)
    ee = _i32(ee, dev).reshape(-1, 2)
    energy = torch.empty(1, dtype=torch.float64, device=dev) if flags & ENERGY else None
    grad = torch.empty(3 * sc.n_node, dtype=torch.float64, device=dev) if flags & GRAD else None
    dense = None
    bsr = None
    if flags & HESS and hess == "dense":
        dense = torch.empty((3 * sc.n_node, 3 * sc.n_node), dtype=torch.float64, device=dev)
    elif flags & HESS and hess == "bsr":
        bsr = _Bsr()
    st = _load().eipc_friction_reduce(ctx.handle, sc.ref, _ptr(q), _ptr(pt), pt.shape[0], _ptr(lag_pt), _ptr(ee),
                                      ee.shape[0], _ptr(lag_ee), float(mu), float(eps_h), int(flags), _ptr(energy),
                                      _ptr(grad), _ptr(dense), None if bsr is None else C.byref(bsr), ctx.stream())
    ctx.check(st)
    H = dense
    if bsr is not None:
        H = _copy_bsr(ctx, bsr)
    return {"energy": energy, "grad": grad, "hess": H}
