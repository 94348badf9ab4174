"""Thin ctypes binding of libhisq (include/hisq.h), for PyTorch-ROCm callers.

Every function here only marshals arguments: torch tensors become device
pointers, ``torch.cuda.current_stream()`` becomes the HIP stream, and the C
entry point of the same name does the work in hand-written HIP kernels.  There
is no CPU fallback: importing this module fails if ``libhisq.so`` is not built,
and the entry points fail if no GPU is visible.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# HISQ_LIBRARY_PATH selects another build of the same library (e.g. an
# experimental tuning variant); the default is the in-tree libhisq.so.
LIB_PATH = os.environ.get("HISQ_LIBRARY_PATH") or os.path.join(_HERE, "libhisq.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libhisq.so is not built (run __graft_entry__.build() or "
                      "python paper_1411_4439_amd/build.py); there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

HISQ_OK = 0
HISQ_EINVAL, HISQ_EGEOM, HISQ_EWORKSPACE, HISQ_EPACK, HISQ_EHIP = -1, -2, -3, -4, -5
HISQ_NOT_CONVERGED, HISQ_BREAKDOWN = 1, 2
HISQ_MAX_RHS, HISQ_MAX_PROBLEMS = 8, 16
PREC_F64, PREC_F32 = 0, 1
NAIK_FULL, NAIK_R14, NAIK_R13, NAIK_R9 = 0, 1, 2, 3
MODE_FP64, MODE_MIXED = 0, 1
LAYOUT_SITE, LAYOUT_COLOUR = 0, 1
K_PUPDATE, K_DSLASH_OE, K_DSLASH_EO, K_RELIABLE, K_FORCE = 0, 1, 2, 3, 4
K_COUNT = 5


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4)]


class Params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("naik", ctypes.c_int32), ("tol", ctypes.c_double),
                ("maxiter", ctypes.c_int32), ("delta", ctypes.c_double),
                ("poll_every", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("profile", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32 * 8), ("status", ctypes.c_int32 * 8),
                ("rel_true_res", ctypes.c_double * 8), ("rel_iter_res", ctypes.c_double * 8),
                ("reliable_updates", ctypes.c_int32), ("polls", ctypes.c_int32),
                ("total_iters", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("rhs_per_thread", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("stage_rows", ctypes.c_int32), ("eo_block_size", ctypes.c_int32),
                ("eo_rhs_per_thread", ctypes.c_int32), ("eo_tile_order", ctypes.c_int32),
                ("eo_stage_rows", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seconds", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * K_COUNT),
                ("kernel_launches", ctypes.c_int32 * K_COUNT)]

    def to_dict(self, nrhs):
        return {
            "iters": list(self.iters[:nrhs]), "status": list(self.status[:nrhs]),
            "rel_true_res": list(self.rel_true_res[:nrhs]),
            "rel_iter_res": list(self.rel_iter_res[:nrhs]),
            "reliable_updates": self.reliable_updates, "polls": self.polls,
            "total_iters": self.total_iters, "block_size": self.block_size,
            "rhs_per_thread": self.rhs_per_thread, "tile_order": self.tile_order,
            "stage_rows": self.stage_rows,
            "eo_block_size": self.eo_block_size, "eo_rhs_per_thread": self.eo_rhs_per_thread,
            "eo_tile_order": self.eo_tile_order, "eo_stage_rows": self.eo_stage_rows,
            "seconds": self.seconds,
            "kernel_ms": list(self.kernel_ms), "kernel_launches": list(self.kernel_launches),
        }


class Problem(ctypes.Structure):
    _fields_ = [("geom", Geom), ("mass", ctypes.c_double), ("nrhs", ctypes.c_int32),
                ("links64", ctypes.c_void_p), ("links32", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


_P = ctypes.c_void_p
_G = ctypes.POINTER(Geom)
_sig = {
    "hisq_default_params": (None, [ctypes.POINTER(Params)]),
    "hisq_links_bytes": (ctypes.c_size_t, [_G, ctypes.c_int, ctypes.c_int]),
    "hisq_workspace_bytes": (ctypes.c_size_t, [_G, ctypes.c_int, ctypes.c_int]),
    "hisq_backward_workspace_bytes": (ctypes.c_size_t, [_G, ctypes.c_int, ctypes.c_int]),
    "hisq_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(Problem),
                                                       ctypes.c_int]),
    "hisq_pack_links": (ctypes.c_int, [_G, _P, _P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "hisq_dslash": (ctypes.c_int, [_G, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, _P, _P, _P, _P]),
    "hisq_cg_solve": (ctypes.c_int, [_G, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Params),
                                     _P, _P, _P, _P, _P, ctypes.c_size_t, ctypes.POINTER(Info), _P]),
    "hisq_cg_solve_backward": (ctypes.c_int, [_G, ctypes.c_double, ctypes.c_int,
                                              ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P, _P,
                                              _P, _P, ctypes.c_size_t, ctypes.POINTER(Info), _P]),
    "hisq_cg_solve_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Problem),
                                             ctypes.POINTER(Params), _P, ctypes.c_size_t,
                                             ctypes.POINTER(Info), _P]),
    "hisq_set_tuning": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int]),
    "hisq_set_tuning_eo": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "hisq_full_workspace_bytes": (ctypes.c_size_t, [_G, ctypes.c_int, ctypes.c_int]),
    "hisq_trace_workspace_bytes": (ctypes.c_size_t, [_G, ctypes.c_int, ctypes.c_int]),
    "hisq_dslash_dmu": (ctypes.c_int, [_G, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P,
                                       _P]),
    "hisq_solve_full": (ctypes.c_int, [_G, ctypes.c_double, ctypes.c_int, ctypes.POINTER(Params),
                                       _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                                       ctypes.POINTER(Info), _P]),
    "hisq_trace_estimate": (ctypes.c_int, [_G, ctypes.c_double, ctypes.c_int,
                                           ctypes.POINTER(Params), _P, _P, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int), _P, _P, _P, _P,
                                           ctypes.c_size_t, ctypes.POINTER(Info), _P]),
    "hisq_cg_solve_noalloc": (ctypes.c_int, [_G, ctypes.c_double, ctypes.c_int,
                                             ctypes.POINTER(Params), _P, _P, _P, _P,
                                             ctypes.POINTER(Info), _P]),
    "hisq_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = tuple(_sig)


class HisqError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib.hisq_last_error().decode(errors="replace")
        super().__init__("%s failed with code %d: %s" % (where, code, msg))
        self.code = code


def _check(rc, where):
    if rc < 0:
        raise HisqError(rc, where)
    return rc


def geom(L):
    L = [int(v) for v in L]
    if len(L) != 4:
        raise ValueError("a lattice has four extents")
    return Geom((ctypes.c_int32 * 4)(*L))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_tensor(t, what):
    if t is not None and not t.is_cuda:
        raise ValueError("%s must be a device tensor (there is no CPU path)" % what)


# --- the C ABI, one wrapper per entry point ---------------------------------

def hisq_default_params(**overrides):
    p = Params()
    _lib.hisq_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def hisq_links_bytes(L, prec, naik=NAIK_FULL):
    return int(_lib.hisq_links_bytes(ctypes.byref(geom(L)), prec, naik))


def hisq_workspace_bytes(L, nrhs, mode):
    return int(_lib.hisq_workspace_bytes(ctypes.byref(geom(L)), nrhs, mode))


def hisq_backward_workspace_bytes(L, nrhs, mode):
    return int(_lib.hisq_backward_workspace_bytes(ctypes.byref(geom(L)), nrhs, mode))


def hisq_batched_workspace_bytes(problems, mode):
    arr = (Problem * len(problems))(*problems)
    return int(_lib.hisq_batched_workspace_bytes(len(problems), arr, mode))


def hisq_pack_links(L, U, N, prec, naik, packed, stream=None):
    _dev_tensor(U, "U")
    _dev_tensor(N, "N")
    return _check(_lib.hisq_pack_links(ctypes.byref(geom(L)), _ptr(U), _ptr(N), prec, naik,
                                       _ptr(packed), _stream(stream)), "hisq_pack_links")


def hisq_dslash(L, out_parity, nrhs, prec, naik, layout, packed, vin, vout, stream=None):
    _dev_tensor(vin, "in")
    _dev_tensor(vout, "out")
    return _check(_lib.hisq_dslash(ctypes.byref(geom(L)), out_parity, nrhs, prec, naik, layout,
                                   _ptr(packed), _ptr(vin), _ptr(vout), _stream(stream)),
                  "hisq_dslash")


def hisq_cg_solve(L, mass, nrhs, params, links64, links32, b, x, ws, info=None, stream=None):
    _dev_tensor(b, "b")
    _dev_tensor(x, "x")
    info = info if info is not None else Info()
    rc = _lib.hisq_cg_solve(ctypes.byref(geom(L)), float(mass), nrhs, ctypes.byref(params),
                            _ptr(links64), _ptr(links32), _ptr(b), _ptr(x), _ptr(ws),
                            ws.numel() * ws.element_size(), ctypes.byref(info), _stream(stream))
    return _check(rc, "hisq_cg_solve"), info


def hisq_cg_solve_noalloc(L, mass, nrhs, params, links64, links32, b, x, info=None, stream=None):
    _dev_tensor(b, "b")
    _dev_tensor(x, "x")
    info = info if info is not None else Info()
    rc = _lib.hisq_cg_solve_noalloc(ctypes.byref(geom(L)), float(mass), nrhs, ctypes.byref(params),
                                    _ptr(links64), _ptr(links32), _ptr(b), _ptr(x),
                                    ctypes.byref(info), _stream(stream))
    return _check(rc, "hisq_cg_solve_noalloc"), info


def hisq_cg_solve_backward(L, mass, nrhs, params, links64, links32, x, grad_x, grad_U, grad_N,
                           grad_m, grad_b, ws, info=None, stream=None):
    info = info if info is not None else Info()
    rc = _lib.hisq_cg_solve_backward(
        ctypes.byref(geom(L)), float(mass), nrhs, ctypes.byref(params), _ptr(links64),
        _ptr(links32), _ptr(x), _ptr(grad_x), _ptr(grad_U), _ptr(grad_N), _ptr(grad_m),
        _ptr(grad_b), _ptr(ws), ws.numel() * ws.element_size(), ctypes.byref(info),
        _stream(stream))
    return _check(rc, "hisq_cg_solve_backward"), info


def hisq_cg_solve_batched(problems, params, ws, stream=None):
    arr = (Problem * len(problems))(*problems)
    infos = (Info * len(problems))()
    rc = _lib.hisq_cg_solve_batched(len(problems), arr, ctypes.byref(params), _ptr(ws),
                                    ws.numel() * ws.element_size(), infos, _stream(stream))
    return _check(rc, "hisq_cg_solve_batched"), list(infos)


def hisq_set_tuning(mode, rhs_per_thread=0, block_size=0, tile_order=1, stage_rows=0):
    return _check(_lib.hisq_set_tuning(mode, rhs_per_thread, block_size, tile_order, stage_rows),
                  "hisq_set_tuning")


def hisq_set_tuning_eo(rhs_per_thread=0, block_size=64, tile_order=1, stage_rows=0):
    return _check(_lib.hisq_set_tuning_eo(rhs_per_thread, block_size, tile_order, stage_rows),
                  "hisq_set_tuning_eo")


def hisq_last_error():
    return _lib.hisq_last_error().decode(errors="replace")


# --- device-memory conveniences (torch allocates, the library computes) -----

def empty_bytes(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Links:
    """Packed link buffers for one gauge field: FP64 full, and optionally FP32
    full, FP32 r14, FP32 r13 and FP32 r9.  U, N: [4][V][3][3] complex128 device
    tensors."""

    def __init__(self, L, U, N, f32=True, r14=True, r13=False, r9=False, stream=None):
        self.L = tuple(int(v) for v in L)
        U = U.contiguous()
        N = N.contiguous()
        self.f64 = empty_bytes(hisq_links_bytes(self.L, PREC_F64, NAIK_FULL), U.device)
        hisq_pack_links(self.L, U, N, PREC_F64, NAIK_FULL, self.f64, stream)
        self.f32 = None
        self.f32r14 = None
        self.f32r13 = None
        self.f32r9 = None
        if f32:
            self.f32 = empty_bytes(hisq_links_bytes(self.L, PREC_F32, NAIK_FULL), U.device)
            hisq_pack_links(self.L, U, N, PREC_F32, NAIK_FULL, self.f32, stream)
        if r14:
            self.f32r14 = empty_bytes(hisq_links_bytes(self.L, PREC_F32, NAIK_R14), U.device)
            hisq_pack_links(self.L, U, N, PREC_F32, NAIK_R14, self.f32r14, stream)
        if r13:
            self.f32r13 = empty_bytes(hisq_links_bytes(self.L, PREC_F32, NAIK_R13), U.device)
            hisq_pack_links(self.L, U, N, PREC_F32, NAIK_R13, self.f32r13, stream)
        if r9:
            self.f32r9 = empty_bytes(hisq_links_bytes(self.L, PREC_F32, NAIK_R9), U.device)
            hisq_pack_links(self.L, U, N, PREC_F32, NAIK_R9, self.f32r9, stream)

    def packed(self, prec, naik=NAIK_FULL):
        if prec == PREC_F64:
            return self.f64
        return {NAIK_R14: self.f32r14, NAIK_R13: self.f32r13, NAIK_R9: self.f32r9}.get(naik, self.f32)


def dslash(links, out_parity, v, prec=PREC_F64, naik=NAIK_FULL, stream=None, layout=LAYOUT_SITE):
    """D_{out, 1-out} v for a half field v (complex128 or complex64), shaped
    [Vh][3][n] for LAYOUT_SITE or [3][Vh][n] for LAYOUT_COLOUR."""
    out = v.new_empty(v.shape)
    hisq_dslash(links.L, out_parity, v.shape[2], prec, naik, layout, links.packed(prec, naik),
                v.contiguous(), out, stream)
    return out


def solve(links, mass, b, mode=MODE_FP64, naik=NAIK_FULL, x0=None, ws=None, stream=None, **kw):
    """x = A^{-1} b for an even bundle b [Vh][3][n] complex128; returns (x, info dict)."""
    n = b.shape[2]
    p = hisq_default_params(mode=mode, naik=naik, **kw)
    x = x0.clone() if x0 is not None else b.new_empty(b.shape)
    p.use_x0 = 1 if x0 is not None else 0
    if ws is None:
        ws = empty_bytes(hisq_workspace_bytes(links.L, n, mode), b.device)
    l32 = links.packed(PREC_F32, naik) if mode == MODE_MIXED else None
    status, info = hisq_cg_solve(links.L, mass, n, p, links.f64, l32, b.contiguous(), x, ws,
                                 stream=stream)
    return x, status, info.to_dict(n)


def hisq_full_workspace_bytes(L, nrhs, mode):
    return int(_lib.hisq_full_workspace_bytes(ctypes.byref(geom(L)), nrhs, mode))


def hisq_trace_workspace_bytes(L, nrhs, mode):
    return int(_lib.hisq_trace_workspace_bytes(ctypes.byref(geom(L)), nrhs, mode))


def hisq_dslash_dmu(L, out_parity, nrhs, nder, links64, vin, vout, stream=None):
    _dev_tensor(vin, "in")
    _dev_tensor(vout, "out")
    return _check(_lib.hisq_dslash_dmu(ctypes.byref(geom(L)), out_parity, nrhs, nder,
                                       _ptr(links64), _ptr(vin), _ptr(vout), _stream(stream)),
                  "hisq_dslash_dmu")


def hisq_solve_full(L, mass, nrhs, params, links64, links32, b_e, b_o, x_e, x_o, ws, info=None,
                    stream=None):
    for t, nm in ((b_e, "b_e"), (b_o, "b_o"), (x_e, "x_e"), (x_o, "x_o")):
        _dev_tensor(t, nm)
    info = info if info is not None else Info()
    rc = _lib.hisq_solve_full(ctypes.byref(geom(L)), float(mass), nrhs, ctypes.byref(params),
                              _ptr(links64), _ptr(links32), _ptr(b_e), _ptr(b_o), _ptr(x_e),
                              _ptr(x_o), _ptr(ws), ws.numel() * ws.element_size(),
                              ctypes.byref(info), _stream(stream))
    return _check(rc, "hisq_solve_full"), info


def hisq_trace_estimate(L, mass, nrhs, params, links64, links32, orders, eta_e, eta_o, est, ws,
                        info=None, stream=None):
    for t, nm in ((eta_e, "eta_e"), (eta_o, "eta_o"), (est, "est")):
        _dev_tensor(t, nm)
    info = info if info is not None else Info()
    arr = (ctypes.c_int * max(1, len(orders)))(*orders)
    rc = _lib.hisq_trace_estimate(ctypes.byref(geom(L)), float(mass), nrhs, ctypes.byref(params),
                                  _ptr(links64), _ptr(links32), len(orders), arr, _ptr(eta_e),
                                  _ptr(eta_o), _ptr(est), _ptr(ws), ws.numel() * ws.element_size(),
                                  ctypes.byref(info), _stream(stream))
    return _check(rc, "hisq_trace_estimate"), info


def dslash_dmu(links, out_parity, v, nder, stream=None):
    """d^n D / d mu^n (mu = 0) for a half field v [Vh][3][n] complex128."""
    out = v.new_empty(v.shape)
    hisq_dslash_dmu(links.L, out_parity, v.shape[2], nder, links.f64, v.contiguous(), out, stream)
    return out


def solve_full(links, mass, b_e, b_o, mode=MODE_FP64, naik=NAIK_FULL, ws=None, stream=None, **kw):
    """(x_e, x_o) = M^-1 (b_e, b_o) on the full lattice; returns (x_e, x_o, status, info dict)."""
    n = b_e.shape[2]
    p = hisq_default_params(mode=mode, naik=naik, **kw)
    if ws is None:
        ws = empty_bytes(hisq_full_workspace_bytes(links.L, n, mode), b_e.device)
    x_e, x_o = b_e.new_empty(b_e.shape), b_o.new_empty(b_o.shape)
    l32 = links.packed(PREC_F32, naik) if mode == MODE_MIXED else None
    status, info = hisq_solve_full(links.L, mass, n, p, links.f64, l32, b_e.contiguous(),
                                   b_o.contiguous(), x_e, x_o, ws, stream=stream)
    return x_e, x_o, status, info.to_dict(n)


def trace_estimate(links, mass, orders, eta_e, eta_o, mode=MODE_FP64, naik=NAIK_FULL, ws=None,
                   stream=None, **kw):
    """Per-vector terms eta_k^dag M^(n_1) M^-1 ... M^(n_j) M^-1 eta_k of eq. (2) for one
    bundle of noise vectors; returns (complex128 numpy array [n], status, info dict)."""
    import torch
    n = eta_e.shape[2]
    p = hisq_default_params(mode=mode, naik=naik, **kw)
    if ws is None:
        ws = empty_bytes(hisq_trace_workspace_bytes(links.L, n, mode), eta_e.device)
    est = torch.empty((n, 2), dtype=torch.float64, device=eta_e.device)
    l32 = links.packed(PREC_F32, naik) if mode == MODE_MIXED else None
    status, info = hisq_trace_estimate(links.L, mass, n, p, links.f64, l32, list(orders),
                                       eta_e.contiguous(), eta_o.contiguous(), est, ws,
                                       stream=stream)
    e = est.cpu().numpy()
    return e[:, 0] + 1j * e[:, 1], status, info.to_dict(n)
