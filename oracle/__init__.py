"""FP64 CPU oracle for the HISQ even-odd CG -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library never does, and this
package never loads the HIP library: the two share no code.

``hisq_oracle.c`` holds the arithmetic (HISQ Dslash of eq. (3) of Kaczmarek et
al., GPUHEP2014, the even-odd operator A = 4m^2 - D_eo D_oe, CG, the link force,
the 14- and 13-real Naik encodings and the mu-derivatives of the Dslash); this
module compiles it with gcc and marshals numpy arrays through ctypes.  The
full-matrix solve and the trace estimator of eq. (2) below only chain those
routines in the order the method states; the 9-real Naik encoding (one scale,
a Hermitian generator) uses scipy's matrix logarithm and exponential.
``oracle.dense`` assembles the same operators as dense matrices for tiny
lattices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hisq_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile hisq_oracle.c into liboracle.so (plain -O2, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=gnu99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            Lp = ctypes.POINTER(ctypes.c_int)
            lib.orc_dslash_full.argtypes = [Lp, I, P, P, P, P]
            lib.orc_dslash_eo.argtypes = [Lp, I, I, P, P, P, P]
            lib.orc_dslash_sites.argtypes = [Lp, I, I, P, P, P, ctypes.c_long, P, P]
            lib.orc_apply_A.argtypes = [Lp, I, D, P, P, P, P]
            lib.orc_cg.argtypes = [Lp, I, D, P, P, P, P, D, I, P, P, P, P]
            lib.orc_residual.argtypes = [Lp, I, D, P, P, P, P, P]
            lib.orc_force.argtypes = [Lp, I, D, P, P, P, P, P, P, P]
            lib.orc_r14_pack.argtypes = [ctypes.c_long, P, P, P]
            lib.orc_r14_unpack.argtypes = [ctypes.c_long, P, P]
            lib.orc_dslash_chem_eo.argtypes = [Lp, I, I, P, P, D, I, P, P]
            lib.orc_r13_pack.argtypes = [ctypes.c_long, P, P, P]
            lib.orc_r13_unpack.argtypes = [ctypes.c_long, P, P]
            lib.orc_num_threads.argtypes = []
            lib.orc_set_threads.argtypes = [I]
            _lib = lib
    return _lib


def _geom(L):
    L = [int(v) for v in L]
    if len(L) != 4:
        raise ValueError("lattice must have 4 extents")
    return (ctypes.c_int * 4)(*L)


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc):
    if rc < 0:
        raise ValueError("oracle call failed with code %d" % rc)
    return rc


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    _check(_load().orc_set_threads(int(k)))


def _links(L, U, N):
    V = int(np.prod(L))
    return _c128(U, (4, V, 3, 3)), _c128(N, (4, V, 3, 3))


def dslash_full(L, U, N, v):
    """w = D v on the full lattice; v is (V, 3, n)."""
    U, N = _links(L, U, N)
    v = _c128(v)
    w = np.empty_like(v)
    _check(_load().orc_dslash_full(_geom(L), v.shape[2], _ptr(U), _ptr(N), _ptr(v), _ptr(w)))
    return w


def dslash_eo(L, U, N, v, out_parity):
    """Half-lattice Dslash: input parity 1-out_parity, output parity out_parity."""
    U, N = _links(L, U, N)
    v = _c128(v)
    w = np.empty_like(v)
    _check(_load().orc_dslash_eo(_geom(L), v.shape[2], int(out_parity), _ptr(U), _ptr(N),
                                 _ptr(v), _ptr(w)))
    return w


def dslash_sites(L, U, N, v, out_parity, sites):
    """Half-lattice Dslash at chosen full-lattice sites of parity out_parity: (count, 3, n)."""
    U, N = _links(L, U, N)
    v = _c128(v)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((sites.size, 3, v.shape[2]), dtype=np.complex128)
    _check(_load().orc_dslash_sites(_geom(L), v.shape[2], int(out_parity), _ptr(U), _ptr(N),
                                    _ptr(v), sites.size, _ptr(sites), _ptr(out)))
    return out


def apply_A(L, U, N, m, x):
    """y = (4 m^2 - D_eo D_oe) x on an even half field (V/2, 3, n)."""
    U, N = _links(L, U, N)
    x = _c128(x)
    y = np.empty_like(x)
    _check(_load().orc_apply_A(_geom(L), x.shape[2], float(m), _ptr(U), _ptr(N), _ptr(x), _ptr(y)))
    return y


def cg(L, U, N, m, b, tol=1e-13, maxiter=20000, x0=None):
    """Plain FP64 CG per rhs; returns (x, info)."""
    U, N = _links(L, U, N)
    b = _c128(b)
    n = b.shape[2]
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    iters = np.zeros(n, dtype=np.int32)
    tres = np.zeros(n)
    ires = np.zeros(n)
    status = np.zeros(n, dtype=np.int32)
    _check(_load().orc_cg(_geom(L), n, float(m), _ptr(U), _ptr(N), _ptr(b), _ptr(x), float(tol),
                          int(maxiter), _ptr(iters), _ptr(tres), _ptr(ires), _ptr(status)))
    return x, {"iters": iters, "true_res": tres, "iter_res": ires, "status": status}


def residual(L, U, N, m, b, x):
    """||b_k - A x_k|| / ||b_k|| per rhs, in FP64."""
    U, N = _links(L, U, N)
    b = _c128(b)
    x = _c128(x, b.shape)
    rel = np.zeros(b.shape[2])
    _check(_load().orc_residual(_geom(L), b.shape[2], float(m), _ptr(U), _ptr(N), _ptr(b),
                                _ptr(x), _ptr(rel)))
    return rel


def force(L, U, N, m, x, y):
    """(G_U, G_N, dL/dm) for L = sum_k Re(phi_k^dag x_k), given x and y = A^{-1} phi."""
    U, N = _links(L, U, N)
    x = _c128(x)
    y = _c128(y, x.shape)
    GU = np.empty_like(U)
    GN = np.empty_like(N)
    dm = np.zeros(1)
    _check(_load().orc_force(_geom(L), x.shape[2], float(m), _ptr(U), _ptr(N), _ptr(x), _ptr(y),
                             _ptr(GU), _ptr(GN), _ptr(dm)))
    return GU, GN, float(dm[0])


def r14_pack(M):
    """Compress (..., 3, 3) complex matrices to (..., 14) reals; returns (packed, max_err)."""
    M = _c128(M)
    lead = M.shape[:-2]
    count = int(np.prod(lead)) if lead else 1
    out = np.empty(lead + (14,), dtype=np.float64)
    err = np.zeros(1)
    _check(_load().orc_r14_pack(count, _ptr(M), _ptr(out), _ptr(err)))
    return out, float(err[0])


def r14_unpack(P):
    """Inverse of r14_pack."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    lead = P.shape[:-1]
    count = int(np.prod(lead)) if lead else 1
    M = np.empty(lead + (3, 3), dtype=np.complex128)
    _check(_load().orc_r14_unpack(count, _ptr(P), _ptr(M)))
    return M


def r13_pack(M):
    """Compress (..., 3, 3) complex matrices to (..., 13) reals; returns (packed, max_err)."""
    M = _c128(M)
    lead = M.shape[:-2]
    count = int(np.prod(lead)) if lead else 1
    out = np.empty(lead + (13,), dtype=np.float64)
    err = np.zeros(1)
    _check(_load().orc_r13_pack(count, _ptr(M), _ptr(out), _ptr(err)))
    return out, float(err[0])


def r13_unpack(P):
    """Inverse of r13_pack."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    lead = P.shape[:-1]
    count = int(np.prod(lead)) if lead else 1
    M = np.empty(lead + (3, 3), dtype=np.complex128)
    _check(_load().orc_r13_unpack(count, _ptr(P), _ptr(M)))
    return M


def r9_pack(M):
    """r9: N = s exp(iH) with one scale s for all matrices, s = |det N|^(1/3)
    (their mean), H = -i log(N / s) Hermitian (9 reals: H00, H11, H22, Re/Im
    H01, H02, H12).  Returns (packed (..., 9), s, max relative round-trip error,
    relative spread of the per-matrix scales).  Uses scipy's matrix log/exp."""
    from scipy.linalg import expm, logm
    M = _c128(M)
    lead = M.shape[:-2]
    flat = M.reshape(-1, 3, 3)
    sj = np.abs(np.linalg.det(flat)) ** (1.0 / 3.0)
    s = float(sj.mean())
    out = np.empty((flat.shape[0], 9))
    worst = 0.0
    for j, m in enumerate(flat):
        H = -1j * logm(m / sj[j])
        H = 0.5 * (H + H.conj().T)
        out[j] = [H[0, 0].real, H[1, 1].real, H[2, 2].real, H[0, 1].real, H[0, 1].imag,
                  H[0, 2].real, H[0, 2].imag, H[1, 2].real, H[1, 2].imag]
        back = sj[j] * expm(1j * H)
        worst = max(worst, np.linalg.norm(back - m) / np.linalg.norm(m))
    spread = float((sj.max() - sj.min()) / sj.max()) if sj.size else 0.0
    return out.reshape(lead + (9,)), s, worst, spread


def r9_unpack(P, s):
    """s exp(iH) from the 9 reals of H."""
    from scipy.linalg import expm
    P = np.ascontiguousarray(P, dtype=np.float64)
    lead = P.shape[:-1]
    flat = P.reshape(-1, 9)
    out = np.empty((flat.shape[0], 3, 3), dtype=np.complex128)
    for j, h in enumerate(flat):
        H = np.array([[h[0], h[3] + 1j * h[4], h[5] + 1j * h[6]],
                      [h[3] - 1j * h[4], h[1], h[7] + 1j * h[8]],
                      [h[5] - 1j * h[6], h[7] - 1j * h[8], h[2]]])
        out[j] = s * expm(1j * H)
    return out.reshape(lead + (3, 3))


def dslash_dmu(L, U, N, v, out_parity, nder, mu=0.0):
    """d^n D(mu) / d mu^n restricted to one output parity (input parity
    1 - out_parity); nder = 0 is D(mu).  Temporal h-hops carry exp(h mu)."""
    U, N = _links(L, U, N)
    v = _c128(v)
    w = np.empty_like(v)
    _check(_load().orc_dslash_chem_eo(_geom(L), v.shape[2], int(out_parity), _ptr(U), _ptr(N),
                                      float(mu), int(nder), _ptr(v), _ptr(w)))
    return w


def apply_M(L, U, N, m, x_e, x_o, nder=0):
    """(y_e, y_o) = d^n M / d mu^n (x_e, x_o) at mu = 0, M = 2m + D: nder = 0 is M
    itself, nder >= 1 the derivative operators of eq. (2) (the mass term does not
    depend on mu)."""
    if nder == 0:
        return (2.0 * m * _c128(x_e) + dslash_eo(L, U, N, x_o, 0),
                2.0 * m * _c128(x_o) + dslash_eo(L, U, N, x_e, 1))
    return dslash_dmu(L, U, N, x_o, 0, nder), dslash_dmu(L, U, N, x_e, 1, nder)


def solve_full(L, U, N, m, b_e, b_o, tol=1e-13, maxiter=20000):
    """x = M^{-1} b on the full lattice through the even-odd reduction:
    (4m^2 - D_eo D_oe) x_e = 2m b_e - D_eo b_o, then x_o = (b_o - D_oe x_e) / (2m)."""
    b_e, b_o = _c128(b_e), _c128(b_o)
    rhs = 2.0 * m * b_e - dslash_eo(L, U, N, b_o, 0)
    x_e, info = cg(L, U, N, m, rhs, tol=tol, maxiter=maxiter)
    x_o = (b_o - dslash_eo(L, U, N, x_e, 1)) / (2.0 * m)
    return x_e, x_o, info


def trace_estimate(L, U, N, m, orders, eta_e, eta_o, tol=1e-13):
    """Per-noise-vector terms of eq. (2):
    eta_k^dag M^(n_1) M^{-1} M^(n_2) M^{-1} ... M^(n_j) M^{-1} eta_k for
    orders = (n_1, ..., n_j), M^(n) = d^n M / d mu^n at mu = 0.  Applied right to
    left: v = eta, then for i = j..1: v = M^{-1} v, v = M^(n_i) v.  Returns the
    n complex terms (their mean over many vectors estimates the trace)."""
    eta_e, eta_o = _c128(eta_e), _c128(eta_o)
    v_e, v_o = eta_e, eta_o
    for nder in reversed(list(orders)):
        v_e, v_o, _ = solve_full(L, U, N, m, v_e, v_o, tol=tol)
        v_e, v_o = apply_M(L, U, N, m, v_e, v_o, nder)
    n = eta_e.shape[2]
    return np.array([np.vdot(eta_e[..., k], v_e[..., k]) + np.vdot(eta_o[..., k], v_o[..., k])
                     for k in range(n)])
