"""Dense-matrix form of the HISQ operator for tiny lattices -- TEST INFRASTRUCTURE ONLY.

A second, independent assembly of the Dslash of Sec. 1 eq. (3) of Kaczmarek et
al. (GPUHEP2014): every term of the sum is written as a 3x3 block of a
(3V) x (3V) complex matrix, so that library routines (LAPACK solve and
eigen-decomposition) can act on it.  From it:

* M = 2 m 1 + D (the reading of the fermion matrix; the paper does not print it),
* A = the even-even block of M^dag M, which must equal 4 m^2 - D_eo D_oe
  (this is checked, not assumed).

Row/column index of a colour component: 3 * s + colour, with the site index
s = x0 + L0*(x1 + L1*(x2 + L2*x3)).
"""
from __future__ import annotations

import numpy as np


def _site(L, x):
    return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))


def _coords(L, s):
    out = []
    for mu in range(4):
        out.append(s % L[mu])
        s //= L[mu]
    return out


def dslash_matrix(L, U, N):
    """D as a dense (3V, 3V) matrix, block (x, y) collecting every term of eq. (3)."""
    L = [int(v) for v in L]
    V = int(np.prod(L))
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for s in range(V):
        x = _coords(L, s)
        for mu in range(4):
            def shifted(h):
                y = list(x)
                y[mu] = (y[mu] + h) % L[mu]
                return _site(L, y)
            fwd1, bwd1, fwd3, bwd3 = shifted(1), shifted(-1), shifted(3), shifted(-3)
            rows = slice(3 * s, 3 * s + 3)
            D[rows, 3 * fwd1:3 * fwd1 + 3] += U[mu, s]
            D[rows, 3 * bwd1:3 * bwd1 + 3] -= U[mu, bwd1].conj().T
            D[rows, 3 * fwd3:3 * fwd3 + 3] += N[mu, s]
            D[rows, 3 * bwd3:3 * bwd3 + 3] -= N[mu, bwd3].conj().T
    return D


def dslash_dmu_matrix(L, U, N, nder):
    """d^n D / d mu^n at mu = 0 as a dense matrix: only the time-direction (mu = 3)
    terms of eq. (3) survive, the h-step hop weighted by h^n (from exp(h mu))."""
    L = [int(v) for v in L]
    V = int(np.prod(L))
    D = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for s in range(V):
        x = _coords(L, s)
        rows = slice(3 * s, 3 * s + 3)
        for h, W, backward in ((1, U, False), (-1, U, True), (3, N, False), (-3, N, True)):
            y = list(x)
            y[3] = (y[3] + h) % L[3]
            t = _site(L, y)
            w = float(h) ** nder
            if backward:
                D[rows, 3 * t:3 * t + 3] -= w * W[3, t].conj().T
            else:
                D[rows, 3 * t:3 * t + 3] += w * W[3, s]
    return D


def parity_indices(L, parity):
    """Dense row indices of one parity, ordered by s // 2 (the half-field order)."""
    L = [int(v) for v in L]
    V = int(np.prod(L))
    sites = [s for s in range(V) if sum(_coords(L, s)) % 2 == parity]
    return np.array([3 * s + c for s in sites for c in range(3)], dtype=np.int64)


def fermion_matrix(L, U, N, m):
    """M = 2 m + D."""
    D = dslash_matrix(L, U, N)
    return 2.0 * m * np.eye(D.shape[0]) + D


def even_normal_matrix(L, U, N, m):
    """Even-even block of M^dag M (the system the even-odd CG solves)."""
    M = fermion_matrix(L, U, N, m)
    MM = M.conj().T @ M
    e = parity_indices(L, 0)
    return MM[np.ix_(e, e)]
