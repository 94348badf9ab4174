"""Pins of the oracle's even-odd operator and CG against library routines and closed forms.

A = 4 m^2 - D_eo D_oe is checked against the even block of M^dag M with
M = 2m + D assembled densely, its spectrum against LAPACK, and the CG against
LAPACK's dense solve and against the free-field closed form.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1411_4439_amd import workload as W


def _A_columns(L, U, N, m):
    Vh = W.half_volume(L)
    eye = np.eye(3 * Vh, dtype=complex).reshape(Vh, 3, 3 * Vh)
    return oracle.apply_A(L, U, N, m, eye).reshape(3 * Vh, 3 * Vh)


@pytest.mark.parametrize("m", [0.1, 0.01])
def test_A_is_even_block_of_MdagM(m):
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 61)
    A = _A_columns(L, U, N, m)
    Ad = dense.even_normal_matrix(L, U, N, m)
    assert np.abs(A - Ad).max() <= 1e-12 * np.abs(Ad).max()
    assert np.abs(A - A.conj().T).max() <= 1e-13 * np.abs(A).max()
    lam = np.linalg.eigvalsh(Ad)
    assert lam.min() >= 4 * m * m * (1 - 1e-10)


@pytest.mark.parametrize("c", [1.0, -1.0 / 24.0])
def test_A_free_field(c):
    L = (4, 6, 4, 4)
    m = 0.05
    U, N = W.free_links(L, c)
    for k in [(1, 0, 0, 0), (1, 1, 2, 3), (0, 5, 1, 0)]:
        v = W.to_half(W.plane_wave(L, k, [1.0, 0.5j, -0.3]), L, 0)
        S = sum(np.sin(2 * np.pi * k[mu] / L[mu]) + c * np.sin(6 * np.pi * k[mu] / L[mu])
                for mu in range(4))
        Av = oracle.apply_A(L, U, N, m, v)
        assert np.linalg.norm(Av - (4 * m * m + 4 * S * S) * v) <= 1e-13 * np.linalg.norm(v)


@pytest.mark.parametrize("m", [0.1, 0.05, 0.01])
def test_cg_matches_dense_solve(m):
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 71)
    b = W.make_sources(L, 2, 72)
    x, info = oracle.cg(L, U, N, m, b, tol=1e-13)
    assert (info["status"] == 0).all()
    assert (info["true_res"] <= 1e-13).all()
    Ad = dense.even_normal_matrix(L, U, N, m)
    xd = np.linalg.solve(Ad, b.reshape(-1, 2)).reshape(b.shape)
    for k in range(2):
        err = np.linalg.norm(x[..., k] - xd[..., k]) / np.linalg.norm(xd[..., k])
        # ||x - x*|| <= ||b - A x|| / lambda_min(A) and lambda_min >= 4 m^2
        bound = 1e-13 * np.linalg.norm(b[..., k]) / (4 * m * m) / np.linalg.norm(xd[..., k])
        assert err <= max(1e-10, 2 * bound)
    assert np.allclose(oracle.residual(L, U, N, m, b, x), info["true_res"], rtol=1e-6, atol=1e-16)


def test_cg_free_field_terminates():
    """Plane-wave sources: one iteration per distinct eigenvalue of A."""
    L = (4, 4, 6, 4)
    m = 0.1
    U, N = W.free_links(L, 1.0)
    k1, k2 = (1, 0, 0, 0), (1, 1, 1, 0)
    S = [sum(np.sin(2 * np.pi * k[mu] / L[mu]) + np.sin(6 * np.pi * k[mu] / L[mu]) for mu in range(4))
         for k in (k1, k2)]
    assert abs(S[0] ** 2 - S[1] ** 2) > 0.1
    b1 = W.to_half(W.plane_wave(L, k1, [1.0, 2.0j, -0.5]), L, 0)
    b2 = W.to_half(W.plane_wave(L, k2, [0.3, -1.0, 1.0j]), L, 0)
    x, info = oracle.cg(L, U, N, m, b1, tol=1e-13)
    assert info["iters"][0] == 1
    assert np.linalg.norm(x - b1 / (4 * m * m + 4 * S[0] ** 2)) <= 1e-13 * np.linalg.norm(x)
    x, info = oracle.cg(L, U, N, m, b1 + b2, tol=1e-13)
    assert info["iters"][0] <= 2
    want = b1 / (4 * m * m + 4 * S[0] ** 2) + b2 / (4 * m * m + 4 * S[1] ** 2)
    assert np.linalg.norm(x - want) <= 1e-13 * np.linalg.norm(want)


def test_cg_start_vector_and_zero_source():
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 81)
    b = W.make_sources(L, 2, 82)
    b[..., 1] = 0
    x, info = oracle.cg(L, U, N, 0.1, b, tol=1e-12)
    assert info["status"][1] == 0 and info["iters"][1] == 0 and not np.any(x[..., 1])
    # restarting from the answer takes no iterations
    x2, info2 = oracle.cg(L, U, N, 0.1, b[..., :1], tol=1e-10, x0=x[..., :1])
    assert info2["iters"][0] == 0


def test_cg_maxiter_and_breakdown_reported():
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 91)
    b = W.make_sources(L, 1, 92)
    _, info = oracle.cg(L, U, N, 0.1, b, tol=1e-12, maxiter=3)
    assert info["status"][0] == oracle.NOT_CONVERGED and info["iters"][0] == 3
    # m = 0 on the free field: A has an exact null space (constant modes)
    U0, N0 = W.free_links(L, 1.0)
    b0 = W.to_half(W.plane_wave(L, (0, 0, 0, 0), [1.0, 0, 0]), L, 0)
    _, info = oracle.cg(L, U0, N0, 0.0, b0, tol=1e-12, maxiter=50)
    assert info["status"][0] == oracle.BREAKDOWN


def test_r14_roundtrip():
    L = (4, 4, 4, 6)
    U, N = W.make_links(L, 0.3, 101)
    P, err = oracle.r14_pack(N)
    assert err <= 1e-14
    assert np.abs(oracle.r14_unpack(P) - N).max() <= 1e-15
    # a general complex matrix is not s * U(3): the round trip must fail loudly
    rng = np.random.default_rng(5)
    Z = rng.standard_normal((10, 3, 3)) + 1j * rng.standard_normal((10, 3, 3))
    _, err = oracle.r14_pack(Z)
    assert err > 1e-3


def test_r13_roundtrip_and_relation_to_r14():
    """r13 keeps rows 0, 1 and one phase: exact for N = s V, V in U(3) (the
    synthetic Naik links, s = 1/24, and a random U(3) times a random scale),
    equal to the r14 decoding, and loudly wrong for a general matrix."""
    L = (4, 4, 4, 6)
    U, N = W.make_links(L, 0.3, 101)
    P, err = oracle.r13_pack(N)
    assert P.shape == N.shape[:-2] + (13,)
    assert err <= 1e-14
    back = oracle.r13_unpack(P)
    assert np.abs(back - N).max() <= 1e-15
    assert np.abs(back - oracle.r14_unpack(oracle.r14_pack(N)[0])).max() <= 1e-15
    rng = np.random.default_rng(6)
    Z = rng.standard_normal((20, 3, 3)) + 1j * rng.standard_normal((20, 3, 3))
    Q, _ = np.linalg.qr(Z)  # a U(3) matrix per entry
    scale = rng.uniform(0.01, 10.0, size=(20, 1, 1))
    _, err = oracle.r13_pack(scale * Q)
    assert err <= 1e-13
    # the phase of c is the phase of det V (row2 = s det(V) conj(v0 x v1))
    P, _ = oracle.r13_pack(scale * Q)
    assert np.allclose(np.exp(1j * P[:, 12]), np.linalg.det(Q), atol=1e-13)
    _, err = oracle.r13_pack(Z)
    assert err > 1e-3


def test_r9_roundtrip():
    """r9 keeps one scale and a Hermitian H per Naik matrix: exact for the
    synthetic links (N = -(1/24) UUU, s = 1/24) and for random U(3) matrices
    times one scale; a general matrix or mixed scales are reported."""
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 102)
    P, s, err, spread = oracle.r9_pack(N[:, :40])
    assert abs(s - 1.0 / 24.0) <= 1e-14 and spread <= 1e-13 and err <= 1e-12
    assert np.abs(oracle.r9_unpack(P, s) - N[:, :40]).max() <= 1e-13
    H = P.reshape(-1, 9)
    # the decoded matrix is s times a unitary one
    Wm = oracle.r9_unpack(P, 1.0).reshape(-1, 3, 3)
    assert np.abs(Wm @ Wm.conj().transpose(0, 2, 1) - np.eye(3)).max() <= 1e-13
    rng = np.random.default_rng(7)
    Z = rng.standard_normal((12, 3, 3)) + 1j * rng.standard_normal((12, 3, 3))
    Q, _ = np.linalg.qr(Z)
    P, s, err, spread = oracle.r9_pack(0.37 * Q)
    assert abs(s - 0.37) <= 1e-13 and err <= 1e-12
    _, _, err, _ = oracle.r9_pack(Z)
    assert err > 1e-3
    _, _, _, spread = oracle.r9_pack(np.concatenate([Q[:6], 2 * Q[6:]]))
    assert spread > 0.4
    assert H.shape[1] == 9


def test_r9_closed_forms():
    """r9 against closed forms: H = diag(a, b, c) decodes to s diag(e^ia, e^ib,
    e^ic); a 2x2 block H = theta * sigma_x decodes to cos(theta) 1 + i sin(theta)
    sigma_x; and packing s diag(e^{i phi}) recovers phi on the principal branch."""
    s = 0.25
    P = np.array([0.3, -1.1, 2.0, 0, 0, 0, 0, 0, 0])
    got = oracle.r9_unpack(P[None], s)[0]
    assert np.allclose(got, s * np.diag(np.exp(1j * P[:3])), atol=1e-15)
    th = 0.7
    P = np.array([0, 0, 0, th, 0, 0, 0, 0, 0])
    want = s * np.array([[np.cos(th), 1j * np.sin(th), 0], [1j * np.sin(th), np.cos(th), 0],
                         [0, 0, 1]])
    assert np.allclose(oracle.r9_unpack(P[None], s)[0], want, atol=1e-15)
    phi = np.array([0.4, -2.5, 1.9])
    Pp, sp, err, spread = oracle.r9_pack((s * np.diag(np.exp(1j * phi)))[None])
    assert abs(sp - s) <= 1e-15 and err <= 1e-13 and spread == 0.0
    assert np.allclose(Pp[0, :3], phi, atol=1e-12) and np.allclose(Pp[0, 3:], 0, atol=1e-12)
