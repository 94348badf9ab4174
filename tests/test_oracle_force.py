"""Pins of the oracle's link force (gradient of L = sum_k Re phi_k^dag x_k, A x_k = eta_k).

Finite differences of L evaluated by a dense LAPACK solve, the Euler identity
(L is homogeneous of degree -2 in (U, N, m)), the free-field closed form for
dL/dm and the gauge covariance of the force.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1411_4439_amd import workload as W


def _loss_dense(L, U, N, m, phi, eta):
    A = dense.even_normal_matrix(L, U, N, m)
    n = eta.shape[2]
    x = np.linalg.solve(A, eta.reshape(-1, n)).reshape(eta.shape)
    return float(np.real(np.vdot(phi, x)))


def _solve_dense(L, U, N, m, rhs):
    A = dense.even_normal_matrix(L, U, N, m)
    n = rhs.shape[2]
    return np.linalg.solve(A, rhs.reshape(-1, n)).reshape(rhs.shape)


def _herm_dirs(shape, seed, imag):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    H = (Z + np.conj(np.swapaxes(Z, -1, -2))) / 2
    return 1j * H if imag else H


def test_force_finite_differences():
    L = (4, 4, 4, 4)
    m = 0.05
    U, N = W.make_links(L, 0.3, 111)
    phi = W.make_sources(L, 2, 112)
    eta = W.make_sources(L, 2, 113)
    x = _solve_dense(L, U, N, m, eta)
    y = _solve_dense(L, U, N, m, phi)
    GU, GN, dm = oracle.force(L, U, N, m, x, y)
    eps = 1e-6
    checked = 0
    for which in ("U", "N"):
        for d in range(8):
            dirn = _herm_dirs(U.shape, 1000 + 10 * d + (which == "N"), imag=(d % 2 == 1))
            G = GU if which == "U" else GN
            pred = float(np.real(np.vdot(G, dirn)))
            if which == "U":
                fp = _loss_dense(L, U + eps * dirn, N, m, phi, eta)
                fm = _loss_dense(L, U - eps * dirn, N, m, phi, eta)
            else:
                fp = _loss_dense(L, U, N + eps * dirn, m, phi, eta)
                fm = _loss_dense(L, U, N - eps * dirn, m, phi, eta)
            fd = (fp - fm) / (2 * eps)
            assert abs(fd - pred) <= 1e-5 * max(abs(pred), 1e-3 * np.linalg.norm(G)), (which, d)
            checked += 1
    fd = (_loss_dense(L, U, N, m + eps, phi, eta) - _loss_dense(L, U, N, m - eps, phi, eta)) / (2 * eps)
    assert abs(fd - dm) <= 1e-5 * abs(dm)
    assert checked == 16


@pytest.mark.parametrize("L,m", [((4, 4, 4, 4), 0.05), ((6, 6, 4, 4), 0.1)])
def test_force_euler_identity(L, m):
    """L(sU, sN, sm) = s^-2 L, so Re<G_U,U> + Re<G_N,N> + m dL/dm = -2 L."""
    U, N = W.make_links(L, 0.3, 121)
    phi = W.make_sources(L, 3, 122)
    eta = W.make_sources(L, 3, 123)
    x, _ = oracle.cg(L, U, N, m, eta, tol=1e-13)
    y, _ = oracle.cg(L, U, N, m, phi, tol=1e-13)
    GU, GN, dm = oracle.force(L, U, N, m, x, y)
    loss = float(np.real(np.vdot(phi, x)))
    lhs = float(np.real(np.vdot(GU, U) + np.vdot(GN, N))) + m * dm
    assert abs(lhs + 2 * loss) <= 1e-8 * abs(loss)


def test_force_free_field_mass_derivative():
    L = (4, 4, 4, 6)
    m = 0.05
    U, N = W.free_links(L, 1.0)
    k = (1, 0, 2, 1)
    pw = W.plane_wave(L, k, [1.0, 0.0, 0.0])[:, 0, 0]
    phi = W.to_half(np.stack([pw * 0.4, pw * (1 - 0.5j), pw * 0.2j], axis=1)[:, :, None], L, 0)
    eta = W.to_half(np.stack([pw * 1.1j, pw * 0.3, pw * (-0.7)], axis=1)[:, :, None], L, 0)
    S = sum(np.sin(2 * np.pi * k[mu] / L[mu]) + np.sin(6 * np.pi * k[mu] / L[mu]) for mu in range(4))
    den = 4 * m * m + 4 * S * S
    x, y = eta / den, phi / den
    _, _, dm = oracle.force(L, U, N, m, x, y)
    want = -8 * m * float(np.real(np.vdot(phi, eta))) / den ** 2
    assert abs(dm - want) <= 1e-10 * abs(want)


def test_force_gauge_covariance():
    L = (4, 4, 6, 4)
    m = 0.1
    U, N = W.make_links(L, 0.3, 131)
    x = W.make_sources(L, 2, 132)
    y = W.make_sources(L, 2, 133)
    g = W.random_su3(W.volume(L), 134)
    GU, GN, _ = oracle.force(L, U, N, m, x, y)
    from tests.test_oracle_dslash import _gauge_transform
    U2, N2 = _gauge_transform(L, U, N, g)
    ge = W.to_half(g, L, 0)
    x2 = np.einsum("sab,sbk->sak", ge, x)
    y2 = np.einsum("sab,sbk->sak", ge, y)
    GU2, GN2, _ = oracle.force(L, U2, N2, m, x2, y2)
    GU_t, GN_t = _gauge_transform(L, GU, GN, g)
    assert np.abs(GU2 - GU_t).max() <= 1e-12 * np.abs(GU).max()
    assert np.abs(GN2 - GN_t).max() <= 1e-12 * np.abs(GN).max()
