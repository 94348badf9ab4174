"""Pins of the oracle's HISQ Dslash (Sec. 1, eq. (3)) that do not use the oracle itself.

Each test fixes something the mathematics fixes: point-source columns read off
eq. (3) by hand, the free-field spectrum (closed form), anti-Hermiticity, gauge
covariance, linearity and the independence of rhs in a bundle (eq. (4)).
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1411_4439_amd import workload as W

LATTICES = [(4, 4, 4, 4), (6, 4, 4, 8), (4, 6, 8, 4)]


def _rand_full(L, n, seed):
    rng = np.random.default_rng(seed)
    V = W.volume(L)
    return rng.standard_normal((V, 3, n)) + 1j * rng.standard_normal((V, 3, n))


def _site(L, x):
    return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))


def _coords(L, s):
    out = []
    for mu in range(4):
        out.append(s % L[mu])
        s //= L[mu]
    return out


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 6, 4)])
def test_point_source_columns(L):
    """Column y of D: which links land on which rows (wrap-aliased sites add)."""
    U, N = W.make_links(L, 0.3, 11)
    V = W.volume(L)
    for y in [0, 5, V // 2 + 3, V - 1]:
        for c in range(3):
            e = np.zeros((V, 3, 1), dtype=complex)
            e[y, c, 0] = 1.0
            col = oracle.dslash_full(L, U, N, e)[:, :, 0]
            want = np.zeros((V, 3), dtype=complex)
            yc = _coords(L, y)
            for mu in range(4):
                def at(h):
                    z = list(yc)
                    z[mu] = (z[mu] + h) % L[mu]
                    return _site(L, z)
                # a site x with x + mu = y picks U_{x,mu} e_y
                want[at(-1)] += U[mu, at(-1)][:, c]
                # a site x with x - mu = y picks -U^dag_{y,mu} e_y
                want[at(+1)] -= np.conj(U[mu, y][c, :])
                want[at(-3)] += N[mu, at(-3)][:, c]
                want[at(+3)] -= np.conj(N[mu, y][c, :])
            assert np.abs(col - want).max() <= 1e-15


def _free_lambda(L, k, c):
    p = [2 * np.pi * k[mu] / L[mu] for mu in range(4)]
    return 2j * sum(np.sin(q) + c * np.sin(3 * q) for q in p)


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("c", [1.0, -1.0 / 24.0])
def test_free_field_plane_waves(L, c):
    """U = 1, N = c: e^{ipx} xi has eigenvalue 2i sum_mu (sin p_mu + c sin 3 p_mu)."""
    U, N = W.free_links(L, c)
    rng = np.random.default_rng(3)
    for k in [(0, 0, 0, 0), (1, 0, 0, 0), (1, 2, 0, 1), (L[0] - 1, 1, 2, 3)]:
        xi = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        v = W.plane_wave(L, k, xi)
        lam = _free_lambda(L, k, c)
        w = oracle.dslash_full(L, U, N, v)
        assert np.linalg.norm(w - lam * v) <= 1e-13 * np.linalg.norm(v)
        # even-odd blocks: D_oe v_e = lam v_o and D_eo v_o = lam v_e
        ve, vo = W.to_half(v, L, 0), W.to_half(v, L, 1)
        assert np.linalg.norm(oracle.dslash_eo(L, U, N, ve, 1) - lam * vo) <= 1e-13 * np.linalg.norm(v)
        assert np.linalg.norm(oracle.dslash_eo(L, U, N, vo, 0) - lam * ve) <= 1e-13 * np.linalg.norm(v)


@pytest.mark.parametrize("L", LATTICES)
def test_anti_hermiticity(L):
    U, N = W.make_links(L, 0.3, 21)
    v = _rand_full(L, 2, 1)
    w = _rand_full(L, 2, 2)
    lhs = np.vdot(w, oracle.dslash_full(L, U, N, v))
    rhs = -np.vdot(oracle.dslash_full(L, U, N, w), v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    ve = W.to_half(w, L, 0)
    vo = W.to_half(v, L, 1)
    lhs = np.vdot(ve, oracle.dslash_eo(L, U, N, vo, 0))
    rhs = -np.vdot(oracle.dslash_eo(L, U, N, ve, 1), vo)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _gauge_transform(L, U, N, g):
    V = W.volume(L)
    U2 = np.empty_like(U)
    N2 = np.empty_like(N)
    gd = np.conj(np.swapaxes(g, -1, -2))
    for mu in range(4):
        for s in range(V):
            x = _coords(L, s)
            x1 = list(x)
            x1[mu] = (x1[mu] + 1) % L[mu]
            x3 = list(x)
            x3[mu] = (x3[mu] + 3) % L[mu]
            U2[mu, s] = g[s] @ U[mu, s] @ gd[_site(L, x1)]
            N2[mu, s] = g[s] @ N[mu, s] @ gd[_site(L, x3)]
    return U2, N2


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 6)])
def test_gauge_covariance(L):
    U, N = W.make_links(L, 0.3, 31)
    g = W.random_su3(W.volume(L), 32)
    U2, N2 = _gauge_transform(L, U, N, g)
    v = _rand_full(L, 3, 4)
    gv = np.einsum("sab,sbk->sak", g, v)
    lhs = oracle.dslash_full(L, U2, N2, gv)
    rhs = np.einsum("sab,sbk->sak", g, oracle.dslash_full(L, U, N, v))
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_linearity_and_bundle():
    L = (4, 4, 6, 4)
    U, N = W.make_links(L, 0.3, 41)
    U2, N2 = W.make_links(L, 0.5, 42)
    v = _rand_full(L, 4, 5)
    w = oracle.dslash_full(L, U, N, v)
    # eq. (4): a bundle equals n independent single-rhs applications
    for k in range(4):
        single = oracle.dslash_full(L, U, N, v[:, :, k:k + 1])
        assert np.abs(single[:, :, 0] - w[:, :, k]).max() <= 1e-15 * np.abs(w).max()
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    lin = oracle.dslash_full(L, U, N, a * v[:, :, :1] + b * v[:, :, 1:2])
    assert np.abs(lin - (a * w[:, :, :1] + b * w[:, :, 1:2])).max() <= 1e-14 * np.abs(w).max()
    sumlinks = oracle.dslash_full(L, U + U2, N + N2, v)
    parts = w + oracle.dslash_full(L, U2, N2, v)
    assert np.abs(sumlinks - parts).max() <= 1e-14 * np.abs(parts).max()


def test_dense_assembly_matches():
    """The dense assembly (used with LAPACK below) is the same operator."""
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 51)
    v = _rand_full(L, 2, 6)
    D = dense.dslash_matrix(L, U, N)
    w = (D @ v.reshape(-1, 2)).reshape(v.shape)
    assert np.abs(w - oracle.dslash_full(L, U, N, v)).max() <= 1e-13


def test_bad_geometry_rejected():
    U, N = W.free_links((4, 4, 4, 4))
    with pytest.raises(ValueError):
        oracle.dslash_eo((5, 4, 4, 4), U, N, np.zeros((40, 3, 1)), 0)


def test_sampled_sites_match_full_pass():
    L = (6, 4, 4, 6)
    U, N = W.make_links(L, 0.3, 141)
    v = W.to_half(_rand_full(L, 3, 7), L, 1)
    full = oracle.dslash_eo(L, U, N, v, 0)
    even = np.flatnonzero(W.even_mask(L))
    pick = even[[0, 5, 17, len(even) - 1]]
    part = oracle.dslash_sites(L, U, N, v, 0, pick)
    assert np.array_equal(part, full[pick // 2])
    with pytest.raises(ValueError):
        oracle.dslash_sites(L, U, N, v, 0, [1])  # site 1 is odd
