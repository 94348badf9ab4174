"""The seeded input generator, checked on the CPU against the recipe it states:
phased SU(3) one-hop links U = eta exp(i eps H), Naik links N = -(1/24) times
the product of three consecutive U, Gaussian sources, Z2 / Gaussian noise, and
the seed scheme.  Site arithmetic is redone here by explicit coordinates."""
import itertools

import numpy as np

from paper_1411_4439_amd import workload as W

L = (4, 6, 4, 6)


def _site(c):
    return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))


def _eta(mu, c):
    return (-1) ** sum(c[:mu])


def test_links_are_phased_special_unitary():
    U, _ = W.make_links(L, 0.3, 11)
    eye = np.eye(3)
    for c in itertools.product(*(range(n) for n in L)):
        s = _site(c)
        for mu in range(4):
            Vm = U[mu, s] * _eta(mu, c)
            assert np.abs(Vm @ Vm.conj().T - eye).max() < 1e-13
            assert abs(np.linalg.det(Vm) - 1.0) < 1e-13


def test_naik_is_the_scaled_three_link_product():
    U, N = W.make_links(L, 0.3, 12)
    for c in itertools.product(*(range(n) for n in L)):
        s = _site(c)
        for mu in range(4):
            hops = []
            for h in range(3):
                d = list(c)
                d[mu] = (d[mu] + h) % L[mu]
                hops.append(U[mu, _site(d)])
            want = -(1.0 / 24.0) * hops[0] @ hops[1] @ hops[2]
            assert np.abs(N[mu, s] - want).max() < 1e-15
            # N = s V with s = 1/24 and V unitary
            Vn = 24.0 * N[mu, s]
            assert np.abs(Vn @ Vn.conj().T - np.eye(3)).max() < 1e-13


def test_smearing_width_sets_the_distance_from_the_identity():
    # ||exp(i eps H) - 1||_F ~ eps ||H||_F, and E ||H||_F^2 = 8 * tr(lambda^2 / 4) = 4
    dist = {}
    for eps in (0.05, 0.2):
        U, _ = W.make_links(L, eps, 13, phases=False)
        dist[eps] = np.linalg.norm(U - np.eye(3), axis=(2, 3)).mean()
    assert 0.7 < dist[0.05] / (0.05 * 2.0) < 1.1
    assert 0.7 < dist[0.2] / (0.2 * 2.0) < 1.1
    assert 3.5 < dist[0.2] / dist[0.05] < 4.1


def test_draws_are_seeded():
    a = W.make_links(L, 0.3, 21)
    b = W.make_links(L, 0.3, 21)
    c = W.make_links(L, 0.3, 22)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])
    assert np.array_equal(W.make_sources(L, 3, 5), W.make_sources(L, 3, 5))
    assert not np.array_equal(W.make_sources(L, 3, 5), W.make_sources(L, 3, 6))


def test_sources_are_unit_complex_gaussians_per_part():
    b = W.make_sources((8, 8, 8, 8), 4, 31)
    assert b.shape == (2048, 3, 4) and b.dtype == np.complex128
    for part in (b.real, b.imag):
        assert abs(part.mean()) < 0.05
        assert abs(part.std() - 1.0) < 0.05


def test_noise_vectors():
    ze, zo = W.make_noise(L, 5, 41, "z2")
    assert ze.shape == zo.shape == (W.half_volume(L), 3, 5)
    for z in (ze, zo):
        assert np.all(z.imag == 0) and np.all(np.abs(z.real) == 1)
    assert 0.4 < (ze.real > 0).mean() < 0.6
    ge, go = W.make_noise(L, 5, 42, "gauss")
    for g in (ge, go):
        assert abs(np.mean(np.abs(g) ** 2) - 1.0) < 0.1


def test_seed_scheme():
    assert W.links_seed(3) == 3000 and W.links_seed(4, 2) == 4002
    assert W.sources_seed(3) == 3500 and W.sources_seed(4, 2) == 4502
