"""GPU half-Dslash (Sec. 1, eqs. (3)-(4)) against the FP64 CPU oracle.

FP64 within 1e-13 and FP32 (full or r14 Naik) within 1e-6 relative L2 per rhs,
for n = 1..8, both output parities, both field orders (site-major [Vh][3][n]
and colour-major [3][Vh][n]), every rhs-per-thread tile and work-group size, on
lattices with wrap aliasing (L = 4: x+3 = x-1; L = 6: x+3 = x-3) and with
ragged last tiles.
"""
import numpy as np
import pytest

import oracle
from paper_1411_4439_amd import workload as W
from tests.gpu_util import dev, gpu_lib, host, rel_l2_per_rhs, say

pytestmark = pytest.mark.gpu

LATTICES = [(4, 4, 4, 4), (6, 4, 6, 4), (8, 6, 4, 10), (16, 16, 16, 4)]
_cache = {}


def _links(H, L):
    if L not in _cache:
        U, N = W.make_links(L, 0.3, 7 + sum(L))
        _cache[L] = (U, N, H.Links(L, dev(U), dev(N), r13=True, r9=True))
    return _cache[L]


def _source(L, n, seed):
    return W.make_sources(L, n, seed)


def _apply(H, links, parity, v, prec, nk=0, layout=0):
    """Dslash of a site-major numpy field through the given field order; the
    result comes back site-major."""
    if layout == H.LAYOUT_COLOUR:
        got = H.dslash(links, parity, dev(np.ascontiguousarray(v.transpose(1, 0, 2))), prec, nk,
                       layout=layout)
        return np.ascontiguousarray(host(got).transpose(1, 0, 2))
    return host(H.dslash(links, parity, dev(v), prec, nk))


def _tiles(n):
    return [n // g for g in (1, 2, 4, 8) if n % g == 0]


@pytest.fixture(autouse=True)
def _reset_tuning():
    yield
    H = gpu_lib()
    H.hisq_set_tuning(0)


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_dslash_f64_all_tiles(L, n):
    H = gpu_lib()
    U, N, links = _links(H, L)
    for parity in (0, 1):
        v = _source(L, n, 100 + n + parity)
        want = oracle.dslash_eo(L, U, N, v, parity)
        outs = []
        for nr in _tiles(n):
            for bs, order in ((64, 0), (64, 2), (256, 1), (256, 2), (64, 3), (256, 3)):
                for lay in (H.LAYOUT_SITE, H.LAYOUT_COLOUR):
                    say("f64", L, n, parity, nr, bs, order, lay)
                    H.hisq_set_tuning(1, nr, bs, order)
                    got = _apply(H, links, parity, v, H.PREC_F64, layout=lay)
                    assert rel_l2_per_rhs(got, want) <= 1e-13, (nr, bs, order, lay)
                    outs.append(got)
        # the per-site arithmetic order depends on neither the tile, the tile
        # order nor the field order: bitwise equal
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("n", [1, 2, 4, 6, 7, 8])
@pytest.mark.parametrize("naik", ["full", "r14", "r13", "r9"])
def test_dslash_f32_all_tiles(L, n, naik):
    H = gpu_lib()
    U, N, links = _links(H, L)
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}.get(naik, H.NAIK_FULL)
    for parity in (0, 1):
        v = _source(L, n, 200 + n + parity).astype(np.complex64)
        want = oracle.dslash_eo(L, U, N, v.astype(np.complex128), parity)
        for nr in _tiles(n):
            for bs, order, lay in ((64, 2, 0), (128, 1, 0), (64, 2, 1), (128, 1, 1), (128, 3, 1)):
                say("f32", naik, L, n, parity, nr, bs, order, lay)
                H.hisq_set_tuning(1, nr, bs, order)
                got = _apply(H, links, parity, v, H.PREC_F32, nk, lay).astype(np.complex128)
                assert rel_l2_per_rhs(got, want) <= 1e-6, (nr, bs, order, lay)


@pytest.mark.parametrize("c", [1.0, -1.0 / 24.0])
def test_dslash_free_field_closed_form(c):
    """Unit links: plane waves are eigenvectors, lambda = 2i sum(sin p + c sin 3p)."""
    H = gpu_lib()
    L = (8, 4, 6, 4)
    U, N = W.free_links(L, c)
    links = H.Links(L, dev(U), dev(N))
    for k in [(1, 0, 0, 0), (2, 1, 3, 1), (7, 3, 5, 2)]:
        pw = W.plane_wave(L, k, [1.0, -0.5j, 0.25])
        lam = 2j * sum(np.sin(2 * np.pi * k[mu] / L[mu]) + c * np.sin(6 * np.pi * k[mu] / L[mu])
                       for mu in range(4))
        ve, vo = W.to_half(pw, L, 0), W.to_half(pw, L, 1)
        got = host(H.dslash(links, 1, dev(ve), H.PREC_F64))
        assert np.linalg.norm(got - lam * vo) <= 1e-13 * np.linalg.norm(vo)


def test_dslash_anti_hermitian_on_gpu():
    H = gpu_lib()
    L = (6, 4, 6, 4)
    U, N, links = _links(H, L)
    v = _source(L, 2, 301)
    w = _source(L, 2, 302)
    lhs = np.vdot(w, host(H.dslash(links, 0, dev(v), H.PREC_F64)))
    rhs = -np.vdot(host(H.dslash(links, 1, dev(w), H.PREC_F64)), v)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_dslash_autotuned_and_bundle_independence():
    H = gpu_lib()
    L = (16, 16, 16, 4)
    U, N, links = _links(H, L)
    v = _source(L, 8, 401)
    H.hisq_set_tuning(0)
    got = host(H.dslash(links, 0, dev(v), H.PREC_F64))
    for k in (0, 3, 7):
        single = host(H.dslash(links, 0, dev(np.ascontiguousarray(v[:, :, k:k + 1])), H.PREC_F64))
        assert np.array_equal(single[:, :, 0], got[:, :, k])


@pytest.mark.parametrize("naik", ["r14", "r13", "r9"])
def test_pack_rejects_non_unitary_naik(naik):
    H = gpu_lib()
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}[naik]
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 5)
    N = N.copy()
    N[2, 17] += 0.1 * np.eye(3) * 1j
    buf = H.empty_bytes(H.hisq_links_bytes(L, H.PREC_F32, nk))
    with pytest.raises(H.HisqError) as e:
        H.hisq_pack_links(L, dev(U), dev(N), H.PREC_F32, nk, buf)
    assert e.value.code == H.HISQ_EPACK


@pytest.mark.parametrize("naik", ["r14", "r13"])
def test_pack_rejects_naik_links_off_by_1e8(naik):
    """r14 / r13 fit row 2 from rows 0 and 1 in FP64: a Naik link that misses
    s*U(3) by 1e-8 of its norm is rejected, the synthetic links (exact to
    rounding) are accepted, and a buffer that failed packing is refused
    afterwards by the Dslash."""
    H = gpu_lib()
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13}[naik]
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 5)
    buf = H.empty_bytes(H.hisq_links_bytes(L, H.PREC_F32, nk))
    H.hisq_pack_links(L, dev(U), dev(N), H.PREC_F32, nk, buf)
    Nb = N.copy()
    Nb[1, 40, 2, 1] += 1e-8 * np.linalg.norm(N[1, 40])
    with pytest.raises(H.HisqError) as e:
        H.hisq_pack_links(L, dev(U), dev(Nb), H.PREC_F32, nk, buf)
    assert e.value.code == H.HISQ_EPACK
    v = dev(_source(L, 2, 11).astype(np.complex64))
    with pytest.raises(H.HisqError) as e:
        H.hisq_dslash(L, 1, 2, H.PREC_F32, nk, H.LAYOUT_SITE, buf, v, v.clone())
    assert e.value.code == H.HISQ_EINVAL


def test_entry_points_check_the_packed_link_header():
    """Links are only accepted for the lattice, precision and Naik storage they
    were packed for: a mismatch in any of them, or a buffer that holds no
    packed links, is HISQ_EINVAL before anything is launched, at the Dslash,
    the solver, the full-matrix solve, the mu-derivative Dslash and the batched
    solver; the matching call still works."""
    H = gpu_lib()
    import torch
    L, n = (8, 8, 4, 4), 2
    U, N = W.make_links(L, 0.3, 7)
    links = H.Links(L, dev(U), dev(N), r13=True)
    v64 = dev(_source(L, n, 12))
    v32 = v64.to(torch.complex64)
    bad = []
    # wrong Naik storage, precision, lattice; not a packed buffer at all
    junk = torch.zeros_like(links.f32r14)
    Lbig = (8, 8, 8, 4)
    vbig = dev(_source(Lbig, n, 13))
    for args in ((L, H.PREC_F32, H.NAIK_FULL, links.f32r14, v32),
                 (L, H.PREC_F32, H.NAIK_R14, links.f32r13, v32),
                 (L, H.PREC_F64, H.NAIK_FULL, links.f32, v64),
                 (L, H.PREC_F32, H.NAIK_FULL, links.f64, v32),
                 (L, H.PREC_F32, H.NAIK_R14, junk, v32),
                 (Lbig, H.PREC_F64, H.NAIK_FULL, links.f64, vbig.to(torch.complex128))):
        Lc, prec, nk, buf, vin = args
        with pytest.raises(H.HisqError) as e:
            H.hisq_dslash(Lc, 1, n, prec, nk, H.LAYOUT_SITE, buf, vin, vin.clone())
        bad.append(e.value.code)
    # solver: links32 packed r14 but params say r13; links64 given an FP32 buffer
    ws = H.empty_bytes(H.hisq_workspace_bytes(L, n, H.MODE_MIXED))
    x = torch.empty_like(v64)
    for l64, l32, nk in ((links.f64, links.f32r14, H.NAIK_R13), (links.f32, links.f32r14, H.NAIK_R14)):
        p = H.hisq_default_params(mode=H.MODE_MIXED, naik=nk)
        with pytest.raises(H.HisqError) as e:
            H.hisq_cg_solve(L, 0.1, n, p, l64, l32, v64, x, ws)
        bad.append(e.value.code)
    with pytest.raises(H.HisqError) as e:
        H.hisq_dslash_dmu(Lbig, 1, n, 1, links.f64, vbig, vbig.clone())
    bad.append(e.value.code)
    eo = dev(_source(L, n, 14))
    swapped = H.Links.__new__(H.Links)
    swapped.__dict__.update(links.__dict__)
    swapped.f32r14 = links.f32r13  # an r13 buffer handed over as r14
    with pytest.raises(H.HisqError) as e:
        H.solve_full(swapped, 0.1, v64, eo, mode=H.MODE_MIXED, naik=H.NAIK_R14)
    bad.append(e.value.code)
    prob = H.Problem(H.geom(L), 0.1, n, links.f64.data_ptr(), links.f32r13.data_ptr(),
                     v64.data_ptr(), x.data_ptr())
    p = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14)
    wsb = H.empty_bytes(H.hisq_batched_workspace_bytes([prob], H.MODE_MIXED))
    with pytest.raises(H.HisqError) as e:
        H.hisq_cg_solve_batched([prob], p, wsb)
    bad.append(e.value.code)
    say("rejections", bad)
    assert all(c == H.HISQ_EINVAL for c in bad), bad
    # the matching calls run
    out = H.dslash(links, 1, v32, H.PREC_F32, H.NAIK_R14)
    assert torch.isfinite(torch.view_as_real(out)).all()
    _, st, _ = H.solve(links, 0.1, v64, mode=H.MODE_MIXED, naik=H.NAIK_R13)
    assert st == H.HISQ_OK


def test_dslash_headline_lattice_sampled_sites():
    """48^3 x 12, n = 8, FP32 and r14, in the autotuned launch shape and the
    colour-major order the solver and the benchmark use (and site-major):
    sampled output sites against the oracle, and the whole output against the
    FP64 GPU Dslash of the same input."""
    H = gpu_lib()
    L = (48, 48, 48, 12)
    U, N = W.make_links(L, 0.2, W.links_seed(3))
    links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
    v = W.make_sources(L, 8, W.sources_seed(3))
    v32 = v.astype(np.complex64)
    rng = np.random.default_rng(9)
    odd = np.flatnonzero(~W.even_mask(L))
    sites = np.sort(rng.choice(odd, 2048, replace=False))
    sites = np.concatenate([odd[:64], sites, odd[-64:]])
    want = oracle.dslash_sites(L, U, N, v32.astype(np.complex128), 1, sites)
    ref64 = H.dslash(links, 1, dev(v), H.PREC_F64)
    assert rel_l2_per_rhs(host(ref64)[sites // 2], oracle.dslash_sites(L, U, N, v, 1, sites)) <= 1e-13
    H.hisq_set_tuning(0)
    for nk in (H.NAIK_FULL, H.NAIK_R14, H.NAIK_R13, H.NAIK_R9):
        for lay in (H.LAYOUT_SITE, H.LAYOUT_COLOUR):
            say("headline", nk, lay)
            g = _apply(H, links, 1, v32, H.PREC_F32, nk, lay).astype(np.complex128)
            assert rel_l2_per_rhs(g[sites // 2], want) <= 1e-6
            assert rel_l2_per_rhs(g, host(ref64)) <= 1e-6


def _staged_block(L, n, G, R, prec):
    """The library's rule for an LDS-staged tile (whole waves, <= 512 threads,
    R | L1, staged rows <= 64 KB); 0 where the tile is not possible."""
    Lh0 = L[0] // 2
    bs = R * Lh0 * G
    lds = 3 * (R + 6) * Lh0 * n * (16 if prec == 0 else 8)
    ok = bs % 64 == 0 and bs <= 512 and L[1] % R == 0 and lds <= 64 * 1024
    return bs if ok else 0


STAGED_LATTICES = [(16, 16, 16, 4), (8, 8, 8, 4), (4, 4, 4, 4), (32, 8, 8, 6)]


@pytest.mark.parametrize("L", STAGED_LATTICES)
@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_dslash_lds_staged_tiles(L, n):
    """LDS-staged Dslash (x and y neighbours from staged rows, periodic in y,
    rows wrapping onto themselves where L1 < rows + 6) in every valid tile and
    tile order, FP64 / FP32 / r14, bitwise equal to the unstaged kernel of the
    same precision (same per-site summation order)."""
    if not any(_staged_block(L, n, G, R, p) for G in (1, 2, 4, 8) if n % G == 0
               for R in range(1, 17) for p in (0, 1)):
        pytest.skip("no staged tile of whole waves fits this lattice and bundle")
    H = gpu_lib()
    U, N, links = _links(H, L)
    ran = 0
    for prec, nk, tol in ((H.PREC_F64, H.NAIK_FULL, 1e-13), (H.PREC_F32, H.NAIK_FULL, 1e-6),
                          (H.PREC_F32, H.NAIK_R14, 1e-6), (H.PREC_F32, H.NAIK_R13, 1e-6),
                          (H.PREC_F32, H.NAIK_R9, 1e-6)):
        for parity in (0, 1):
            v = _source(L, n, 500 + n + parity)
            if prec == H.PREC_F32:
                v = v.astype(np.complex64)
            want = oracle.dslash_eo(L, U, N, v.astype(np.complex128), parity)
            for nr in _tiles(n):
                G = n // nr
                H.hisq_set_tuning(1, nr, 64, 1, 0)
                plain = _apply(H, links, parity, v, prec, nk, H.LAYOUT_COLOUR)
                for R in range(1, 17):
                    if not _staged_block(L, n, G, R, prec):
                        continue
                    for order in (0, 1, 3):
                        say("staged", L, n, prec, nk, parity, nr, R, order)
                        H.hisq_set_tuning(1, nr, 64, order, R)
                        got = _apply(H, links, parity, v, prec, nk, H.LAYOUT_COLOUR)
                        assert rel_l2_per_rhs(got.astype(np.complex128), want) <= tol, (nr, R, order)
                        assert np.array_equal(got, plain), (nr, R, order)
                        ran += 1
    assert ran > 0


def test_pack_r9_rejects_mixed_naik_scales():
    """r9 stores one scale for the whole field: Naik links that are multiples of
    U(3) matrices with different scales are reported, not silently rescaled."""
    H = gpu_lib()
    L = (4, 4, 4, 4)
    U, N = W.make_links(L, 0.3, 5)
    N = N.copy()
    N[1, 3] *= 1.5
    buf = H.empty_bytes(H.hisq_links_bytes(L, H.PREC_F32, H.NAIK_R9))
    with pytest.raises(H.HisqError) as e:
        H.hisq_pack_links(L, dev(U), dev(N), H.PREC_F32, H.NAIK_R9, buf)
    assert e.value.code == H.HISQ_EPACK and "scale" in str(e.value)


def test_dslash_free_field_64x16_all_storages():
    """The paper's production lattice size (64^3 x 16, Vh = 2 097 152, three
    times the headline volume): with unit U and N = -1/24, plane waves are
    eigenvectors with lambda = 2i sum(sin p - sin 3p / 24), a property that
    holds at any size.  A two-rhs bundle of two momenta through the FP64, FP32,
    r14, r13 and r9 Dslash in the colour-major order the solver uses."""
    H = gpu_lib()
    import torch
    L, c = (64, 64, 64, 16), -1.0 / 24.0
    U, N = W.free_links(L, c)
    links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
    del U, N
    ks = [(1, 2, 3, 1), (63, 5, 32, 7)]
    vo = np.concatenate([W.to_half(W.plane_wave(L, k, [1.0, -0.5j, 0.25]), L, 1) for k in ks], axis=2)
    ve = np.concatenate([W.to_half(W.plane_wave(L, k, [1.0, -0.5j, 0.25]), L, 0) for k in ks], axis=2)
    lam = np.array([2j * sum(np.sin(2 * np.pi * k[mu] / L[mu]) + c * np.sin(6 * np.pi * k[mu] / L[mu])
                             for mu in range(4)) for k in ks])
    want = vo * lam[None, None, :]
    ved = torch.from_numpy(np.ascontiguousarray(ve.transpose(1, 0, 2))).cuda()
    for prec, nk, tol in ((H.PREC_F64, H.NAIK_FULL, 1e-13), (H.PREC_F32, H.NAIK_FULL, 1e-6),
                          (H.PREC_F32, H.NAIK_R14, 1e-6), (H.PREC_F32, H.NAIK_R13, 1e-6),
                          (H.PREC_F32, H.NAIK_R9, 1e-6)):
        vin = ved if prec == H.PREC_F64 else ved.to(torch.complex64)
        got = H.dslash(links, 1, vin, prec, nk, layout=H.LAYOUT_COLOUR)
        got = np.ascontiguousarray(host(got).transpose(1, 0, 2)).astype(np.complex128)
        err = rel_l2_per_rhs(got, want)
        say("64^3x16 free field", prec, nk, err)
        assert err <= tol, (prec, nk, err)
