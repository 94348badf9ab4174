"""GPU full-matrix solve (M = 2m + D through the even-odd reduction), the
mu-derivative Dslash and the trace estimator of Sec. 1 eq. (2), against the
FP64 CPU oracle (and LAPACK / the exact trace on 4^4)."""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1411_4439_amd import workload as W
from tests.gpu_util import dev, gpu_lib, host, rel_l2_per_rhs, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 6, 6), (8, 6, 4, 10)])
@pytest.mark.parametrize("n", [1, 3, 8])
def test_dslash_dmu_vs_oracle(L, n):
    H = gpu_lib()
    U, N = W.make_links(L, 0.3, 70 + sum(L))
    links = H.Links(L, dev(U), dev(N))
    for nder in (0, 1, 2, 3, 4):
        for par in (0, 1):
            v = W.make_sources(L, n, 80 + nder + par)
            say("dmu", L, n, nder, par)
            got = host(H.dslash_dmu(links, par, dev(v), nder))
            want = oracle.dslash_dmu(L, U, N, v, par, nder)
            assert rel_l2_per_rhs(got, want) <= 1e-13, (nder, par)


@pytest.mark.parametrize("mode,naik", [("fp64", "full"), ("mixed", "r14"), ("mixed", "r13"),
                                       ("mixed", "r9")])
def test_solve_full_vs_lapack(mode, naik):
    H = gpu_lib()
    L, m, n = (4, 4, 4, 4), 0.1, 3
    U, N = W.make_links(L, 0.3, 90)
    links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
    b_e, b_o = W.make_noise(L, n, 91, "gauss")
    md = H.MODE_MIXED if mode == "mixed" else H.MODE_FP64
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}.get(naik, H.NAIK_FULL)
    x_e, x_o, st, info = H.solve_full(links, m, dev(b_e), dev(b_o), mode=md, naik=nk)
    say(mode, info["iters"])
    assert st == H.HISQ_OK
    M = dense.fermion_matrix(L, U, N, m)
    e, o = dense.parity_indices(L, 0), dense.parity_indices(L, 1)
    b = np.zeros((M.shape[0], n), dtype=np.complex128)
    b[e], b[o] = b_e.reshape(-1, n), b_o.reshape(-1, n)
    x = np.linalg.solve(M, b)
    got = np.zeros_like(x)
    got[e], got[o] = host(x_e).reshape(-1, n), host(x_o).reshape(-1, n)
    for k in range(n):
        assert np.linalg.norm(got[:, k] - x[:, k]) <= 1e-8 * np.linalg.norm(x[:, k])


def test_solve_full_residual_medium_lattice():
    """16^3 x 4, m = 0.02, n = 8, mixed precision: ||b - M x|| / ||b|| from the
    oracle's M, and the even part against the oracle's own full solve."""
    H = gpu_lib()
    L, m, n = (16, 16, 16, 4), 0.02, 8
    U, N = W.make_links(L, 0.3, 92)
    links = H.Links(L, dev(U), dev(N))
    b_e, b_o = W.make_noise(L, n, 93, "z2")
    x_e, x_o, st, info = H.solve_full(links, m, dev(b_e), dev(b_o), mode=H.MODE_MIXED,
                                      naik=H.NAIK_R14)
    assert st == H.HISQ_OK
    xe, xo = host(x_e), host(x_o)
    y_e, y_o = oracle.apply_M(L, U, N, m, xe, xo)
    for k in range(n):
        r = np.sqrt(np.linalg.norm(y_e[..., k] - b_e[..., k]) ** 2 + np.linalg.norm(y_o[..., k] - b_o[..., k]) ** 2)
        bn = np.sqrt(np.linalg.norm(b_e[..., k]) ** 2 + np.linalg.norm(b_o[..., k]) ** 2)
        # the even solve stops at 1e-10 relative on the reduced system; M's
        # residual is bounded by it up to the norm of the reduction
        assert r / bn <= 1e-8, (k, r / bn)
    oe, oo, _ = oracle.solve_full(L, U, N, m, b_e, b_o, tol=1e-12)
    assert rel_l2_per_rhs(xe, oe) <= 1e-7
    assert rel_l2_per_rhs(xo, oo) <= 1e-7


@pytest.mark.parametrize("orders", [(1,), (2,), (1, 1), (0,), (2, 1)])
def test_trace_estimate_vs_oracle(orders):
    H = gpu_lib()
    L, m, n = (8, 8, 8, 4), 0.05, 8
    U, N = W.make_links(L, 0.3, 94)
    links = H.Links(L, dev(U), dev(N))
    eta_e, eta_o = W.make_noise(L, n, 95, "z2")
    got, st, info = H.trace_estimate(links, m, orders, dev(eta_e), dev(eta_o), mode=H.MODE_MIXED,
                                     naik=H.NAIK_R14, tol=1e-12)
    say(orders, info["total_iters"], got[:2])
    assert st == H.HISQ_OK
    want = oracle.trace_estimate(L, U, N, m, orders, eta_e, eta_o, tol=1e-13)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-8 * scale, (got, want)


def test_trace_estimate_exact_on_unit_basis():
    """4^4: with the complete unit basis as noise (96 bundles of 8) the terms sum
    to Tr(M' M^-1 M' M^-1) from dense LAPACK."""
    H = gpu_lib()
    L, m = (4, 4, 4, 4), 0.15
    U, N = W.make_links(L, 0.3, 96)
    links = H.Links(L, dev(U), dev(N))
    M = dense.fermion_matrix(L, U, N, m)
    Mp = dense.dslash_dmu_matrix(L, U, N, 1)
    Minv = np.linalg.inv(M)
    exact = np.trace(Mp @ Minv @ Mp @ Minv)
    e, o = dense.parity_indices(L, 0), dense.parity_indices(L, 1)
    dim = M.shape[0]
    ws = H.empty_bytes(H.hisq_trace_workspace_bytes(L, 8, H.MODE_FP64))
    total = 0j
    for start in range(0, dim, 8):
        basis = np.zeros((dim, 8), dtype=np.complex128)
        basis[np.arange(start, start + 8), np.arange(8)] = 1.0
        eta_e = np.ascontiguousarray(basis[e].reshape(-1, 3, 8))
        eta_o = np.ascontiguousarray(basis[o].reshape(-1, 3, 8))
        got, st, _ = H.trace_estimate(links, m, (1, 1), dev(eta_e), dev(eta_o), ws=ws, tol=1e-12)
        assert st == H.HISQ_OK
        total += got.sum()
    say(total, exact)
    assert abs(total - exact) <= 1e-8 * max(1.0, abs(exact))
