"""GPU backward (adjoint CG + link force + dL/dm) against the oracle and
against finite differences; the torch.autograd.Function on top of it."""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1411_4439_amd import workload as W
from tests.gpu_util import dev, gpu_lib, host, say

pytestmark = pytest.mark.gpu


def _backward(H, L, U, N, m, x, phi, mode=0, naik=0, tol=1e-10):
    import torch
    n = x.shape[2]
    V = W.volume(L)
    links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
    gU = torch.empty((4, V, 3, 3), dtype=torch.complex128, device="cuda")
    gN = torch.empty_like(gU)
    gm = torch.zeros((), dtype=torch.float64, device="cuda")
    gb = torch.empty_like(dev(x))
    ws = H.empty_bytes(H.hisq_backward_workspace_bytes(L, n, mode))
    p = H.hisq_default_params(mode=mode, naik=naik, tol=tol)
    l32 = links.packed(H.PREC_F32, naik) if mode == H.MODE_MIXED else None
    status, info = H.hisq_cg_solve_backward(L, m, n, p, links.f64, l32, dev(x), dev(phi), gU, gN,
                                            gm, gb, ws)
    assert status == H.HISQ_OK, info.to_dict(n)
    return host(gU), host(gN), float(gm.item()), host(gb)


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 6, 4), (6, 6, 6, 6), (8, 8, 8, 4)])
@pytest.mark.parametrize("mode", [0, 1])
def test_force_matches_oracle(L, mode):
    """6^4 leaves a ragged last work-group (1296 sites, 32 per group); 8^3 x 4
    runs the XCD-ordered site blocks (z extent a multiple of 8)."""
    H = gpu_lib()
    m, n = 0.05, 3
    U, N = W.make_links(L, 0.3, 201)
    eta = W.make_sources(L, n, 202)
    phi = W.make_sources(L, n, 203)
    x, _ = oracle.cg(L, U, N, m, eta, tol=1e-13)
    y, _ = oracle.cg(L, U, N, m, phi, tol=1e-13)
    GU, GN, dm = oracle.force(L, U, N, m, x, y)
    gU, gN, gm, gb = _backward(H, L, U, N, m, x, phi, mode=mode, tol=1e-12)
    tol = 1e-8 if mode == 0 else 1e-7
    assert np.linalg.norm(gU - GU) <= tol * np.linalg.norm(GU)
    assert np.linalg.norm(gN - GN) <= tol * np.linalg.norm(GN)
    assert abs(gm - dm) <= tol * abs(dm)
    assert np.linalg.norm(gb - y) <= tol * np.linalg.norm(y)


@pytest.mark.parametrize("naik", ["r14", "r13", "r9"])
def test_force_mixed_compressed_naik(naik):
    """Mixed-precision backward with compressed FP32 Naik links: the adjoint
    solve runs on the compressed links, the force in FP64."""
    H = gpu_lib()
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}[naik]
    L, m, n = (4, 4, 4, 4), 0.05, 2
    U, N = W.make_links(L, 0.3, 211)
    eta = W.make_sources(L, n, 212)
    phi = W.make_sources(L, n, 213)
    x, _ = oracle.cg(L, U, N, m, eta, tol=1e-13)
    y, _ = oracle.cg(L, U, N, m, phi, tol=1e-13)
    GU, GN, dm = oracle.force(L, U, N, m, x, y)
    gU, gN, gm, gb = _backward(H, L, U, N, m, x, phi, mode=H.MODE_MIXED, naik=nk, tol=1e-12)
    say(naik, np.linalg.norm(gU - GU) / np.linalg.norm(GU))
    assert np.linalg.norm(gU - GU) <= 1e-7 * np.linalg.norm(GU)
    assert np.linalg.norm(gN - GN) <= 1e-7 * np.linalg.norm(GN)
    assert abs(gm - dm) <= 1e-7 * abs(dm)


def test_autograd_finite_differences():
    """HisqSolve through torch.autograd on 4^4, checked by central differences of
    L = sum Re(phi^dag x) evaluated with LAPACK (step 1e-6, Hermitian and
    anti-Hermitian link directions, and the mass)."""
    H = gpu_lib()
    import torch
    from paper_1411_4439_amd.autograd import HisqSolve
    L, m, n = (4, 4, 4, 4), 0.05, 2
    U, N = W.make_links(L, 0.3, 211)
    eta = W.make_sources(L, n, 212)
    phi = W.make_sources(L, n, 213)
    Ut = dev(U).requires_grad_(True)
    Nt = dev(N).requires_grad_(True)
    mt = torch.tensor(m, dtype=torch.float64, requires_grad=True)
    bt = dev(eta).requires_grad_(True)
    x = HisqSolve.apply(Ut, Nt, mt, bt, L, H.MODE_FP64, H.NAIK_FULL, 1e-12)
    loss = torch.real(torch.sum(torch.conj(dev(phi)) * x))
    loss.backward()
    gU, gN, gm, gb = host(Ut.grad), host(Nt.grad), float(mt.grad), host(bt.grad)

    def Lval(U_, N_, m_, b_):
        A = dense.even_normal_matrix(L, U_, N_, m_)
        xs = np.linalg.solve(A, b_.reshape(-1, n)).reshape(b_.shape)
        return float(np.real(np.vdot(phi, xs)))

    eps = 1e-6
    rng = np.random.default_rng(5)
    for d in range(8):
        Z = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        Hd = (Z + np.conj(np.swapaxes(Z, -1, -2))) / 2
        if d % 2:
            Hd = 1j * Hd
        for which, G in (("U", gU), ("N", gN)):
            if which == "U":
                fd = (Lval(U + eps * Hd, N, m, eta) - Lval(U - eps * Hd, N, m, eta)) / (2 * eps)
            else:
                fd = (Lval(U, N + eps * Hd, m, eta) - Lval(U, N - eps * Hd, m, eta)) / (2 * eps)
            pred = float(np.real(np.vdot(G, Hd)))
            say(which, d, fd, pred)
            assert abs(fd - pred) <= 1e-5 * max(abs(pred), 1e-3 * np.linalg.norm(G))
    fd = (Lval(U, N, m + eps, eta) - Lval(U, N, m - eps, eta)) / (2 * eps)
    assert abs(fd - gm) <= 1e-5 * abs(gm)
    db = rng.standard_normal(eta.shape) + 1j * rng.standard_normal(eta.shape)
    fd = (Lval(U, N, m, eta + eps * db) - Lval(U, N, m, eta - eps * db)) / (2 * eps)
    assert abs(fd - float(np.real(np.vdot(gb, db)))) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("mode", [0, 1])
def test_config5_gradient_24x6(mode):
    """24^3 x 6, n = 4, m = 0.05: the GPU force equals the oracle's force formula
    evaluated on the GPU's own x and y; the Euler identity (L is homogeneous of
    degree -2 in (U, N, m)) holds; the solves pass the oracle's true residual."""
    H = gpu_lib()
    L, m, n = (24, 24, 24, 6), 0.05, 4
    U, N = W.make_links(L, 0.3, W.links_seed(5))
    eta = W.make_sources(L, n, W.sources_seed(5))
    phi = W.make_sources(L, n, W.sources_seed(5, 1))
    links = H.Links(L, dev(U), dev(N))
    tol = 1e-12 if mode == 0 else 1e-11
    x, st, info = H.solve(links, m, dev(eta), mode=mode, tol=tol)
    assert st == H.HISQ_OK
    xh = host(x)
    gU, gN, gm, y = _backward(H, L, U, N, m, xh, phi, mode=mode, tol=tol)
    assert oracle.residual(L, U, N, m, eta, xh).max() <= tol * 1.0001
    assert oracle.residual(L, U, N, m, phi, y).max() <= tol * 1.0001
    GU, GN, dm = oracle.force(L, U, N, m, xh, y)
    assert np.linalg.norm(gU - GU) <= 1e-12 * np.linalg.norm(GU)
    assert np.linalg.norm(gN - GN) <= 1e-12 * np.linalg.norm(GN)
    assert abs(gm - dm) <= 1e-12 * abs(dm)
    loss = float(np.real(np.vdot(phi, xh)))
    euler = float(np.real(np.vdot(gU, U) + np.vdot(gN, N))) + m * gm
    say("euler", euler, -2 * loss)
    assert abs(euler + 2 * loss) <= 1e-6 * abs(loss)


@pytest.mark.parametrize("naik", ["r14", "r9"])
def test_autograd_mixed_compressed_naik(naik):
    """HisqSolve in mixed precision with compressed FP32 Naik links (the forward
    and adjoint solves iterate on them, the force runs in FP64): the gradients
    through torch.autograd equal the oracle's force for the oracle's x and y."""
    H = gpu_lib()
    import torch
    from paper_1411_4439_amd.autograd import HisqSolve
    nk = {"r14": H.NAIK_R14, "r9": H.NAIK_R9}[naik]
    L, m, n = (4, 4, 4, 4), 0.05, 2
    U, N = W.make_links(L, 0.3, 221)
    eta = W.make_sources(L, n, 222)
    phi = W.make_sources(L, n, 223)
    Ut = dev(U).requires_grad_(True)
    Nt = dev(N).requires_grad_(True)
    mt = torch.tensor(m, dtype=torch.float64, requires_grad=True)
    x = HisqSolve.apply(Ut, Nt, mt, dev(eta), L, H.MODE_MIXED, nk, 1e-12)
    loss = torch.real(torch.sum(torch.conj(dev(phi)) * x))
    loss.backward()
    xo, _ = oracle.cg(L, U, N, m, eta, tol=1e-13)
    yo, _ = oracle.cg(L, U, N, m, phi, tol=1e-13)
    GU, GN, dm = oracle.force(L, U, N, m, xo, yo)
    eU = np.linalg.norm(host(Ut.grad) - GU) / np.linalg.norm(GU)
    eN = np.linalg.norm(host(Nt.grad) - GN) / np.linalg.norm(GN)
    say(naik, eU, eN, float(mt.grad), dm)
    assert eU <= 1e-7 and eN <= 1e-7
    assert abs(float(mt.grad) - dm) <= 1e-7 * abs(dm)
