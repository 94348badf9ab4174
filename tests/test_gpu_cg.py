"""GPU even-odd CG against the FP64 CPU oracle.

Gates: the true residual ||b - A x|| / ||b|| of the GPU solution, recomputed by
the oracle in FP64, is <= 1e-10 (the solver's tolerance); the solution matches
the oracle's (tol 1e-13) or LAPACK's within 1e-8, or within the a-posteriori
bound ||x - x*|| <= ||b - A x|| / (4 m^2) where the conditioning allows no more.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_1411_4439_amd import workload as W
from tests.gpu_util import dev, gpu_lib, host, rel_l2_per_rhs, say

pytestmark = pytest.mark.gpu


def _setup(H, L, eps, seed, n, sseed):
    U, N = W.make_links(L, eps, seed)
    links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
    b = W.make_sources(L, n, sseed)
    return U, N, links, b


def _check_solution(L, U, N, m, b, x, x_ref, tol=1e-10):
    res = oracle.residual(L, U, N, m, b, x)
    assert res.max() <= tol * 1.0001, res
    for k in range(b.shape[2]):
        err = np.linalg.norm(x[..., k] - x_ref[..., k]) / np.linalg.norm(x_ref[..., k])
        bound = res[k] * np.linalg.norm(b[..., k]) / (4 * m * m) / np.linalg.norm(x_ref[..., k])
        assert err <= max(1e-8, 2 * bound), (k, err, bound)


def test_config1_fp64_8x4():
    """8^4, m = 0.1, one rhs, plain FP64, stop at 1e-10."""
    H = gpu_lib()
    L, m = (8, 8, 8, 8), 0.1
    U, N, links, b = _setup(H, L, 0.3, W.links_seed(1), 1, W.sources_seed(1))
    x, status, info = H.solve(links, m, dev(b))
    say(info)
    assert status == H.HISQ_OK
    xo, oinfo = oracle.cg(L, U, N, m, b, tol=1e-13)
    _check_solution(L, U, N, m, b, host(x), xo)
    # same method, same stopping rule: iteration counts agree closely
    _, o10 = oracle.cg(L, U, N, m, b, tol=1e-10)
    assert abs(info["iters"][0] - o10["iters"][0]) <= 0.05 * o10["iters"][0] + 3


@pytest.mark.parametrize("mode,naik", [("fp64", "full"), ("mixed", "full"), ("mixed", "r14"),
                                       ("mixed", "r13"), ("mixed", "r9")])
@pytest.mark.parametrize("n", [1, 3, 4, 8])
def test_bundles_vs_lapack(mode, naik, n):
    """4^4 (wrap aliasing): every rhs against LAPACK's dense solve."""
    H = gpu_lib()
    L, m = (4, 4, 4, 4), 0.05
    U, N, links, b = _setup(H, L, 0.3, 21, n, 22 + n)
    md = H.MODE_MIXED if mode == "mixed" else H.MODE_FP64
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}.get(naik, H.NAIK_FULL)
    x, status, info = H.solve(links, m, dev(b), mode=md, naik=nk)
    say(mode, naik, n, info["iters"], info["reliable_updates"])
    assert status == H.HISQ_OK
    A = dense.even_normal_matrix(L, U, N, m)
    xd = np.linalg.solve(A, b.reshape(-1, n)).reshape(b.shape)
    _check_solution(L, U, N, m, b, host(x), xd)
    if mode == "mixed":
        assert info["reliable_updates"] >= 1


@pytest.mark.parametrize("mode,naik", [("fp64", "full"), ("mixed", "full"), ("mixed", "r14"),
                                       ("mixed", "r13"), ("mixed", "r9")])
def test_medium_lattice_small_mass(mode, naik):
    """16^3 x 4 (ragged tiles in every tile shape), m = 0.01, n = 5."""
    H = gpu_lib()
    L, m, n = (16, 16, 16, 4), 0.01, 5
    U, N, links, b = _setup(H, L, 0.3, 31, n, 32)
    md = H.MODE_MIXED if mode == "mixed" else H.MODE_FP64
    nk = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}.get(naik, H.NAIK_FULL)
    x, status, info = H.solve(links, m, dev(b), mode=md, naik=nk)
    say(mode, naik, info["iters"], info["reliable_updates"], info["rel_true_res"])
    assert status == H.HISQ_OK
    res = oracle.residual(L, U, N, m, b, host(x))
    assert res.max() <= 1e-10
    assert np.allclose(res, info["rel_true_res"], rtol=1e-3, atol=1e-14)


def test_mixed_matches_fp64_solution():
    H = gpu_lib()
    L, m, n = (8, 8, 8, 4), 0.02, 8
    U, N, links, b = _setup(H, L, 0.3, 41, n, 42)
    x64, s1, i1 = H.solve(links, m, dev(b), mode=H.MODE_FP64, tol=1e-12)
    xmx, s2, i2 = H.solve(links, m, dev(b), mode=H.MODE_MIXED, tol=1e-12)
    assert s1 == s2 == H.HISQ_OK
    assert rel_l2_per_rhs(host(xmx), host(x64)) <= 1e-8


def test_deterministic_and_graph_equals_stream():
    """Fixed-order FP64 reductions: repeated solves are bitwise identical, and
    the hipGraph path gives the same bits as plain stream launches."""
    H = gpu_lib()
    L, m, n = (8, 8, 8, 8), 0.05, 4
    U, N, links, b = _setup(H, L, 0.3, 51, n, 52)
    bd = dev(b)
    for mode in (H.MODE_FP64, H.MODE_MIXED):
        xa, _, _ = H.solve(links, m, bd, mode=mode)
        xb, _, _ = H.solve(links, m, bd, mode=mode)
        xc, _, _ = H.solve(links, m, bd, mode=mode, use_graph=0)
        assert np.array_equal(host(xa), host(xb))
        assert np.array_equal(host(xa), host(xc))


def test_profile_counts_launches():
    H = gpu_lib()
    L, m, n = (8, 8, 8, 4), 0.1, 2
    U, N, links, b = _setup(H, L, 0.3, 61, n, 62)
    for g in (1, 0):
        x, status, info = H.solve(links, m, dev(b), mode=H.MODE_MIXED, profile=1, use_graph=g)
        assert status == H.HISQ_OK
        launches = info["kernel_launches"]
        # a profiled solve runs without a graph; every iteration is timed
        assert launches[H.K_DSLASH_OE] == launches[H.K_DSLASH_EO] >= max(info["iters"])
        assert all(t > 0 for t in info["kernel_ms"][:3])
        assert launches[H.K_RELIABLE] == info["reliable_updates"] >= 1


def test_start_vector_zero_source_and_maxiter():
    H = gpu_lib()
    L, m = (4, 4, 4, 6), 0.1
    U, N, links, b = _setup(H, L, 0.3, 71, 3, 72)
    b[..., 1] = 0
    x0 = W.make_sources(L, 3, 73)  # non-zero start, also for the zero rhs
    x, status, info = H.solve(links, m, dev(b), x0=dev(x0))
    assert status == H.HISQ_OK
    xh = host(x)
    assert not np.any(xh[..., 1]), "b = 0 must give x = 0"
    assert oracle.residual(L, U, N, m, b, xh)[[0, 2]].max() <= 1e-10
    # restarting from the solution needs no iteration
    x2, status, info = H.solve(links, m, dev(b), x0=x)
    assert status == H.HISQ_OK and max(info["iters"]) == 0
    # maxiter cap: reported, and x is the last iterate
    x3, status, info = H.solve(links, m, dev(b), maxiter=5)
    assert status == H.HISQ_NOT_CONVERGED
    assert info["iters"][0] <= 5 and info["status"][0] == H.HISQ_NOT_CONVERGED
    assert info["status"][1] == H.HISQ_OK


def test_failure_paths_end_cleanly():
    """Singular and non-finite inputs end with a positive status, never a hang."""
    H = gpu_lib()
    L = (4, 4, 4, 4)
    U, N = W.free_links(L, 1.0)
    links = H.Links(L, dev(U), dev(N))
    b = W.to_half(W.plane_wave(L, (0, 0, 0, 0), [1.0, 0, 0]), L, 0)
    for mode in (H.MODE_FP64, H.MODE_MIXED):
        x, status, info = H.solve(links, 0.0, dev(b), mode=mode, maxiter=200)
        assert status in (H.HISQ_BREAKDOWN, H.HISQ_NOT_CONVERGED)
    U, N = W.make_links(L, 0.3, 81)
    links = H.Links(L, dev(U), dev(N))
    bn = W.make_sources(L, 2, 82)
    bn[3, 1, 0] = np.nan
    x, status, info = H.solve(links, 0.1, dev(bn), maxiter=100)
    assert status > 0 and info["status"][0] > 0


def test_batched_equals_separate_solves():
    """Several lattices, masses and bundle sizes in one batched launch per phase."""
    H = gpu_lib()
    import torch
    specs = [((8, 8, 8, 4), 3, 0.05), ((6, 6, 6, 4), 5, 0.01), ((8, 8, 4, 4), 8, 0.05),
             ((4, 4, 4, 4), 1, 0.1)]
    for mode, naik in ((H.MODE_MIXED, H.NAIK_FULL), (H.MODE_MIXED, H.NAIK_R14),
                       (H.MODE_MIXED, H.NAIK_R13), (H.MODE_MIXED, H.NAIK_R9),
                       (H.MODE_FP64, H.NAIK_FULL)):
        probs, keep, refs = [], [], []
        for j, (L, n, m) in enumerate(specs):
            U, N = W.make_links(L, 0.3, 90 + j)
            links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
            b = W.make_sources(L, n, 95 + j)
            bd = dev(b)
            x = torch.empty_like(bd)
            keep.append((links, bd, x, U, N, b))
            probs.append(H.Problem(H.geom(L), m, n, links.f64.data_ptr(),
                                   links.packed(H.PREC_F32, naik).data_ptr() if mode == H.MODE_MIXED else None,
                                   bd.data_ptr(), x.data_ptr()))
            refs.append(H.solve(links, m, bd, mode=mode, naik=naik)[0])
        p = H.hisq_default_params(mode=mode, naik=naik)
        ws = H.empty_bytes(H.hisq_batched_workspace_bytes(probs, mode))
        status, infos = H.hisq_cg_solve_batched(probs, p, ws)
        assert status == H.HISQ_OK
        for j, (L, n, m) in enumerate(specs):
            links, bd, x, U, N, b = keep[j]
            xh = host(x)
            res = oracle.residual(L, U, N, m, b, xh)
            say("batched", mode, naik, L, n, infos[j].iters[:n], res.max())
            assert res.max() <= 1e-10
            assert rel_l2_per_rhs(xh, host(refs[j])) <= 1e-7


@pytest.mark.parametrize("specs", [
    [((8, 8, 8, 4), 3, 0.05), ((4, 4, 4, 4), 1, 0.1)],           # 3 and 1 rhs per thread
    [((6, 6, 6, 4), 5, 0.01), ((8, 8, 8, 4), 3, 0.05)],           # 5 rhs per thread
    [((8, 8, 4, 4), 8, 0.05), ((6, 6, 6, 4), 5, 0.01)],           # 8 rhs per thread
])
def test_batched_builtin_tiles(specs):
    """Batches on the built-in tiles (every problem n rhs per thread, 128
    threads): 3 and 1, 5 and 3, 8 and 5 rhs per thread side by side, the
    lattices with z extent 8 on the XCD-ordered tile walk; each problem agrees
    with its own solve and reaches the oracle's residual."""
    H = gpu_lib()
    import torch
    H.hisq_set_tuning(2)
    try:
        probs, keep, refs = [], [], []
        for j, (L, n, m) in enumerate(specs):
            U, N = W.make_links(L, 0.3, 300 + j)
            links = H.Links(L, dev(U), dev(N), f32=False, r14=True)
            b = W.make_sources(L, n, 310 + j)
            bd = dev(b)
            x = torch.empty_like(bd)
            keep.append((U, N, b, x))
            probs.append(H.Problem(H.geom(L), m, n, links.f64.data_ptr(), links.f32r14.data_ptr(),
                                   bd.data_ptr(), x.data_ptr()))
            refs.append((links, bd, H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14)[0]))
        p = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14)
        ws = H.empty_bytes(H.hisq_batched_workspace_bytes(probs, H.MODE_MIXED))
        status, infos = H.hisq_cg_solve_batched(probs, p, ws)
        assert status == H.HISQ_OK
        for j, (L, n, m) in enumerate(specs):
            U, N, b, x = keep[j]
            xh = host(x)
            res = oracle.residual(L, U, N, m, b, xh)
            say("class batch", L, n, infos[j].iters[:n], res.max())
            assert res.max() <= 1e-10
            assert rel_l2_per_rhs(xh, host(refs[j][2])) <= 1e-7
    finally:
        H.hisq_set_tuning(0)


def test_headline_mixed_8rhs_true_residual():
    """48^3 x 12, m = 0.01, eps = 0.2, 8 rhs, in every precision form the
    benchmark times (mixed precision with r14, full, r13 and r9 Naik links, and
    FP64 throughout): the oracle's FP64 true residual of the returned x is
    <= 1e-10 for every rhs."""
    H = gpu_lib()
    L, m, n = (48, 48, 48, 12), 0.01, 8
    U, N = W.make_links(L, 0.2, W.links_seed(3))
    links = H.Links(L, dev(U), dev(N), r13=True, r9=True)
    b = W.make_sources(L, n, W.sources_seed(3))
    for mode, nk in ((H.MODE_MIXED, H.NAIK_R14), (H.MODE_MIXED, H.NAIK_FULL),
                     (H.MODE_MIXED, H.NAIK_R13), (H.MODE_MIXED, H.NAIK_R9),
                     (H.MODE_FP64, H.NAIK_FULL)):
        x, status, info = H.solve(links, m, dev(b), mode=mode, naik=nk)
        say("headline", mode, nk, info["iters"], info["reliable_updates"], info["seconds"])
        assert status == H.HISQ_OK
        res = oracle.residual(L, U, N, m, b, host(x))
        say("oracle true residual", res)
        assert res.max() <= 1e-10


def test_paper_lattice_64x16_mixed_8rhs_true_residual():
    """64^3 x 16, the size of the paper's production lattices, m = 0.01,
    eps = 0.2, 8 rhs, mixed precision with r14 Naik links and autotuned tiles
    (the benchmark's 64^3 x 16 block): the oracle's FP64 true residual of the
    returned x is <= 1e-10 for every rhs."""
    H = gpu_lib()
    L, m, n = (64, 64, 64, 16), 0.01, 8
    U, N = W.make_links(L, 0.2, W.links_seed(6))
    links = H.Links(L, dev(U), dev(N), f32=False, r14=True)
    b = W.make_sources(L, n, W.sources_seed(6))
    x, status, info = H.solve(links, m, dev(b), mode=H.MODE_MIXED, naik=H.NAIK_R14)
    say("64^3 x 16", info["iters"], info["reliable_updates"], info["seconds"])
    assert status == H.HISQ_OK
    res = oracle.residual(L, U, N, m, b, host(x))
    say("oracle true residual", res)
    assert res.max() <= 1e-10


def test_headline_solve_in_the_benchmark_launch_configuration():
    """48^3 x 12, n = 8, m = 0.01, mixed r14 with the tiles bench.py pins: the
    oracle's FP64 true residual of the returned x is <= 1e-10 for every rhs."""
    H = gpu_lib()
    import bench
    L, m, n = (48, 48, 48, 12), 0.01, 8
    U, N = W.make_links(L, 0.2, W.links_seed(3))
    links = H.Links(L, dev(U), dev(N))
    b = W.make_sources(L, n, W.sources_seed(3))
    nr, order, rows = (int(v) for v in bench.DEFAULT_TILE.split(","))
    try:
        H.hisq_set_tuning(1, nr, 64, order, rows)
        H.hisq_set_tuning_eo(*(int(v) for v in bench.DEFAULT_TILE_EO.split(",")))
        x, status, info = H.solve(links, m, dev(b), mode=H.MODE_MIXED, naik=H.NAIK_R14)
    finally:
        H.hisq_set_tuning(0)
    say("bench tiles", info["rhs_per_thread"], info["block_size"], info["stage_rows"],
        info["eo_rhs_per_thread"], info["eo_block_size"], info["iters"])
    assert status == H.HISQ_OK
    assert (info["rhs_per_thread"], info["stage_rows"]) == (nr, rows)
    res = oracle.residual(L, U, N, m, b, host(x))
    say("oracle true residual", res)
    assert res.max() <= 1e-10


def test_lds_staged_solve_matches_unstaged():
    """A mixed-precision solve forced onto LDS-staged Dslash tiles reports the
    staged shape and returns the same bits as the unstaged tiles (the staged
    kernel sums the 16 slots in the same order)."""
    H = gpu_lib()
    L, m, n = (16, 16, 16, 4), 0.02, 8
    U, N, links, b = _setup(H, L, 0.3, 61, n, 62)
    bd = dev(b)
    try:
        H.hisq_set_tuning(1, 4, 64, 3, 0)
        x0, s0, i0 = H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14)
        H.hisq_set_tuning(1, 4, 64, 3, 4)
        x1, s1, i1 = H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14)
    finally:
        H.hisq_set_tuning(0)
    say(i0["stage_rows"], i1["stage_rows"], i1["block_size"], i1["iters"])
    assert s0 == s1 == H.HISQ_OK
    assert i0["stage_rows"] == 0 and i1["stage_rows"] == 4 and i1["block_size"] == 4 * 8 * 2
    assert np.array_equal(host(x0), host(x1))
    res = oracle.residual(L, U, N, m, b, host(x1))
    assert res.max() <= 1e-10


def test_wide_staged_tile_with_unstaged_kernels():
    """A forced LDS-staged FP32 Dslash tile of 384 threads (6 rhs, 3 per
    thread, 16 staged rows of a 24 x 16 x 8 x 4 lattice) is wider than the
    p-update and batched kernels are built for: those fall back to an unstaged
    tile, the single solve still reports the staged tile, and single and
    batched mixed-precision solves converge."""
    H = gpu_lib()
    import torch
    m = 0.05
    L, n = (24, 16, 8, 4), 6
    U, N, links, b = _setup(H, L, 0.3, 71, n, 72)
    L2, n2 = (8, 8, 8, 4), 3
    U2, N2, links2, b2 = _setup(H, L2, 0.3, 73, n2, 74)
    bd, bd2 = dev(b), dev(b2)
    try:
        H.hisq_set_tuning(1, 3, 64, 3, 16)
        x, s, info = H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14)
        say("wide staged single", info["block_size"], info["stage_rows"], info["iters"])
        assert s == H.HISQ_OK
        assert info["block_size"] == 16 * 12 * 2 and info["stage_rows"] == 16
        assert oracle.residual(L, U, N, m, b, host(x)).max() <= 1e-10
        xs = [torch.empty_like(bd), torch.empty_like(bd2)]
        probs = [H.Problem(H.geom(Lq), m, nq, lq.f64.data_ptr(),
                           lq.packed(H.PREC_F32, H.NAIK_R14).data_ptr(), bq.data_ptr(),
                           xq.data_ptr())
                 for Lq, nq, lq, bq, xq in ((L, n, links, bd, xs[0]), (L2, n2, links2, bd2, xs[1]))]
        p = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14)
        ws = H.empty_bytes(H.hisq_batched_workspace_bytes(probs, H.MODE_MIXED))
        s, infos = H.hisq_cg_solve_batched(probs, p, ws)
        say("wide staged batched", infos[0].block_size)
        assert s == H.HISQ_OK and 64 <= infos[0].block_size <= 256
        for Lq, Uq, Nq, bq, xq in ((L, U, N, b, xs[0]), (L2, U2, N2, b2, xs[1])):
            assert oracle.residual(Lq, Uq, Nq, m, bq, host(xq)).max() <= 1e-10
    finally:
        H.hisq_set_tuning(0)


def test_separate_tile_for_the_cg_epilogue_kernel():
    """The D_eo kernel with the CG epilogue takes a tile of its own: forced
    (LDS-staged D_oe, unstaged 2-rhs D_eo) and autotuned, both reported in the
    info, and the solves reach the oracle's true residual."""
    H = gpu_lib()
    L, m, n = (16, 16, 16, 4), 0.02, 8
    U, N, links, b = _setup(H, L, 0.3, 81, n, 82)
    bd = dev(b)
    try:
        H.hisq_set_tuning(1, 4, 64, 3, 4)
        H.hisq_set_tuning_eo(2, 256, 3, 0)
        x, s, info = H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14)
        say("forced", info["block_size"], info["stage_rows"], info["eo_block_size"],
            info["eo_rhs_per_thread"], info["iters"])
        assert s == H.HISQ_OK
        assert (info["rhs_per_thread"], info["stage_rows"]) == (4, 4)
        assert (info["eo_rhs_per_thread"], info["eo_block_size"], info["eo_stage_rows"]) == (2, 256, 0)
        assert oracle.residual(L, U, N, m, b, host(x)).max() <= 1e-10
        H.hisq_set_tuning(0)
        for mode in (H.MODE_MIXED, H.MODE_FP64):
            x, s, info = H.solve(links, m, bd, mode=mode, naik=H.NAIK_R14)
            say("autotuned", mode, info)
            assert s == H.HISQ_OK
            assert info["eo_block_size"] >= 64 and n % info["eo_rhs_per_thread"] == 0
            assert oracle.residual(L, U, N, m, b, host(x)).max() <= 1e-10
    finally:
        H.hisq_set_tuning(0)


def test_config2_32x8_fp64_vs_mixed_bundles():
    """32^3 x 8, m = 0.02, complex Gaussian sources, bundles of 1, 2, 4 and 8:
    plain FP64 against FP32 storage (r14 Naik) with FP64 reliable updates, both
    to true residual 1e-10 (recomputed by the oracle), solutions within 1e-8
    of each other or the a-posteriori bound."""
    H = gpu_lib()
    L, m = (32, 32, 32, 8), 0.02
    U, N = W.make_links(L, 0.3, W.links_seed(2))
    links = H.Links(L, dev(U), dev(N))
    b8 = W.make_sources(L, 8, W.sources_seed(2))
    for n in (1, 2, 4, 8):
        b = np.ascontiguousarray(b8[:, :, :n])
        x64, s64, i64 = H.solve(links, m, dev(b), mode=H.MODE_FP64)
        xmx, smx, imx = H.solve(links, m, dev(b), mode=H.MODE_MIXED, naik=H.NAIK_R14)
        say("config2 n=%d" % n, "fp64", i64["iters"], "%.3f s" % i64["seconds"],
            "mixed", imx["iters"], imx["reliable_updates"], "%.3f s" % imx["seconds"])
        assert s64 == smx == H.HISQ_OK
        r64 = oracle.residual(L, U, N, m, b, host(x64))
        rmx = oracle.residual(L, U, N, m, b, host(xmx))
        assert r64.max() <= 1e-10 and rmx.max() <= 1e-10
        _check_solution(L, U, N, m, b, host(xmx), host(x64))


def test_concurrent_solves_from_two_threads():
    """Two host threads, each with its own stream, workspace and problem, solve
    at the same time (per-thread capture streams and host state, a shared
    autotune cache); each result equals the same solve run alone, bit for bit."""
    H = gpu_lib()
    import threading
    import torch
    cases = [((8, 8, 8, 4), 0.05, 4, 301), ((6, 6, 6, 4), 0.02, 3, 302)]
    inputs = []
    for L, m, n, seed in cases:
        U, N = W.make_links(L, 0.3, seed)
        links = H.Links(L, dev(U), dev(N))
        b = dev(W.make_sources(L, n, seed + 10))
        inputs.append((L, m, n, links, b, U, N))
    ref = [host(H.solve(links, m, b, mode=H.MODE_MIXED, naik=H.NAIK_R14)[0])
           for L, m, n, links, b, U, N in inputs]
    torch.cuda.synchronize()
    got, errors = [None, None], []

    def run(j):
        try:
            L, m, n, links, b, U, N = inputs[j]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    x, st, info = H.solve(links, m, b, mode=H.MODE_MIXED, naik=H.NAIK_R14,
                                          stream=s.cuda_stream)
                    assert st == H.HISQ_OK
                s.synchronize()
                got[j] = host(x)
        except Exception as e:  # reported in the main thread
            errors.append(repr(e))

    threads = [threading.Thread(target=run, args=(j,)) for j in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors, errors
    for j in range(2):
        assert got[j] is not None and np.array_equal(got[j], ref[j]), j


def test_batched_workload_at_its_own_sizes():
    """The batched workload exactly as the benchmark runs it: 16^3 x 4 (3 rhs),
    24^3 x 6 (5 rhs) and 32^3 x 8 (8 rhs), each at m = 0.05 and 0.01, links
    with eps = 0.3, the benchmark's seeds, mixed precision with r14 Naik links,
    all six in one batched solve.  Every rhs reaches the oracle's FP64 true
    residual <= 1e-10, and every solution agrees with the same problem solved
    on its own within 1e-7 (or the a-posteriori bound of the two residuals)."""
    H = gpu_lib()
    import torch
    probs, keep = [], []
    j = 0
    for L, n in W.BATCHED_PROBLEMS:
        for m in W.BATCHED_MASSES:
            U, N = W.make_links(L, 0.3, W.links_seed(4, j))
            links = H.Links(L, dev(U), dev(N), f32=False, r14=True)
            b = W.make_sources(L, n, W.sources_seed(4, j))
            bd = dev(b)
            x = torch.empty_like(bd)
            keep.append((L, n, m, U, N, b, links, bd, x))
            probs.append(H.Problem(H.geom(L), m, n, links.f64.data_ptr(),
                                   links.f32r14.data_ptr(), bd.data_ptr(), x.data_ptr()))
            j += 1
    p = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14)
    ws = H.empty_bytes(H.hisq_batched_workspace_bytes(probs, H.MODE_MIXED))
    status, infos = H.hisq_cg_solve_batched(probs, p, ws)
    say("batched workload", status, [i.total_iters for i in infos])
    assert status == H.HISQ_OK
    for j, (L, n, m, U, N, b, links, bd, x) in enumerate(keep):
        xb = host(x)
        res = oracle.residual(L, U, N, m, b, xb)
        xs, st, info = H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14)
        assert st == H.HISQ_OK
        xs = host(xs)
        rs = oracle.residual(L, U, N, m, b, xs)
        say("problem", j, L, n, m, "true residual", res.max(), "separate", rs.max())
        assert res.max() <= 1e-10, (j, res)
        for k in range(n):
            err = np.linalg.norm(xb[..., k] - xs[..., k]) / np.linalg.norm(xs[..., k])
            # both solutions are within ||b - A x|| / (4 m^2) of the exact one
            bound = (res[k] + rs[k]) * np.linalg.norm(b[..., k]) / (4 * m * m) / np.linalg.norm(xs[..., k])
            assert err <= max(1e-7, bound), (j, k, err, bound)
