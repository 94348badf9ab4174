"""hisq_cg_solve_noalloc (scratch in a static device array, no allocation)
against hisq_cg_solve with a caller workspace, through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_1411_4439_amd import workload as W
from tests.gpu_util import dev, gpu_lib, host, say

pytestmark = pytest.mark.gpu


def _solve_both(H, L, m, n, mode, naik, seed):
    import torch
    U, N = W.make_links(L, 0.3, seed)
    links = H.Links(L, dev(U), dev(N))
    b = W.make_sources(L, n, seed + 1)
    bd = dev(b)
    l32 = links.packed(H.PREC_F32, naik) if mode == H.MODE_MIXED else None
    p = H.hisq_default_params(mode=mode, naik=naik)
    ws = H.empty_bytes(H.hisq_workspace_bytes(L, n, mode))
    x_ws = torch.empty_like(bd)
    st_ws, info_ws = H.hisq_cg_solve(L, m, n, p, links.f64, l32, bd, x_ws, ws)
    x_na = torch.empty_like(bd)
    st_na, info_na = H.hisq_cg_solve_noalloc(L, m, n, p, links.f64, l32, bd, x_na)
    torch.cuda.synchronize()
    return U, N, b, host(x_ws), st_ws, info_ws, host(x_na), st_na, info_na


def test_noalloc_matches_workspace_solve_twice():
    """Two calls in a row, the second on a smaller lattice and bundle (the
    static scratch keeps the first call's contents): each result equals the
    workspace solve of the same problem bit for bit (same kernels, tiles and
    fixed-order reductions) and passes the oracle's FP64 true residual."""
    H = gpu_lib()
    cases = [((16, 16, 16, 4), 0.05, 4, H.MODE_MIXED, H.NAIK_R14, 611),
             ((8, 8, 8, 4), 0.1, 2, H.MODE_FP64, H.NAIK_FULL, 621)]
    for L, m, n, mode, naik, seed in cases:
        U, N, b, x_ws, st_ws, i_ws, x_na, st_na, i_na = _solve_both(H, L, m, n, mode, naik, seed)
        say("noalloc", L, n, mode, list(i_na.iters[:n]), list(i_ws.iters[:n]))
        assert st_ws == st_na == H.HISQ_OK
        assert list(i_na.iters[:n]) == list(i_ws.iters[:n])
        assert np.array_equal(x_na, x_ws)
        assert oracle.residual(L, U, N, m, b, x_na).max() <= 1e-10


def test_noalloc_rejects_solves_beyond_its_scratch():
    """A solve whose workspace exceeds the static scratch is refused with
    HISQ_EWORKSPACE before anything is launched."""
    H = gpu_lib()
    import torch
    Ls = (8, 8, 8, 4)
    U, N = W.make_links(Ls, 0.3, 631)
    links = H.Links(Ls, dev(U), dev(N))
    Lbig, n = (32, 32, 32, 8), 8
    assert H.hisq_workspace_bytes(Lbig, n, H.MODE_MIXED) > 64 << 20
    b = torch.zeros((4, 3, n), dtype=torch.complex128, device="cuda")
    x = torch.empty_like(b)
    p = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14)
    with pytest.raises(H.HisqError) as e:
        H.hisq_cg_solve_noalloc(Lbig, 0.1, n, p, links.f64, links.f32r14, b, x)
    assert e.value.code == H.HISQ_EWORKSPACE
