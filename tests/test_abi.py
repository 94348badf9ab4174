"""The C ABI without a GPU: the library loads, exports every entry point that
include/hisq.h declares, and its host-only logic (size queries, argument and
geometry checks) behaves as documented.  No call here launches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hisq.h")


@pytest.fixture(scope="module")
def H():
    from paper_1411_4439_amd import hisq
    return hisq


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(hisq_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("hisq_dslash", "hisq_cg_solve", "hisq_cg_solve_backward", "hisq_solve_full",
                     "hisq_dslash_dmu", "hisq_trace_estimate",
                     "hisq_cg_solve_batched", "hisq_pack_links", "hisq_links_bytes",
                     "hisq_workspace_bytes", "hisq_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(H):
    lib = ctypes.CDLL(H.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared_functions()) == set(H.EXPORTS)


def test_struct_layouts_match_header(H):
    # sizes follow the C declarations (natural alignment)
    assert ctypes.sizeof(H.Geom) == 16
    assert ctypes.sizeof(H.Params) == 48
    assert ctypes.sizeof(H.Problem) == 16 + 8 + 8 + 4 * 8
    # five timed kernel classes; 4 bytes of tail padding to the struct's 8-byte alignment
    assert ctypes.sizeof(H.Info) == 8 * 4 * 2 + 8 * 8 * 2 + 12 * 4 + 8 + 5 * 8 + 5 * 4 + 4


def test_default_params(H):
    p = H.hisq_default_params()
    assert p.mode == H.MODE_FP64 and p.tol == 1e-10 and p.maxiter == 20000
    assert p.delta == 0.1 and p.use_graph == 1 and p.use_x0 == 0


def test_links_bytes(H):
    L = (8, 8, 8, 8)
    Vh = 8 ** 4 // 2
    assert H.hisq_links_bytes(L, H.PREC_F64, H.NAIK_FULL) == 256 + 2 * 144 * Vh * 16
    assert H.hisq_links_bytes(L, H.PREC_F32, H.NAIK_FULL) == 256 + 2 * 144 * Vh * 8
    assert H.hisq_links_bytes(L, H.PREC_F32, H.NAIK_R14) == 256 + 2 * 128 * Vh * 8
    # r13: 8 U slots of 18 reals, 8 Naik slots of 13, four bytes each
    assert H.hisq_links_bytes(L, H.PREC_F32, H.NAIK_R13) == 256 + 2 * (8 * 18 + 8 * 13) * Vh * 4
    assert H.hisq_links_bytes(L, H.PREC_F32, H.NAIK_R9) == 256 + 2 * (8 * 18 + 8 * 9) * Vh * 4
    # r14 is an FP32 format; odd or small extents are rejected
    assert H.hisq_links_bytes(L, H.PREC_F64, H.NAIK_R14) == 0
    assert H.hisq_links_bytes(L, H.PREC_F64, H.NAIK_R13) == 0
    assert H.hisq_links_bytes(L, H.PREC_F32, 4) == 0
    assert H.hisq_links_bytes((8, 8, 8, 7), H.PREC_F64, H.NAIK_FULL) == 0
    assert H.hisq_links_bytes((2, 8, 8, 8), H.PREC_F64, H.NAIK_FULL) == 0


def test_workspace_bytes(H):
    L = (8, 8, 8, 8)
    w64 = H.hisq_workspace_bytes(L, 4, H.MODE_FP64)
    wmx = H.hisq_workspace_bytes(L, 4, H.MODE_MIXED)
    Vh = 8 ** 4 // 2
    assert w64 >= 3 * Vh * 3 * 4 * 16
    assert wmx >= 2 * Vh * 3 * 4 * 16 + 4 * Vh * 3 * 4 * 8
    assert H.hisq_backward_workspace_bytes(L, 4, H.MODE_FP64) >= w64 + 3 * Vh * 3 * 4 * 16
    assert H.hisq_workspace_bytes(L, 0, H.MODE_FP64) == 0
    assert H.hisq_workspace_bytes(L, 9, H.MODE_FP64) == 0
    assert H.hisq_workspace_bytes(L, 1, 7) == 0
    wf = H.hisq_full_workspace_bytes(L, 4, H.MODE_MIXED)
    assert wf >= wmx + 2 * Vh * 3 * 4 * 16
    assert H.hisq_trace_workspace_bytes(L, 4, H.MODE_MIXED) >= wf + 4 * Vh * 3 * 4 * 16


def test_errors_before_any_launch(H):
    """Invalid calls return a negative code and a message without touching a GPU."""
    lib = H._lib
    g = H.geom((8, 8, 8, 6))
    bad = H.geom((8, 8, 5, 6))
    p = H.hisq_default_params()
    info = H.Info()
    fake = ctypes.c_void_p(0x1000)
    rc = lib.hisq_cg_solve(ctypes.byref(bad), 0.1, 1, ctypes.byref(p), fake, None, fake, fake,
                           fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EGEOM and "L[2]" in H.hisq_last_error()
    rc = lib.hisq_cg_solve(ctypes.byref(g), 0.1, 9, ctypes.byref(p), fake, None, fake, fake,
                           fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL
    p.tol = 0.0
    rc = lib.hisq_cg_solve(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, fake, fake,
                           fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL
    p = H.hisq_default_params(mode=H.MODE_MIXED)
    rc = lib.hisq_cg_solve(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, fake, fake,
                           fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL and "FP32" in H.hisq_last_error()
    p = H.hisq_default_params()
    rc = lib.hisq_cg_solve(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, fake, fake,
                           fake, 16, ctypes.byref(info), None)
    assert rc == H.HISQ_EWORKSPACE
    rc = lib.hisq_dslash(ctypes.byref(g), 2, 1, H.PREC_F64, H.NAIK_FULL, 0, fake, fake, fake, None)
    assert rc == H.HISQ_EINVAL
    rc = lib.hisq_dslash(ctypes.byref(g), 0, 1, H.PREC_F64, H.NAIK_FULL, 2, fake, fake, fake, None)
    assert rc == H.HISQ_EINVAL and "layout" in H.hisq_last_error()
    rc = lib.hisq_pack_links(ctypes.byref(g), fake, fake, H.PREC_F64, H.NAIK_R14, fake, None)
    assert rc == H.HISQ_EINVAL
    rc = lib.hisq_cg_solve_batched(0, None, ctypes.byref(p), fake, 0, None, None)
    assert rc == H.HISQ_EINVAL
    # 16-byte alignment of every field, link and workspace buffer
    odd = ctypes.c_void_p(0x1008)
    rc = lib.hisq_dslash(ctypes.byref(g), 0, 1, H.PREC_F64, H.NAIK_FULL, 0, fake, odd, fake, None)
    assert rc == H.HISQ_EINVAL and "aligned" in H.hisq_last_error()
    rc = lib.hisq_cg_solve(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, fake, fake,
                           odd, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL and "aligned" in H.hisq_last_error()
    # full solve and trace estimator: mass 0 cannot give x_o; bad insertion lists
    rc = lib.hisq_solve_full(ctypes.byref(g), 0.0, 1, ctypes.byref(p), fake, None, fake, fake, fake,
                             fake, fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL and "mass" in H.hisq_last_error()
    orders = (ctypes.c_int * 2)(1, 9)
    rc = lib.hisq_trace_estimate(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, 2, orders,
                                 fake, fake, fake, fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL and "orders[1]" in H.hisq_last_error()
    rc = lib.hisq_trace_estimate(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, 0, orders,
                                 fake, fake, fake, fake, 1 << 30, ctypes.byref(info), None)
    assert rc == H.HISQ_EINVAL
    rc = lib.hisq_dslash_dmu(ctypes.byref(g), 0, 1, -1, fake, fake, fake, None)
    assert rc == H.HISQ_EINVAL
    rc = lib.hisq_solve_full(ctypes.byref(g), 0.1, 1, ctypes.byref(p), fake, None, fake, fake, fake,
                             fake, fake, 16, ctypes.byref(info), None)
    assert rc == H.HISQ_EWORKSPACE


def test_tuning_control(H):
    assert H.hisq_set_tuning(2) == 0
    with pytest.raises(H.HisqError):
        H.hisq_set_tuning(1, 3, 100, 1)
    with pytest.raises(H.HisqError):
        H.hisq_set_tuning(5)
    with pytest.raises(H.HisqError):
        H.hisq_set_tuning(1, 4, 64, 3, -1)
    assert H.hisq_set_tuning(1, 4, 64, 3, 8) == 0
    assert H.hisq_set_tuning_eo(2, 256, 3, 0) == 0
    with pytest.raises(H.HisqError):
        H.hisq_set_tuning_eo(2, 96, 3, 0)
    with pytest.raises(H.HisqError):
        H.hisq_set_tuning_eo(9, 64, 3, 0)
    assert H.hisq_set_tuning_eo(0) == 0
    assert H.hisq_set_tuning(0) == 0


def test_solver_refuses_host_tensors(H):
    import torch
    L = (4, 4, 4, 4)
    b = torch.zeros((128, 3, 1), dtype=torch.complex128)
    with pytest.raises(ValueError):
        H.hisq_dslash(L, 0, 1, H.PREC_F64, H.NAIK_FULL, H.LAYOUT_SITE,
                      torch.zeros(16, dtype=torch.uint8), b, b)


def test_lattice_size_limit(H):
    """Packed links are indexed with 32-bit offsets per parity block (144
    complex numbers per site): a lattice with V/2 * 144 >= 2^31 is refused
    before any launch, and the largest production-style shapes below it are
    accepted."""
    lib = H._lib
    fake = ctypes.c_void_p(0x1000)
    big = H.geom((128, 128, 128, 16))          # V/2 * 144 = 2.4e9
    rc = lib.hisq_dslash(ctypes.byref(big), 0, 1, H.PREC_F64, H.NAIK_FULL, 0, fake, fake, fake, None)
    assert rc == H.HISQ_EGEOM and "too large" in H.hisq_last_error()
    assert H.hisq_links_bytes((128, 128, 128, 16), H.PREC_F32, H.NAIK_R14) == 0
    for L in ((96, 96, 96, 24), (64, 64, 64, 16)):
        V = L[0] * L[1] * L[2] * L[3]
        assert V // 2 * 144 < 2 ** 31
        assert H.hisq_links_bytes(L, H.PREC_F64, H.NAIK_FULL) >= 2 * (V // 2) * 16 * 9 * 16
