"""torch.autograd.Function over the HISQ even-odd CG (forward and adjoint solve).

x = A(U, N, m)^{-1} b with A = 4m^2 - D_eo D_oe.  The backward pass calls
hisq_cg_solve_backward, which solves A y = dL/dx (A is Hermitian, so the
adjoint solve uses the same operator) and accumulates the per-link outer
products into dL/dU and dL/dN with a dedicated HIP kernel, plus dL/dm and
dL/db = y.  Gradients follow PyTorch's complex convention dL/dRe + i dL/dIm.
U and N are independent inputs (N is not differentiated through any product
of U links).  All arithmetic runs in libhisq; this module only allocates
device buffers and passes pointers.
"""
from __future__ import annotations

import torch

from . import hisq as H


class HisqSolve(torch.autograd.Function):
    """x = HisqSolve.apply(U, N, m, b, L, mode, naik, tol).

    U, N: [4][V][3][3] complex128 device tensors; m: 0-dim float64 tensor (or a
    float); b: [V/2][3][n] complex128 even-site bundle; L: lattice extents.
    """

    @staticmethod
    def forward(ctx, U, N, m, b, L, mode=H.MODE_FP64, naik=H.NAIK_FULL, tol=1e-10):
        L = tuple(int(v) for v in L)
        mass = float(m)
        mixed = mode == H.MODE_MIXED
        links = H.Links(L, U, N, f32=(mixed and naik == H.NAIK_FULL),
                        r14=(mixed and naik == H.NAIK_R14), r13=(mixed and naik == H.NAIK_R13),
                        r9=(mixed and naik == H.NAIK_R9))
        x, status, info = H.solve(links, mass, b, mode=mode, naik=naik, tol=tol)
        if status != H.HISQ_OK:
            raise RuntimeError("forward solve did not converge: %s" % (info,))
        ctx.links = links
        ctx.L, ctx.mass, ctx.mode, ctx.naik, ctx.tol = L, mass, mode, naik, tol
        ctx.m_is_tensor = isinstance(m, torch.Tensor)
        ctx.m_device = m.device if ctx.m_is_tensor else None
        ctx.save_for_backward(x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        links = ctx.links
        n = x.shape[2]
        V = 2 * x.shape[0]
        dev = x.device
        grad_x = grad_x.contiguous().to(torch.complex128)
        gU = torch.empty((4, V, 3, 3), dtype=torch.complex128, device=dev)
        gN = torch.empty_like(gU)
        gm = torch.zeros((), dtype=torch.float64, device=dev)
        gb = torch.empty_like(x)
        ws = H.empty_bytes(H.hisq_backward_workspace_bytes(ctx.L, n, ctx.mode), dev)
        p = H.hisq_default_params(mode=ctx.mode, naik=ctx.naik, tol=ctx.tol)
        l32 = links.packed(H.PREC_F32, ctx.naik) if ctx.mode == H.MODE_MIXED else None
        status, info = H.hisq_cg_solve_backward(ctx.L, ctx.mass, n, p, links.f64, l32, x, grad_x,
                                                gU, gN, gm, gb, ws)
        if status != H.HISQ_OK:
            raise RuntimeError("adjoint solve did not converge: %s" % (info.to_dict(n),))
        gm_out = gm.to(ctx.m_device) if ctx.m_is_tensor else None
        return gU, gN, gm_out, gb, None, None, None, None


def solve(U, N, m, b, L, mode=H.MODE_FP64, naik=H.NAIK_FULL, tol=1e-10):
    return HisqSolve.apply(U, N, m, b, L, mode, naik, tol)
