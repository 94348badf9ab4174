"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import sys

import numpy as np
import pytest


def gpu_lib():
    """The HIP binding; skip cleanly where no GPU is visible, fail loudly if the
    library is missing on a machine with a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1411_4439_amd import hisq
    return hisq


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_l2_per_rhs(a, b):
    """max over rhs k of ||a_k - b_k|| / ||b_k|| for [sites][3][n] arrays."""
    n = b.shape[-1]
    out = []
    for k in range(n):
        den = np.linalg.norm(b[..., k])
        out.append(np.linalg.norm(a[..., k] - b[..., k]) / (den if den > 0 else 1.0))
    return max(out)


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
