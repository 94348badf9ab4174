"""Flop and byte accounting for the HISQ Dslash and the CG iteration.

The paper prints only flop/byte ratios (Sec. 1, Table 1), in single precision,
for 1..8 rhs with full or 14-real ("r14") Naik storage, and states that double
precision halves them.  The counts below reproduce all fourteen printed values
to the two decimals shown:

* flops per output site and rhs: 16 SU(3)-shaped mat-vecs of 66 flops (9 complex
  multiplies of 6 flops, 6 complex adds of 2) plus 15 adds of 3-vectors (6 flops)
  = 1146;
* bytes per output site, the paper's model: 16 links (72 B each, or 56 B for an
  r14 Naik link) read once, plus per rhs 16 neighbour vectors and one output
  vector of 24 B, i.e. 1152 (or 1024) + 408 n.

For the roofline of this library a second byte count is used, the *algorithmic*
minimum: links once, every input vector once, every output vector once, i.e.
1152 (1024) + 48 n per output site in FP32 and twice that in FP64.
"""
from __future__ import annotations

FLOPS_PER_SITE_RHS = 16 * 66 + 15 * 6  # 1146
LINK_BYTES_F32 = {"full": 16 * 72, "r14": 8 * 72 + 8 * 56, "r13": 8 * 72 + 8 * 52,
                  "r9": 8 * 72 + 8 * 36}  # 1152, 1024, 992, 864
VEC_BYTES_F32 = 24  # one colour vector, 3 complex FP32 numbers

MI355X_HBM_GBPS = 8000.0
MI355X_FP64_VECTOR_TFLOPS = 78.6
MI355X_FP32_VECTOR_TFLOPS = 157.3


def _scale(prec: str) -> int:
    if prec not in ("f32", "f64"):
        raise ValueError("prec must be 'f32' or 'f64'")
    return 1 if prec == "f32" else 2


def dslash_flops_per_site(nrhs: int) -> int:
    return FLOPS_PER_SITE_RHS * nrhs


def paper_bytes_per_site(nrhs: int, naik: str = "full", prec: str = "f32") -> int:
    """Table 1 byte model: no reuse of neighbour vectors."""
    return _scale(prec) * (LINK_BYTES_F32[naik] + (16 + 1) * VEC_BYTES_F32 * nrhs)


def paper_flop_per_byte(nrhs: int, naik: str = "full", prec: str = "f32") -> float:
    return dslash_flops_per_site(nrhs) / paper_bytes_per_site(nrhs, naik, prec)


def dslash_algorithmic_bytes_per_site(nrhs: int, naik: str = "full", prec: str = "f32") -> int:
    """Minimum traffic of one half-Dslash per output site: links + input + output once."""
    return _scale(prec) * (LINK_BYTES_F32[naik] + 2 * VEC_BYTES_F32 * nrhs)


def cg_iteration_bytes_per_site(nrhs: int, naik: str = "full", prec: str = "f32") -> int:
    """Minimum traffic of one fused CG iteration per even site.

    p-update: read r, p, write p (3 vectors); D_oe: links, read p, write t (2);
    D_eo + epilogue: links, read t, p, x, r, write x, r (6).  11 vectors in all.
    """
    return _scale(prec) * (2 * LINK_BYTES_F32[naik] + 11 * VEC_BYTES_F32 * nrhs)


def cg_iteration_flops_per_site(nrhs: int) -> int:
    """Two half-Dslash (paper count) plus 72 flops of vector algebra per rhs."""
    return 2 * FLOPS_PER_SITE_RHS * nrhs + 72 * nrhs
