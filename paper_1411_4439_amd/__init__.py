"""MI355X-native multi-rhs HISQ even-odd conjugate gradient.

``paper_1411_4439_amd.hisq`` is the thin Python binding of ``libhisq.so`` (the
HIP library); importing it fails loudly if the library is not built.
``workload`` draws seeded synthetic inputs and ``roofline`` holds the flop/byte
accounting; neither touches the GPU.
"""
__all__ = ["hisq", "workload", "roofline", "autograd"]
