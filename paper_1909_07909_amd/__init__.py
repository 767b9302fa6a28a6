"""MI355X-native HSS matrix x block product and implicit ULV solve.

The compute path is ``libhss.so`` (HIP kernels for gfx950 behind the C ABI of
``include/hss.h``); ``paper_1909_07909_amd.hss`` is its Python binding and
``paper_1909_07909_amd.inputs`` draws seeded synthetic generators.
"""
__all__ = ["hss", "inputs"]
