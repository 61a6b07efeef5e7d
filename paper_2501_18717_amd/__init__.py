"""MI355X-native randomized (augmented) block-CG.

The solver library is ``librbcg.so`` (HIP for gfx950, C ABI in
``include/rbcg.h``); ``paper_2501_18717_amd.rbcg`` is its Python binding.
Build with ``python -m paper_2501_18717_amd.build``.
"""
__all__ = ["rbcg", "build"]
