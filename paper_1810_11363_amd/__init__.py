"""MI355X (gfx950) split search for oblivious gradient-boosted trees and
ordered target statistics (CatBoost, arXiv:1810.11363).

``cbhip``   ctypes binding of libcbhip (include/cbhip.h), same names as the C-ABI
``booster`` boosting driver: device buffers from PyTorch, every step in libcbhip
``build``   compiles libcbhip.so with hipcc for gfx950
"""
__all__ = ["cbhip", "booster", "build"]
