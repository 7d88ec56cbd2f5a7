"""MI355X-native G-BM3D hot path (block matching, transform-domain patch
stacks, hard-threshold and Wiener collaborative filtering, aggregation).

The HIP library lives in ``libgbm3d.so`` beside this file; ``gbm3d`` is the
thin ctypes binding to its C ABI.  ``synth`` draws seeded synthetic inputs.
"""
__all__ = ["gbm3d", "synth"]
