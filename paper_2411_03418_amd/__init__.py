"""MI355X-native eleven-grid line-by-line absorption (MARFA hot path).

The HIP library is loaded on first use of :mod:`paper_2411_03418_amd.marfa`;
importing this package (or its input generator) does not touch the GPU.
"""
__all__ = ["marfa", "synth"]
