"""Oracle: plain CPU evaluation of the paper's formulas (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package; the GPU library and its Python binding never do.
"""
from . import hs_oracle

__all__ = ["hs_oracle"]
