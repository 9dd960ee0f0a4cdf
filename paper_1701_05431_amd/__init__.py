"""MI355X (gfx950) first-order finite-volume time step.

Importing the package loads nothing: the HIP library is loaded on first use
(``paper_1701_05431_amd._lib.lib()``) and fails loudly if it is not built.
"""
__all__ = ["inputs", "solver", "build"]
