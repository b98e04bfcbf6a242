"""FP64 CPU oracle of fKK-EC (arXiv 2005.07132).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The library never imports it and
it imports nothing from the library.
"""
from . import operators, workflows
from .operators import hilbert, als_baseline, whittaker, savgol_matrix, ridge
from .workflows import Params, fit, plain, transform, reconstruct, basis_from_factors

__all__ = [
    "operators", "workflows", "hilbert", "als_baseline", "whittaker",
    "savgol_matrix", "ridge", "Params", "fit", "plain", "transform",
    "reconstruct", "basis_from_factors",
]
