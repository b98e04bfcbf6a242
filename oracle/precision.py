"""Operand rounding of the BF16 matrix-core mode, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py): imported by the tests,
the smoke check and the benchmark's CPU-baseline leg, never by the library.

The BF16 mode is defined by one rule: every operand of a matrix contraction
of the method is a BF16 number (the FP64 / FP32 value rounded to the nearest
number with 8 significant bits, ties to even) and the products are summed
without further rounding.  The contractions are Eq. 6 (l^T l), the
projection of Eq. 13 / Eq. 25 (l times the projection weights) and the two
products of Eq. 23 (Z times B_re and Z times B_im).  ``contract`` states the
rule once; the models below only say which matrices enter which
contraction, following workflows.py, so they hold for any kernel layout.
A device result differs from them by its FP32 accumulation and by operands
whose FP32 value sits at a BF16 rounding boundary.  The error of the BF16
mode as such is measured against workflows.py directly.
"""
from __future__ import annotations

import numpy as np

from . import workflows as wf


def round_bf16(x) -> np.ndarray:
    """Nearest number with 8 significant bits (BF16: 1 implicit + 7 stored),
    ties to even; the exponent range of the data here is far inside BF16's,
    so overflow and subnormals do not arise."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                    # x = m 2^e, 1/2 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def contract(a, b) -> np.ndarray:
    """A B with both operands rounded to BF16 and the sum of products exact
    (FP64 holds every product of two BF16 numbers exactly)."""
    return round_bf16(a) @ round_bf16(b)


def gram(i_cars, i_ref, floor: float) -> np.ndarray:
    """G_L = l^T l (Eq. 6) as a BF16 contraction."""
    ell, _ = wf.log_ratio(i_cars, i_ref, floor)
    return contract(ell.T, ell)


def projection_weights(basis) -> np.ndarray:
    """W (N x k) with Z_new = A_new V S^2 (S^2 + lam)^-1 = l diag(f) W-columns:
    the regression of Eq. 24-25 rewritten with X = S V^T and the identity
    (X^T X + lam I)^-1 X^T = V S (S^2 + lam)^-1; lam = 0 keeps the columns
    with s > 1e-15 max(s) (pseudo-inverse)."""
    s = np.asarray(basis["s"], dtype=np.float64)
    lam = basis["ml_lambda"]
    if lam > 0.0:
        shrink = s * s / (s * s + lam)
    else:
        shrink = (s > 1e-15 * s.max()).astype(np.float64)
    return basis["f"][:, None] * basis["v"] * shrink[None, :]


def project(i_new, basis) -> np.ndarray:
    """Z_new = l W (Eq. 25 through the weights above) as a BF16 contraction."""
    ell, _ = wf.log_ratio(i_new, basis["i_ref"], basis["ratio_floor"])
    return contract(np.atleast_2d(ell), projection_weights(basis))


def reconstruct(z, basis) -> dict:
    """Eq. 23: both exponent matrices as BF16 contractions of Z with the
    corrected bases."""
    return wf.retrieve(contract(z, basis["b_re"]), contract(z, basis["b_im"]))


def transform(i_new, basis) -> dict:
    """ML:fKK-EC (Eq. 24-25, then Eq. 23) in the BF16 mode: the projection's
    result Z is the left operand of the two contractions of Eq. 23, so the
    rule rounds it there like any other operand."""
    z = project(i_new, basis)
    out = reconstruct(z, basis)
    out["z"] = z
    return out


def transform_full_precision_z(i_new, basis) -> dict:
    """A variant outside the BF16 mode's rule, kept as a labelled
    comparison: BF16 projection operands and BF16 bases, but Z entering
    Eq. 23 unrounded.  It measures how much of the mode's error comes from
    rounding Z."""
    z = project(i_new, basis)
    out = wf.retrieve(z @ round_bf16(basis["b_re"]), z @ round_bf16(basis["b_im"]))
    out["z"] = z
    return out
