"""Operand rounding of the BF16 matrix-core mode, in FP64.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py): imported by the tests,
the smoke check and the benchmark's CPU-baseline leg, never by the library.

In BF16 mode the operands of the three contractions (the log ratio l in the
Gram of Eq. 6; l and the projection weights in Eq. 13 / Eq. 25; Z and the
corrected bases in Eq. 23) are rounded to BF16 and the products are
accumulated in FP32.  The functions below round the FP64 operands the same
way and then evaluate the definitions of workflows.py exactly (FP64), so a
device result differs from them only by FP32 accumulation and by operands
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


def gram(i_cars, i_ref, floor: float) -> np.ndarray:
    """G_L = l^T l (Eq. 6) with l rounded to BF16."""
    ell, _ = wf.log_ratio(i_cars, i_ref, floor)
    l16 = round_bf16(ell)
    return l16.T @ l16


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
    """Z_new = l W with both operands rounded to BF16."""
    ell, _ = wf.log_ratio(i_new, basis["i_ref"], basis["ratio_floor"])
    return round_bf16(np.atleast_2d(ell)) @ round_bf16(projection_weights(basis))


def reconstruct(z, basis) -> dict:
    """Eq. 23 with Z and the corrected bases rounded to BF16."""
    z16 = round_bf16(z)
    return wf.retrieve(z16 @ round_bf16(basis["b_re"]), z16 @ round_bf16(basis["b_im"]))


def transform(i_new, basis) -> dict:
    """ML:fKK-EC with every contraction operand rounded to BF16 (Z rounded
    again before the reconstruction, as the fused kernel stages it)."""
    z = project(i_new, basis)
    out = reconstruct(z, basis)
    out["z"] = z
    return out
