"""FP64 reference operators of fKK-EC (Camp, Bender & Lee, arXiv 2005.07132).

TEST INFRASTRUCTURE ONLY.  This package is the oracle that the HIP path is
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the library itself never does.  It
shares no code with the HIP path.

Every function is written from its mathematical definition in plain NumPy /
SciPy FP64 so that it can be read against the paper by eye.  Rows are
spectra, the last axis is the wavenumber axis (the orientation of Sec. 2.2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


# ---------------------------------------------------------------------------
# Discrete Hilbert transform (Eq. 2, Eq. 7): the operator applied along the
# frequency axis in KK, PEC and SEC.  The paper names the transform only; the
# discrete form (padding, sign, Nyquist) is this build's reading:
#   pad x to length L, DFT, multiply bin nu by -i*sgn(nu) (0 at DC and at
#   the Nyquist bin), inverse DFT, keep the real part, crop.
# With this sign H{cos} = sin, which is the convention under which the phase
# of a causal, minimum-phase response equals H{ln|K|}.
# ---------------------------------------------------------------------------

PAD_EDGE = 0
PAD_ZERO = 1


def default_fft_len(n: int) -> int:
    """Smallest power of two that is at least 3*n (padding reading)."""
    length = 1
    while length < 3 * n:
        length *= 2
    return length


def hilbert_multiplier(length: int) -> np.ndarray:
    """-i*sgn(nu) for the DFT bins of a length-`length` transform."""
    nu = np.fft.fftfreq(length) * length  # signed bin index
    mult = -1j * np.sign(nu)
    mult[0] = 0.0
    if length % 2 == 0:
        mult[length // 2] = 0.0
    return mult


def pad_rows(x: np.ndarray, length: int, pad_mode: int = PAD_EDGE):
    """Pad each row of x (..., N) to `length` points, centred.

    Returns the padded array and the left offset P_l = floor((L - N) / 2).
    """
    n = x.shape[-1]
    if length < n:
        raise ValueError("fft length shorter than the spectrum")
    p_left = (length - n) // 2
    p_right = length - n - p_left
    if pad_mode == PAD_EDGE:
        left = np.repeat(x[..., :1], p_left, axis=-1)
        right = np.repeat(x[..., -1:], p_right, axis=-1)
    elif pad_mode == PAD_ZERO:
        left = np.zeros(x.shape[:-1] + (p_left,))
        right = np.zeros(x.shape[:-1] + (p_right,))
    else:
        raise ValueError("unknown pad mode")
    return np.concatenate([left, x, right], axis=-1), p_left


def hilbert(x, fft_len: int | None = None, pad_mode: int = PAD_EDGE) -> np.ndarray:
    """Row-wise discrete Hilbert transform H{x} along the last axis."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    length = default_fft_len(n) if not fft_len else int(fft_len)
    xp, p_left = pad_rows(x, length, pad_mode)
    spec = np.fft.fft(xp, axis=-1) * hilbert_multiplier(length)
    y = np.fft.ifft(spec, axis=-1).real
    return y[..., p_left:p_left + n]


# ---------------------------------------------------------------------------
# Detrending operator D (Eq. 12, Eq. 16): asymmetric least squares (ALS),
# the method the paper names for PEC (Eilers 2003/2005).  The baseline z of a
# signal y minimises  sum_i w_i (y_i - z_i)^2 + lam * sum_i (z_{i-1} - 2 z_i
# + z_{i+1})^2, i.e. (diag(w) + lam D^T D) z = w * y with D the second
# difference matrix; the weights are re-set after each solve to p where the
# signal lies above the baseline and 1 - p elsewhere (ties count as "not
# above").  The number of solves is fixed (no early exit).
# ---------------------------------------------------------------------------

DETREND_ALS = 0
DETREND_WHITTAKER = 1


def default_als_lambda(n: int) -> float:
    """ALS smoothness 1e5 * (n / 1000)^4 (reading; the paper gives none).

    The penalty sum of squared second differences of a fixed curve sampled at
    n points scales as n^-3 against n for the data term, so lam ~ n^4 keeps
    the same physical smoothness at every spectral length.
    """
    return 1.0e5 * (n / 1000.0) ** 4


def second_difference(n: int) -> np.ndarray:
    """Dense (n-2) x n second-difference matrix D."""
    d = np.zeros((n - 2, n))
    for i in range(n - 2):
        d[i, i] = 1.0
        d[i, i + 1] = -2.0
        d[i, i + 2] = 1.0
    return d


def _penalty_bands(n: int, lam: float) -> np.ndarray:
    """Upper banded storage (solveh_banded layout) of lam * D^T D."""
    # Diagonals of D^T D for the second difference operator.
    main = np.full(n, 6.0)
    main[[0, -1]] = 1.0
    main[[1, -2]] = 5.0
    off1 = np.full(n - 1, -4.0)
    off1[[0, -1]] = -2.0
    off2 = np.ones(n - 2)
    ab = np.zeros((3, n))
    ab[2] = lam * main
    ab[1, 1:] = lam * off1
    ab[0, 2:] = lam * off2
    return ab


def weighted_smooth(y: np.ndarray, w: np.ndarray, lam: float) -> np.ndarray:
    """Solve (diag(w) + lam D^T D) z = w * y (banded SPD solve)."""
    ab = _penalty_bands(y.shape[-1], lam)
    ab[2] += w
    return scipy.linalg.solveh_banded(ab, w * y)


def als_baseline(y, lam: float, p: float, n_iter: int) -> np.ndarray:
    """ALS baseline of one spectrum y (1-D)."""
    y = np.asarray(y, dtype=np.float64)
    w = np.ones_like(y)
    z = y
    for _ in range(n_iter):
        z = weighted_smooth(y, w, lam)
        w = np.where(y > z, p, 1.0 - p)
    return z


def whittaker(y, lam: float) -> np.ndarray:
    """Linear (weights fixed at one) Whittaker smoother of one spectrum."""
    y = np.asarray(y, dtype=np.float64)
    return weighted_smooth(y, np.ones_like(y), lam)


def detrend_rows(y, mode: int, lam: float, p: float, n_iter: int) -> np.ndarray:
    """Apply the detrending operator D to every row of y."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    out = np.empty_like(y)
    for r in range(y.shape[0]):
        if mode == DETREND_ALS:
            out[r] = als_baseline(y[r], lam, p, n_iter)
        elif mode == DETREND_WHITTAKER:
            out[r] = whittaker(y[r], lam)
        else:
            raise ValueError("unknown detrend mode")
    return out


# ---------------------------------------------------------------------------
# Trendline operator M (Eq. 4, Eq. 22): the paper uses a large-window,
# low-order Savitzky-Golay filter, or the plain mean.  At an interior point
# the trendline is the value at the window centre of the least-squares
# polynomial fitted to the window; within half a window of either end the
# polynomial fitted to the first (last) full window is evaluated at the point.
# ---------------------------------------------------------------------------

SEC_SAVGOL = 0
SEC_MEAN = 1


def default_sg_window(n: int) -> int:
    """Largest odd window not above n / 2 (reading of 'large window')."""
    w = n // 2
    if w % 2 == 0:
        w -= 1
    return max(w, 3)


def savgol_matrix(n: int, window: int, order: int) -> np.ndarray:
    """Dense n x n Savitzky-Golay trendline operator S (row i: output i)."""
    if window % 2 == 0 or window > n or window <= order:
        raise ValueError("invalid Savitzky-Golay window")
    half = window // 2
    s = np.zeros((n, n))
    for i in range(n):
        start = min(max(i - half, 0), n - window)
        pos = np.arange(start, start + window, dtype=np.float64)
        # Least-squares polynomial through the window, evaluated at i:
        # value = e(i)^T pinv(V) y_window, V the Vandermonde of the window.
        vander = np.vander(pos - i, order + 1, increasing=True)
        coeffs = np.linalg.pinv(vander)[0]  # constant term at x = i
        s[i, start:start + window] = coeffs
    return s


def trendline_rows(y, mode: int, window: int, order: int) -> np.ndarray:
    """Apply the trendline operator M to every row of y."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    if mode == SEC_MEAN:
        return np.repeat(y.mean(axis=-1, keepdims=True), y.shape[-1], axis=-1)
    if mode == SEC_SAVGOL:
        s = savgol_matrix(y.shape[-1], window, order)
        return y @ s.T
    raise ValueError("unknown trendline mode")


# ---------------------------------------------------------------------------
# Ridge regression (Eq. 17, Eq. 25): (X^T X + lam I)^-1 X^T Y.
# lam = 0 is read as the minimum-norm least-squares solution.
# ---------------------------------------------------------------------------

def ridge(x: np.ndarray, y: np.ndarray, lam: float) -> np.ndarray:
    """Return (X^T X + lam I)^-1 X^T Y; min-norm lstsq when lam == 0."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if lam == 0.0:
        return np.linalg.lstsq(x, y, rcond=None)[0]
    gram = x.T @ x + lam * np.eye(x.shape[1])
    return np.linalg.solve(gram, x.T @ y)
