"""Pins of the oracle's operators against closed forms, published tables,
brute force and library routines (CPU only)."""
import os

import numpy as np
import pytest
import scipy.signal

from oracle import operators as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Hilbert transform (Eq. 2, Eq. 7)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [32, 33, 64])
@pytest.mark.parametrize("j", [1, 3, 7])
def test_hilbert_cos_is_sin_periodic(n, j):
    t = np.arange(n)
    x = np.cos(2 * np.pi * j * t / n)
    y = op.hilbert(x, fft_len=n, pad_mode=op.PAD_ZERO)
    np.testing.assert_allclose(y, np.sin(2 * np.pi * j * t / n), atol=1e-13)


def test_hilbert_matches_scipy_analytic_signal():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(128)
    y = op.hilbert(x, fft_len=128, pad_mode=op.PAD_ZERO)
    np.testing.assert_allclose(y, np.imag(scipy.signal.hilbert(x)), atol=1e-12)


def test_hilbert_brute_force_dft_with_edge_padding():
    # Explicit O(L^2) DFT and explicit edge replication on a tiny input.
    rng = np.random.default_rng(1)
    n, length = 7, 21
    x = rng.standard_normal(n)
    pl = (length - n) // 2
    xp = np.array([x[min(max(i - pl, 0), n - 1)] for i in range(length)])
    a = np.arange(length)
    dft = np.exp(-2j * np.pi * np.outer(a, a) / length)
    spec = dft @ xp
    for b in range(length):
        nu = b if b <= length // 2 else b - length
        spec[b] *= -1j * np.sign(nu)
    y = (np.conj(dft) @ spec / length).real[pl:pl + n]
    np.testing.assert_allclose(op.hilbert(x, fft_len=length), y, atol=1e-13)


def test_hilbert_of_constant_is_zero():
    # Sec. 2.1: the Hilbert transform of a constant vanishes.
    y = op.hilbert(np.full((3, 100), 2.5))
    assert np.abs(y).max() < 1e-14


@pytest.mark.parametrize("n", [31, 63])
def test_hilbert_squared_is_minus_identity_on_zero_mean(n):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n)
    hh = op.hilbert(op.hilbert(x, fft_len=n, pad_mode=op.PAD_ZERO), fft_len=n, pad_mode=op.PAD_ZERO)
    np.testing.assert_allclose(hh, -(x - x.mean()), atol=1e-13)


def test_hilbert_is_linear_rowwise():
    # Eq. 7 rests on linearity: H{U S V^T} = U S H{V^T}.
    rng = np.random.default_rng(3)
    vt = rng.standard_normal((4, 200))
    us = rng.standard_normal((9, 4))
    np.testing.assert_allclose(op.hilbert(us @ vt), us @ op.hilbert(vt), atol=1e-12)


def test_hilbert_of_lorentzian_closed_form():
    # H{G/(x^2+G^2)} = x/(x^2+G^2): the Lorentzian line shape of Eq. 19's
    # model.  Discretisation error depends on resolution (G / dw = 10 here)
    # and on how far the padding reaches; 2e-3 of the peak at L >= 3N.
    w = np.linspace(500.0, 3800.0, 1000)
    gamma = 33.0
    x = w - 2150.0
    lor = gamma / (x ** 2 + gamma ** 2)
    y = op.hilbert(lor)
    exact = x / (x ** 2 + gamma ** 2)
    assert np.abs(y - exact).max() / lor.max() < 2e-3


def test_kk_phase_of_single_resonance():
    # K = 1 + A/(W - w - iG) is zero- and pole-free in the upper half plane,
    # so its phase is the Hilbert transform of ln|K| (Eq. 2).
    w = np.linspace(500.0, 3800.0, 1000)
    k = 1.0 + 0.8 / (1800.0 - w - 1j * 15.0)
    phase = op.hilbert(np.log(np.abs(k)))
    assert np.abs(phase - np.angle(k)).max() < 5e-3


def test_hilbert_pad_modes_and_lengths():
    x = np.linspace(0, 1, 50) ** 2
    assert op.default_fft_len(50) == 256
    assert op.default_fft_len(1000) == 4096
    assert op.default_fft_len(512) == 2048
    assert op.default_fft_len(1600) == 8192
    y0 = op.hilbert(x, pad_mode=op.PAD_ZERO)
    y1 = op.hilbert(x, pad_mode=op.PAD_EDGE)
    assert y0.shape == y1.shape == (50,)
    assert not np.allclose(y0, y1)
    with pytest.raises(ValueError):
        op.hilbert(x, fft_len=40)


# --------------------------------------------------------------------------
# ALS / Whittaker detrender
# --------------------------------------------------------------------------

def test_penalty_matches_published_stencil():
    rows = {}
    for line in open(os.path.join(GOLDEN, "second_difference_penalty.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, *vals = line.split()
        rows[name] = [float(v) for v in vals]
    d = op.second_difference(12)
    dtd = d.T @ d
    np.testing.assert_array_equal(dtd[5, 3:8], rows["interior"])
    np.testing.assert_array_equal(dtd[0, :3], rows["row0"])
    np.testing.assert_array_equal(dtd[1, :4], rows["row1"])
    # banded storage used by the solver agrees with the dense operator
    ab = op._penalty_bands(12, 1.0)
    dense = np.diag(ab[2]) + np.diag(ab[1, 1:], 1) + np.diag(ab[1, 1:], -1) \
        + np.diag(ab[0, 2:], 2) + np.diag(ab[0, 2:], -2)
    np.testing.assert_array_equal(dense, dtd)


@pytest.mark.parametrize("lam,p", [(1e2, 1e-3), (1e6, 0.1), (10.0, 0.5)])
def test_als_returns_linear_input(lam, p):
    y = 0.3 - 0.002 * np.arange(300)
    np.testing.assert_allclose(op.als_baseline(y, lam, p, 10), y, atol=1e-9)


def test_als_single_pass_is_whittaker_dense():
    rng = np.random.default_rng(4)
    n, lam = 40, 50.0
    y = rng.standard_normal(n)
    d = op.second_difference(n)
    z = np.linalg.solve(np.eye(n) + lam * d.T @ d, y)
    np.testing.assert_allclose(op.als_baseline(y, lam, 0.01, 1), z, atol=1e-11)
    np.testing.assert_allclose(op.whittaker(y, lam), z, atol=1e-11)


def test_als_satisfies_its_normal_equations():
    rng = np.random.default_rng(5)
    n, lam, p, it = 60, 300.0, 0.02, 6
    y = np.cumsum(rng.standard_normal(n)) * 0.1
    z = op.als_baseline(y, lam, p, it)
    # weights of the last solve are those set from the previous iterate
    zprev = op.als_baseline(y, lam, p, it - 1)
    w = np.where(y > zprev, p, 1 - p)
    d = op.second_difference(n)
    np.testing.assert_allclose((np.diag(w) + lam * d.T @ d) @ z, w * y, atol=1e-9)


def test_als_finds_baseline_under_positive_peaks():
    # Small p puts the baseline under positive features (Eilers 2005);
    # inverting the weights would put it over them.
    t = np.linspace(0, 1, 800)
    base = 0.3 * np.sin(2 * t) + 0.1 * t
    peaks = sum(a * np.exp(-0.5 * ((t - c) / 0.004) ** 2) for a, c in [(1.0, 0.2), (0.6, 0.45), (0.8, 0.7)])
    z = op.als_baseline(base + peaks, 1e5, 1e-3, 10)
    assert np.abs(z - base).max() < 0.01
    z_bad = op.als_baseline(base + peaks, 1e5, 1 - 1e-3, 10)
    assert np.abs(z_bad - base).max() > 0.1


# --------------------------------------------------------------------------
# Savitzky-Golay trendline
# --------------------------------------------------------------------------

def test_savgol_interior_weights_match_published_table():
    for line in open(os.path.join(GOLDEN, "savgol_quadratic.txt")):
        if line.startswith("#") or not line.strip():
            continue
        window, norm, *weights = (int(v) for v in line.split())
        s = op.savgol_matrix(41, window, 2)
        half = window // 2
        np.testing.assert_allclose(s[20, 20 - half:20 + half + 1], np.array(weights) / norm, atol=1e-14)


@pytest.mark.parametrize("n,window", [(100, 31), (1000, 499), (512, 255)])
def test_savgol_matches_scipy_interp(n, window):
    rng = np.random.default_rng(6)
    y = rng.standard_normal(n)
    s = op.savgol_matrix(n, window, 2)
    np.testing.assert_allclose(s @ y, scipy.signal.savgol_filter(y, window, 2, mode="interp"), atol=1e-11)


def test_savgol_passes_quadratics():
    n = 200
    t = np.arange(n, dtype=float)
    s = op.savgol_matrix(n, op.default_sg_window(n), 2)
    for y in (np.ones(n), t, 1e-3 * t ** 2 - 0.1 * t + 2):
        np.testing.assert_allclose(s @ y, y, atol=1e-9 * np.abs(y).max())


def test_trendline_mean_mode():
    y = np.arange(12.0).reshape(2, 6)
    m = op.trendline_rows(y, op.SEC_MEAN, 3, 2)
    np.testing.assert_allclose(m, [[2.5] * 6, [8.5] * 6])


# --------------------------------------------------------------------------
# Ridge regression (Eq. 17, Eq. 25)
# --------------------------------------------------------------------------

def test_ridge_zero_is_lstsq_and_normal_equations_hold():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((30, 5))
    y = rng.standard_normal((30, 8))
    np.testing.assert_allclose(op.ridge(x, y, 0.0), np.linalg.lstsq(x, y, rcond=None)[0], atol=1e-12)
    b = op.ridge(x, y, 2.0)
    # stationarity of ||Y - X B||^2 + lam ||B||^2
    np.testing.assert_allclose(x.T @ (x @ b - y) + 2.0 * b, 0.0, atol=1e-11)


def test_ridge_push_through():
    # A (X^T X + lam I)^-1 X^T with X = S V^T equals A V diag(s / (s^2 + lam))
    rng = np.random.default_rng(8)
    n, k = 40, 6
    v, _ = np.linalg.qr(rng.standard_normal((n, k)))
    s = np.sort(rng.uniform(0.5, 3.0, k))[::-1]
    a = rng.standard_normal((10, n))
    lam = 0.3
    x = np.diag(s) @ v.T
    lhs = a @ np.linalg.solve(x.T @ x + lam * np.eye(n), x.T)
    np.testing.assert_allclose(lhs, a @ v * (s / (s ** 2 + lam)), atol=1e-12)
