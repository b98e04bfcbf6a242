"""FP64 reference workflows of fKK-EC and of the conventional method.

TEST INFRASTRUCTURE ONLY (see oracle/operators.py): imported by the tests,
the smoke check and the benchmark's CPU-baseline leg, never by the library.

Implements, step by step in the paper's order and notation:
  * ``plain``      conventional per-spectrum KK -> PEC -> SEC (Eq. 2-5, with
                   SEC in the log form of Eq. 19),
  * ``fit``        fKK-EC: truncated SVD of A (Eq. 6, 10), fKK (Eq. 7, 11),
                   fPEC (Eq. 13-17), fSEC (Eq. 20-22) and the reconstruction
                   of Eq. 23,
  * ``transform``  ML:fKK-EC: regression of U_new on a stored basis
                   (Eq. 24-25) followed by Eq. 23.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import operators as op

F_ONE = 0
F_NOISE = 1


@dataclass
class Params:
    """Method parameters (names follow the C parameter block).

    Values the paper leaves open are this build's readings:
      fft_len 0 -> smallest power of two >= 3N; edge-replicate padding;
      ALS lam (0 -> 1e5 (N/1000)^4) / p / iterations; ridge weight relative to the largest
      eigenvalue of X^T X; Savitzky-Golay order 2 with window 0 -> the largest
      odd number <= N/2; ratios not above ``ratio_floor`` are clamped.
    """

    k: int = 50
    f_mode: int = F_ONE
    alpha: float = 0.0
    sigma_g: float = 1.0
    pad_mode: int = op.PAD_EDGE
    fft_len: int = 0
    detrend: int = op.DETREND_ALS
    als_lambda: float = 0.0
    als_p: float = 1.0e-3
    als_iters: int = 10
    ridge_rel: float = 1.0e-6
    sec_mode: int = op.SEC_SAVGOL
    sg_window: int = 0
    sg_order: int = 2
    ml_lambda: float = 0.0
    ratio_floor: float = 1.0e-6
    k_max: int = 128        # k = 0: at most this many vectors from the rank rule
    sec_form: int = 0       # plain workflow: 0 log form (Eq. 19), 1 real-part form (Eq. 4-5)
    q_between: int = 0      # rows per column between the extrema added to q (Sec. 2.3)
    q_override: np.ndarray | None = field(default=None, repr=False)

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


# ---------------------------------------------------------------------------
# Shared steps.
# ---------------------------------------------------------------------------

def log_ratio(i_cars, i_ref, floor: float):
    """l = 1/2 ln(I_CARS / I_ref) (Eq. 2), with non-finite or non-positive
    ratios (ratio not above ``floor``) replaced by ``floor``.

    Returns (l, number_of_clamped_entries).
    """
    ratio = np.asarray(i_cars, dtype=np.float64) / np.asarray(i_ref, dtype=np.float64)
    bad = ~((ratio > floor) & np.isfinite(ratio))
    ratio = np.where(bad, floor, ratio)
    return 0.5 * np.log(ratio), int(bad.sum())


def scaling_f(i_cars, p: Params) -> np.ndarray:
    """f(omega) = 2<I> / sqrt(alpha <I> + sigma_g^2) (Eq. 9), or 1."""
    n = np.asarray(i_cars).shape[-1]
    if p.f_mode == F_ONE:
        return np.ones(n)
    mean = np.asarray(i_cars, dtype=np.float64).mean(axis=0)
    return 2.0 * mean / np.sqrt(p.alpha * mean + p.sigma_g ** 2)


def fix_signs(v: np.ndarray, u: np.ndarray | None = None):
    """Make the largest-magnitude entry of every column of v positive
    (first occurrence on ties) and flip the matching column of u."""
    v = v.copy()
    u = None if u is None else u.copy()
    for i in range(v.shape[1]):
        j = int(np.argmax(np.abs(v[:, i])))
        if v[j, i] < 0:
            v[:, i] = -v[:, i]
            if u is not None:
                u[:, i] = -u[:, i]
    return v, u


def randomized_svd(a: np.ndarray, k: int, omega: np.ndarray, power_iters: int = 1):
    """Rank-k SVD of A from a randomized range finder (the alternative the
    paper names for very large data, Sec. 5): Halko, Martinsson & Tropp
    (2011), randomized subspace iteration (their Algorithm 4.4) on the test
    matrix omega (N x l, l >= k), then the SVD of B = Q^T A (Algorithm 5.1).
    Returns (U_k, s_k, V_k) before the sign rule."""
    q, _ = np.linalg.qr(a @ omega)                    # range of A Omega
    for _ in range(power_iters):
        z, _ = np.linalg.qr(a.T @ q)                  # re-orthonormalised each half step
        q, _ = np.linalg.qr(a @ z)
    b = q.T @ a                                       # l x N
    ub, s, vt = np.linalg.svd(b, full_matrices=False)
    return (q @ ub)[:, :k], s[:k], vt[:k].T


def truncated_svd(a: np.ndarray, k: int, method: str = "gesdd", omega=None, power_iters: int = 1):
    """Rank-k SVD of A (Eq. 6): returns (U_k, s_k, V_k), descending s.

    method 'gesdd' is LAPACK's SVD of A itself; 'gram' is the symmetric
    eigendecomposition of A^T A with s = sqrt(eigenvalue) and U = A V / s;
    'randomized' is randomized_svd with the test matrix omega.
    """
    if method == "randomized":
        u, s, v = randomized_svd(a, k, omega, power_iters)
    elif method == "gesdd":
        u, s, vt = np.linalg.svd(a, full_matrices=False)
        u, s, v = u[:, :k], s[:k], vt[:k].T
    elif method == "gram":
        lam, vec = np.linalg.eigh(a.T @ a)
        order = np.argsort(lam)[::-1][:k]
        s = np.sqrt(np.maximum(lam[order], 0.0))
        v = vec[:, order]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = np.where(s > 0, (a @ v) / s, 0.0)
    else:
        raise ValueError(method)
    v, u = fix_signs(v, u)
    return u, s, v


def rank_cutoff(s: np.ndarray, m: int, n: int, eps: float) -> int:
    """Number of singular values larger than s_max * max(M, N) * eps, eps
    the machine epsilon of the data type of the SVD input (Sec. 4.1: the
    cut-off of NumPy's and MATLAB's rank estimate)."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0 or not s.max() > 0.0:
        return 0
    return int(np.count_nonzero(s > s.max() * max(m, n) * eps))


def subsample_rows(z: np.ndarray, between: int = 0) -> np.ndarray:
    """q = union over columns of argmax and argmin over rows (Eq. 13-15).

    Z = U S with s > 0 has the same per-column arg-extrema as U.  Ties take
    the first row; the union is returned sorted ascending.

    between > 0 adds the optional sub-sample between the extrema (Sec. 2.3,
    after Eq. 15), read as: for each column, the rows whose values lie
    nearest to the `between` evenly spaced levels min + (max - min) j /
    (between + 1), j = 1..between (first row on ties).  Z = U S scales each
    column by s > 0, which maps these levels and rows onto U's.
    """
    qmax = np.argmax(z, axis=0)
    qmin = np.argmin(z, axis=0)
    picked = [qmax, qmin]
    for c in range(z.shape[1]):
        lo, hi = z[qmin[c], c], z[qmax[c], c]
        for j in range(1, between + 1):
            level = lo + (hi - lo) * (j / (between + 1))
            picked.append(np.array([np.argmin(np.abs(z[:, c] - level))]))
    return np.unique(np.concatenate(picked))


def ridge_lambda(x: np.ndarray, rel: float) -> float:
    """Ridge weight lam = rel * largest eigenvalue of X^T X."""
    if rel == 0.0 or x.size == 0:
        return 0.0
    return rel * float(np.linalg.eigvalsh(x.T @ x)[-1])


def _hilbert(x, p: Params):
    return op.hilbert(x, p.fft_len or None, p.pad_mode)


def _detrend(y, p: Params):
    n = np.atleast_2d(y).shape[-1]
    lam = p.als_lambda or op.default_als_lambda(n)
    return op.detrend_rows(y, p.detrend, lam, p.als_p, p.als_iters)


def _trend(y, p: Params):
    n = np.atleast_2d(y).shape[-1]
    window = p.sg_window or op.default_sg_window(n)
    return op.trendline_rows(y, p.sec_mode, window, p.sg_order)


def retrieve(re_part: np.ndarray, im_part: np.ndarray) -> dict:
    """K_CARS = exp(re_part) * exp(i im_part): Im, Re and |K|."""
    mag = np.exp(re_part)
    return {"im": mag * np.sin(im_part), "re": mag * np.cos(im_part), "abs": mag}


# ---------------------------------------------------------------------------
# Conventional per-spectrum workflow (Eq. 2-5, SEC of Eq. 19).
# ---------------------------------------------------------------------------

def plain(i_cars, i_ref, p: Params) -> dict:
    """Per-spectrum KK, PEC and SEC for every row of I_CARS."""
    ell, clamps = log_ratio(i_cars, i_ref, p.ratio_floor)
    ell = np.atleast_2d(ell)
    phi = _hilbert(ell, p)                     # KK phase, Eq. 2
    phi_err = _detrend(phi, p)                 # PEC: phase error by D
    amp_log = ell + _hilbert(phi_err, p)       # ln|K| + H{phi_err}, Eq. 5
    if p.sec_form == 1:
        # SEC as Eq. 4-5: K e^{H{phi_err}} e^{-i phi_err} divided by the
        # trendline (or mean) of its real part
        out = retrieve(amp_log, phi - phi_err)
        scale = _trend(out["re"], p)
        out = {"im": out["im"] / scale, "re": out["re"] / scale, "abs": out["abs"] / np.abs(scale)}
    else:
        amp_log = amp_log - _trend(amp_log, p)     # SEC, log form (Eq. 19)
        out = retrieve(amp_log, phi - phi_err)
    out.update(phi=phi, phi_err=phi_err, clamps=clamps)
    return out


# ---------------------------------------------------------------------------
# fKK-EC (Eq. 6-23).
# ---------------------------------------------------------------------------

def basis_from_factors(f, s, v, z, p: Params, q=None) -> dict:
    """fKK, fPEC and fSEC on the k right singular vectors.

    f (N), s (k), v = V_k (N x k), z = U_k S_k (M x k).  Returns the basis
    dictionary, including the corrected exponent bases
      B_re = V^T/f + H{Phi_PEC^T} - V_SEC^T   and   B_im = H{V^T/f} - Phi_PEC^T
    of Eq. 23.
    """
    vt_f = v.T / f                                   # V^T / f (k x N)
    h_v = _hilbert(vt_f, p)                          # fKK, Eq. 7 / 11
    if q is None:
        q = p.q_override if p.q_override is not None else subsample_rows(z, p.q_between)
    q = np.asarray(q, dtype=np.int64)
    x = z[q, :]                                      # X = U_ss S (Eq. 16)
    phi_raw = x @ h_v                                # U_ss S H{V^T/f}
    phi_err = _detrend(phi_raw, p)                   # D{...}, Eq. 16
    lam = ridge_lambda(x, p.ridge_rel)
    if x.size == 0 or not np.any(x):
        phi_pec_t = np.zeros_like(vt_f)              # X = 0: no phase error
    else:
        phi_pec_t = op.ridge(x, phi_err, lam)        # Eq. 17 (k x N)
    h_phi = _hilbert(phi_pec_t, p)                   # H{Phi_PEC}
    t = vt_f + h_phi                                 # Eq. 18 amplitude basis
    v_sec_t = _trend(t, p)                           # Eq. 22
    return {
        "f": np.asarray(f, dtype=np.float64), "s": s, "v": v, "q": q, "x": x,
        "h_v": h_v, "phi_err": phi_err, "ridge_lambda": lam,
        "phi_pec_t": phi_pec_t, "v_sec_t": v_sec_t,
        "b_re": t - v_sec_t, "b_im": h_v - phi_pec_t,
    }


def reconstruct(z, basis) -> dict:
    """K_CARS of Eq. 23 for the rows of Z = U S."""
    return retrieve(z @ basis["b_re"], z @ basis["b_im"])


def fit(i_cars, i_ref, p: Params, svd: str = "gesdd", omega=None, power_iters: int = 1) -> dict:
    """Full fKK-EC on I_CARS (M x N).  Returns basis, Z and outputs.

    k = 0 keeps the singular vectors the rank rule of Sec. 4.1 selects
    (rank_cutoff with the machine epsilon of I_CARS's data type), at least
    one and at most p.k_max."""
    in_type = np.asarray(i_cars).dtype
    eps = float(np.finfo(in_type).eps) if np.issubdtype(in_type, np.floating) else float(np.finfo(np.float64).eps)
    i_cars = np.asarray(i_cars, dtype=np.float64)
    ell, clamps = log_ratio(i_cars, i_ref, p.ratio_floor)
    f = scaling_f(i_cars, p)
    a = ell * f                                       # Eq. 10
    if p.k == 0:
        u, s, v = truncated_svd(a, min(a.shape), svd, omega, power_iters)
        k = min(max(rank_cutoff(s, a.shape[0], a.shape[1], eps), 1), p.k_max)
        u, s, v = u[:, :k], s[:k], v[:, :k]
    else:
        u, s, v = truncated_svd(a, p.k, svd, omega, power_iters)
    z = u * s                                         # U_k S_k
    basis = basis_from_factors(f, s, v, z, p)
    basis["i_ref"] = np.asarray(i_ref, dtype=np.float64)
    basis["ml_lambda"] = p.ml_lambda
    basis["ratio_floor"] = p.ratio_floor
    out = reconstruct(z, basis)
    out.update(basis=basis, z=z, u=u, clamps=clamps)
    return out


# ---------------------------------------------------------------------------
# ML:fKK-EC (Eq. 24-25).
# ---------------------------------------------------------------------------

def regress_z(i_new, basis) -> np.ndarray:
    """Z_new = U_new S with U_new = A_new (X^T X + lam I)^-1 X^T, X = S V^T.

    lam = 0 is read as the pseudo-inverse of X.
    """
    ell, _ = log_ratio(i_new, basis["i_ref"], basis["ratio_floor"])
    a_new = np.atleast_2d(ell) * basis["f"]
    x = np.diag(basis["s"]) @ basis["v"].T            # S V^T (k x N)
    lam = basis["ml_lambda"]
    if lam == 0.0:
        u_new = a_new @ np.linalg.pinv(x)
    else:
        n = x.shape[1]
        u_new = a_new @ np.linalg.solve(x.T @ x + lam * np.eye(n), x.T)
    return u_new * basis["s"]


def basis_residual(i_new, basis) -> float:
    """How well a stored basis supports new spectra (the retraining
    criterion of Sec. 5): with A = l diag(f) of the new spectra,
    ||A - A V V^T||_F / ||A||_F."""
    ell, _ = log_ratio(i_new, basis["i_ref"], basis["ratio_floor"])
    a = np.atleast_2d(ell) * basis["f"]
    v = basis["v"]
    return float(np.linalg.norm(a - (a @ v) @ v.T) / np.linalg.norm(a))


def transform(i_new, basis) -> dict:
    """Apply a stored basis to new spectra."""
    z = regress_z(i_new, basis)
    out = reconstruct(z, basis)
    out["z"] = z
    return out
