"""Seeded synthetic CARS hyperspectral cubes.

This module only draws inputs: intensities of the CARS forward model
(Eq. 1 with a constant system response, chi_nr = 1) and of a surrogate
reference.  It holds none of the retrieval method's arithmetic, and both the
HIP path and the oracle consume what it returns.

Spectra follow the paper's simulation recipe: each Raman susceptibility is a
sum of complex Lorentzians A / (Omega - w - i Gamma) with A, Gamma > 0
(the model under Eq. 19), chi_nr is real and constant, and the surrogate
reference differs from the true NRB by a constant amplitude factor Xi and a
smooth frequency-dependent factor xi(w) (Eq. 3).  Noise is mixed
Poisson-Gaussian (Sec. 2.2, Eq. 9); at the counts used here the Poisson
part is drawn in its Gaussian limit, variance I / c.

All randomness comes from numpy PCG64 streams keyed by SeedSequence spawn
keys, so a cube is bit-identical for a given (seed, key) on every machine.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import scipy.ndimage
import scipy.special

ROOT_SEED = 20200514

# spawn-key roles
ROLE_COMPONENTS = 1
ROLE_ABUNDANCE = 2
ROLE_SNR = 3
ROLE_NOISE = 4
ROLE_PIXEL_PEAKS = 5


def rng_for(*key: int) -> np.random.Generator:
    """Independent PCG64 stream for a spawn key."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(key))))


def wavenumbers(n: int, lo: float = 500.0, hi: float = 3800.0) -> np.ndarray:
    return np.linspace(lo, hi, n)


def envelope(w: np.ndarray) -> np.ndarray:
    """Gaussian excitation envelope E(w), >= 0.61 over 500-3800 cm^-1."""
    mid = 0.5 * (w[0] + w[-1])
    half = 0.5 * (w[-1] - w[0])
    return np.exp(-((w - mid) ** 2) / (2.0 * half ** 2))


def reference(w: np.ndarray, xi_const: float = 1.1, slope: float = 0.2) -> np.ndarray:
    """Surrogate reference I_ref = Xi * xi(w) * chi_nr^2 * E(w), noiseless.

    xi(w) = (1 + slope * wt)^2 with wt in [-1, 1]: the intensity of a linear
    chi_ref, as in the paper's simulation.
    """
    mid = 0.5 * (w[0] + w[-1])
    half = 0.5 * (w[-1] - w[0])
    wt = (w - mid) / half
    return xi_const * (1.0 + slope * wt) ** 2 * envelope(w)


def lorentz_chi(w: np.ndarray, amp, centre, width) -> np.ndarray:
    """chi_R(w) = sum_j amp_j / (centre_j - w - i width_j)."""
    amp = np.atleast_1d(amp)[:, None]
    centre = np.atleast_1d(centre)[:, None]
    width = np.atleast_1d(width)[:, None]
    return (amp / (centre - w[None, :] - 1j * width)).sum(axis=0)


def draw_peaks(rng: np.random.Generator, n_peaks: int, w: np.ndarray):
    """Amplitudes U(0.05, 1), widths U(5, 20) cm^-1, centres with a 10%
    peak-free margin at both ends of the grid."""
    span = w[-1] - w[0]
    amp = rng.uniform(0.05, 1.0, n_peaks)
    width = rng.uniform(5.0, 20.0, n_peaks)
    centre = rng.uniform(w[0] + 0.1 * span, w[-1] - 0.1 * span, n_peaks)
    return amp, centre, width


@dataclass
class Cube:
    """A synthetic cube: intensities (M x N), reference, grid and metadata."""

    i_cars: np.ndarray
    i_ref: np.ndarray
    w: np.ndarray
    alpha: float = 0.0
    sigma_g: float = 0.0
    chi_components: np.ndarray | None = None   # (C x N) complex
    abundance: np.ndarray | None = None        # (M x C)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.i_cars.shape

    def ideal_im(self, rows) -> np.ndarray:
        """Known Im{chi / chi_nr} for the given rows (chi_nr = 1)."""
        if self.chi_components is not None:
            a = self.abundance[rows].astype(np.float64)
            im = a @ self.chi_components.imag
            if "nrb_components" in self.meta:
                im /= a @ self.meta["nrb_components"]
            return im
        return self.meta["ideal_im"][rows]


# ---------------------------------------------------------------------------
# Small plain-method cube: one random 8-peak spectrum per pixel, AWGN.
# ---------------------------------------------------------------------------

def pixel_cube(side: int = 64, n: int = 512, peaks: int = 8, snr: float = 50.0,
               key: int = 1, dtype=np.float64) -> Cube:
    w = wavenumbers(n)
    env = envelope(w)
    m = side * side
    rng = rng_for(key, ROLE_PIXEL_PEAKS)
    chi = np.empty((m, n), dtype=np.complex128)
    for r in range(m):
        chi[r] = lorentz_chi(w, *draw_peaks(rng, peaks, w))
    clean = np.abs(chi + 1.0) ** 2 * env
    sigma = clean.mean(axis=0).max() / snr
    noise = rng_for(key, ROLE_NOISE).standard_normal((m, n))
    i_cars = (clean + sigma * noise).astype(dtype)
    return Cube(i_cars=i_cars, i_ref=reference(w), w=w, alpha=0.0, sigma_g=sigma,
                meta={"ideal_im": chi.imag, "side": side, "snr": snr})


# ---------------------------------------------------------------------------
# Tissue-like mixture cube.
# ---------------------------------------------------------------------------

def smooth_field(rng: np.random.Generator, rows: int, cols: int, blur: float) -> np.ndarray:
    """White N(0,1) field blurred by a Gaussian of `blur` px, standardised."""
    z = scipy.ndimage.gaussian_filter(rng.standard_normal((rows, cols)), blur, mode="wrap")
    sd = z.std()
    # a one-pixel grid has no spread to standardise: a flat field
    return (z - z.mean()) / sd if sd > 0.0 else np.zeros_like(z)


def abundances(rng: np.random.Generator, rows: int, cols: int, n_comp: int,
               blur: float = 16.0) -> np.ndarray:
    """Spatially smooth maps whose per-pixel marginal is Dirichlet(1,...,1):
    u = Phi(z) of each standardised field, g = -ln(1 - u), a = g / sum g."""
    g = np.empty((rows * cols, n_comp))
    for c in range(n_comp):
        u = scipy.special.ndtr(smooth_field(rng, rows, cols, blur)).ravel()
        g[:, c] = -np.log1p(-np.minimum(u, 1.0 - 1e-16))
    return g / g.sum(axis=1, keepdims=True)


def components(n: int, n_comp: int = 5, key: int = 2, lo: float = 500.0,
               hi: float = 3800.0) -> np.ndarray:
    """Component susceptibilities chi_c (C x N), 10-25 peaks each."""
    w = wavenumbers(n, lo, hi)
    rng = rng_for(key, ROLE_COMPONENTS)
    chi = np.empty((n_comp, n), dtype=np.complex128)
    for c in range(n_comp):
        chi[c] = lorentz_chi(w, *draw_peaks(rng, int(rng.integers(10, 26)), w))
    return chi


def _mix_chunk(args):
    (i0, i1, ab, chi_re, chi_im, env, c_pix, sigma_g, noise_key, out) = args
    a = ab[i0:i1]
    re = 1.0 + a @ chi_re
    im = a @ chi_im
    clean = (re * re + im * im) * env
    rng = rng_for(*noise_key, i0)
    std = np.sqrt(clean / c_pix[i0:i1, None] + sigma_g ** 2)
    out[i0:i1] = clean + std * rng.standard_normal(clean.shape)


def tissue_cube(rows: int = 838, cols: int = 839, m: int | None = None, n: int = 1000,
                n_comp: int = 5, comp_key: int = 2, map_key: int = 2, noise_key: int = 2,
                sigma_g: float = 0.005, snr_lo: float = 20.0, snr_hi: float = 100.0,
                blur: float = 16.0, dtype=np.float32, chunk: int = 16384,
                threads: int | None = None) -> Cube:
    """Mixture cube on a rows x cols grid, truncated to the first m pixels.

    Each pixel's chi_R is sum_c a_c chi_c, mixed coherently at the
    susceptibility level; the SNR map runs from snr_lo to snr_hi.
    """
    m = rows * cols if m is None else min(m, rows * cols)
    w = wavenumbers(n)
    env = envelope(w)
    chi = components(n, n_comp, comp_key)
    ab = abundances(rng_for(map_key, ROLE_ABUNDANCE), rows, cols, n_comp, blur)[:m]
    us = smooth_field(rng_for(map_key, ROLE_SNR), rows, cols, blur).ravel()[:m]
    us = (us - us.min()) / max(us.max() - us.min(), 1e-300)
    snr = snr_lo * (snr_hi / snr_lo) ** us
    c_pix = snr ** 2
    out = np.empty((m, n), dtype=dtype)
    jobs = [(i0, min(i0 + chunk, m), ab, chi.real.copy(), chi.imag.copy(), env, c_pix,
             sigma_g, (noise_key, ROLE_NOISE), out) for i0 in range(0, m, chunk)]
    threads = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as pool:
        list(pool.map(_mix_chunk, jobs))
    return Cube(i_cars=out, i_ref=reference(w), w=w, alpha=float(np.mean(1.0 / c_pix)),
                sigma_g=sigma_g, chi_components=chi, abundance=ab.astype(np.float32),
                meta={"rows": rows, "cols": cols, "snr": (snr_lo, snr_hi)})


def tissue_703k(**kw) -> Cube:
    """The paper-scale cube: 838 x 839 grid truncated to 703,026 spectra x
    1,000 points (the pixel count of the stitched tissue image, Sec. 4.2)."""
    return tissue_cube(rows=838, cols=839, m=703026, n=1000, **kw)


def frame(i: int, side: int = 256, n: int = 1000, **kw) -> Cube:
    """Stored-basis stream frame i: same components, new maps and noise."""
    return tissue_cube(rows=side, cols=side, m=None, n=n, map_key=1000 + i,
                       noise_key=2000 + i, **kw)


# ---------------------------------------------------------------------------
# Controlled-spectrum cube: log-ratio of exact rank r plus small noise, so the
# gap between singular values r and r+1 is large.
# ---------------------------------------------------------------------------

def lowrank_log_cube(m: int, n: int, rank: int, noise: float = 1e-6, key: int = 7,
                     dtype=np.float64, decay: float = 0.7) -> Cube:
    w = wavenumbers(n)
    ref = reference(w)
    rng = rng_for(key, ROLE_COMPONENTS)
    basis = np.empty((rank, n))
    for r in range(rank):
        chi = lorentz_chi(w, *draw_peaks(rng, 6, w))
        basis[r] = np.log(np.abs(1.0 + chi))
    weights = rng_for(key, ROLE_ABUNDANCE).uniform(0.0, 1.0, (m, rank)) * decay ** np.arange(rank)
    ell = weights @ basis + noise * rng_for(key, ROLE_NOISE).standard_normal((m, n))
    i_cars = (ref * np.exp(2.0 * ell)).astype(dtype)
    return Cube(i_cars=i_cars, i_ref=ref, w=w, meta={"rank": rank})


# ---------------------------------------------------------------------------
# Replica of the paper's simulation workload (Sec. 4.1): a noiseless mixture
# of three chemicals whose NRBs differ, on a 74 x 246 base map side-scaled by
# 0.5, 1, 2, 3 or 4.
# ---------------------------------------------------------------------------

PAPER_SIM_BASE = (74, 246)
PAPER_SIM_SCALES = (0.5, 1.0, 2.0, 3.0, 4.0)
PAPER_SIM_PEAKS = (22, 25, 10)
ROLE_SIM_NRB = 6


def paper_sim_shape(scale: float) -> tuple[int, int]:
    """Map of the base 74 x 246 grid side-scaled by `scale`."""
    return int(round(PAPER_SIM_BASE[0] * scale)), int(round(PAPER_SIM_BASE[1] * scale))


def paper_sim_cube(scale: float = 1.0, n: int = 810, lo: float = -500.0, hi: float = 2500.0,
                   peak_lo: float = 500.0, peak_hi: float = 1700.0, key: int = 11, blur: float = 8.0,
                   constant_nrb: bool = False, dtype=np.float32, chunk: int = 16384) -> Cube:
    """Noiseless three-chemical mixture cube of (74 s) x (246 s) spectra.

    Chemical c has a Raman susceptibility of 22, 25 or 10 complex Lorentzians
    with centres in [peak_lo, peak_hi] and a real NRB chi_nr,c(w) that is a
    quadratic in wt = (w - lo) / (hi - lo) with non-negative coefficients.  A
    pixel's susceptibility is the abundance-weighted sum of the chemicals'
    chi_R,c + chi_nr,c, so its NRB is the same mixture of the chi_nr,c.  The
    reference is |chi_ref|^2 of a linear chi_ref, and the stimulation profile
    is constant (1).  The abundance maps are drawn once on the 74 x 246 base
    grid and resampled bilinearly, so every scale shows the same image.
    ideal_im(rows) is the known Im{chi / chi_nr} of those pixels.
    constant_nrb sets every chi_nr,c and chi_ref to 1 (same peaks and maps).
    """
    rows, cols = paper_sim_shape(scale)
    w = wavenumbers(n, lo, hi)
    wt = (w - lo) / (hi - lo)
    rng = rng_for(key, ROLE_COMPONENTS)
    chi = np.empty((3, n), dtype=np.complex128)
    for c, n_peaks in enumerate(PAPER_SIM_PEAKS):
        amp = rng.uniform(0.05, 1.0, n_peaks)
        width = rng.uniform(5.0, 20.0, n_peaks)
        centre = rng.uniform(peak_lo, peak_hi, n_peaks)
        chi[c] = lorentz_chi(w, amp, centre, width)
    nrng = rng_for(key, ROLE_SIM_NRB)
    coef = np.column_stack([nrng.uniform(0.25, 1.0, 3), nrng.uniform(0.0, 1.0, (3, 2))])
    nrb = coef[:, :1] + coef[:, 1:2] * wt + coef[:, 2:3] * wt ** 2
    ref_coef = np.array([nrng.uniform(0.25, 1.0), nrng.uniform(0.0, 1.0)])
    i_ref = (ref_coef[0] + ref_coef[1] * wt) ** 2
    if constant_nrb:
        nrb = np.ones_like(nrb)
        i_ref = np.ones_like(i_ref)

    base = abundances(rng_for(key, ROLE_ABUNDANCE), *PAPER_SIM_BASE, 3, blur)
    base = base.reshape(*PAPER_SIM_BASE, 3)
    ab = np.stack([scipy.ndimage.zoom(base[..., c], (rows / PAPER_SIM_BASE[0], cols / PAPER_SIM_BASE[1]),
                                      order=1, mode="nearest", grid_mode=True) for c in range(3)], axis=-1)
    assert ab.shape[:2] == (rows, cols), ab.shape
    ab = np.maximum(ab.reshape(rows * cols, 3), 0.0)
    ab /= ab.sum(axis=1, keepdims=True)

    m = rows * cols
    out = np.empty((m, n), dtype=dtype)
    chi_tot = chi + nrb
    for i0 in range(0, m, chunk):
        x = ab[i0:i0 + chunk] @ chi_tot
        out[i0:i0 + chunk] = x.real ** 2 + x.imag ** 2
    return Cube(i_cars=out, i_ref=i_ref, w=w, chi_components=chi, abundance=ab,
                meta={"rows": rows, "cols": cols, "scale": scale, "nrb_components": nrb,
                      "ref_coef": ref_coef, "nrb_coef": coef})
