"""Parity of the BF16 matrix-core mode, called through the C ABI.

Two kinds of checks:
* the kernels are exact up to FP32 accumulation: inputs whose contraction
  operands are BF16 numbers already (log ratios, Z, projection weights and
  bases with 8 significant bits; |l| >= 1/4 keeps the FP32 log ratio far
  from a BF16 rounding boundary), compared with the oracle's FP64 product of
  the same operands to the FP32-mode bar: 1e-5 per spectrum, 2e-6 of the
  largest Gram entry;
* the error of the mode itself on tissue-like cubes against the FP64
  oracle, reported with a sanity bound only (operands rounded to 2^-9
  relative).
Where a rounding decision depends on FP32 arithmetic that the oracle does
in FP64 (Z rounded again inside the fused transform; the log ratio of
general data, whose FP32 logarithm has an absolute error near 2^-24), an
operand can land on the other side of a BF16 rounding boundary and change
by 2^-8 of itself.  Spectra touched by such a flip are held to the sanity
bound (1e-2); the others, at least FRAC of them, to 1e-5.  On small log
ratios (|l| ~ 1e-2) about 3% of spectra of a rank-6 fit see a flip.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import precision as pr
from oracle import workflows as wf

torch = pytest.importorskip("torch")
fk = pytest.importorskip("paper_2005_07132_amd")

pytestmark = pytest.mark.gpu
TOL = 1e-5
FRAC = 0.9


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def spectrum_err(y, ref):
    return np.abs(y - ref).max(axis=1) / np.maximum(np.abs(ref).max(axis=1), 1e-30)


@pytest.fixture(scope="module")
def ctx():
    c = fk.Context(0)
    yield c
    c.close()


def bf16_values(rng, shape, lo=0.25, hi=1.0):
    """BF16 numbers with magnitudes in [lo, hi] and random signs."""
    mag = rng.uniform(lo, hi, shape)
    return pr.round_bf16(np.where(rng.random(shape) < 0.5, -mag, mag))


def exact_intensities(ell16, rng):
    """FP32 intensities whose log ratio rounds to ell16 (BF16)."""
    n = ell16.shape[1]
    i_ref = rng.uniform(0.5, 2.0, n)
    data = (i_ref * np.exp(2.0 * ell16)).astype(np.float32)
    ell, _ = wf.log_ratio(data.astype(np.float64), i_ref, 1e-6)
    np.testing.assert_array_equal(pr.round_bf16(ell), ell16)
    return data, i_ref


def synthetic_basis(rng, n, k, i_ref, phase=1.0):
    """Basis with f = 1, s = 1 (so W = V) and BF16-valued V, B_re, B_im."""
    return {"i_ref": i_ref, "f": np.ones(n), "s": np.ones(k), "v": bf16_values(rng, (n, k), 0.01, 0.1),
            "b_re": bf16_values(rng, (k, n), 0.001, 0.05), "b_im": bf16_values(rng, (k, n), 0.01, phase),
            "ml_lambda": 0.0, "ratio_floor": 1e-6}


def strided(data, ld_pad):
    if not ld_pad:
        return dev(data)
    m, n = data.shape
    full = np.zeros((m, n + ld_pad), dtype=np.float32)
    full[:, :n] = data
    return dev(full)[:, :n]


# --------------------------------------------------------------------------
# Gram (Eq. 6)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,ld_pad", [(37, 20, 0), (5000, 300, 0), (3001, 1000, 0), (777, 129, 3),
                                         (8191, 128, 0)])
def test_bf16_gram_exact_operands(ctx, m, n, ld_pad):
    say(f"bf16 gram m={m} n={n} ld_pad={ld_pad}")
    rng = synth.rng_for(901, m, n)
    ell16 = bf16_values(rng, (m, n))
    data, i_ref = exact_intensities(ell16, rng)
    g, cs, clamps = ctx.gram(strided(data, ld_pad), i_ref, prec=fk.PREC_BF16)
    ref = ell16.T @ ell16
    assert np.abs(g - ref).max() / np.abs(ref).max() < 2e-6
    np.testing.assert_array_equal(g, g.T)
    np.testing.assert_allclose(cs, data.astype(np.float64).sum(axis=0), rtol=1e-12)
    assert clamps == 0


def test_bf16_gram_tissue_error_and_clamps(ctx):
    say("bf16 gram tissue")
    cube = synth.tissue_cube(rows=60, cols=50, n=400, map_key=17, noise_key=17, blur=3.0)
    data = cube.i_cars.copy()
    data[5, 7] = 0.0
    data[9, 100] = np.nan
    g, cs, clamps = ctx.gram(dev(data), cube.i_ref, prec=fk.PREC_BF16)
    ell, bad = wf.log_ratio(data.astype(np.float64), cube.i_ref, 1e-6)
    assert clamps == bad == 2
    exact = ell.T @ ell
    rounded = pr.gram(data.astype(np.float64), cube.i_ref, 1e-6)
    err_exact = np.abs(g - exact).max() / np.abs(exact).max()
    err_rounded = np.abs(g - rounded).max() / np.abs(rounded).max()
    say(f"bf16 gram tissue: rel err vs FP64 {err_exact:.2e}, vs rounded operands {err_rounded:.2e}")
    assert err_rounded < 2e-5
    assert err_exact < 1e-2


# --------------------------------------------------------------------------
# Projection, reconstruction, fused transform (Eq. 13, 23, 25)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k,m,n", [(8, 1000, 300), (20, 129, 1000), (50, 3000, 257), (100, 700, 400)])
def test_bf16_projection_exact_operands(ctx, k, m, n):
    say(f"bf16 project k={k} m={m} n={n}")
    rng = synth.rng_for(902, k, m, n)
    ell16 = bf16_values(rng, (m, n))
    data, i_ref = exact_intensities(ell16, rng)
    basis = synthetic_basis(rng, n, k, i_ref)
    b = ctx.basis_import(basis)
    b.precision = fk.PREC_BF16
    assert b.precision == fk.PREC_BF16
    z, qmax, qmin = ctx.project(b, dev(data))
    zg = host(z)
    zref = pr.project(data.astype(np.float64), basis)
    np.testing.assert_array_equal(zref, ell16 @ basis["v"])
    assert spectrum_err(zg.T, zref.T).max() < TOL
    for c in range(k):
        scale = np.abs(zref[:, c]).max()
        assert zref[qmax[c], c] >= zref[:, c].max() - 4 * TOL * scale
        assert zref[qmin[c], c] <= zref[:, c].min() + 4 * TOL * scale


@pytest.mark.parametrize("k,phase,n", [(8, 1.0, 333), (30, 1.0, 333), (64, 0.5, 333), (100, 0.3, 333),
                                         (30, 1.0, 300)])
def test_bf16_reconstruction_exact_operands(ctx, k, phase, n):
    # n = 300: rows of the BF16 basis planes end at 320 (N rounded up to 64)
    say(f"bf16 reconstruct k={k} n={n}")
    rng = synth.rng_for(903, k)
    m = 2000
    basis = synthetic_basis(rng, n, k, np.ones(n), phase=phase)
    z16 = bf16_values(rng, (m, k), 0.25, 2.0)
    b = ctx.basis_import(basis)
    b.precision = fk.PREC_BF16
    phase_range = np.abs(z16 @ basis["b_im"]).max()
    for plane, key in ((fk.OUT_IM, "im"), (fk.OUT_RE, "re"), (fk.OUT_ABS, "abs")):
        out = host(ctx.reconstruct(b, dev(z16), plane))
        ref = wf.reconstruct(z16, basis)[key]
        err = spectrum_err(out, ref).max()
        assert err < TOL, (key, err, phase_range)


@pytest.mark.parametrize("k,m,n", [(10, 1, 300), (10, 129, 300), (50, 1000, 1000), (100, 513, 200)])
def test_bf16_transform_exact_operands(ctx, k, m, n):
    say(f"bf16 transform k={k} m={m} n={n}")
    rng = synth.rng_for(904, k, m, n)
    ell16 = bf16_values(rng, (m, n))
    data, i_ref = exact_intensities(ell16, rng)
    basis = synthetic_basis(rng, n, k, i_ref, phase=0.5)
    b = ctx.basis_import(basis)
    b.precision = fk.PREC_BF16
    out = host(ctx.transform(b, dev(data)))
    ref = pr.transform(data.astype(np.float64), basis)["im"]
    err = spectrum_err(out, ref)
    assert np.mean(err < TOL) >= 0.99 and err.max() < 1e-2, (np.mean(err < TOL), err.max())


def test_bf16_transform_tissue_error_vs_fp64(ctx):
    say("bf16 transform tissue")
    cube = synth.tissue_cube(rows=48, cols=40, n=256, map_key=3, noise_key=3, blur=4.0)
    p = wf.Params(k=12, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    res = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)
    b = ctx.basis_import(res["basis"])
    out32 = host(ctx.transform(b, dev(cube.i_cars)))
    b.precision = fk.PREC_BF16
    out16 = host(ctx.transform(b, dev(cube.i_cars)))
    ref = wf.transform(cube.i_cars.astype(np.float64), res["basis"])["im"]
    e32, e16 = spectrum_err(out32, ref), spectrum_err(out16, ref)
    say(f"bf16 transform tissue: max {e16.max():.2e} rms {np.sqrt(np.mean(e16 ** 2)):.2e} (fp32 max {e32.max():.2e})")
    assert e32.max() < TOL
    assert 1e-5 < e16.max() < 5e-2


# --------------------------------------------------------------------------
# End to end and serving
# --------------------------------------------------------------------------

def test_bf16_fit_lowrank(ctx):
    say("bf16 fit low-rank")
    cube = synth.lowrank_log_cube(4000, 300, rank=6, dtype=np.float32)
    p = wf.Params(k=6)
    ref = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)
    b, out, rep = ctx.fit(dev(cube.i_cars), cube.i_ref,
                          fk.params(k=6, gram_prec=fk.PREC_BF16, recon_prec=fk.PREC_BF16))
    out = host(out)
    assert b.precision == fk.PREC_BF16
    e = b.export()
    angle = np.linalg.norm(e["v"] @ e["v"].T - ref["basis"]["v"] @ ref["basis"]["v"].T, 2)
    err = spectrum_err(out, ref["im"])
    say(f"bf16 fit low-rank: subspace {angle:.2e}, output max {err.max():.2e} rms {np.sqrt(np.mean(err ** 2)):.2e}")
    assert angle < 1e-2 and err.max() < 5e-2
    # the device output equals Eq. 23 of its own basis with BF16 operands
    ell, _ = wf.log_ratio(cube.i_cars.astype(np.float64), e["i_ref"], e["ratio_floor"])
    z = pr.round_bf16(ell) @ pr.round_bf16(e["f"][:, None] * e["v"])
    own = pr.reconstruct(z, e)["im"]
    err_own = spectrum_err(out, own)
    say(f"bf16 fit low-rank: {np.mean(err_own < TOL):.4f} of spectra within {TOL} of the BF16 operand model")
    assert np.mean(err_own < TOL) >= FRAC and err_own.max() < 1e-2


@pytest.mark.parametrize("gram_prec,recon_prec", [(1, 0), (0, 1), (1, 1), (3, 3), (0, 3)])
def test_mixed_precision_fit(ctx, gram_prec, recon_prec):
    # Eq. 23 of the device's own (exported) basis is the parity target; the
    # distance to the FP64 oracle's fit, which also moves with the
    # eigenvectors past the retained spectrum, is reported.
    say(f"fit gram_prec={gram_prec} recon_prec={recon_prec}")
    cube = synth.tissue_cube(rows=40, cols=40, n=256, map_key=8, noise_key=8, blur=3.0)
    p = wf.Params(k=10, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    ref = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)
    b, out, rep = ctx.fit(dev(cube.i_cars), cube.i_ref,
                          fk.params(k=10, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g,
                                    gram_prec=gram_prec, recon_prec=recon_prec))
    out = host(out)
    assert b.precision == recon_prec
    e = b.export()
    ell, _ = wf.log_ratio(cube.i_cars.astype(np.float64), e["i_ref"], e["ratio_floor"])
    if recon_prec in (fk.PREC_FP32, fk.PREC_SPLIT):  # FP32-accurate projection and reconstruction
        own = wf.reconstruct((ell * e["f"]) @ e["v"], e)["im"]
        assert spectrum_err(out, own).max() < TOL
    else:
        own = pr.reconstruct(pr.round_bf16(ell) @ pr.round_bf16(e["f"][:, None] * e["v"]), e)["im"]
        err_own = spectrum_err(out, own)
        say(f"mixed fit: {np.mean(err_own < TOL):.4f} of spectra within {TOL} of the BF16 operand model")
        assert np.mean(err_own < TOL) >= FRAC and err_own.max() < 1e-2
    err = spectrum_err(out, ref["im"])
    say(f"mixed fit vs FP64 fit: max {err.max():.2e} rms {np.sqrt(np.mean(err ** 2)):.2e}")
    assert err.max() < 0.2


def test_bf16_server_tiles_equal_alone(ctx):
    say("bf16 server")
    rng = synth.rng_for(905, 1)
    n, k = 320, 12
    cube = synth.tissue_cube(rows=40, cols=40, n=n, map_key=31, noise_key=31, blur=3.0)
    p = wf.Params(k=k, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    basis = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)["basis"]
    b = ctx.basis_import(basis)
    b.precision = fk.PREC_BF16
    srv = fk.Server(0, hbm_budget_bytes=3 << 19, max_inflight=8, max_batch_rows=4096)
    bid = srv.add_basis(b)
    tiles = []
    for t in range(16):
        side = int(rng.integers(4, 17))
        c = synth.tissue_cube(rows=side, cols=side, n=n, map_key=500 + t, noise_key=600 + t, blur=1.0)
        tin = torch.empty((side * side, n), dtype=torch.float32, pin_memory=True)
        tin.copy_(torch.from_numpy(c.i_cars))
        tiles.append((c.i_cars, tin, torch.empty((side * side, n), pin_memory=True)))
    tickets = [srv.submit(bid, tin, tout) for (_, tin, tout) in tiles]
    for t in tickets:
        srv.wait(t)
    assert srv.stats()["completed"] == len(tiles)
    for arr, tin, tout in tiles:
        alone = ctx.transform(b, torch.from_numpy(arr).cuda())
        torch.cuda.synchronize()
        assert torch.equal(tout, alone.cpu())
    srv.close()
