"""Pins of the oracle's workflows (conventional, fKK-EC, ML:fKK-EC) against
identities the paper's derivation fixes and physical closed forms."""
import numpy as np
import pytest

import synth
from oracle import operators as op
from oracle import workflows as wf

LINEAR = dict(detrend=op.DETREND_WHITTAKER, als_lambda=1e4, ridge_rel=0.0)


def _small_cube(m_side=24, n=256, key=11):
    return synth.tissue_cube(rows=m_side, cols=m_side, n=n, map_key=key, noise_key=key,
                             blur=3.0, dtype=np.float64)


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


# --------------------------------------------------------------------------
# Factorisation (Eq. 6)
# --------------------------------------------------------------------------

def test_svd_routes_agree_and_full_rank_reconstructs():
    cube = _small_cube()
    ell, _ = wf.log_ratio(cube.i_cars, cube.i_ref, 1e-6)
    u1, s1, v1 = wf.truncated_svd(ell, 8, "gesdd")
    u2, s2, v2 = wf.truncated_svd(ell, 8, "gram")
    np.testing.assert_allclose(s1, s2, rtol=1e-10)
    # principal angles between the two 8-dim subspaces
    # distance between the two 8-dim subspaces (projector difference)
    assert np.linalg.norm(v1 @ v1.T - v2 @ v2.T, 2) < 1e-9
    # sign convention: largest-magnitude entry of each v positive
    idx = np.argmax(np.abs(v1), axis=0)
    assert np.all(v1[idx, np.arange(8)] > 0)
    n = ell.shape[1]
    u, s, v = wf.truncated_svd(ell, n, "gesdd")
    np.testing.assert_allclose((u * s) @ v.T, ell, atol=1e-12)


# --------------------------------------------------------------------------
# Factorisation identity: with a linear detrender and unregularised
# regression, fKK-EC on k vectors equals the conventional workflow on the
# rank-k log ratio (Eq. 7, 12, 16-18, 21-23 chained); at full rank it is the
# conventional workflow itself.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("sec_mode", [op.SEC_SAVGOL, op.SEC_MEAN])
def test_factorised_equals_conventional_on_rank_k_data(sec_mode):
    cube = _small_cube()
    p = wf.Params(k=6, sec_mode=sec_mode, **LINEAR)
    res = wf.fit(cube.i_cars, cube.i_ref, p)
    b = res["basis"]
    assert len(b["q"]) >= p.k
    ell_k = res["z"] @ b["v"].T / b["f"]            # rank-k log ratio
    i_k = cube.i_ref * np.exp(2.0 * ell_k)
    ref = wf.plain(i_k, cube.i_ref, p)
    for key in ("im", "re", "abs"):
        assert _rel(res[key], ref[key]) < 1e-11


def test_factorised_equals_conventional_at_full_rank_with_noise_scaling():
    cube = _small_cube(m_side=16, n=64, key=12)
    p = wf.Params(k=64, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g,
                  sg_window=21, **LINEAR)
    res = wf.fit(cube.i_cars, cube.i_ref, p)
    assert not np.allclose(res["basis"]["f"], res["basis"]["f"][0])
    ref = wf.plain(cube.i_cars, cube.i_ref, p)
    assert _rel(res["im"], ref["im"]) < 1e-9


# --------------------------------------------------------------------------
# NRB-only inputs (spec closed form): no Raman signal -> zero output.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("detrend", [op.DETREND_ALS, op.DETREND_WHITTAKER])
def test_nrb_only_returns_zero(detrend):
    w = synth.wavenumbers(200)
    ref = synth.reference(w)
    cube = np.tile(ref, (50, 1))
    p = wf.Params(k=5, detrend=detrend, als_lambda=1e4)
    assert np.abs(wf.fit(cube, ref, p)["im"]).max() == 0.0
    assert np.abs(wf.plain(cube, ref, p)["im"]).max() < 1e-15


def test_nrb_only_with_surrogate_error_is_small():
    # I = I_NRB but I_ref = Xi xi(w) I_NRB: only the smooth phase error
    # remains, which PEC removes up to the detrender's fit error.
    w = synth.wavenumbers(400)
    env = synth.envelope(w)
    ref = synth.reference(w)
    cube = np.tile(env, (40, 1)) * np.linspace(0.9, 1.1, 40)[:, None]
    p = wf.Params(k=3)
    no_pec = np.sin(op.hilbert(0.5 * np.log(env / ref)))
    assert np.abs(no_pec).max() > 0.2
    assert np.abs(wf.plain(cube, ref, p)["im"]).max() < 0.02
    assert np.abs(wf.fit(cube, ref, p)["im"]).max() < 0.02


# --------------------------------------------------------------------------
# Physics: retrieval of the known Im{chi/chi_nr}.
# --------------------------------------------------------------------------

def _mixture(n=1000, m=100, xi_slope=0.2, key=13):
    w = synth.wavenumbers(n)
    chi = synth.components(n, 3, key=key)
    ab = synth.rng_for(key, 99).dirichlet(np.ones(3), m)
    chi_r = ab @ chi
    env = synth.envelope(w)
    i_cars = np.abs(chi_r + 1.0) ** 2 * env
    ref = synth.reference(w, 1.1, xi_slope)
    return i_cars, ref, chi_r.imag


def _kk_floor(i_cars, ideal):
    """RSS of KK alone with the exact reference: the discretisation floor of
    a Hilbert transform over a finite window (Sec. 2.1)."""
    w = synth.wavenumbers(i_cars.shape[1])
    ell, _ = wf.log_ratio(i_cars, synth.envelope(w), 1e-6)
    kk = np.exp(ell) * np.sin(op.hilbert(ell))
    return ((kk - ideal) ** 2).sum(axis=1).mean()


def test_conventional_retrieves_raman_with_surrogate_reference():
    # RSS against the known Im{chi/chi_nr} (the paper's metric, Sec. 4.1).
    i_cars, ref, ideal = _mixture()
    p = wf.Params(k=20)
    out = wf.plain(i_cars, ref, p)["im"]
    rss = ((out - ideal) ** 2).sum(axis=1).mean()
    null = (ideal ** 2).sum(axis=1).mean()
    assert _kk_floor(i_cars, ideal) < 0.01 * null
    assert rss < 0.04 * null
    # without PEC/SEC (KK alone) the error is much larger
    ell, _ = wf.log_ratio(i_cars, ref, 1e-6)
    kk_only = np.exp(ell) * np.sin(op.hilbert(ell))
    assert ((kk_only - ideal) ** 2).sum(axis=1).mean() > 5 * rss


def test_factorised_close_to_conventional_and_ideal():
    # Sec. 4.1: similar RSS, the factorised one slightly lower.
    i_cars, ref, ideal = _mixture()
    p = wf.Params(k=20)
    fk = wf.fit(i_cars, ref, p)["im"]
    cv = wf.plain(i_cars, ref, p)["im"]
    null = (ideal ** 2).sum(axis=1).mean()
    rss_f = ((fk - ideal) ** 2).sum(axis=1).mean()
    rss_c = ((cv - ideal) ** 2).sum(axis=1).mean()
    assert rss_f < 0.04 * null and rss_c < 0.04 * null
    assert rss_f <= 1.05 * rss_c


def test_constant_nrb_agreement():
    # Sec. 4.1: with constant NRBs (xi = 1) the ideal, conventional and
    # factorised results agree.  Over a finite window they agree with the
    # ideal only down to the KK discretisation floor; with each other, far
    # below it.
    i_cars, ref, ideal = _mixture(xi_slope=0.0)
    p = wf.Params(k=40)
    fk = wf.fit(i_cars, ref, p)["im"]
    cv = wf.plain(i_cars, ref, p)["im"]
    floor = _kk_floor(i_cars, ideal)
    for out in (fk, cv):
        assert ((out - ideal) ** 2).sum(axis=1).mean() < 2.0 * floor
    assert ((fk - cv) ** 2).sum(axis=1).mean() < 0.05 * floor


# --------------------------------------------------------------------------
# SEC invariant, ML reuse, symmetries.
# --------------------------------------------------------------------------

def test_sec_mean_mode_zeroes_mean_log_magnitude():
    cube = _small_cube(key=14)
    p = wf.Params(k=8, sec_mode=op.SEC_MEAN, als_lambda=1e4)
    for res in (wf.fit(cube.i_cars, cube.i_ref, p), wf.plain(cube.i_cars, cube.i_ref, p)):
        assert np.abs(np.log(res["abs"]).mean(axis=1)).max() < 1e-13


def test_ml_transform_of_training_data_equals_fit():
    cube = _small_cube(key=15)
    p = wf.Params(k=10, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g, als_lambda=1e4)
    res = wf.fit(cube.i_cars, cube.i_ref, p)
    tr = wf.transform(cube.i_cars, res["basis"])
    assert _rel(tr["im"], res["im"]) < 1e-10
    # ridge in the regression shrinks Z by s^2/(s^2+lam) (Eq. 25 push-through)
    b = dict(res["basis"], ml_lambda=float(res["basis"]["s"][-1] ** 2))
    z = wf.regress_z(cube.i_cars, b)
    shrink = b["s"] ** 2 / (b["s"] ** 2 + b["ml_lambda"])
    np.testing.assert_allclose(z, res["z"] * shrink, atol=1e-10 * np.abs(res["z"]).max())


def test_scale_of_f_cancels():
    cube = _small_cube(key=16)
    p = wf.Params(k=8, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g, als_lambda=1e4)
    a = wf.fit(cube.i_cars, cube.i_ref, p)
    c = 7.0  # f(alpha / c^2, sigma / c) = c f
    b = wf.fit(cube.i_cars, cube.i_ref, p.with_(alpha=cube.alpha / c ** 2, sigma_g=cube.sigma_g / c))
    np.testing.assert_allclose(b["basis"]["f"], c * a["basis"]["f"], rtol=1e-12)
    assert _rel(b["im"], a["im"]) < 1e-9


def test_singular_vector_sign_flip_invariance():
    cube = _small_cube(key=17)
    p = wf.Params(k=8, als_lambda=1e4)
    res = wf.fit(cube.i_cars, cube.i_ref, p)
    b = res["basis"]
    flip = np.where(np.arange(8) % 3 == 0, -1.0, 1.0)
    b2 = wf.basis_from_factors(b["f"], b["s"], b["v"] * flip, res["z"] * flip, p)
    np.testing.assert_array_equal(np.sort(b2["q"]), np.sort(b["q"]))
    out2 = wf.reconstruct(res["z"] * flip, b2)
    assert _rel(out2["im"], res["im"]) < 1e-10


def test_rows_are_independent_under_transform_and_permutation():
    cube = _small_cube(key=18)
    p = wf.Params(k=8, als_lambda=1e4)
    res = wf.fit(cube.i_cars, cube.i_ref, p)
    perm = synth.rng_for(18, 1).permutation(cube.shape[0])
    tr = wf.transform(cube.i_cars[perm], res["basis"])
    assert _rel(tr["im"], res["im"][perm]) < 1e-10
    refit = wf.fit(cube.i_cars[perm], cube.i_ref, p)
    assert _rel(refit["im"], res["im"][perm]) < 1e-8


def test_clamping_of_invalid_ratios():
    ref = np.ones(5)
    i = np.array([[1.0, 0.0, -1.0, np.nan, np.inf]])
    ell, n_bad = wf.log_ratio(i, ref, 1e-6)
    assert n_bad == 4
    np.testing.assert_allclose(ell[0, 1:], 0.5 * np.log(1e-6))
    assert ell[0, 0] == 0.0


def test_q_is_union_of_column_extrema():
    z = np.array([[0.0, 5.0], [3.0, -1.0], [3.0, 2.0], [-2.0, -1.0]])
    # col 0: max first at row 1, min at row 3; col 1: max row 0, min first at row 1
    np.testing.assert_array_equal(wf.subsample_rows(z), [0, 1, 3])


def test_q_between_on_monotone_columns_is_evenly_spaced():
    # a column rising linearly from row 0 to row 60 has the level
    # min + (max - min) j / (s + 1) at row 60 j / (s + 1) exactly; a falling
    # column takes the mirrored rows; s = 0 is Eq. 13-15 alone
    m = 61
    z = np.column_stack([np.arange(m, dtype=float), 2.5 * (m - 1 - np.arange(m))])
    np.testing.assert_array_equal(wf.subsample_rows(z, 0), [0, 60])
    np.testing.assert_array_equal(wf.subsample_rows(z, 3), [0, 15, 30, 45, 60])
    np.testing.assert_array_equal(wf.subsample_rows(z, 2), [0, 20, 40, 60])
    # s = 4 puts the levels at 12, 24, 36, 48 of the rising column and at
    # the same rows of the falling one
    np.testing.assert_array_equal(wf.subsample_rows(z[:, 1:], 4), [0, 12, 24, 36, 48, 60])


def test_q_between_is_the_nearest_row_to_each_level_by_brute_force():
    # tiny random columns: every level's nearest row (first on ties), found
    # by checking all rows, is in q, and q holds nothing else
    rng = np.random.default_rng(9)
    z = np.round(rng.standard_normal((23, 3)), 1)  # repeated values: ties
    s = 3
    expect = set()
    for c in range(3):
        col = list(z[:, c])
        hi, lo = max(col), min(col)
        expect.add(col.index(hi))
        expect.add(col.index(lo))
        for j in range(1, s + 1):
            level = lo + (hi - lo) * j / (s + 1)
            dist = [abs(v - level) for v in col]
            expect.add(dist.index(min(dist)))
    np.testing.assert_array_equal(wf.subsample_rows(z, s), sorted(expect))


def test_q_between_keeps_the_factorisation_identity():
    # with linear detrending and no ridge, Phi_PEC solves the regression
    # exactly for any q of full column rank, so the extra rows leave the
    # output equal to the conventional workflow on the rank-k data
    cube = _small_cube()
    p = wf.Params(k=6, q_between=3, **LINEAR)
    res = wf.fit(cube.i_cars, cube.i_ref, p)
    b = res["basis"]
    assert len(b["q"]) > len(wf.subsample_rows(res["z"]))
    ell_k = res["z"] @ b["v"].T / b["f"]
    ref = wf.plain(cube.i_ref * np.exp(2.0 * ell_k), cube.i_ref, p)
    assert _rel(res["im"], ref["im"]) < 1e-11


# --------------------------------------------------------------------------
# Rank rule of Sec. 4.1 (k = 0)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,m,n", [(np.float32, 300, 120), (np.float64, 200, 90), (np.float32, 80, 150)])
def test_rank_rule_matches_numpy_matrix_rank(dtype, m, n):
    # singular values built around the cut-off s_max max(M, N) eps: seven
    # well above it, the rest well below; NumPy's own rank estimate on the
    # same matrix in its own data type must agree
    rng = np.random.default_rng(3)
    r = min(m, n)
    u, _ = np.linalg.qr(rng.standard_normal((m, r)))
    v, _ = np.linalg.qr(rng.standard_normal((n, r)))
    tol = max(m, n) * float(np.finfo(dtype).eps)
    s = np.concatenate([np.geomspace(1.0, 30 * tol, 7), np.geomspace(tol / 30, tol / 3000, r - 7)])
    a = ((u * s) @ v.T).astype(dtype)
    expected = int(np.linalg.matrix_rank(a))
    assert expected == 7
    sv = np.linalg.svd(a.astype(np.float64), compute_uv=False)
    assert wf.rank_cutoff(sv, m, n, float(np.finfo(dtype).eps)) == expected
    # "larger than": a value exactly at the cut-off is not counted
    assert wf.rank_cutoff(np.array([2.0, 2.0 * 10 * 1e-3]), 10, 4, 1e-3) == 1


def test_fit_with_rank_rule_equals_fit_at_that_rank():
    cube = synth.lowrank_log_cube(1500, 256, rank=4, noise=1e-6, dtype=np.float32)
    p = wf.Params(k=0, sg_window=101)
    auto = wf.fit(cube.i_cars, cube.i_ref, p)
    assert auto["basis"]["s"].shape == (4,)
    fixed = wf.fit(cube.i_cars, cube.i_ref, p.with_(k=4))
    np.testing.assert_array_equal(auto["im"], fixed["im"])
    # the same data in FP64 has a smaller epsilon: the noise floor is kept
    # too, up to k_max
    auto64 = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p.with_(k_max=12))
    assert auto64["basis"]["s"].shape == (12,)


# --------------------------------------------------------------------------
# Randomized range finder (Halko, Martinsson & Tropp 2011)
# --------------------------------------------------------------------------

def _matrix_with_spectrum(m, n, s, seed):
    rng = np.random.default_rng(seed)
    u, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    v, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    return (u * s) @ v.T, u, v


@pytest.mark.parametrize("power_iters", [0, 1, 2])
def test_randomized_svd_exact_on_low_rank(power_iters):
    # rank r <= l: the range of A Omega is the range of A, so the factors
    # are the exact ones
    s_true = np.array([50.0, 20.0, 7.0, 3.0, 1.0, 0.4])
    a, u, v = _matrix_with_spectrum(400, 120, s_true, 1)
    omega = np.random.default_rng(2).standard_normal((120, 10))
    ur, sr, vr = wf.randomized_svd(a, 6, omega, power_iters)
    np.testing.assert_allclose(sr, s_true, rtol=1e-12)
    assert np.linalg.norm(vr @ vr.T - v @ v.T, 2) < 1e-12
    assert np.linalg.norm(ur @ ur.T - u @ u.T, 2) < 1e-12
    np.testing.assert_allclose((ur * sr) @ vr.T, a, atol=1e-11)


def test_randomized_svd_interlaces_and_improves_with_iterations():
    # singular values of Q^T A never exceed those of A (Q orthonormal);
    # with a test matrix spanning the top right singular vectors the result
    # is exact; subspace iteration brings the estimates towards the truth
    s_true = 1.0 / np.arange(1, 81) ** 1.5
    a, u, v = _matrix_with_spectrum(300, 80, s_true, 3)
    omega = np.random.default_rng(4).standard_normal((80, 15))
    errs = []
    for q in (0, 1, 3):
        _, sr, _ = wf.randomized_svd(a, 10, omega, q)
        assert np.all(sr <= s_true[:10] * (1 + 1e-12))
        errs.append(np.max(np.abs(sr - s_true[:10]) / s_true[:10]))
    assert errs[0] > errs[1] > errs[2]
    _, sr, vr = wf.randomized_svd(a, 10, v[:, :15] @ np.random.default_rng(5).standard_normal((15, 15)), 0)
    np.testing.assert_allclose(sr, s_true[:10], rtol=1e-10)


def test_fit_with_randomized_svd_equals_exact_on_low_rank_data():
    cube = synth.lowrank_log_cube(1200, 200, rank=5, noise=0.0)
    p = wf.Params(k=5, sg_window=61)
    omega = np.random.default_rng(6).standard_normal((200, 15))
    exact = wf.fit(cube.i_cars, cube.i_ref, p)
    rr = wf.fit(cube.i_cars, cube.i_ref, p, svd="randomized", omega=omega, power_iters=1)
    assert np.array_equal(np.sort(rr["basis"]["q"]), np.sort(exact["basis"]["q"]))
    assert _rel(rr["im"], exact["im"]) < 1e-10


# --------------------------------------------------------------------------
# Basis adequacy (retraining criterion, Sec. 5)
# --------------------------------------------------------------------------

def test_basis_residual_in_span_orthogonal_and_mixed():
    rng = np.random.default_rng(9)
    n, k = 120, 5
    v, _ = np.linalg.qr(rng.standard_normal((n, k)))
    f = rng.uniform(0.5, 2.0, n)
    i_ref = rng.uniform(1.0, 2.0, n)
    basis = {"v": v, "f": f, "i_ref": i_ref, "ratio_floor": 1e-6}

    def spectra(a):  # intensities whose A = l diag(f) is a
        return i_ref * np.exp(2.0 * a / f)

    inside = rng.standard_normal((40, k)) @ v.T
    outside = rng.standard_normal((40, n))
    outside -= (outside @ v) @ v.T
    assert wf.basis_residual(spectra(inside), basis) < 1e-12
    assert abs(wf.basis_residual(spectra(outside), basis) - 1.0) < 1e-12
    mix = inside + 0.3 * outside
    expected = np.linalg.norm(0.3 * outside) / np.linalg.norm(mix)
    assert abs(wf.basis_residual(spectra(mix), basis) - expected) < 1e-12


# --------------------------------------------------------------------------
# SEC in the real-part form of Eq. 4-5 (conventional workflow)
# --------------------------------------------------------------------------

def test_sec_real_part_form_mean_and_scale():
    cube = _small_cube(key=16)
    p = wf.Params(sec_mode=op.SEC_MEAN, sec_form=1, als_lambda=1e4)
    out = wf.plain(cube.i_cars, cube.i_ref, p)
    # Eq. 4: after correction the mean real part over frequency is 1
    assert np.abs(out["re"].mean(axis=1) - 1.0).max() < 1e-13
    # SEC removes the constant amplitude error Xi of the reference (Sec. 2.1)
    for sec_mode in (op.SEC_MEAN, op.SEC_SAVGOL):
        q = p.with_(sec_mode=sec_mode, sg_window=51)
        a = wf.plain(cube.i_cars, cube.i_ref, q)
        b = wf.plain(cube.i_cars, 3.7 * cube.i_ref, q)
        assert _rel(b["im"], a["im"]) < 1e-11
    # the phase (and so Im/Re up to the positive scale) is the log form's
    lg = wf.plain(cube.i_cars, cube.i_ref, p.with_(sec_form=0))
    np.testing.assert_allclose(np.arctan2(out["im"], out["re"]), np.arctan2(lg["im"], lg["re"]), atol=1e-12)
    # NRB-only input: zero Raman
    w = synth.wavenumbers(200)
    ref = synth.reference(w)
    nrb = wf.plain(np.tile(ref, (20, 1)), ref, wf.Params(sec_form=1, als_lambda=1e4))
    assert np.abs(nrb["im"]).max() < 1e-15 and np.abs(nrb["re"] - 1.0).max() < 1e-14


# --------------------------------------------------------------------------
# Ridge weight of Eq. 17 on hand-worked cases
# --------------------------------------------------------------------------

def test_ridge_lambda_hand_cases():
    # X = diag(3, 1): X^T X = diag(9, 1), largest eigenvalue 9 (not the trace
    # 10, the largest singular value 3 or the smallest eigenvalue 1)
    x = np.array([[3.0, 0.0], [0.0, 1.0]])
    assert wf.ridge_lambda(x, 1e-6) == pytest.approx(9e-6, rel=1e-14)
    # rank one: rows (1, 2) and (2, 4): X^T X = [[5, 10], [10, 20]], eigenvalues 25 and 0
    x = np.array([[1.0, 2.0], [2.0, 4.0]])
    assert wf.ridge_lambda(x, 0.5) == pytest.approx(12.5, rel=1e-14)
    # 3 x 2 with orthogonal columns of norms 2 and sqrt(2): X^T X = diag(4, 2)
    x = np.array([[2.0, 0.0], [0.0, 1.0], [0.0, -1.0]])
    assert wf.ridge_lambda(x, 1.0) == pytest.approx(4.0, rel=1e-14)
    # rel = 0 (the identity tests) and X = 0 give no regularisation
    assert wf.ridge_lambda(x, 0.0) == 0.0
    assert wf.ridge_lambda(np.zeros((4, 3)), 1e-6) == 0.0


def test_ridge_lambda_is_what_the_fit_uses():
    cube = _small_cube(m_side=12, n=128, key=21)
    p = wf.Params(k=5, ridge_rel=1e-3)
    b = wf.fit(cube.i_cars, cube.i_ref, p)["basis"]
    x = b["x"]
    assert b["ridge_lambda"] == pytest.approx(1e-3 * np.linalg.norm(x, 2) ** 2, rel=1e-12)


# --------------------------------------------------------------------------
# Variance scaling f of Eq. 9: its purpose is unit variance of f A over an
# image of one repeated spectrum under Poisson + Gaussian noise (first-order
# error propagation through the logarithm)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,sigma_g", [(4e-4, 5e-3), (1e-5, 2e-2), (5e-4, 0.0)])
def test_scaling_f_gives_unit_variance_on_repeated_spectrum(alpha, sigma_g):
    n, m = 64, 200_000
    w = np.linspace(0.0, 1.0, n)
    i0 = 2.0 + 6.0 * np.exp(-((w - 0.4) / 0.15) ** 2)      # 2 ... 8: I0^2 differs from I0
    i_ref = 1.5 + w                                          # noiseless reference
    rng = np.random.default_rng(909)
    sd = np.sqrt(alpha * i0 + sigma_g ** 2)                  # Poisson (Gaussian limit) + Gaussian
    assert np.all(sd / i0 < 0.02)                            # inside the first-order regime
    i_cars = i0 + sd * rng.standard_normal((m, n))
    p = wf.Params(f_mode=wf.F_NOISE, alpha=alpha, sigma_g=sigma_g)
    f = wf.scaling_f(i_cars, p)
    ell, _ = wf.log_ratio(i_cars, i_ref, 1e-6)
    std = (ell * f).std(axis=0)
    # sampling error of a standard deviation over 2e5 rows: 0.16 %
    assert np.all(np.abs(std - 1.0) < 0.01), (std.min(), std.max())
    # f itself: 2 <I> / sqrt(alpha <I> + sigma_g^2), computed per wavenumber
    mean = i_cars.mean(axis=0)
    np.testing.assert_allclose(f, 2.0 * mean / np.sqrt(alpha * mean + sigma_g ** 2), rtol=1e-14)


def test_scaling_f_one_mode_and_awgn_form():
    # f_mode one gives f = 1; with alpha = 0 (AWGN) f = 2 <I> / sigma_g
    rng = np.random.default_rng(3)
    i_cars = 1.0 + rng.random((50, 16))
    np.testing.assert_array_equal(wf.scaling_f(i_cars, wf.Params()), np.ones(16))
    f = wf.scaling_f(i_cars, wf.Params(f_mode=wf.F_NOISE, alpha=0.0, sigma_g=0.25))
    np.testing.assert_allclose(f, 8.0 * i_cars.mean(axis=0), rtol=1e-14)
