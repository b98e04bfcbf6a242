"""Pins of the BF16 operand model (oracle/precision.py): the rounding against
hand-worked values, torch's own BF16 conversion and its error bound; the
rewritten regression weights against the oracle's regression route."""
import numpy as np
import pytest

import synth
from oracle import precision as pr
from oracle import workflows as wf


def test_round_bf16_hand_values():
    u = 2.0 ** -7  # spacing of BF16 in [1, 2)
    cases = [
        (1.0, 1.0),
        (1.0 + u / 2, 1.0),               # tie -> even (mantissa 0)
        (1.0 + 3 * u / 2, 1.0 + 2 * u),   # tie -> even (mantissa 2)
        (1.0 + u / 2 + 1e-12, 1.0 + u),   # just above the tie
        (-(1.0 + 3 * u / 2), -(1.0 + 2 * u)),
        (2.0 - u / 4, 2.0),               # carry into the exponent
        (0.0, 0.0),
        (3.0, 3.0),
        (1.0 / 3.0, 0.333984375),         # 171 / 512
        (1e-3, 0.00099945068359375),      # 131 / 2^17
    ]
    for x, want in cases:
        assert pr.round_bf16(x) == want, x


def test_round_bf16_matches_torch_on_float32_values():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 6, 20000),
                        rng.uniform(-2, 2, 20000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(pr.round_bf16(x.astype(np.float64)), ref)


def test_round_bf16_error_bound_and_idempotence():
    rng = np.random.default_rng(6)
    x = rng.standard_normal(50000) * 10.0 ** rng.uniform(-4, 4, 50000)
    r = pr.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))  # half a unit of 8 bits
    np.testing.assert_array_equal(pr.round_bf16(r), r)
    assert np.mean(r != x) > 0.99


def test_bf16_gram_within_rounding_bound():
    cube = synth.tissue_cube(rows=12, cols=12, n=96, map_key=3, noise_key=3, blur=2.0, dtype=np.float64)
    ell, _ = wf.log_ratio(cube.i_cars, cube.i_ref, 1e-6)
    g = ell.T @ ell
    g16 = pr.gram(cube.i_cars, cube.i_ref, 1e-6)
    bound = (2 * 2.0 ** -8 + 2.0 ** -16) * (np.abs(ell).T @ np.abs(ell))
    assert np.all(np.abs(g16 - g) <= bound + 1e-300)
    assert np.abs(g16 - g).max() > 0  # the rounding is applied
    np.testing.assert_array_equal(g16, g16.T)


@pytest.mark.parametrize("lam", [0.0, 3.0])
def test_projection_weights_equal_the_regression(lam):
    cube = synth.tissue_cube(rows=10, cols=10, n=80, map_key=4, noise_key=4, blur=2.0, dtype=np.float64)
    p = wf.Params(k=6, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g, ml_lambda=lam)
    basis = wf.fit(cube.i_cars, cube.i_ref, p)["basis"]
    new = synth.tissue_cube(rows=5, cols=5, n=80, map_key=40, noise_key=41, blur=2.0, dtype=np.float64)
    ell, _ = wf.log_ratio(new.i_cars, basis["i_ref"], basis["ratio_floor"])
    z_w = ell @ pr.projection_weights(basis)
    z_r = wf.regress_z(new.i_cars, basis)
    np.testing.assert_allclose(z_w, z_r, rtol=1e-9, atol=1e-9 * np.abs(z_r).max())


def test_bf16_transform_close_to_fp64_transform():
    cube = synth.tissue_cube(rows=10, cols=10, n=128, map_key=7, noise_key=7, blur=2.0, dtype=np.float64)
    p = wf.Params(k=8, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    basis = wf.fit(cube.i_cars, cube.i_ref, p)["basis"]
    exact = wf.transform(cube.i_cars, basis)
    low = pr.transform(cube.i_cars, basis)
    err = np.abs(low["im"] - exact["im"]).max(axis=1) / np.abs(exact["im"]).max(axis=1)
    assert 1e-5 < err.max() < 5e-2  # BF16 operands: ~1e-3, not exact


def test_contract_rule_exact_on_bf16_operands_and_bounded_otherwise():
    rng = np.random.default_rng(8)
    a16 = pr.round_bf16(rng.standard_normal((30, 20)))
    b16 = pr.round_bf16(rng.standard_normal((20, 10)))
    np.testing.assert_array_equal(pr.contract(a16, b16), a16 @ b16)  # operands already BF16
    a = rng.standard_normal((30, 20))
    b = rng.standard_normal((20, 10))
    err = np.abs(pr.contract(a, b) - a @ b)
    assert np.all(err <= (2 * 2.0 ** -8 + 2.0 ** -16) * (np.abs(a) @ np.abs(b)))
    assert err.max() > 0


def test_bf16_transform_is_the_rule_applied_to_each_contraction():
    cube = synth.tissue_cube(rows=8, cols=8, n=96, map_key=9, noise_key=9, blur=2.0, dtype=np.float64)
    p = wf.Params(k=6, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    basis = wf.fit(cube.i_cars, cube.i_ref, p)["basis"]
    ell, _ = wf.log_ratio(cube.i_cars, basis["i_ref"], basis["ratio_floor"])
    # written out: every operand of the three products rounded, sums exact
    z = pr.round_bf16(ell) @ pr.round_bf16(pr.projection_weights(basis))
    z16 = pr.round_bf16(z)
    want = wf.retrieve(z16 @ pr.round_bf16(basis["b_re"]), z16 @ pr.round_bf16(basis["b_im"]))["im"]
    np.testing.assert_array_equal(pr.transform(cube.i_cars, basis)["im"], want)
    # the labelled variant that leaves Z unrounded differs, by about one BF16 rounding of Z
    other = pr.transform_full_precision_z(cube.i_cars, basis)["im"]
    assert 0 < np.abs(other - want).max() < 5e-2 * np.abs(want).max()
