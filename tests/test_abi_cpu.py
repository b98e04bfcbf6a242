"""C ABI checks that need no GPU: the library loads and exports every
declared symbol, parameter defaults and validation, and the host FP64 stages
(eigensolver, basis-vector KK/PEC/SEC) against the oracle."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import operators as op
from oracle import workflows as wf

fk = pytest.importorskip("paper_2005_07132_amd")

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fkkec.h")

if not os.path.exists(fk.LIB_PATH):
    pytest.skip("libfkkec.so not built", allow_module_level=True)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fkk_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    L = fk.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(fk.SYMBOLS)
    assert L.fkk_version() == 1


def test_status_strings():
    L = fk.lib()
    assert L.fkk_status_string(0) == b"ok"
    assert L.fkk_status_string(-1) == b"invalid argument"


def test_param_defaults_match_oracle_readings():
    p = fk.params()
    q = wf.Params()
    for name in ("k", "f_mode", "pad_mode", "fft_len", "detrend", "als_lambda", "als_p", "als_iters",
                 "ridge_rel", "sec_mode", "sg_window", "sg_order", "ml_lambda", "ratio_floor"):
        assert getattr(p, name) == getattr(q, name), name


@pytest.mark.parametrize("n,k", [(50, 5), (257, 20), (1000, 50)])
def test_eigh_topk_matches_lapack(n, k):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n + 30, n))
    g = a.T @ a
    vals, vecs = fk.eigh_topk(g, k)
    w, v = np.linalg.eigh(g)
    ref_vals = w[::-1][:k]
    np.testing.assert_allclose(vals, ref_vals, rtol=0, atol=1e-12 * w[-1])
    ref = v[:, ::-1][:, :k]
    assert np.linalg.norm(vecs @ vecs.T - ref @ ref.T, 2) < 1e-10
    np.testing.assert_allclose(vecs.T @ vecs, np.eye(k), atol=1e-12)
    idx = np.argmax(np.abs(vecs), axis=0)
    assert np.all(vecs[idx, np.arange(k)] > 0)


def test_eigh_topk_degenerate_and_zero():
    vals, vecs = fk.eigh_topk(np.zeros((10, 10)), 3)
    assert np.all(vals == 0)
    np.testing.assert_allclose(vecs.T @ vecs, np.eye(3))
    d = np.diag([5.0, 5.0, 5.0, 1.0, 0.5])
    vals, vecs = fk.eigh_topk(d, 3)
    np.testing.assert_allclose(vals, [5, 5, 5], atol=1e-14)
    np.testing.assert_allclose(vecs.T @ vecs, np.eye(3), atol=1e-12)
    assert np.abs(vecs[3:]).max() < 1e-12


def _oracle_basis(detrend, sec, n=256, k=8, **kw):
    cube = synth.tissue_cube(rows=32, cols=32, n=n, blur=3.0, dtype=np.float64)
    p = wf.Params(k=k, detrend=detrend, sec_mode=sec, f_mode=wf.F_NOISE, alpha=cube.alpha,
                  sigma_g=cube.sigma_g, **kw)
    return cube, p, wf.fit(cube.i_cars, cube.i_ref, p)["basis"]


@pytest.mark.parametrize("detrend,tol", [(op.DETREND_ALS, 1e-8), (op.DETREND_WHITTAKER, 1e-11)])
@pytest.mark.parametrize("sec", [op.SEC_SAVGOL, op.SEC_MEAN])
def test_host_basis_math_matches_oracle(detrend, tol, sec):
    # ALS solves are ill-conditioned (lam / p ~ 1e7): rounding differences
    # between two banded solvers grow to ~1e-10 relative.
    cube, p, b = _oracle_basis(detrend, sec)
    cp = fk.params(k=p.k, detrend=detrend, sec_mode=sec, f_mode=1, alpha=cube.alpha, sigma_g=cube.sigma_g)
    e = fk.basis_from_factors(None, cube.i_ref, b["f"], b["s"], b["v"], b["x"], cp).export()
    for key in ("h_v", "phi_pec_t", "v_sec_t", "b_re", "b_im"):
        err = np.abs(e[key] - b[key]).max() / np.abs(b[key]).max()
        assert err < tol, (key, err)
    assert e["ridge_lambda"] == pytest.approx(b["ridge_lambda"], rel=1e-12)


def test_host_basis_zero_pad_custom_fft_and_window():
    cube, p, b = _oracle_basis(op.DETREND_ALS, op.SEC_SAVGOL, n=200, k=6, pad_mode=op.PAD_ZERO, fft_len=1024,
                               sg_window=51, sg_order=3, als_lambda=300.0, ridge_rel=1e-4)
    cp = fk.params(k=6, f_mode=1, alpha=cube.alpha, sigma_g=cube.sigma_g, pad_mode=1, fft_len=1024, sg_window=51,
                   sg_order=3, als_lambda=300.0, ridge_rel=1e-4)
    e = fk.basis_from_factors(None, cube.i_ref, b["f"], b["s"], b["v"], b["x"], cp).export()
    for key in ("h_v", "b_re", "b_im"):
        assert np.abs(e[key] - b[key]).max() / np.abs(b[key]).max() < 1e-8, key


def test_host_basis_zero_x_gives_no_phase_error():
    n, k = 64, 3
    rng = np.random.default_rng(9)
    v, _ = np.linalg.qr(rng.standard_normal((n, k)))
    e = fk.basis_from_factors(None, np.ones(n), np.ones(n), np.ones(k), v, np.zeros((4, k)),
                              fk.params(k=k, sg_window=21)).export()
    assert np.all(e["phi_pec_t"] == 0.0)
    ref = wf.basis_from_factors(np.ones(n), np.ones(k), v, np.zeros((4, k)), wf.Params(k=k, sg_window=21), q=[0, 1, 2, 3])
    np.testing.assert_allclose(e["b_re"], ref["b_re"], atol=1e-13)


@pytest.mark.parametrize("kw", [dict(k=0), dict(k=300), dict(sg_window=10), dict(sg_window=2001),
                                dict(fft_len=1000), dict(als_p=0.0), dict(als_iters=0), dict(ratio_floor=0.0), dict(ratio_floor=1e-39),
                                dict(output=7), dict(detrend=5), dict(ridge_rel=-1.0),
                                dict(f_mode=1, alpha=0.0, sigma_g=0.0), dict(gram_prec=4), dict(recon_prec=2), dict(recon_prec=-1),
                                dict(svd_mode=2), dict(svd_mode=1, rrf_power_iters=-1),
                                dict(svd_mode=1, rrf_oversample=-1), dict(svd_mode=1, k=120, rrf_oversample=10),
                                dict(sec_form=1), dict(sec_form=2), dict(q_between=-1), dict(q_between=17)])
def test_parameter_validation(kw):
    n = 256
    base = dict(k=4)
    base.update(kw)
    p = fk.params(**base)
    k = 4
    v = np.linalg.qr(np.random.default_rng(1).standard_normal((n, k)))[0]
    with pytest.raises(fk.FkkError) as err:
        fk.basis_from_factors(None, np.ones(n), np.ones(n), np.ones(k), v, np.ones((3, k)), p)
    assert err.value.status in (-1, -7)


def test_basis_precision_accessors():
    n, k = 64, 3
    v = np.linalg.qr(np.random.default_rng(2).standard_normal((n, k)))[0]
    b = fk.basis_from_factors(None, np.ones(n), np.ones(n), np.ones(k), v, np.ones((3, k)),
                              fk.params(k=k, sg_window=21))
    assert b.precision == fk.PREC_FP32
    b.precision = fk.PREC_BF16
    assert b.precision == fk.PREC_BF16
    with pytest.raises(fk.FkkError):
        b.precision = 2
    assert b.precision == fk.PREC_BF16


def test_host_stages_from_two_threads_at_once():
    # separate contexts on separate host threads share the library's host
    # thread pool: concurrent host stages must give the results of the same
    # calls made one after the other
    import threading
    cube, p, b = _oracle_basis(op.DETREND_ALS, op.SEC_SAVGOL, n=256, k=8)
    cp = fk.params(k=p.k, f_mode=1, alpha=cube.alpha, sigma_g=cube.sigma_g)
    rng = np.random.default_rng(12)
    a = rng.standard_normal((700, 600))
    g = a.T @ a
    ref_basis = fk.basis_from_factors(None, cube.i_ref, b["f"], b["s"], b["v"], b["x"], cp).export()
    ref_vals, ref_vecs = fk.eigh_topk(g, 30)
    errors = []

    def basis_worker():
        try:
            for _ in range(12):
                e = fk.basis_from_factors(None, cube.i_ref, b["f"], b["s"], b["v"], b["x"], cp).export()
                for key in ("h_v", "phi_pec_t", "b_re", "b_im"):
                    np.testing.assert_array_equal(e[key], ref_basis[key])
        except Exception as exc:  # pragma: no cover - reported below
            errors.append(exc)

    def eig_worker():
        try:
            for _ in range(12):
                vals, vecs = fk.eigh_topk(g, 30)
                np.testing.assert_array_equal(vals, ref_vals)
                np.testing.assert_array_equal(vecs, ref_vecs)
        except Exception as exc:  # pragma: no cover - reported below
            errors.append(exc)

    threads = [threading.Thread(target=basis_worker), threading.Thread(target=eig_worker),
               threading.Thread(target=basis_worker)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors


def test_workspace_sizes():
    p = fk.params(k=50)
    fit_small = fk.workspace_size(fk.OP_FIT, 4096, 512, p)
    fit_large = fk.workspace_size(fk.OP_FIT, 703026, 1000, p)
    # the log ratio alone is M x npad floats; the whole fit stays well under twice that plus the Gram partials
    assert 703026 * 1024 * 4 < fit_large < 2 * 703026 * 1024 * 4 + (1 << 30)
    assert fit_small < fit_large
    assert fk.workspace_size(fk.OP_FIT, 4096, 512, fk.params(k=0)) >= fit_small  # rank rule sizes for 128 vectors
    assert fk.workspace_size(fk.OP_TRANSFORM, 703026, 1000) == 0
    plain = fk.workspace_size(fk.OP_PLAIN, 703026, 1000, p)
    assert plain >= 131072 * 1000 * 8 * 7  # batches of 131,072 spectra, seven FP64 rows each
    assert fk.workspace_size(fk.OP_PLAIN, 300, 1000, p) < plain
    for bad in (lambda: fk.workspace_size(7, 10, 100, p), lambda: fk.workspace_size(fk.OP_FIT, 0, 100, p),
                lambda: fk.workspace_size(fk.OP_FIT, 10, 100, fk.params(k=500))):
        with pytest.raises(fk.FkkError):
            bad()
