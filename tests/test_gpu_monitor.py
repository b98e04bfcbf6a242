"""Basis adequacy on the device (the retraining criterion of Sec. 5: retrain
when the stored basis no longer supports new data): the per-spectrum sums
the fused transform writes, against the FP64 oracle on the same basis, and
the serving runtime's per-tile residuals and flags on frames drawn from the
training components and from other components."""
import sys

import numpy as np
import pytest

import synth
from oracle import precision as pr
from oracle import workflows as wf

torch = pytest.importorskip("torch")
fk = pytest.importorskip("paper_2005_07132_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def pinned(a):
    t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)))
    return t


def oracle_norms(i_cars, basis):
    """||A_m||^2 and ||A_m V||^2 per spectrum, A = l diag(f) (FP64)."""
    ell, _ = wf.log_ratio(i_cars.astype(np.float64), basis["i_ref"], basis["ratio_floor"])
    a = ell * basis["f"]
    return (a * a).sum(axis=1), ((a @ basis["v"]) ** 2).sum(axis=1)


@pytest.fixture(scope="module")
def trained():
    ctx = fk.Context(0)
    cube = synth.tissue_cube(rows=48, cols=48, n=256, map_key=41, noise_key=41, blur=4.0)
    p = wf.Params(k=10, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    basis = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)["basis"]
    yield ctx, cube, basis
    ctx.close()


@pytest.mark.parametrize("ml_lambda", [0.0, 1.0])
def test_fused_transform_norms_match_oracle(trained, ml_lambda):
    ctx, cube, basis = trained
    say(f"transform norms ml_lambda={ml_lambda}")
    basis = dict(basis, ml_lambda=ml_lambda * float(basis["s"][5] ** 2))
    b = ctx.basis_import(basis)
    # 1,000 spectra: several blocks and a ragged last one
    new = synth.tissue_cube(rows=20, cols=50, n=256, map_key=44, noise_key=44, blur=3.0)
    t = dev(new.i_cars)
    ref_a, ref_z = oracle_norms(new.i_cars, basis)
    for prec in (fk.PREC_FP32, fk.PREC_BF16):
        b.precision = prec
        norms = torch.empty((t.shape[0], 2), dtype=torch.float32, device="cuda")
        out = ctx.transform(b, t, norms=norms)
        plain = ctx.transform(b, t)
        torch.cuda.synchronize()
        assert torch.equal(out, plain)  # the sums change nothing in the output
        got = norms.cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got[:, 0], ref_a, rtol=1e-5)  # FP32 log ratio, FP32 sums
        if prec == fk.PREC_FP32:
            np.testing.assert_allclose(got[:, 1], ref_z, rtol=1e-5)
            # 1 - sum z / sum a: the residual of the oracle
            r = np.sqrt(max(0.0, 1.0 - got[:, 1].sum() / got[:, 0].sum()))
            ref_r = wf.basis_residual(new.i_cars.astype(np.float64), basis)
            assert abs(r - ref_r) <= 1e-4 * ref_r + 1e-3
        else:
            # BF16 projection operands: the sums of the BF16 operand model
            ell, _ = wf.log_ratio(new.i_cars.astype(np.float64), basis["i_ref"], basis["ratio_floor"])
            s = np.asarray(basis["s"])
            shrink = s * s / (s * s + basis["ml_lambda"]) if basis["ml_lambda"] > 0 else np.ones_like(s)
            z16 = pr.contract(ell, pr.projection_weights(basis)) / shrink
            np.testing.assert_allclose(got[:, 1], (z16 ** 2).sum(axis=1), rtol=2e-3)


def test_basis_residual_call_matches_transform_sums(trained):
    ctx, cube, basis = trained
    say("basis residual vs transform sums")
    b = ctx.basis_import(basis)
    new = synth.tissue_cube(rows=33, cols=31, n=256, map_key=45, noise_key=45, blur=3.0)
    t = dev(new.i_cars)
    norms = torch.empty((t.shape[0], 2), dtype=torch.float32, device="cuda")
    ctx.transform(b, t, norms=norms)
    got = norms.double().sum(dim=0).cpu().numpy()
    r_sums = np.sqrt(1.0 - got[1] / got[0])
    r_call = ctx.residual(b, t)
    assert abs(r_call - r_sums) < 1e-6
    assert abs(r_call - wf.basis_residual(new.i_cars.astype(np.float64), basis)) < 1e-3


@pytest.mark.parametrize("prec", [fk.PREC_FP32, fk.PREC_BF16])
def test_server_flags_tiles_the_basis_does_not_support(trained, prec):
    ctx, cube, basis = trained
    say(f"server residual flags prec={prec}")
    b = ctx.basis_import(basis)
    b.precision = prec
    # tiles of new frames: the training components (supported) and other
    # components (not); the threshold sits between the two oracle residuals
    same = [synth.tissue_cube(rows=24, cols=24, n=256, map_key=500 + i, noise_key=600 + i, blur=3.0)
            for i in range(6)]
    other = [synth.tissue_cube(rows=24, cols=24, n=256, map_key=700 + i, noise_key=800 + i, comp_key=43, blur=3.0)
             for i in range(6)]
    r_same = [wf.basis_residual(c.i_cars.astype(np.float64), basis) for c in same]
    r_other = [wf.basis_residual(c.i_cars.astype(np.float64), basis) for c in other]
    say(f"oracle residuals same {min(r_same):.4f}-{max(r_same):.4f}, other {min(r_other):.4f}-{max(r_other):.4f}")
    assert max(r_same) * 1.2 < min(r_other)
    thr = 0.5 * (max(r_same) + min(r_other))
    srv = fk.Server(0, hbm_budget_bytes=64 << 20, max_inflight=8, max_batch_rows=8192, residual_threshold=thr)
    bid = srv.add_basis(b)
    tiles = []
    for i, c in enumerate(same + other):
        tiles.append((i >= len(same), c, pinned(c.i_cars), torch.empty(c.i_cars.shape, pin_memory=True)))
    tickets = [srv.submit(bid, tin, tout) for (_, _, tin, tout) in tiles]
    tol = 1e-3 if prec == fk.PREC_FP32 else 2e-2
    for (is_other, c, _, _), tk in zip(tiles, tickets):
        _, r = srv.wait(tk, with_residual=True)
        ref = wf.basis_residual(c.i_cars.astype(np.float64), basis)
        assert abs(r - ref) <= tol, (r, ref)
        assert (r > thr) == is_other
    st = srv.stats()
    assert st["flagged"] == len(other)
    assert st["max_residual"] == pytest.approx(max(r_other), abs=tol)
    srv.close()
