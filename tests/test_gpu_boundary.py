"""The C ABI's ownership rules on the GPU: a fit, the plain method and the
transform running in a caller-owned (torch-allocated) workspace with no
device allocation during the call; the output plane of the transform; a
basis held by a server cannot be freed; the server's host-buffer checks."""
import sys

import numpy as np
import pytest

import synth
from oracle import workflows as wf

torch = pytest.importorskip("torch")
fk = pytest.importorskip("paper_2005_07132_amd")

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


def cube_and_params(rows=48, cols=40, n=256, key=41, **kw):
    cube = synth.tissue_cube(rows=rows, cols=cols, n=n, map_key=key, noise_key=key, blur=4.0)
    args = dict(k=12, f_mode=fk.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    args.update(kw)
    return cube, fk.params(**args)


@pytest.mark.parametrize("kw", [dict(), dict(gram_prec=fk.PREC_FP64, q_between=2), dict(recon_prec=fk.PREC_BF16),
                                dict(svd_mode=fk.SVD_RANDOMIZED), dict(k=0)])
def test_fit_in_caller_workspace_allocates_nothing(kw):
    say(f"fit in caller workspace {kw}")
    cube, p = cube_and_params(**kw)
    m, n = cube.shape
    t = dev(cube.i_cars)
    own = fk.Context(0)
    b_ref, out_ref, _ = own.fit(t, cube.i_ref, p)
    ref = host(out_ref)
    assert own.workspace_bytes() > 0
    need = fk.workspace_size(fk.OP_FIT, m, n, p)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = torch.empty_like(t)
    ctx = fk.Context(0)
    ctx.fit(t, cube.i_ref, p, out=out, ws=ws, want_basis=False)  # first call: one-time runtime set-up
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(2):
        b, _, _ = ctx.fit(t, cube.i_ref, p, out=out, ws=ws, want_basis=False)
        assert b is None
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0  # no device allocation during the call
        np.testing.assert_array_equal(host(out), ref)  # same layout, same arithmetic
    assert ctx.workspace_bytes() == 0
    # one byte short, or misaligned: refused before any launch
    with pytest.raises(fk.FkkError):
        ctx.fit(t, cube.i_ref, p, out=out, ws=ws[: need - 1])
    with pytest.raises(fk.FkkError):
        ctx.fit(t, cube.i_ref, p, out=out, ws=ws[16:])
    b_ref.free()
    own.close()
    ctx.close()


def test_plain_in_small_caller_workspace_runs_in_batches():
    say("plain in caller workspace")
    cube, _ = cube_and_params(rows=30, cols=30, n=200, key=42)
    p = fk.params(k=4)
    m, n = cube.shape
    t = dev(cube.i_cars)
    ctx = fk.Context(0)
    ref = host(ctx.plain(t, cube.i_ref, p))
    full = fk.workspace_size(fk.OP_PLAIN, m, n, p)
    small = full // 3  # room for batches of a few hundred rows only
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    out = ctx.plain(t, cube.i_ref, p, ws=ws)
    np.testing.assert_array_equal(host(out), ref)
    with pytest.raises(fk.FkkError):
        ctx.plain(t, cube.i_ref, p, ws=ws[:1024])
    ctx.close()


@pytest.mark.parametrize("prec", [fk.PREC_FP32, fk.PREC_BF16])
def test_transform_output_planes(prec):
    say(f"transform planes prec={prec}")
    cube, _ = cube_and_params(rows=40, cols=40, n=256, key=43)
    op = wf.Params(k=10, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    basis = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, op)["basis"]
    ctx = fk.Context(0)
    b = ctx.basis_import(basis)
    b.precision = prec
    new = synth.tissue_cube(rows=20, cols=30, n=256, map_key=44, noise_key=45, blur=3.0)
    t = dev(new.i_cars)
    ref = wf.transform(new.i_cars.astype(np.float64), basis)
    im = host(ctx.transform(b, t))
    for plane, key in ((fk.OUT_IM, "im"), (fk.OUT_RE, "re"), (fk.OUT_ABS, "abs")):
        got = host(ctx.transform(b, t, plane=plane))
        if prec == fk.PREC_FP32:
            assert spectrum_err(got, ref[key]).max() < TOL, key
        else:  # BF16 operands: the planes agree with each other exactly where they share a result
            assert spectrum_err(got, ref[key]).max() < 5e-2, key
        if plane == fk.OUT_IM:
            np.testing.assert_array_equal(got, im)
    with pytest.raises(fk.FkkError):
        ctx.transform(b, t, plane=3)
    ctx.close()


def test_basis_held_by_server_is_busy():
    say("basis busy while served")
    cube, _ = cube_and_params(rows=16, cols=16, n=128, key=46)
    op = wf.Params(k=6, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    ctx = fk.Context(0)
    b = ctx.basis_import(wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, op)["basis"])
    srv = fk.Server(0, hbm_budget_bytes=64 << 20)
    bid = srv.add_basis(b)
    with pytest.raises(fk.FkkError) as err:
        b.free()
    assert err.value.status == -9
    tile = torch.empty((10, 128), dtype=torch.float32, pin_memory=True).fill_(1.0)
    out = torch.empty((10, 128), dtype=torch.float32, pin_memory=True)
    srv.wait(srv.submit(bid, tile, out))  # the basis still works
    # host-buffer checks: dtype, column count, output rows
    with pytest.raises(TypeError):
        srv.submit(bid, tile.double(), out)
    with pytest.raises(fk.FkkError):
        srv.submit(bid, tile[:, :100], out)
    with pytest.raises(fk.FkkError):
        srv.submit(bid, tile, out[:5])
    with pytest.raises(TypeError):
        srv.submit(bid, tile.cuda(), out)
    srv.close()
    b.free()  # released with the server
    ctx.close()
