"""fkk_basis_residual_noalloc, the entry point for callers that cannot
allocate device memory, against fkk_basis_residual (the same kernels with
the context's workspace): two calls in a row, the second on fewer spectra,
with no device allocation during either; sizes past the fixed array are
refused before any launch."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from oracle import workflows as wf

torch = pytest.importorskip("torch")
fk = pytest.importorskip("paper_2005_07132_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_residual_noalloc_matches_the_allocating_call():
    say("residual noalloc vs residual")
    cube = synth.tissue_cube(rows=40, cols=40, n=256, map_key=51, noise_key=51, blur=4.0)
    p = wf.Params(k=10, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    basis = wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)["basis"]
    ref_ctx = fk.Context(0)
    b = ref_ctx.basis_import(basis)
    big = synth.tissue_cube(rows=100, cols=103, n=256, map_key=52, noise_key=52, blur=3.0)  # 10,300: ragged
    small = synth.tissue_cube(rows=7, cols=9, n=256, map_key=53, noise_key=53, comp_key=43, blur=2.0)  # 63
    inputs = [dev(big.i_cars), dev(small.i_cars)]
    want = [ref_ctx.residual(b, t) for t in inputs]
    ctx = fk.Context(0)  # a context that never needs its own workspace
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = [ctx.residual_noalloc(b, t) for t in inputs]  # large, then smaller
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert ctx.workspace_bytes() == 0
    # same kernels, same order of summation: the same numbers
    assert got == want, (got, want)
    for g, c in zip(got, (big, small)):
        assert abs(g - wf.basis_residual(c.i_cars.astype(np.float64), basis)) < 1e-3
    # again, in the opposite order: nothing left over from the previous call matters
    assert [ctx.residual_noalloc(b, t) for t in inputs[::-1]] == want[::-1]
    # past the fixed array: refused before any launch (the pointer is never read)
    r = ctypes.c_double()
    st = fk.lib().fkk_basis_residual_noalloc(ctx.handle, b.handle, inputs[1].data_ptr(), 128 * 65536 + 1, 256,
                                             ctypes.byref(r))
    assert st == -1
    ctx.close()
    ref_ctx.close()
