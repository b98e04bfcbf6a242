import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size case, minutes on the CPU")


def pytest_collection_modifyitems(config, items):
    # GPU tests are skipped, not failed, where no GPU is visible.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover - torch missing
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def oracle_case(cube, k):
    """The FP64 oracle's fit of `cube` (Gram route, noise scaling of Eq. 9)
    and the FP64 Gram of A = l diag(f) (Eq. 6, 10) with its whole spectrum,
    descending; only the outputs the GPU tests compare with are kept."""
    from oracle import workflows as wf
    p = wf.Params(k=k, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    i64 = cube.i_cars.astype(np.float64)
    ref = wf.fit(i64, cube.i_ref, p, svd="gram")
    basis, im = ref["basis"], ref["im"]
    del ref
    f = wf.scaling_f(i64, p)
    g = np.zeros((cube.shape[1], cube.shape[1]))
    for i in range(0, cube.shape[0], 65536):
        ell, _ = wf.log_ratio(i64[i:i + 65536], cube.i_ref, p.ratio_floor)
        a = ell * f
        g += a.T @ a
    del i64
    lam = np.linalg.eigvalsh(g)[::-1]
    return SimpleNamespace(cube=cube, p=p, basis=basis, im=im, g_a=g, lam=lam)


@pytest.fixture(scope="session")
def tissue703_oracle():
    """The 703,026 x 1,000 tissue cube and its oracle case at k = 50."""
    import synth
    return oracle_case(synth.tissue_703k(), 50)


@pytest.fixture(scope="session")
def tissue262_oracle():
    """A 512 x 512 x 1,600 tissue cube (262,144 spectra) and its oracle case
    at k = 50."""
    import synth
    return oracle_case(synth.tissue_cube(rows=512, cols=512, n=1600, map_key=3, noise_key=3), 50)
