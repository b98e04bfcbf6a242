"""Serving runtime (continuous batching of stored-basis transforms), checked
through the C ABI: every tile's result equals the same tile transformed
alone (bitwise) and the oracle (to the FP32 tolerance), with two resident
bases, ragged tiles, and an HBM budget smaller than the submitted work."""
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


def basis_for(n, key):
    cube = synth.tissue_cube(rows=40, cols=40, n=n, map_key=key, noise_key=key, blur=3.0)
    p = wf.Params(k=12, f_mode=wf.F_NOISE, alpha=cube.alpha, sigma_g=cube.sigma_g)
    return wf.fit(cube.i_cars.astype(np.float64), cube.i_ref, p)["basis"]


def pinned(a):
    t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)))
    return t


@pytest.fixture(scope="module")
def setup():
    ctx = fk.Context(0)
    bases = [basis_for(256, 31), basis_for(320, 32)]
    dev_bases = [ctx.basis_import(b) for b in bases]
    yield ctx, bases, dev_bases
    ctx.close()


def test_server_batches_ragged_tiles_from_two_bases(setup):
    say("server two bases")
    ctx, bases, dev_bases = setup
    budget = 3 << 19  # ~1.5 MB: the tiles below (about 8 MB in total) must queue
    rng = synth.rng_for(33, 1)
    tiles = []
    # first a tile of basis 0 that fills the whole budget (its bytes as the
    # server counts them: 4 (2 rows n + 2 rows) + 512), so that every tile
    # submitted while it runs waits in the queue and is batched with the
    # queued tiles of its basis when it completes
    n0 = bases[0]["i_ref"].shape[0]
    big_rows = (budget - 512) // (4 * (2 * n0 + 2))
    big = synth.tissue_cube(rows=28, cols=28, n=n0, map_key=299, noise_key=299, blur=1.0).i_cars[:big_rows]
    tiles.append((0, big, pinned(big), torch.empty((big_rows, n0), pin_memory=True)))
    for t in range(40):
        which = int(rng.integers(0, 2))
        side = int(rng.integers(4, 17))
        n = bases[which]["i_ref"].shape[0]
        cube = synth.tissue_cube(rows=side, cols=side, n=n, map_key=300 + t, noise_key=400 + t, blur=1.0)
        tiles.append((which, cube.i_cars, pinned(cube.i_cars), torch.empty((side * side, n), pin_memory=True)))
    alone = [None] * len(tiles)
    batched = False
    for attempt in range(3):  # batching depends on timing: a round without it is run again
        srv = fk.Server(0, hbm_budget_bytes=budget, max_inflight=8, max_batch_rows=4096)
        ids = [srv.add_basis(b) for b in dev_bases]
        for (_, _, _, tout) in tiles:
            tout.zero_()
        tickets = [srv.submit(ids[w], tin, tout) for (w, _, tin, tout) in tiles]
        lat = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert st["completed"] == len(tiles) and st["rejected"] == 0
        assert min(lat) > 0 and st["p99_ms"] >= st["p50_ms"] > 0
        for i, (w, arr, tin, tout) in enumerate(tiles):
            if alone[i] is None:
                alone[i] = ctx.transform(dev_bases[w], torch.from_numpy(arr).cuda()).cpu()
                ref = wf.transform(arr.astype(np.float64), bases[w])["im"]
                err = np.abs(alone[i].numpy() - ref).max(axis=1) / np.abs(ref).max(axis=1)
                assert err.max() < TOL
            assert torch.equal(tout, alone[i])
        srv.close()
        say(f"  round {attempt}: {st['launches']} launches for {len(tiles)} tiles")
        if st["launches"] < len(tiles):  # some tiles were batched together
            batched = True
            break
    assert batched


def test_server_rejects_oversized_tile_and_drains(setup):
    say("server admission")
    ctx, bases, dev_bases = setup
    srv = fk.Server(0, hbm_budget_bytes=1 << 20, max_inflight=4, max_batch_rows=100000)
    bid = srv.add_basis(dev_bases[0])
    big = pinned(np.ones((2000, 256)))
    with pytest.raises(fk.FkkError) as e:
        srv.submit(bid, big, torch.empty((2000, 256), pin_memory=True))
    assert e.value.status == -2
    small = pinned(synth.tissue_cube(rows=10, cols=10, n=256, map_key=5, noise_key=5).i_cars)
    outs = [torch.empty((100, 256), pin_memory=True) for _ in range(12)]
    for o in outs:
        srv.submit(bid, small, o)
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 12 and st["rejected"] == 1
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    srv.reset_stats()
    assert srv.stats()["completed"] == 0
    srv.close()
