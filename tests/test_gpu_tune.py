"""GPU tests of the launch-shape autotuner: a first call times candidates and
writes the cache, a second call applies the cached shapes without timing,
and the transfer stays within 1e-5 of the oracle under every spreading tile
edge the grid allows (re-cut in place)."""
import numpy as np
import pytest

from parity import F_TOL, PHI_TOL, normwise, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_01113_amd import mls
    mls.load()
    return torch


def _spread_vs_oracle(orc, torch, ctx, gs, x, y, z, area, F, label):
    from paper_1805_01113_amd import mls
    n = len(x)
    home, phi, _ = ctx.build(to_dev(x), to_dev(y), to_dev(z), method=mls.MLS_EXACT)
    fo = [torch.zeros(gs.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
    ctx.spread(home, phi, to_dev(area), to_dev(F), fo)
    ctx.sync()
    g = orc.Grid(gs.faces, gs.periodic)
    p = mls.unpack_phi(phi.cpu().numpy(), n)
    errs = []
    for c in range(3):
        ref = orc.build_exact(g, c, x, y, z)
        assert normwise(p[c], ref["phi"]) <= PHI_TOL
        fref, _ = orc.spread(g, c, ref["home"], ref["phi"], area, F[c])
        errs.append(normwise(fo[c].cpu().numpy(), fref))
    say("%s spread normwise rel err %s" % (label, ["%.2e" % e for e in errs]))
    assert max(errs) <= F_TOL


def test_autotune_then_cache(orc, torch_cuda, tmp_path):
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    torch = torch_cuda
    wl = W.single_sphere(n=64, subdiv=4)
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    x0, y0, z0, area = [torch.from_numpy(a).cuda() for a in (wl.x, wl.y, wl.z, wl.area)]
    fields = wl.fields("cuda")
    forcing = [torch.zeros(wl.grid.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
    bufs = mls.StepBuffers(ctx, x0, y0, z0, area, fields, forcing)
    cache = str(tmp_path / "tune.jsonl")
    r1 = ctx.autotune(bufs, method=mls.MLS_EXACT, cache_path=cache)
    say("autotune: %s" % r1)
    assert not r1["from_cache"] and r1["candidates"] >= 8
    assert 4 <= r1["spread_tile"] <= 12
    assert ctx.tune_get()["spread_tile"] == r1["spread_tile"]
    with open(cache) as f:
        assert len(f.read().strip().splitlines()) == 1
    r2 = ctx.autotune(bufs, method=mls.MLS_EXACT, cache_path=cache)
    assert r2["from_cache"] and r2["candidates"] == 0
    for k in ("spread_tile", "spread_blocks_per_cu", "build_blocks_per_cu", "interp_blocks_per_cu", "spread_threads"):
        assert r2[k] == r1[k]
    # the compact exact step is tuned under its own key, then served from the cache
    r3 = ctx.autotune(bufs, method=mls.MLS_EXACT, cache_path=cache, compact=True)
    assert not r3["from_cache"] and r3["candidates"] >= 8
    r4 = ctx.autotune(bufs, method=mls.MLS_EXACT, cache_path=cache, compact=True)
    assert r4["from_cache"]
    with open(cache) as f:
        assert len(f.read().strip().splitlines()) == 2
    # fast-MLS ignores the flag: served from the entry tuned without it
    ctx.autotune(bufs, method=mls.MLS_FAST, cache_path=cache)
    r5 = ctx.autotune(bufs, method=mls.MLS_FAST, cache_path=cache, compact=True)
    assert r5["from_cache"]
    with pytest.raises(mls.MLSError):
        ctx._raise(ctx._lib.mls_autotune(ctx.h, mls.MLS_EXACT, 4, None, None, None, None), "mls_autotune")
    # the tuned context still computes the transfer of the oracle, and the
    # compact step is still the default step bit for bit
    _spread_vs_oracle(orc, torch, ctx, wl.grid, wl.x, wl.y, wl.z, wl.area, wl.force, "tuned")


def test_every_tile_edge_matches_oracle(orc, torch_cuda):
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    gs = W.GridSpec([W.uniform_faces(48), W.uniform_faces(48), W.uniform_faces(48)], [True, True, True])
    r = np.random.default_rng(5)
    n = 4000
    x, y, z = [r.uniform(0, 1, n).astype(np.float32) for _ in range(3)]
    area = r.uniform(0.5, 1.5, n).astype(np.float32) / 48 ** 2
    F = r.normal(size=(3, n)).astype(np.float32)
    ctx = mls.Context(gs.faces, gs.periodic)
    for tile in (4, 6, 8, 12, 16):
        ctx.tune_set(spread_tile=tile, spread_blocks_per_cu=4)
        assert ctx.tune_get()["spread_tile"] == tile
        _spread_vs_oracle(orc, torch_cuda, ctx, gs, x, y, z, area, F, "tile %d" % tile)
    with pytest.raises(mls.MLSError):
        ctx.tune_set(spread_tile=17)
    with pytest.raises(mls.MLSError):
        ctx.tune_set(build_blocks_per_cu=0)
    assert ctx.tune_get()["spread_tile"] == 16


def test_spread_shapes_give_identical_forcing(torch_cuda):
    """The compact exact step's forcing is the same bit for bit for 128-, 192-
    and 256-thread spreading workgroups and any number of them per compute
    unit (fixed-point sums per tile), and out-of-range shapes are rejected."""
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    torch = torch_cuda
    wl = W.ellipsoids(n_bodies=40, n=128, cfg_id=320)
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    x0, y0, z0, area = [torch.from_numpy(a).cuda() for a in (wl.x, wl.y, wl.z, wl.area)]
    fields = wl.fields("cuda")
    forcing = [torch.zeros(wl.grid.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
    bufs = mls.StepBuffers(ctx, x0, y0, z0, area, fields, forcing)
    outs = []
    for th, bpc in ((128, 16), (256, 1), (256, 8), (192, 10), (128, 2)):
        ctx.tune_set(spread_threads=th, spread_blocks_per_cu=bpc)
        for f in forcing:
            f.zero_()
        mls.step_counter_set(ctx, 3)
        mls.step(ctx, bufs, method=mls.MLS_EXACT, dt=1.0, jitter=0.1 / 128, seed=2, compact=True)
        ctx.sync()
        outs.append([f.cpu().numpy().copy() for f in forcing])
    for o in outs[1:]:
        for c in range(3):
            assert np.array_equal(o[c], outs[0][c])
    for bad in (64, 320, 512):
        with pytest.raises(mls.MLSError):
            ctx.tune_set(spread_threads=bad)


def test_tile_handout_regimes_give_identical_forcing(torch_cuda):
    """The spreading hands a colour's tiles out through a shared counter, or
    its first round by position when the colour has fewer than four tiles per
    workgroup.  On 1000 ellipsoids in 512^3 (about 1300 non-empty tiles of 8^3
    cells per colour) 256 workgroups take the counter only, 512 a first round
    by position and the counter, 2048 and more by position only (some get no
    tile); the forcing of the compact exact step is the same bit for bit in
    every case."""
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    torch = torch_cuda
    wl = W.ellipsoids()
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    x0, y0, z0, area = [torch.from_numpy(a).cuda() for a in (wl.x, wl.y, wl.z, wl.area)]
    fields = wl.fields("cuda")
    forcing = [torch.zeros(wl.grid.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
    bufs = mls.StepBuffers(ctx, x0, y0, z0, area, fields, forcing)
    outs = []
    shapes = ((192, 1), (192, 2), (256, 4), (192, 8), (128, 32))
    for th, bpc in shapes:
        ctx.tune_set(spread_tile=8, spread_threads=th, spread_blocks_per_cu=bpc)
        for f in forcing:
            f.zero_()
        mls.step_counter_set(ctx, 5)
        mls.step(ctx, bufs, method=mls.MLS_EXACT, dt=1.0, jitter=0.2 / 512, seed=7, compact=True)
        ctx.sync()
        outs.append([f.cpu().numpy().copy() for f in forcing])
        say("threads %d, %d per CU: forcing sum %s" % (th, bpc, ["%.6e" % float(o.sum(dtype=np.float64))
                                                               for o in outs[-1]]))
    assert max(float(np.abs(o).max()) for o in outs[0]) > 0.0
    for o in outs[1:]:
        for c in range(3):
            assert np.array_equal(o[c], outs[0][c])
