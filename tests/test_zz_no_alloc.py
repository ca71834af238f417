"""GPU: the allocation-free spreading (mls_spread_noalloc) against mls_spread.

Both entry points run the same kernels on the same inputs, so their fields
must agree bit for bit; each is also held to the oracle's eq. 7-8 forcing
within F_TOL.  Two calls in a row share the library's fixed scratch array,
the second with fewer markers (a ragged count) than the first, so whatever
the first call left there must not leak into the second; a third call comes
from another context on a smaller grid.  A request larger than the fixed
array is refused on the host, before anything is launched.
"""
import ctypes

import numpy as np
import pytest

from paper_1805_01113_amd import workloads as W
from parity import F_TOL, normwise, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_01113_amd import mls
    mls.load()
    return torch


def _fields(torch, ctx):
    return [torch.zeros(ctx.shape(c), device="cuda") for c in range(3)]


def _both(torch, orc, ctx, gs, x, y, z, area, F, label):
    """Spreads through both entry points (no-alloc first) and checks them
    against each other and the oracle."""
    home, phi, _ = ctx.build(to_dev(x), to_dev(y), to_dev(z))
    fa = _fields(torch, ctx)
    ctx.spread_noalloc(home, phi, to_dev(area), to_dev(F), fa)
    ctx.sync()
    fb = _fields(torch, ctx)
    ctx.spread(home, phi, to_dev(area), to_dev(F), fb)
    ctx.sync()
    g = orc.Grid(gs.faces, gs.periodic)
    for c in range(3):
        a = fa[c].cpu().numpy()
        b = fb[c].cpu().numpy()
        assert np.array_equal(a, b), "%s comp %d: no-alloc and allocating spreads differ at %d nodes" % (
            label, c, int(np.count_nonzero(a != b)))
        ref = orc.build_exact(g, c, x, y, z)
        fo, _ = orc.spread(g, c, ref["home"], ref["phi"], area, F[c])
        e = normwise(a, fo)
        say("%s comp %d: %d markers, bitwise equal to mls_spread, err vs oracle %.2e" % (label, c, len(x), e))
        assert e <= F_TOL
    return fa


def test_noalloc_matches_spread_on_two_calls(orc, torch_cuda):
    torch = torch_cuda
    from paper_1805_01113_amd import mls
    # 72^3 periodic: 9 tiles of 8 per axis, so the third colour is used too
    wl = W.ellipsoids(n_bodies=40, n=72, cfg_id=420)
    gs = wl.grid
    ctx = mls.Context(gs.faces, gs.periodic)
    say("no-alloc call 1: %s, %d markers" % (wl.name, wl.n))
    _both(torch, orc, ctx, gs, wl.x, wl.y, wl.z, wl.area, wl.force, "call 1")
    m = 7777                                     # fewer markers, not a multiple of 64
    sel = np.random.default_rng(421).choice(wl.n, size=m, replace=False)
    F2 = np.ascontiguousarray(wl.force[:, sel]) * np.float32(-3.0)
    say("no-alloc call 2: %d markers of the same workload" % m)
    _both(torch, orc, ctx, gs, wl.x[sel], wl.y[sel], wl.z[sel], wl.area[sel], F2, "call 2")
    ctx.close()
    # another context on the same array: a smaller channel, walls and tanh clustering in z
    wl3 = W.stretched_channel(n_bodies=4, nxy=48, nz=40, lz=1.0, beta=1.5, cfg_id=422)
    gs3 = wl3.grid
    ctx3 = mls.Context(gs3.faces, gs3.periodic)
    say("no-alloc call 3: %s, %d markers" % (wl3.name, wl3.n))
    _both(torch, orc, ctx3, gs3, wl3.x, wl3.y, wl3.z, wl3.area, wl3.force, "call 3")
    ctx3.close()


def test_noalloc_refuses_requests_beyond_the_array(torch_cuda):
    """A marker count whose scratch exceeds the fixed array is refused with
    MLS_E_ARG on the host (nothing launched, fields untouched); the next call
    that fits works as before."""
    torch = torch_cuda
    from paper_1805_01113_amd import mls
    wl = W.single_sphere(n=32, subdiv=2, radius=0.15, cfg_id=423)
    gs = wl.grid
    ctx = mls.Context(gs.faces, gs.periodic)
    home, phi, _ = ctx.build(to_dev(wl.x), to_dev(wl.y), to_dev(wl.z))
    area, F = to_dev(wl.area), to_dev(wl.force)
    f = _fields(torch, ctx)
    ctx.sync()
    big = mls.SPREAD_NOALLOC_BYTES // 20 + 1     # 20 bytes of scratch per marker alone exceed it
    p = ctypes.c_void_p
    st = ctx._lib.mls_spread_noalloc(ctx.h, ctypes.c_int64(big), p(home.data_ptr()), p(phi.data_ptr()),
                                     p(area.data_ptr()), p(F[0].data_ptr()), p(F[1].data_ptr()), p(F[2].data_ptr()),
                                     p(f[0].data_ptr()), p(f[1].data_ptr()), p(f[2].data_ptr()), None)
    msg = ctx._lib.mls_last_error(ctx.h).decode()
    say("oversized no-alloc request (%d markers): status %d, %s" % (big, st, msg))
    assert st == mls.MLS_E_ARG
    assert "MLS_SPREAD_NOALLOC_BYTES" in msg
    ctx.sync()
    assert all(float(t.abs().max()) == 0.0 for t in f)
    ctx.spread_noalloc(home, phi, area, F, f)
    g = _fields(torch, ctx)
    ctx.spread(home, phi, area, F, g)
    ctx.sync()
    for c in range(3):
        assert torch.equal(f[c], g[c])
    ctx.close()
