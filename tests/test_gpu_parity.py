"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Support indices must match bit for bit; shape functions,
interpolated velocities and spread forcing within 1e-5 normwise relative
error (max |gpu - oracle| / max |oracle|), printed per result."""
import numpy as np
import pytest

from paper_1805_01113_amd import workloads as W
from parity import F_TOL, PHI_TOL, U_TOL, compare_build, gpu_build, normwise, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_01113_amd import mls
    mls.load()      # raises if the HIP library is missing
    return torch


def _ctx(gs, **kw):
    from paper_1805_01113_amd import mls
    return mls.Context(gs.faces, gs.periodic, **kw)


def _ogrid(orc, gs):
    return orc.Grid(gs.faces, gs.periodic)


def _full_check(orc, torch, gs, x, y, z, area, F, fields_np, method=0, label="", kw=None):
    """build + interp + spread against the oracle; returns the GPU outputs."""
    ctx = _ctx(gs, **(kw or {}))
    g = _ogrid(orc, gs)
    home, phi, refs = compare_build(orc, g, ctx, x, y, z, method=method, label=label,
                                    kind=(kw or {}).get("kind", 0))
    n = len(x)
    # interpolation with the GPU's own Phi vs the oracle's interpolation with its own Phi
    u, v, w = [to_dev(q) for q in fields_np]
    U = ctx.interp(home, phi, u, v, w, n)
    ctx.sync()
    Ug = U.cpu().numpy()
    errs = []
    for c in range(3):
        Uo = orc.interp(g, c, refs[c]["home"], refs[c]["phi"], fields_np[c])
        errs.append(normwise(Ug[c], Uo))
    say("%s interp normwise rel err: %s" % (label, ["%.2e" % e for e in errs]))
    assert max(errs) <= U_TOL
    # spreading into zero fields
    fo = [torch.zeros(gs.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
    ctx.spread(home, phi, to_dev(area), to_dev(F), fo)
    ctx.sync()
    errs = []
    for c in range(3):
        fref, _ = orc.spread(g, c, refs[c]["home"], refs[c]["phi"], area, F[c])
        errs.append(normwise(fo[c].cpu().numpy(), fref))
    say("%s spread normwise rel err: %s" % (label, ["%.2e" % e for e in errs]))
    assert max(errs) <= F_TOL
    return ctx, home, phi, fo


def test_single_sphere_64_exact(orc, torch_cuda):
    """5120 centroid markers of one icosphere, uniform periodic 64^3 grid."""
    wl = W.single_sphere()
    fields = [f.numpy() for f in wl.fields("cpu")]
    _full_check(orc, torch_cuda, wl.grid, wl.x, wl.y, wl.z, wl.area, wl.force, fields, label="sphere64 exact")


def test_single_sphere_64_fast(orc, torch_cuda):
    wl = W.single_sphere()
    fields = [f.numpy() for f in wl.fields("cpu")]
    _full_check(orc, torch_cuda, wl.grid, wl.x, wl.y, wl.z, wl.area, wl.force, fields, method=1,
                label="sphere64 fast")


def test_single_sphere_64_fast_trilinear(orc, torch_cuda):
    wl = W.single_sphere()
    fields = [f.numpy() for f in wl.fields("cpu")]
    _full_check(orc, torch_cuda, wl.grid, wl.x, wl.y, wl.z, wl.area, wl.force, fields, method=3,
                label="sphere64 fast trilinear")


def _ragged_markers(n_grid, n, seed):
    r = np.random.default_rng(seed)
    x = r.uniform(-0.5, 1.5, n)
    y = r.uniform(0, 1, n)
    z = r.uniform(0, 1, n)
    # markers exactly on control-volume boundaries (ties go to the upper node)
    i = r.integers(0, n_grid, 40)
    x[:20] = i[:20] / n_grid
    y[20:40] = (i[20:40] + 0.5) / n_grid
    z[40:50] = 1.0 - 1e-7
    return [a.astype(np.float32) for a in (x, y, z)]


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_ragged_periodic_32(orc, torch_cuda, kind):
    """1037 markers (a ragged tail for 256-lane blocks), ties and wrapped
    coordinates, several spreading tiles, all three weight kinds."""
    gs = W.GridSpec([W.uniform_faces(32)] * 3, [True] * 3)
    x, y, z = _ragged_markers(32, 1037, 3 + kind)
    r = np.random.default_rng(7)
    area = r.uniform(0.2, 1.0, len(x)).astype(np.float32) / 32 ** 2
    F = r.normal(size=(3, len(x))).astype(np.float32)
    fields = [r.normal(size=gs.shape(c)).astype(np.float32) for c in range(3)]
    _full_check(orc, torch_cuda, gs, x, y, z, area, F, fields, label="ragged32 kind%d" % kind,
                kw=dict(kind=kind))


@pytest.mark.parametrize("dims,tile", [((24, 40, 12), 8), ((48, 20, 36), 12), ((36, 28, 44), 4)])
def test_uneven_grid_tiles(orc, torch_cuda, dims, tile):
    """Non-power-of-two periodic grids: odd tile counts (three tile colours),
    single-tile axes and every tile edge."""
    gs = W.GridSpec([W.uniform_faces(n) for n in dims], [True] * 3)
    r = np.random.default_rng(sum(dims))
    n = 2000
    x, y, z = [r.uniform(-0.2, 1.2, n).astype(np.float32) for _ in range(3)]
    area = r.uniform(0.2, 1.0, n).astype(np.float32) / 900
    F = r.normal(size=(3, n)).astype(np.float32)
    fields = [r.normal(size=gs.shape(c)).astype(np.float32) for c in range(3)]
    _full_check(orc, torch_cuda, gs, x, y, z, area, F, fields, label="grid%s tile%d" % (dims, tile),
                kw=dict(spread_tile=tile))


def test_face_and_centre_markers_non_power_of_two(orc, torch_cuda):
    """Markers at the faces and centres of a 24 x 40 x 36 periodic grid, as
    FP32 coordinates: the FP64 faces i/n are not FP32 values, so every marker
    lies within one FP32 rounding below or above a control-volume boundary.
    Homes must follow the oracle's control-volume rule bit for bit on either
    side, and the interpolation and spreading stay within tolerance."""
    dims = (24, 40, 36)
    gs = W.GridSpec([W.uniform_faces(n) for n in dims], [True] * 3)
    r = np.random.default_rng(2024)
    n = 3000
    coords = []
    for d, nd in enumerate(dims):
        i = r.integers(0, nd, n)
        half = r.integers(0, 2, n) * 0.5          # faces and centres
        coords.append(((i + half) / nd).astype(np.float32))
    x, y, z = coords
    area = r.uniform(0.2, 1.0, n).astype(np.float32) / 900
    F = r.normal(size=(3, n)).astype(np.float32)
    fields = [r.normal(size=gs.shape(c)).astype(np.float32) for c in range(3)]
    _full_check(orc, torch_cuda, gs, x, y, z, area, F, fields, label="faces and centres 24x40x36",
                kw=dict(spread_tile=4))


def test_grid_rejected_without_tile_divisor(torch_cuda):
    """A periodic axis of 17 cells has no tile edge between 4 and 12."""
    from paper_1805_01113_amd import mls
    gs = W.GridSpec([W.uniform_faces(17), W.uniform_faces(16), W.uniform_faces(16)], [True] * 3)
    with pytest.raises(mls.MLSError):
        _ctx(gs)


def _stretched(nxy=48, nz=72, n_bodies=12, seed=4):
    wl = W.stretched_channel(n_bodies=n_bodies, nxy=nxy, nz=nz, cfg_id=100 + seed)
    return wl


def test_stretched_exact_and_fast(orc, torch_cuda):
    """Wall-bounded tanh-stretched z axis (beta 2.5): FP64 offsets, per-plane
    fast-MLS tables."""
    wl = _stretched()
    fields = [f.numpy() for f in wl.fields("cpu")]
    for method in (0, 1, 3):
        _full_check(orc, torch_cuda, wl.grid, wl.x, wl.y, wl.z, wl.area, wl.force, fields, method=method,
                    label="stretched m%d" % method)


def test_fast_tables_match_oracle(orc, torch_cuda):
    """fast-MLS tables (built once on the GPU) against the oracle's tables."""
    import torch
    wl = _stretched()
    ctx = _ctx(wl.grid)
    Td, first, axis = ctx.fast_tables()
    assert axis == 2 and Td.shape[0] == 72 + 73
    torch.cuda.synchronize()
    T = Td.cpu().numpy()
    g = _ogrid(orc, wl.grid)
    worst = 0.0
    for comp, ttype in ((0, 0), (2, 1)):
        for plane in (1, 5, 20, 36, 60, 70):
            home = np.array([3, 4, plane], dtype=np.int32)
            node, lo, hi = orc.home_support(g, comp, home)
            ref = orc.fast_table(node, lo, hi, 9)
            worst = max(worst, normwise(T[first[ttype] + plane], ref))
    say("fast table normwise rel err: %.2e" % worst)
    assert worst <= PHI_TOL


def test_empty_and_single_marker(orc, torch_cuda):
    import torch
    gs = W.GridSpec([W.uniform_faces(16)] * 3, [True] * 3)
    ctx = _ctx(gs)
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    home, phi, _ = ctx.build(e, e, e)
    U = ctx.interp(home, phi, *[torch.zeros(gs.shape(c), device="cuda") for c in range(3)], n=0)
    ctx.spread(home, phi, e, torch.empty((3, 0), device="cuda"), [torch.zeros(gs.shape(c), device="cuda") for c in range(3)])
    ctx.sync()
    assert U.numel() == 0
    x, y, z = [np.array([v], np.float32) for v in (0.3, 0.71, 0.999)]
    compare_build(orc, _ogrid(orc, gs), ctx, x, y, z, label="single")


def test_forced_fp64_route(orc, torch_cuda):
    """kappa_tau = 0 sends every (marker, component) solve to FP64; results
    still match the oracle and every route flag is set."""
    gs = W.GridSpec([W.uniform_faces(32)] * 3, [True] * 3)
    x, y, z = _ragged_markers(32, 700, 9)
    ctx = _ctx(gs, kappa_tau=0.0)
    ctx.stats_reset()
    compare_build(orc, _ogrid(orc, gs), ctx, x, y, z, label="tau=0")
    _, _, _, _, route = gpu_build(ctx, x, y, z, route=True)
    assert np.all(route & 1)
    st = ctx.stats()
    assert st["fp64_solves"] == 2 * 3 * 700
    ctx2 = _ctx(gs)
    ctx2.stats_reset()
    _, _, _, _, route = gpu_build(ctx2, x, y, z, route=True)
    assert not np.any(route & 1)
    st = ctx2.stats()
    say("default route: fp64 solves %d, kappa_max %.3g" % (st["fp64_solves"], st["kappa_max"]))
    assert st["fp64_solves"] == 0 and 1.0 < st["kappa_max"] < 200.0


def test_support_error_reports_lowest_marker(orc, torch_cuda):
    """A marker whose support leaves a wall axis gets MLS_E_SUPPORT with the
    lowest offending index; the others are still built."""
    from paper_1805_01113_amd import mls
    wl = _stretched()
    ctx = _ctx(wl.grid)
    x, y, z = wl.x[:300].copy(), wl.y[:300].copy(), wl.z[:300].copy()
    z[123] = 0.0
    z[200] = np.float32(wl.grid.faces[2][-1])
    home, phi, _ = ctx.build(to_dev(x), to_dev(y), to_dev(z))
    st, bad = ctx.sync(raise_on_error=False)
    assert st == -2 and bad == 123
    p = mls.unpack_phi(phi.cpu().numpy(), 300)      # [3, n, 27]
    assert np.all(np.isnan(p[:, 123])) and np.all(np.isfinite(p[:, :123]))
    assert ctx.sync(raise_on_error=False) == (0, -1)   # the error word was cleared


def test_spread_deterministic_and_order_independent(orc, torch_cuda):
    """Spreading is bitwise reproducible, also when the markers are permuted
    (the per-tile fixed-point sums do not depend on order)."""
    import torch
    wl = W.ellipsoids(n_bodies=60, n=128, cfg_id=200)
    gs = wl.grid
    ctx = _ctx(gs)
    home, phi, _ = ctx.build(to_dev(wl.x), to_dev(wl.y), to_dev(wl.z))
    outs = []
    for rep in range(2):
        f = [torch.zeros(gs.shape(c), device="cuda") for c in range(3)]
        ctx.spread(home, phi, to_dev(wl.area), to_dev(wl.force), f)
        ctx.sync()
        outs.append([t.cpu().numpy() for t in f])
    perm = np.random.default_rng(1).permutation(wl.n)
    h2, p2, _ = ctx.build(to_dev(wl.x[perm]), to_dev(wl.y[perm]), to_dev(wl.z[perm]))
    f = [torch.zeros(gs.shape(c), device="cuda") for c in range(3)]
    ctx.spread(h2, p2, to_dev(wl.area[perm]), to_dev(np.ascontiguousarray(wl.force[:, perm])), f)
    ctx.sync()
    outs.append([t.cpu().numpy() for t in f])
    for c in range(3):
        assert np.array_equal(outs[0][c], outs[1][c])
        assert np.array_equal(outs[0][c], outs[2][c])
    say("spread bitwise identical over reruns and permutation (%d markers)" % wl.n)


def test_spread_conserves_force_full_ellipsoids(orc, torch_cuda):
    """eq. 7 on a 128^3 grid with 60 ellipsoids: sum_k f_k dV_k equals
    sum_l F_l A_l h_l (GPU fields, oracle Phi) to FP32 accuracy."""
    import torch
    wl = W.ellipsoids(n_bodies=60, n=128, cfg_id=201)
    gs = wl.grid
    g = _ogrid(orc, gs)
    ctx = _ctx(gs)
    home, phi, _ = ctx.build(to_dev(wl.x), to_dev(wl.y), to_dev(wl.z))
    f = [torch.zeros(gs.shape(c), device="cuda") for c in range(3)]
    ctx.spread(home, phi, to_dev(wl.area), to_dev(wl.force), f)
    ctx.sync()
    h = 1.0 / 128
    for c in range(3):
        ref = orc.build_exact(g, c, wl.x, wl.y, wl.z)
        lhs = float(f[c].double().sum().item()) * h ** 3
        rhs = float(np.sum(wl.force[c].astype(np.float64) * wl.area.astype(np.float64) * h * ref["phi"].sum(1)))
        scale = float(np.sum(np.abs(wl.force[c]) * wl.area * h))
        say("conservation comp %d: |lhs-rhs|/sum|F dV| = %.2e" % (c, abs(lhs - rhs) / scale))
        assert abs(lhs - rhs) <= 1e-5 * scale


def test_spread_range_errors_report_the_marker(orc, torch_cuda):
    """A non-finite force, or a non-finite shape-function value of a marker with
    a valid support, is reported as MLS_E_RANGE with the lowest offending
    marker; a clean rerun reports nothing and matches the oracle."""
    import torch
    from paper_1805_01113_amd import mls
    wl = W.ellipsoids(n_bodies=20, n=64, cfg_id=202)
    gs = wl.grid
    ctx = _ctx(gs)
    home, phi, _ = ctx.build(to_dev(wl.x), to_dev(wl.y), to_dev(wl.z))
    ctx.sync()
    fields = lambda: [torch.zeros(gs.shape(c), device="cuda") for c in range(3)]
    F = wl.force.copy()
    F[1, 37] = np.nan
    F[2, 90] = np.inf
    ctx.spread(home, phi, to_dev(wl.area), to_dev(F), fields())
    assert ctx.sync(raise_on_error=False) == (mls.MLS_E_RANGE, 37)
    # phi of marker 50, component 0, node 13 -> NaN (blocked layout [block][comp][node][lane])
    bad_phi = phi.clone()
    b, r = divmod(50, 64)
    bad_phi[((b * 3 + 0) * 27 + 13) * 64 + r] = float("nan")
    ctx.spread(home, bad_phi, to_dev(wl.area), to_dev(wl.force), fields())
    assert ctx.sync(raise_on_error=False) == (mls.MLS_E_RANGE, 50)
    fo = fields()
    ctx.spread(home, phi, to_dev(wl.area), to_dev(wl.force), fo)
    assert ctx.sync(raise_on_error=False) == (0, -1)
    g = _ogrid(orc, gs)
    errs = []
    for c in range(3):
        ref = orc.build_exact(g, c, wl.x, wl.y, wl.z)
        fref, _ = orc.spread(g, c, ref["home"], ref["phi"], wl.area, wl.force[c])
        errs.append(normwise(fo[c].cpu().numpy(), fref))
    assert max(errs) <= F_TOL
