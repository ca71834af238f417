"""GPU parity of adaptive Lagrangian mesh refinement (Sec. 3) against the
oracle: levels, marker counts and parent triangles bit for bit; positions,
areas and normals within one FP32 rounding of the FP64 oracle (both evaluate
the construction in FP64; the GPU rounds to FP32 once)."""
import numpy as np
import pytest

from parity import say, to_dev

pytestmark = pytest.mark.gpu

# one FP32 rounding of an FP64 value, plus slack for a last-bit difference in
# the FP64 evaluation: 2 ulp relative
REL = 2.0 ** -22


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1805_01113_amd import mls
    mls.load()
    return torch


def _compare(orc, torch, gs, tri, v, ratio, level, label):
    from paper_1805_01113_amd import mls
    ctx = mls.Context(gs.faces, gs.periodic)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    td = torch.from_numpy(tri).cuda()
    vd = [to_dev(np.ascontiguousarray(v[:, d])) for d in range(3)]
    r = ctx.refine(td, *vd, ratio=ratio, level=level)
    ctx.sync()
    ref = orc.refine(orc.Grid(gs.faces, gs.periodic), tri, v[:, 0], v[:, 1], v[:, 2], ratio=ratio, level=level)
    assert r["count"] == ref["count"]
    np.testing.assert_array_equal(r["level"].cpu().numpy(), ref["level"])
    np.testing.assert_array_equal(r["parent"].cpu().numpy(), ref["parent"])
    errs = {}
    for k in ("x", "y", "z", "area"):
        g = r[k].cpu().numpy().astype(np.float64)
        o = ref[k]
        err = np.abs(g - o) / np.maximum(np.abs(o), 1e-30)
        errs[k] = float(err.max()) if len(err) else 0.0
        assert errs[k] <= REL, (k, errs[k])
    gn = r["normal"].cpu().numpy().T.astype(np.float64)
    en = float(np.abs(gn - ref["normal"]).max()) if ref["count"] else 0.0
    assert en <= REL
    hist = np.bincount(ref["level"], minlength=4).tolist()
    say("%s: %d triangles -> %d markers, levels %s, max rel err %s, normal %.1e" %
        (label, len(tri), ref["count"], hist, {k: "%.1e" % e for k, e in errs.items()}, en))
    return ctx, r, ref


def test_unit_triangle_every_level(orc, torch_cuda):
    from paper_1805_01113_amd import workloads as W
    gs = W.GridSpec([W.uniform_faces(16)] * 3, [True] * 3)
    v = np.array([[0.1, 0.1, 0.3], [0.6, 0.1, 0.3], [0.1, 0.6, 0.3]], dtype=np.float32)
    for level in range(4):
        _compare(orc, torch_cuda, gs, [[0, 1, 2]], v, 1.0, level, "unit triangle level %d" % level)


def test_random_triangles_adaptive_stretched(orc, torch_cuda):
    """Triangles of random size and shape over a tanh-stretched wall axis:
    every level occurs, several workgroups and a ragged tail."""
    from paper_1805_01113_amd import workloads as W
    fz = W.tanh_faces(64, 1.5, 2.5)
    gs = W.GridSpec([W.uniform_faces(48), W.uniform_faces(40), fz], [True, True, False])
    rng = np.random.default_rng(3)
    T = 5000 + 77
    c = np.stack([rng.uniform(-0.5, 1.5, T), rng.uniform(0, 1, T), rng.uniform(0.05, 1.45, T)], axis=1)
    size = rng.uniform(0.2, 3.0, T)[:, None, None] / 48
    v = (c[:, None, :] + size * rng.normal(size=(T, 3, 3)) * 0.5).reshape(-1, 3)
    v[:, 2] = np.clip(v[:, 2], 0.001, 1.499)
    v = v.astype(np.float32)
    tri = np.arange(3 * T).reshape(T, 3)
    for ratio in (1.0, 0.7):
        _, _, ref = _compare(orc, torch_cuda, gs, tri, v, ratio, -1, "random adaptive ratio %.1f" % ratio)
        assert set(np.unique(ref["level"]).tolist()) == {0, 1, 2, 3}
    for level in range(4):
        _compare(orc, torch_cuda, gs, tri[:1000], v, 1.0, level, "random forced level %d" % level)


def test_stretched_channel_full_mesh(orc, torch_cuda):
    """The 2000 spheres of the stretched channel (2.56 M base triangles):
    refined where the wall-normal cells shrink."""
    from paper_1805_01113_amd import workloads as W
    wl = W.stretched_channel()
    v, t = W.body_mesh(wl)
    ctx, r, ref = _compare(orc, torch_cuda, wl.grid, t, v, 1.0, -1, "stretched channel")
    assert ref["count"] > len(t)


def test_refined_markers_feed_the_build(orc, torch_cuda):
    """Refined markers of a sphere go through the exact build and the
    interpolation like any other markers (against the oracle on the same
    FP32 positions)."""
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    from parity import U_TOL, normwise
    torch = torch_cuda
    wl = W.single_sphere(n=64, subdiv=3)
    v, t = W.body_mesh(wl)
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    r = ctx.refine(torch.from_numpy(t).cuda(), *[to_dev(np.ascontiguousarray(v[:, d])) for d in range(3)], level=3)
    n = r["count"]
    assert n == 4 * len(t)
    x, y, z = (r[k].contiguous() for k in ("x", "y", "z"))
    home, phi, _ = ctx.build(x, y, z, method=mls.MLS_EXACT)
    fields = wl.fields("cuda")
    U = ctx.interp(home, phi, *fields, n)
    ctx.sync()
    g = orc.Grid(wl.grid.faces, wl.grid.periodic)
    xs, ys, zs = (a.cpu().numpy() for a in (x, y, z))
    for c in range(3):
        ref = orc.build_exact(g, c, xs, ys, zs)
        Uo = orc.interp(g, c, ref["home"], ref["phi"], fields[c].cpu().numpy())
        e = normwise(U[c].cpu().numpy(), Uo)
        say("refined sphere comp %d: %d markers, U err %.2e" % (c, n, e))
        assert e <= U_TOL


def test_errors_and_empty(torch_cuda):
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    torch = torch_cuda
    gs = W.GridSpec([W.uniform_faces(8)] * 3, [True, True, False])
    ctx = mls.Context(gs.faces, gs.periodic)
    vx = to_dev(np.array([0.5, 0.6, 0.5, 0.5], dtype=np.float32))
    vz = to_dev(np.array([0.5, 0.5, 0.6, 1.2], dtype=np.float32))
    tri = np.zeros((600, 3), dtype=np.int32)
    tri[:] = [0, 1, 2]
    tri[400] = [0, 1, 9]
    tri[500] = [3, 3, 3]
    r = ctx.refine(torch.from_numpy(tri).cuda(), vx, vx, vz)
    st, bad = ctx.sync(raise_on_error=False)
    assert st == mls.MLS_E_ARG and bad == 400
    lev = r["level"].cpu().numpy().astype(int)
    assert lev[400] == 0 and lev[500] == 0
    assert r["count"] == int((lev + 1).sum())
    par = r["parent"].cpu().numpy()
    assert np.isnan(r["x"].cpu().numpy()[par == 400]).all()
    tri[400] = [0, 1, 2]
    ctx.refine(torch.from_numpy(tri).cuda(), vx, vx, vz)
    st, bad = ctx.sync(raise_on_error=False)
    assert st == mls.MLS_E_SUPPORT and bad == 500
    r = ctx.refine(torch.from_numpy(tri).cuda(), vx, vx, vz, level=2)   # forced: no cell needed
    ctx.sync()
    assert r["count"] == 1800
    r = ctx.refine(torch.zeros((0, 3), dtype=torch.int32, device="cuda"), vx, vx, vz)
    ctx.sync()
    assert r["count"] == 0
    with pytest.raises(mls.MLSError):
        ctx.refine(torch.from_numpy(tri).cuda(), vx, vx, vz, level=4)


@pytest.mark.slow
def test_uneven_bodies_full_mesh(orc, torch_cuda):
    """The 10,000 bodies of the 1024^3 workload (22.66 M base triangles)."""
    from paper_1805_01113_amd import workloads as W
    wl = W.uneven_bodies()
    v, t = W.body_mesh(wl)
    _compare(orc, torch_cuda, wl.grid, t, v, 1.0, -1, "uneven bodies")
