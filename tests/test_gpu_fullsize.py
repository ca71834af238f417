"""GPU parity at the full workload sizes, in the configuration bench.py
times: the autotuned launch shapes and one replay of the captured step.  The
exact step is checked in both forms: with compact transfer functions (gamma
and the support offsets per row, the form bench.py times, with the launch
shapes the autotuner picks for it) and with the 27-value rows.

The FP64 oracle cannot process 22.66 M markers in a test, so it checks
samples it can compute one by one:
  * interpolated velocity U of sampled markers (oracle jitter of the same
    counter, oracle exact build and interpolation on the full fields);
  * forcing at probe nodes: the oracle spreads every marker whose support
    can reach a probe node (all markers whose cell lies within two cells);
and, at full size on a uniform grid, the conservation of the total force per
component (eq. 7-8: sum_k f_k dV_k = sum_l c_l F_l sum_k phi_k dV_k =
sum_l A_l h_l F_l, with h_l = h sum_k phi_k = h).  For the learned method only
U is compared (the gate bounds the consistency residuals, not the nodal
shape-function values the forcing depends on).
"""
import numpy as np
import pytest

from parity import F_TOL, U_TOL, normwise, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _widths(faces, periodic, is_face):
    """Control-volume widths of the nodes along one axis."""
    f = np.asarray(faces, dtype=np.float64)
    c = 0.5 * (f[:-1] + f[1:])
    if not is_face:
        return np.diff(f)
    if periodic:
        L = f[-1] - f[0]
        return c - np.concatenate([[c[-1] - L], c[:-1]])
    return np.diff(np.concatenate([[f[0]], c, [f[-1]]]))


def _cells(faces, periodic, x):
    f = np.asarray(faces)
    xx = np.asarray(x, dtype=np.float64)
    if periodic:
        L = f[-1] - f[0]
        xx = f[0] + np.mod(xx - f[0], L)
    return np.clip(np.searchsorted(f, xx, side="right") - 1, 0, len(f) - 2)


def _run_step(torch, wl, method, cache, counter=11, compact=False):
    from paper_1805_01113_amd import mls, train_mlp
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    ctx.reserve(wl.n)
    if method == mls.MLS_LEARNED:
        p, q, _ = train_mlp.load_weights()
        ctx.mlp_load(p, q)
    x0, y0, z0, area = [torch.from_numpy(a).cuda() for a in (wl.x, wl.y, wl.z, wl.area)]
    fields = wl.fields("cuda")
    forcing = [torch.zeros(wl.grid.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
    bufs = mls.StepBuffers(ctx, x0, y0, z0, area, fields, forcing)
    tune = ctx.autotune(bufs, method=method, cache_path=cache, compact=compact)
    for f in forcing:
        f.zero_()
    amp = 0.1 * wl.grid.h_min
    graph = mls.StepGraph(ctx, bufs, method=method, dt=1.0, jitter=amp, seed=20180503, compact=compact)
    mls.step_counter_set(ctx, counter)
    graph.launch(1)
    ctx.sync()
    graph.close()
    say("%s: %d markers, compact %s, shapes %s" % (wl.name, wl.n, compact, {
        k: tune[k] for k in ("spread_tile", "spread_blocks_per_cu", "build_blocks_per_cu", "spread_threads")}))
    return ctx, bufs, fields, forcing, amp, counter


def _near(cells, probes, dims, periodic, reach=2):
    """Markers whose cell lies within `reach` cells of any probe node (wrapped
    distance on periodic axes)."""
    near = np.zeros(len(cells[0]), dtype=bool)
    for p in probes:
        ok = np.ones(len(cells[0]), dtype=bool)
        for d in range(3):
            dist = np.abs(cells[d] - p[d])
            if periodic[d]:
                dist = np.minimum(dist, dims[d] - dist)
            ok &= dist <= reach
        near |= ok
    return near


def _check(orc, torch, wl, bufs, fields, forcing, amp, counter, u_tol, label, forcing_check=True, n_sample=1500,
           n_probe=40, build=None):
    """build(g, c, x, y, z) -> dict(home, phi): the oracle's shape functions
    for the method under test (exact MLS by default)."""
    if build is None:
        build = orc.build_exact
    g = orc.Grid(wl.grid.faces, wl.grid.periodic)
    xj = orc.jitter(wl.x, wl.y, wl.z, counter, np.float32(amp), 20180503)
    r = np.random.default_rng(7)
    sample = np.sort(r.choice(wl.n, n_sample, replace=False))
    Ug = bufs.U.cpu().numpy()
    Fg = bufs.F.cpu().numpy()
    ncell = [len(f) - 1 for f in wl.grid.faces]
    uniform = all(np.allclose(np.diff(f), np.diff(f)[0], rtol=1e-12, atol=0) for f in wl.grid.faces)
    cells = [_cells(wl.grid.faces[d], wl.grid.periodic[d], xj[d]) for d in range(3)]
    for c in range(3):
        q = fields[c].cpu().numpy()
        ref = build(g, c, *[a[sample] for a in xj])
        Uo = orc.interp(g, c, ref["home"], ref["phi"], q)
        del q
        eu = normwise(Ug[c][sample], Uo)
        msg = "%s comp %d: U err %.2e over %d markers" % (label, c, eu, n_sample)
        assert eu <= u_tol, msg
        if forcing_check:
            # forcing at probe nodes: home nodes of some sampled markers
            probes = ref["home"][r.choice(n_sample, n_probe, replace=False)]
            idx = np.nonzero(_near(cells, probes, ncell, wl.grid.periodic))[0]
            refn = build(g, c, *[a[idx] for a in xj])
            fo, _ = orc.spread(g, c, refn["home"], refn["phi"], wl.area[idx], Fg[c][idx])
            pv_o = np.array([fo[k, j, i] for i, j, k in probes])
            del fo
            fg = forcing[c]
            pv_g = np.array([float(fg[k, j, i]) for i, j, k in probes])
            ef = normwise(pv_g, pv_o)
            msg += "; forcing err %.2e at %d probes (%d markers spread)" % (ef, n_probe, len(idx))
            assert ef <= F_TOL, msg
        if forcing_check and uniform:
            wx = torch.from_numpy(_widths(wl.grid.faces[0], wl.grid.periodic[0], c == 0)).cuda()
            wy = torch.from_numpy(_widths(wl.grid.faces[1], wl.grid.periodic[1], c == 1)).cuda()
            wz = torch.from_numpy(_widths(wl.grid.faces[2], wl.grid.periodic[2], c == 2)).cuda()
            tot = 0.0
            for z0 in range(0, forcing[c].shape[0], 64):
                blk = forcing[c][z0:z0 + 64].double()
                tot += float(((blk @ wx) @ wy) @ wz[z0:z0 + 64])
            h = float(np.diff(wl.grid.faces[0])[0])
            af = torch.from_numpy(wl.area).cuda().double() * bufs.F[c].double()
            rhs = h * float(af.sum())
            scale = h * float(af.abs().sum())
            msg += "; total force %.9e vs sum A h F %.9e" % (tot, rhs)
            assert abs(tot - rhs) <= 1e-6 * scale, msg
        say(msg)


@pytest.mark.parametrize("compact", [True, False], ids=["compact", "full_rows"])
def test_uneven_bodies_full_size_exact(orc, tmp_path, compact):
    import torch
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    wl = W.uneven_bodies()
    ctx, bufs, fields, forcing, amp, counter = _run_step(torch, wl, mls.MLS_EXACT, str(tmp_path / "t.jsonl"),
                                                         compact=compact)
    _check(orc, torch, wl, bufs, fields, forcing, amp, counter, U_TOL,
           "uneven exact (%s)" % ("compact" if compact else "full rows"))
    ctx.close()


def test_stretched_channel_full_size_exact_and_learned(orc, tmp_path):
    import torch
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    wl = W.stretched_channel()
    for method, tol, label, compact in ((mls.MLS_EXACT, U_TOL, "stretched exact (compact)", True),
                                        (mls.MLS_EXACT, U_TOL, "stretched exact (full rows)", False),
                                        (mls.MLS_LEARNED, 1e-4, "stretched learned", False)):
        # the learned method keeps network shape functions where the gate passes
        ctx, bufs, fields, forcing, amp, counter = _run_step(torch, wl, method, str(tmp_path / "t.jsonl"),
                                                             compact=compact)
        st = ctx.stats()
        if method == mls.MLS_LEARNED:
            say("learned: %d kept, %d fell back to exact" % (st["learned"], st["fallbacks"]))
            assert st["learned"] > 0
        _check(orc, torch, wl, bufs, fields, forcing, amp, counter, tol, label,
               forcing_check=(method == mls.MLS_EXACT))
        ctx.close()
        del bufs, fields, forcing
        torch.cuda.empty_cache()


def test_uneven_bodies_full_size_fast_trilinear(orc, tmp_path):
    """The fused fast-MLS step (trilinear blend, octant table in LDS) at full
    size: U of sampled markers, forcing at probe nodes and conservation
    against the oracle's table blend."""
    import torch
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    wl = W.uneven_bodies()
    ctx, bufs, fields, forcing, amp, counter = _run_step(torch, wl, mls.MLS_FAST_LINEAR, str(tmp_path / "t.jsonl"))

    def build(g, c, x, y, z):
        return orc.build_fast(g, c, x, y, z, blend=orc.BLEND_TRILINEAR)

    _check(orc, torch, wl, bufs, fields, forcing, amp, counter, U_TOL, "uneven fast trilinear", build=build)
    ctx.close()
