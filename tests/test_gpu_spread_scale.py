"""GPU: the spreading's fixed-point scale follows each tile's own forces
(eq. 7-8), so weakly forced bodies keep FP32-level accuracy beside strongly
forced ones.

Two groups of spheres sit in separate slabs of a periodic grid (more than a
spreading tile and a support apart), one with forces 10^6 times weaker than
the other.  The forcing is compared with the oracle node by node, normwise on
the nodes of each group separately: a scale shared by the whole grid would
leave the weak group's nodes with errors of order 1e-2.  Checked for the
standalone spreading (forces given) and for the compact exact step (forces
F = -U/dt from a velocity field 10^6 times weaker over the weak slab).
"""
import numpy as np
import pytest

from paper_1805_01113_amd import workloads as W
from parity import F_TOL, U_TOL, normwise, say, to_dev

pytestmark = pytest.mark.gpu

WEAK = 1e-6


def _two_groups(n=128, per_group=12, subdiv=3, cfg_id=410):
    """Spheres of radius 5.31 h: group 0 centred in x in [0.10, 0.35), group 1
    in [0.60, 0.85); y, z anywhere (periodic).  Returns the workload and the
    group of every marker."""
    h = 1.0 / n
    r = W.rng("placement", cfg_id)
    radius = 5.31 * h
    cen = []
    for lo in (0.10, 0.60):
        got = []
        while len(got) < per_group:
            c = np.array([r.uniform(lo, lo + 0.25), r.random(), r.random()])
            d = [np.abs(c - o) for o in got]
            d = [np.minimum(v, 1.0 - v) for v in d]
            if all(np.linalg.norm(v) > 2 * radius + 3 * h for v in d):
                got.append(c)
        cen.extend(got)
    cen = np.array(cen)
    axes = np.full((len(cen), 3), radius)
    rots = np.repeat(np.eye(3)[None], len(cen), axis=0)
    pos, area, nrm = W.surface_markers(subdiv, cen, axes, rots)
    nf = len(area) // len(cen)
    g = W.GridSpec([W.uniform_faces(n)] * 3, [True] * 3)
    wl = W._finish("two_groups_%d^3" % n, g, [1.0] * 3, pos, area, nrm, np.arange(len(cen) + 1) * nf, cfg_id, 8)
    group = np.repeat(np.arange(len(cen)) >= per_group, nf).astype(np.int64)
    return wl, group


def _groupwise(fg, fo_groups):
    """Normwise error of the GPU forcing on the nodes each group touches."""
    errs = []
    for fo in fo_groups:
        mask = fo != 0.0
        errs.append(normwise(fg[mask], fo[mask]))
    return errs


def test_weak_and_strong_forces_standalone_spread(orc):
    import torch
    from paper_1805_01113_amd import mls
    wl, group = _two_groups()
    F = wl.force.copy()
    F[:, group == 1] *= np.float32(WEAK)
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    home, phi, _ = ctx.build(to_dev(wl.x), to_dev(wl.y), to_dev(wl.z))
    fg = [torch.zeros(wl.grid.shape(c), device="cuda") for c in range(3)]
    ctx.spread(home, phi, to_dev(wl.area), to_dev(F), fg)
    ctx.sync()
    g = orc.Grid(wl.grid.faces, wl.grid.periodic)
    for c in range(3):
        ref = orc.build_exact(g, c, wl.x, wl.y, wl.z)
        fo = []
        for k in (0, 1):
            sel = group == k
            f, _ = orc.spread(g, c, ref["home"][sel], ref["phi"][sel], wl.area[sel], F[c][sel])
            fo.append(f)
        assert not np.any((fo[0] != 0) & (fo[1] != 0)), "the groups share nodes"
        errs = _groupwise(fg[c].cpu().numpy(), fo)
        say("standalone spread comp %d: strong group err %.2e, weak group (x%.0e) err %.2e"
            % (c, errs[0], WEAK, errs[1]))
        assert max(errs) <= F_TOL
    ctx.close()


def test_weak_and_strong_forces_compact_step(orc):
    import torch
    from paper_1805_01113_amd import mls
    wl, group = _two_groups(cfg_id=411)
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    fields = wl.fields("cuda")
    for c in range(3):
        xn = torch.from_numpy(wl.grid.node_coords(c, 0)).cuda()
        fields[c][:, :, xn >= 0.5] *= WEAK          # the weak slab (group 1 lies in x in [0.6, 0.85))
    forcing = [torch.zeros(wl.grid.shape(c), device="cuda") for c in range(3)]
    bufs = mls.StepBuffers(ctx, to_dev(wl.x), to_dev(wl.y), to_dev(wl.z), to_dev(wl.area), fields, forcing)
    dt = 0.5
    mls.step(ctx, bufs, method=mls.MLS_EXACT, dt=dt, jitter=0.0, seed=0, compact=True)
    ctx.sync()
    g = orc.Grid(wl.grid.faces, wl.grid.periodic)
    Ug = bufs.U.cpu().numpy()
    for c in range(3):
        q = fields[c].cpu().numpy()
        ref = orc.build_exact(g, c, wl.x, wl.y, wl.z)
        Uo = orc.interp(g, c, ref["home"], ref["phi"], q)
        Fo = ((0.0 - Uo) / dt).astype(np.float32)
        eu = [normwise(Ug[c][group == k], Uo[group == k]) for k in (0, 1)]
        fo = []
        for k in (0, 1):
            sel = group == k
            f, _ = orc.spread(g, c, ref["home"][sel], ref["phi"][sel], wl.area[sel], Fo[sel])
            fo.append(f)
        errs = _groupwise(forcing[c].cpu().numpy(), fo)
        ratio = np.abs(fo[1]).max() / np.abs(fo[0]).max()
        say("compact step comp %d: U err %.2e / %.2e; forcing err strong %.2e, weak %.2e (forcing ratio %.1e)"
            % (c, eu[0], eu[1], errs[0], errs[1], ratio))
        assert max(eu) <= U_TOL
        assert ratio < 1e-4
        assert max(errs) <= F_TOL
    ctx.close()
