"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare them."""
import sys

import numpy as np

PHI_TOL = 1e-5      # normwise relative (max |d| / max |ref|), FP32 path vs FP64 oracle
U_TOL = 1e-5
F_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def normwise(a, ref):
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - ref)) / den)


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_build(ctx, x, y, z, method=0, route=False):
    import torch
    from paper_1805_01113_amd import mls
    xd, yd, zd = to_dev(x), to_dev(y), to_dev(z)
    n = len(x)
    r = torch.zeros(3 * mls.npad(n), dtype=torch.uint8, device="cuda") if route else None
    home, phi, r = ctx.build(xd, yd, zd, method=method, route=r)
    ctx.sync()
    h = mls.unpack_home(home.cpu().numpy().view(np.uint32), n)      # [3, n, 3]
    p = mls.unpack_phi(phi.cpu().numpy(), n)                        # [3, n, 27]
    return home, phi, h, p, (mls.unpack_route(r.cpu().numpy(), n) if route else None)


def compare_build(orc, grid, ctx, x, y, z, method=0, nsub=9, label="", kind=0):
    """Bit-exact homes and Phi within PHI_TOL for all three components."""
    home, phi, h, p, _ = gpu_build(ctx, x, y, z, method=method)
    errs = []
    refs = []
    for c in range(3):
        if method == 0:
            ref = orc.build_exact(grid, c, x, y, z, kind=kind)
        else:
            # method 1: Shepard blend (eq. 9-10); method 3: trilinear blend of the same tables
            ref = orc.build_fast(grid, c, x, y, z, nsub=nsub, kind=kind, blend=1 if method == 3 else 0)
        assert np.array_equal(h[c], ref["home"]), "%s comp %d: home mismatch at %s" % (
            label, c, np.nonzero(np.any(h[c] != ref["home"], axis=1))[0][:10])
        e = normwise(p[c], ref["phi"])
        errs.append(e)
        refs.append(ref)
    say("%s build(method=%d) phi normwise rel err per component: %s" % (label, method, ["%.2e" % e for e in errs]))
    assert max(errs) <= PHI_TOL, errs
    return home, phi, refs
