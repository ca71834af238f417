"""Pins of the FP64 surrogate reference: gradients against central finite
differences of the loss, the GELU derivative against differences of GELU,
and the support geometry against the grid-based oracle."""
import numpy as np

from oracle import mlp as M


def _feat(n, seed):
    r = np.random.default_rng(seed)
    xi = r.uniform(-0.5, 0.5, (n, 3))
    rho = 1.0 + r.uniform(-0.05, 0.05, (n, 3))
    return np.concatenate([xi, rho], 1)


def test_gelu_derivative_matches_differences():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, rtol=0, atol=1e-8)
    # closed values: gelu(0) = 0, gelu'(0) = 1/2
    assert M.gelu(np.array([0.0]))[0] == 0.0 and abs(M.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_gradient_matches_central_differences():
    feat = _feat(16, 1)
    tgt = np.random.default_rng(2).normal(size=(16, 27)) * 0.1
    p = M.init_params(3, shift=np.array([0, 0, 0, 1, 1, 1.0]), scale=np.array([2, 2, 2, 20, 20, 20.0]))
    L, g = M.loss_and_grad(p, feat, tgt, mu=0.7)
    v = p.flat()
    r = np.random.default_rng(4)
    idx = r.choice(len(v), 60, replace=False)
    h = 1e-6
    for i in idx:
        vp = v.copy(); vp[i] += h
        vm = v.copy(); vm[i] -= h
        Lp, _ = M.loss_and_grad(M.Params.unflat(vp, p.shift, p.scale), feat, tgt, mu=0.7)
        Lm, _ = M.loss_and_grad(M.Params.unflat(vm, p.shift, p.scale), feat, tgt, mu=0.7)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_support_offsets_agree_with_grid_oracle(orc):
    """xi and rho (as the oracle build reports them) fix the normalised node
    offsets of the exact MLS shape function; exact MLS from those offsets
    equals the grid-based build."""
    from paper_1805_01113_amd import workloads as W
    gs = W.GridSpec([W.uniform_faces(16), W.uniform_faces(16), W.tanh_faces(24, 1.5, 2.5)], [True, True, False])
    g = orc.Grid(gs.faces, gs.periodic)
    r = np.random.default_rng(5)
    fz = gs.faces[2]
    x, y = r.uniform(0, 1, 50), r.uniform(0, 1, 50)
    z = r.uniform(fz[3], fz[-4], 50)
    for comp in range(3):
        out = orc.build_exact(g, comp, x, y, z)
        feat = np.concatenate([out["xi"], out["rho"]], 1)
        s = M.support_offsets(feat)
        for b in range(50):
            phi = orc.mls_shape(s[b])
            np.testing.assert_allclose(phi, out["phi"][b], rtol=0, atol=1e-12)


def test_exact_shape_functions_have_zero_residual(orc):
    feat = _feat(40, 6)
    s = M.support_offsets(feat)
    y = np.stack([orc.mls_shape(s[b]) for b in range(40)])
    r0, r1 = M.residuals(y, feat)
    assert r0.max() < 1e-13 and r1.max() < 1e-13
