"""Pins of the oracle's derivative shape functions (eq. 6 differentiated in
the marker position) and of the cell-centred (pressure) staggering.

Against what the mathematics fixes, not the oracle's product-rule formula:
central differences of the (separately pinned) shape functions, the
derivatives of the MLS consistency conditions (partition of unity and
linear reproduction hold for every marker position, so their derivatives
vanish or give the identity), the closed form of the constant weight on a
uniform grid, exact gradients of linear fields on a stretched grid, and the
home cells of the pressure staggering."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1805_01113_amd import workloads as W

K = np.arange(27)
OFF = np.stack([K % 3 - 1, (K // 3) % 3 - 1, K // 9 - 1], axis=1).astype(np.float64)


def _offsets(rng, stretched):
    """Normalised node offsets of a random marker: s[d, a] = node_a - xi."""
    s = np.empty((3, 3))
    for d in range(3):
        if stretched:
            r = rng.uniform(0.6, 1.6)          # spacing ratio of the two intervals
            hm, hp = 2.0 / (1 + r), 2.0 * r / (1 + r)
            nodes = np.array([-hm, 0.0, hp])
        else:
            nodes = np.array([-1.0, 0.0, 1.0])
        s[d] = nodes - rng.uniform(-0.5, 0.5)
    return s


@pytest.mark.parametrize("kind", [orc.W_GAUSS_SHIFTED, orc.W_GAUSS, orc.W_CONST])
@pytest.mark.parametrize("stretched", [False, True])
def test_central_differences(kind, stretched):
    rng = np.random.default_rng(10 + kind + 3 * stretched)
    dl = 1e-6
    for _ in range(20):
        s = _offsets(rng, stretched)
        phi, dphi = orc.mls_shape_grad(s, kind=kind)
        np.testing.assert_allclose(phi, orc.mls_shape(s, kind=kind), rtol=0, atol=1e-14)
        for d in range(3):
            sp, sm = s.copy(), s.copy()
            sp[d] -= dl                         # marker moves by +dl: offsets by -dl
            sm[d] += dl
            fd = (orc.mls_shape(sp, kind=kind) - orc.mls_shape(sm, kind=kind)) / (2 * dl)
            assert np.abs(fd - dphi[d]).max() <= 1e-7 * max(1.0, np.abs(dphi[d]).max())


@pytest.mark.parametrize("stretched", [False, True])
def test_derivatives_of_consistency_conditions(stretched):
    """sum_k phi_k = 1 and sum_k phi_k s_ek = 0 for every position, so
    sum_k dphi_dk = 0 and sum_k dphi_dk s_ek = delta_de."""
    rng = np.random.default_rng(20 + stretched)
    for _ in range(50):
        s = _offsets(rng, stretched)
        _, dphi = orc.mls_shape_grad(s)
        S = np.stack([s[e][OFF[:, e].astype(int) + 1] for e in range(3)], axis=1)   # s_ek per node
        np.testing.assert_allclose(dphi.sum(axis=1), 0.0, atol=1e-12)
        np.testing.assert_allclose(dphi @ S, np.eye(3), atol=1e-12)


def test_constant_weight_closed_form():
    """Constant weight on a uniform stencil: phi_k = 1/27 + a_k . xi / 18, so
    d phi_k / d xi_d = a_kd / 18 everywhere."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        xi = rng.uniform(-0.5, 0.5, 3)
        s = np.array([[-1.0, 0.0, 1.0]] * 3) - xi[:, None]
        _, dphi = orc.mls_shape_grad(s, kind=orc.W_CONST)
        np.testing.assert_allclose(dphi, OFF.T / 18.0, atol=1e-14)


@pytest.mark.parametrize("comp", [0, 1, 2, 3])
def test_linear_field_gradient_on_stretched_grid(comp):
    """The gradient of a linear field is reproduced exactly on every
    staggering, in physical units (checks the 1/H scaling)."""
    fz = W.tanh_faces(32, 1.5, 2.5)
    faces = [W.uniform_faces(24), W.uniform_faces(20, 2.0), fz]
    g = orc.Grid(faces, (False, False, False))
    rng = np.random.default_rng(comp)
    n = 300
    x = rng.uniform(0.2, 0.8, n).astype(np.float32)
    y = rng.uniform(0.4, 1.6, n).astype(np.float32)
    z = rng.uniform(0.3, 1.2, n).astype(np.float32)
    alpha, beta = 0.7, np.array([1.3, -0.4, 2.1])
    nodes = [g.axis_nodes(comp, d) for d in range(3)]
    q = (alpha + beta[0] * nodes[0][None, None, :] + beta[1] * nodes[1][None, :, None]
         + beta[2] * nodes[2][:, None, None]).astype(np.float64)
    # the interpolation reads FP32 fields: keep q exactly representable
    q32 = q.astype(np.float32)
    U, G = orc.interp_grad(g, comp, x, y, z, q32)
    # reference from the FP32-rounded nodal values: their plane fit is not exact,
    # so compare against the exact field with a tolerance set by that rounding
    Xl = np.stack([x, y, z], axis=1).astype(np.float64)
    np.testing.assert_allclose(U, alpha + Xl @ beta, rtol=0, atol=1e-5)
    np.testing.assert_allclose(G, np.tile(beta, (n, 1)), rtol=0, atol=5e-4)
    # in FP64 nodal values the reproduction is exact to rounding
    r = orc.build_grad(g, comp, x, y, z)
    for d in range(3):
        gd = np.einsum("lk,lk->l", r["dphi"][:, d, :], _gather(g, comp, r["home"], q))
        np.testing.assert_allclose(gd, beta[d], rtol=1e-11)


def _gather(g, comp, home, q):
    """q at the 27 support nodes of each marker (wall axes, no wrap)."""
    out = np.empty((len(home), 27))
    for k in range(27):
        i = home[:, 0] + int(OFF[k, 0])
        j = home[:, 1] + int(OFF[k, 1])
        kk = home[:, 2] + int(OFF[k, 2])
        out[:, k] = q[kk, j, i]
    return out


def test_pressure_staggering_homes_and_consistency():
    """Cell-centred staggering: the home node is the cell holding the marker
    (floor(X n) on the periodic unit cube) and the shape functions keep
    partition of unity and linear reproduction."""
    n = 32
    g = orc.Grid([W.uniform_faces(n)] * 3, (True, True, True))
    rng = np.random.default_rng(5)
    x, y, z = (rng.uniform(-1, 2, 500).astype(np.float32) for _ in range(3))
    r = orc.build_grad(g, orc.COMP_CELL, x, y, z)
    for d, a in enumerate((x, y, z)):
        np.testing.assert_array_equal(r["home"][:, d], np.floor(np.mod(a.astype(np.float64), 1.0) * n))
    np.testing.assert_allclose(r["phi"].sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(r["dphi"].sum(axis=2), 0.0, atol=1e-9)
    e = orc.build_exact(g, orc.COMP_CELL, x, y, z)
    np.testing.assert_allclose(r["phi"], e["phi"], atol=1e-15)
