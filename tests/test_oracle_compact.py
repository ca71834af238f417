"""The identity behind the compact transfer functions of a time step (eq. 5):
phi_k = W_k (gamma . p_k) with gamma = A^{-1} e_0, A = sum_k W_k p_k p_k^T, so
that gamma and the support offsets fix the 27 shape functions.  Checked
against the oracle's exact shape functions, with gamma solved here by a
library routine from the oracle's 1-D weights; on a uniform axis the three
offsets follow from the centre one."""
import itertools

import numpy as np

from oracle import oracle as orc


def _phi_from_gamma(s):
    w = np.array([[orc.weight_1d(s[d, a]) for a in range(3)] for d in range(3)])
    nodes = list(itertools.product(range(3), repeat=3))     # (cz, by, ax) -> node k = ax + 3 by + 9 cz
    W = np.empty(27)
    P = np.empty((27, 4))
    for cz, by, ax in nodes:
        k = ax + 3 * by + 9 * cz
        W[k] = w[0, ax] * w[1, by] * w[2, cz]
        P[k] = [1.0, s[0, ax], s[1, by], s[2, cz]]
    A = (P * W[:, None]).T @ P
    gamma = np.linalg.solve(A, np.array([1.0, 0.0, 0.0, 0.0]))
    return W * (P @ gamma), gamma


def test_phi_equals_weights_times_gamma_dot_p():
    rng = np.random.default_rng(5)
    for trial in range(200):
        if trial % 2 == 0:
            # uniform axes: offsets (a - 1) - xi, xi in the home control volume
            xi = rng.uniform(-0.5, 0.5, 3)
            s = np.array([[a - 1.0 - xi[d] for a in range(3)] for d in range(3)])
        else:
            # stretched axes: node spacing ratio up to 2, offsets scaled by half the support
            s = np.empty((3, 3))
            for d in range(3):
                hm, hp = rng.uniform(0.6, 1.2, 2)
                x0 = rng.uniform(-0.5 * hm, 0.5 * hp)
                H = 0.5 * (hm + hp)
                s[d] = np.array([-hm - x0, -x0, hp - x0]) / H
        ref = orc.mls_shape(s)
        phi, gamma = _phi_from_gamma(s)
        assert np.max(np.abs(phi - ref)) <= 1e-12 * np.max(np.abs(ref)), trial
        # partition of unity and linear reproduction hold for the reconstruction too
        assert abs(phi.sum() - 1.0) <= 1e-12
        assert np.all(np.abs(gamma) < 1e6)


def test_uniform_offsets_follow_from_the_centre_one():
    """On a uniform axis s_{-1} = s_0 - 1 and s_{+1} = s_0 + 1: a row that
    stores s_0 alone reproduces the shape functions of the three offsets."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        xi = rng.uniform(-0.5, 0.5, 3)
        s0 = -xi
        s = np.stack([s0 - 1.0, s0, s0 + 1.0], axis=1)
        ref = orc.mls_shape(np.array([[a - 1.0 - xi[d] for a in range(3)] for d in range(3)]))
        assert np.max(np.abs(orc.mls_shape(s) - ref)) <= 1e-13
