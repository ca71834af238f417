"""FP64 reference of the learned shape-function surrogate (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's checks, never
by the product path; shares no code with the HIP kernels.

The surrogate is not part of the paper: it maps the features of one (marker,
component) support -- the in-cell offsets xi_d = (X - X_0)/H_d and the spacing
ratios rho_d = (X_{+1} - X_0)/(X_0 - X_{-1}) per axis, which determine the
exact MLS shape function (Sec. 2, eq. 3-6) completely -- to its 27 shape-
function values:

    u  = (x - shift) * scale                      (6 normalised inputs)
    z1 = u W1 + b1,   h1 = gelu(z1)               (128)
    z2 = h1 W2 + b2,  h2 = gelu(z2)               (128)
    y  = h2 W3 + b3                               (27)

with gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.  Training minimises

    L = mean_{b,k} (y_bk - t_bk)^2
        + mu * mean_b [ (sum_k y_bk - 1)^2 + sum_d (sum_k y_bk s_dk(b))^2 ],

the squared error plus the squared consistency residuals that gate the
surrogate at run time (partition of unity and reproduction of linear fields,
with s_dk the normalised offset of support node k from the marker along d).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_IN, N_H, N_OUT = 6, 128, 27
K = np.arange(27)
A_OFF = np.stack([K % 3, (K // 3) % 3, K // 9], axis=1)   # node index a_d in {0,1,2} per axis


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def support_offsets(feat):
    """s[b, d, a]: normalised position of support node a (0,1,2 = -1,0,+1)
    along axis d relative to the marker, from xi and rho.  With node spacings
    h- and h+ = rho h- and H = (h- + h+)/2 the nodes sit at -2/(1+rho),
    0, 2 rho/(1+rho) relative to the home node."""
    feat = np.asarray(feat, dtype=np.float64)
    xi, rho = feat[:, 0:3], feat[:, 3:6]
    s = np.empty((len(feat), 3, 3))
    s[:, :, 0] = -2.0 / (1.0 + rho) - xi
    s[:, :, 1] = -xi
    s[:, :, 2] = 2.0 * rho / (1.0 + rho) - xi
    return s


def node_offsets(feat):
    """s_dk[b, d, k] for the 27 support nodes (k = a_x + 3 a_y + 9 a_z)."""
    s = support_offsets(feat)
    return np.stack([s[:, d, A_OFF[:, d]] for d in range(3)], axis=1)


def residuals(y, feat):
    """Partition-of-unity and linear-reproduction residuals of shape functions y."""
    sk = node_offsets(feat)
    r0 = np.abs(y.sum(1) - 1.0)
    r1 = np.abs(np.einsum("bk,bdk->bd", y, sk)).max(1)
    return r0, r1


class Params:
    def __init__(self, w1, b1, w2, b2, w3, b3, shift, scale):
        self.w1, self.b1, self.w2, self.b2, self.w3, self.b3 = [np.asarray(a, dtype=np.float64) for a in
                                                                  (w1, b1, w2, b2, w3, b3)]
        self.shift = np.asarray(shift, dtype=np.float64)
        self.scale = np.asarray(scale, dtype=np.float64)

    def flat(self):
        return np.concatenate([a.ravel() for a in (self.w1, self.b1, self.w2, self.b2, self.w3, self.b3)])

    @classmethod
    def unflat(cls, v, shift, scale):
        shapes = [(N_IN, N_H), (N_H,), (N_H, N_H), (N_H,), (N_H, N_OUT), (N_OUT,)]
        out, o = [], 0
        for sh in shapes:
            n = int(np.prod(sh))
            out.append(np.asarray(v[o:o + n]).reshape(sh))
            o += n
        return cls(*out, shift, scale)


def forward(p: Params, feat):
    u = (np.asarray(feat, dtype=np.float64) - p.shift) * p.scale
    z1 = u @ p.w1 + p.b1
    h1 = gelu(z1)
    z2 = h1 @ p.w2 + p.b2
    h2 = gelu(z2)
    y = h2 @ p.w3 + p.b3
    return y, dict(u=u, z1=z1, h1=h1, z2=z2, h2=h2)


def loss_and_grad(p: Params, feat, target, mu=1.0):
    """Loss L (definition in the module docstring) and its gradient, by the
    chain rule written out layer by layer."""
    y, c = forward(p, feat)
    B = len(y)
    sk = node_offsets(feat)
    e = y - target
    r0 = y.sum(1) - 1.0
    r1 = np.einsum("bk,bdk->bd", y, sk)
    L = np.mean(e * e) + mu * np.mean(r0 * r0 + (r1 * r1).sum(1))
    dy = 2.0 * e / (B * N_OUT) + mu * (2.0 / B) * (r0[:, None] + np.einsum("bd,bdk->bk", r1, sk))
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = dy.sum(0)
    d2 = (dy @ p.w3.T) * gelu_grad(c["z2"])
    g["w2"] = c["h1"].T @ d2
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p.w2.T) * gelu_grad(c["z1"])
    g["w1"] = c["u"].T @ d1
    g["b1"] = d1.sum(0)
    flat = np.concatenate([g[k].ravel() for k in ("w1", "b1", "w2", "b2", "w3", "b3")])
    return L, flat


def init_params(seed=0, shift=None, scale=None):
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    r = np.random.default_rng(seed)
    w1 = r.normal(0, math.sqrt(2.0 / N_IN), (N_IN, N_H))
    w2 = r.normal(0, math.sqrt(2.0 / N_H), (N_H, N_H))
    w3 = r.normal(0, math.sqrt(2.0 / N_H), (N_H, N_OUT)) * 0.1
    return Params(w1, np.zeros(N_H), w2, np.zeros(N_H), w3, np.zeros(N_OUT),
                  np.zeros(N_IN) if shift is None else shift, np.ones(N_IN) if scale is None else scale)
