"""Python access to the FP64 CPU oracle (``mls_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this module; the product library never does.  It
shares no code with the HIP library.

The grid is described as the paper states the problem (Sec. 2): per axis the
cell-face coordinates ``faces[d]`` (n_d + 1 values, FP64) and a periodic flag.
Velocity component c lives on the faces along axis c and on cell centres
along the other axes (marker-and-cell staggering).

Arrays returned here are in "marker-major" order: ``home[l, d]`` (wrapped node
index along axis d), ``phi[l, k]`` with support node k = a_x + 3 a_y + 9 a_z
(a_d = offset + 1, x fastest).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mls_oracle.c")
_LIB = os.path.join(_HERE, "liborc_mls.so")
_lock = threading.Lock()
_lib = None

W_GAUSS_SHIFTED = 0
W_GAUSS = 1
W_CONST = 2

E_SUPPORT = -2
E_SINGULAR = -3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, IEEE double)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, i64, f64 = ctypes.c_int, ctypes.c_long, ctypes.c_double
            L.orc_weight_1d.argtypes = [i32, f64, f64, f64]
            L.orc_weight_1d.restype = f64
            L.orc_mls_shape.argtypes = [i32, P, i32, f64, f64, P, P]
            L.orc_mls_shape_literal.argtypes = [i32, P, P, P, i32, f64, f64, P]
            L.orc_locate_axis.argtypes = [P, i32, i32, i32, f64, P, P]
            L.orc_build_exact.argtypes = [P, P, P, i32, i32, f64, f64, i64, P, P, P, P, P, P, P, P, P]
            L.orc_fast_table.argtypes = [i32, P, P, P, i32, i32, f64, f64, P]
            L.orc_fast_shape.argtypes = [i32, P, P, P, i32, P, P]
            L.orc_build_fast.argtypes = [P, P, P, i32, i32, f64, f64, i32, i64, P, P, P, P, P, P]
            L.orc_fast_shape_trilinear.argtypes = [i32, P, P, P, i32, P, P]
            L.orc_build_fast_blend.argtypes = [P, P, P, i32, i32, f64, f64, i32, i32, i64, P, P, P, P, P, P]
            L.orc_home_support.argtypes = [P, P, P, i32, P, P, P, P]
            L.orc_interp.argtypes = [P, P, P, i32, i64, P, P, P, P]
            L.orc_spread.argtypes = [P, P, P, i32, i64, P, P, P, P, P, P]
            L.orc_node_volumes.argtypes = [P, P, P, i32, P]
            L.orc_axis_nodes.argtypes = [P, P, P, i32, i32, P]
            L.orc_collide.argtypes = [P, P, P, i64, P, P, P, P, P, P, P, P]
            L.orc_refine.argtypes = [P, P, P, i64, P, i64, P, P, P, f64, i32, P, P, P, P, P, P, P, P, P]
            L.orc_weight_1d_deriv.argtypes = [i32, f64, f64, f64]
            L.orc_weight_1d_deriv.restype = f64
            L.orc_mls_shape_grad.argtypes = [i32, P, i32, f64, f64, P, P]
            L.orc_build_grad.argtypes = [P, P, P, i32, i32, f64, f64, i64, P, P, P, P, P, P]
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Grid:
    """Staggered Eulerian grid: faces per axis (FP64) and periodic flags."""

    def __init__(self, faces, periodic):
        self.faces = [np.ascontiguousarray(f, dtype=np.float64) for f in faces]
        self.n = np.array([len(f) - 1 for f in self.faces], dtype=np.int32)
        self.periodic = np.array([1 if p else 0 for p in periodic], dtype=np.int32)
        self._cat = np.ascontiguousarray(np.concatenate(self.faces))

    def args(self):
        return _p(self._cat), _p(self.n), _p(self.periodic)

    def dims(self, comp: int):
        """Node counts (x, y, z) of component comp's grid."""
        return tuple(int(self.n[d] + (1 if (d == comp and not self.periodic[d]) else 0)) for d in range(3))

    def shape(self, comp: int):
        """Array shape (z, y, x) of component comp's field."""
        nx, ny, nz = self.dims(comp)
        return (nz, ny, nx)

    def axis_nodes(self, comp: int, axis: int) -> np.ndarray:
        out = np.empty(self.dims(comp)[axis], dtype=np.float64)
        lib().orc_axis_nodes(*self.args(), comp, axis, _p(out))
        return out

    def node_volumes(self, comp: int) -> np.ndarray:
        out = np.empty(self.shape(comp), dtype=np.float64)
        lib().orc_node_volumes(*self.args(), comp, _p(out))
        return out


class OracleError(RuntimeError):
    def __init__(self, rc, bad):
        super().__init__("oracle error %d at marker %d" % (rc, bad))
        self.rc = rc
        self.bad = bad


def weight_1d(s, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5):
    return lib().orc_weight_1d(kind, eps, R, float(s))


def mls_shape(s, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5, with_kappa=False):
    """Exact MLS shape function from normalised support offsets s[d, a]."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    dim = s.shape[0]
    phi = np.empty(3 ** dim)
    kap = ctypes.c_double(0.0)
    rc = lib().orc_mls_shape(dim, _p(s), kind, eps, R, _p(phi), ctypes.byref(kap))
    if rc != 0:
        raise OracleError(rc, 0)
    return (phi, kap.value) if with_kappa else phi


def mls_shape_literal(xl, xn, H, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5):
    xl = np.ascontiguousarray(xl, dtype=np.float64)
    xn = np.ascontiguousarray(xn, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    dim = xl.shape[0]
    phi = np.empty(3 ** dim)
    rc = lib().orc_mls_shape_literal(dim, _p(xl), _p(xn), _p(H), kind, eps, R, _p(phi))
    if rc != 0:
        raise OracleError(rc, 0)
    return phi


def locate_axis(faces, periodic, is_face, x):
    faces = np.ascontiguousarray(faces, dtype=np.float64)
    ih = ctypes.c_long(0)
    X = ctypes.c_double(0.0)
    rc = lib().orc_locate_axis(_p(faces), len(faces) - 1, int(periodic), int(is_face), float(x),
                               ctypes.byref(ih), ctypes.byref(X))
    if rc != 0:
        raise OracleError(rc, 0)
    return ih.value, X.value


def _markers(x, y, z):
    return [np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, z)]


def build_exact(grid: Grid, comp, x, y, z, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5, check=True):
    """Exact MLS per marker: returns dict(home [N,3] int32, phi [N,27], kappa [N], xi, rho)."""
    x, y, z = _markers(x, y, z)
    n = len(x)
    home = np.empty((n, 3), dtype=np.int32)
    phi = np.empty((n, 27))
    kappa = np.empty(n)
    xi = np.empty((n, 3))
    rho = np.empty((n, 3))
    bad = ctypes.c_long(-1)
    rc = lib().orc_build_exact(*grid.args(), comp, kind, eps, R, n, _p(x), _p(y), _p(z),
                               _p(home), _p(phi), _p(kappa), _p(xi), _p(rho), ctypes.byref(bad))
    if rc != 0 and check:
        raise OracleError(rc, bad.value)
    return dict(home=home, phi=phi, kappa=kappa, xi=xi, rho=rho, rc=rc, bad=bad.value)


def fast_table(node, cvlo, cvhi, nsub, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5):
    node = np.ascontiguousarray(node, dtype=np.float64)
    dim = node.shape[0]
    cvlo = np.ascontiguousarray(cvlo, dtype=np.float64)
    cvhi = np.ascontiguousarray(cvhi, dtype=np.float64)
    ne = 3 ** dim
    table = np.empty((nsub ** dim, ne))
    rc = lib().orc_fast_table(dim, _p(node), _p(cvlo), _p(cvhi), nsub, kind, eps, R, _p(table))
    if rc != 0:
        raise OracleError(rc, 0)
    return table


BLEND_SHEPARD, BLEND_TRILINEAR = 0, 1


def fast_shape(xi, cvlo, cvhi, nsub, table, blend=BLEND_SHEPARD):
    """fast-MLS value at xi from a sub-node table: Shepard (eq. 9-10) or trilinear blend."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    dim = xi.shape[0]
    cvlo = np.ascontiguousarray(cvlo, dtype=np.float64)
    cvhi = np.ascontiguousarray(cvhi, dtype=np.float64)
    table = np.ascontiguousarray(table, dtype=np.float64)
    phi = np.empty(3 ** dim)
    f = lib().orc_fast_shape_trilinear if blend == BLEND_TRILINEAR else lib().orc_fast_shape
    f(dim, _p(xi), _p(cvlo), _p(cvhi), nsub, _p(table), _p(phi))
    return phi


def home_support(grid: Grid, comp, home):
    home = np.ascontiguousarray(home, dtype=np.int32)
    node = np.empty((3, 3))
    lo = np.empty(3)
    hi = np.empty(3)
    lib().orc_home_support(*grid.args(), comp, _p(home), _p(node), _p(lo), _p(hi))
    return node, lo, hi


def build_fast(grid: Grid, comp, x, y, z, nsub=9, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5, check=True,
               blend=BLEND_SHEPARD):
    x, y, z = _markers(x, y, z)
    n = len(x)
    home = np.empty((n, 3), dtype=np.int32)
    phi = np.empty((n, 27))
    bad = ctypes.c_long(-1)
    rc = lib().orc_build_fast_blend(*grid.args(), comp, kind, eps, R, nsub, blend, n, _p(x), _p(y), _p(z),
                                    _p(home), _p(phi), ctypes.byref(bad))
    if rc != 0 and check:
        raise OracleError(rc, bad.value)
    return dict(home=home, phi=phi, rc=rc, bad=bad.value)


def interp(grid: Grid, comp, home, phi, q):
    home = np.ascontiguousarray(home, dtype=np.int32)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float32)
    assert q.shape == grid.shape(comp)
    n = home.shape[0]
    U = np.empty(n)
    lib().orc_interp(*grid.args(), comp, n, _p(home), _p(phi), _p(q), _p(U))
    return U


def spread(grid: Grid, comp, home, phi, area, F, f=None):
    """Adds the eq. 7-8 forcing of component comp into the FP64 field f."""
    home = np.ascontiguousarray(home, dtype=np.int32)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    area = np.ascontiguousarray(area, dtype=np.float32)
    F = np.ascontiguousarray(F, dtype=np.float32)
    n = home.shape[0]
    if f is None:
        f = np.zeros(grid.shape(comp))
    assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == grid.shape(comp)
    cl = np.empty(n)
    lib().orc_spread(*grid.args(), comp, n, _p(home), _p(phi), _p(area), _p(F), _p(f), _p(cl))
    return f, cl


def collide(grid: Grid, x, y, z, body, check=True):
    """Coarse-grained collision detection (Sec. 4): returns dict(coll
    [nz, ny, nx] int32 with 0 = empty cell, b + 1 = markers of body b only,
    -1 = markers of several bodies; flag [N] uint8 = 1 where the marker's
    cell holds -1; cell [N] linear cell index)."""
    x, y, z = _markers(x, y, z)
    body = np.ascontiguousarray(body, dtype=np.int32)
    n = len(x)
    assert len(body) == n
    nx, ny, nz = (int(v) for v in grid.n)
    coll = np.empty((nz, ny, nx), dtype=np.int32)
    cell = np.empty(n, dtype=np.int64)
    flag = np.empty(n, dtype=np.uint8)
    bad = ctypes.c_long(-1)
    rc = lib().orc_collide(*grid.args(), n, _p(x), _p(y), _p(z), _p(body), _p(coll), _p(cell), _p(flag),
                           ctypes.byref(bad))
    if rc != 0 and check:
        raise OracleError(rc, bad.value)
    return dict(coll=coll, flag=flag, cell=cell, rc=rc, bad=bad.value)


def refine(grid: Grid, tri, xv, yv, zv, ratio=1.0, level=-1, check=True):
    """Adaptive Lagrangian mesh refinement (Sec. 3): returns dict(x, y, z,
    area [M] FP64, normal [M, 3], parent [M] int32, level [T] uint8, count)
    for the base triangles tri [T, 3] over FP32 vertices; level -1 chooses
    each triangle's level from its size against the local cell size."""
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    xv, yv, zv = _markers(xv, yv, zv)
    T = tri.shape[0]
    M = 4 * T
    x, y, z, area = (np.empty(M) for _ in range(4))
    normal = np.empty((M, 3))
    parent = np.empty(M, dtype=np.int32)
    lev = np.empty(T, dtype=np.uint8)
    count = ctypes.c_long(0)
    bad = ctypes.c_long(-1)
    rc = lib().orc_refine(*grid.args(), T, _p(tri), len(xv), _p(xv), _p(yv), _p(zv), float(ratio), int(level),
                          _p(x), _p(y), _p(z), _p(area), _p(normal), _p(parent), _p(lev), ctypes.byref(count),
                          ctypes.byref(bad))
    if rc != 0 and check:
        raise OracleError(rc, bad.value)
    m = count.value
    return dict(x=x[:m], y=y[:m], z=z[:m], area=area[:m], normal=normal[:m], parent=parent[:m], level=lev,
                count=m, rc=rc, bad=bad.value)


COMP_CELL = 3   # staggering of cell-centred fields (pressure): no face axis


def mls_shape_grad(s, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5):
    """phi [3^dim] and d phi / d xi [dim, 3^dim] for node offsets s [dim, 3]
    (normalised units; the marker's normalised coordinate xi moves the
    offsets by -xi)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    dim = s.shape[0]
    phi = np.empty(3 ** dim)
    dphi = np.empty((dim, 3 ** dim))
    rc = lib().orc_mls_shape_grad(dim, _p(s), kind, eps, R, _p(phi), _p(dphi))
    if rc != 0:
        raise OracleError(rc, 0)
    return phi, dphi


def build_grad(grid: Grid, comp, x, y, z, kind=W_GAUSS_SHIFTED, eps=1.0, R=1.5, check=True):
    """Exact shape functions and their derivatives in the marker position:
    dict(home [N,3], phi [N,27], dphi [N,3,27] (d phi_k / d x_d)); comp 3 is
    the cell-centred (pressure) staggering."""
    x, y, z = _markers(x, y, z)
    n = len(x)
    home = np.empty((n, 3), dtype=np.int32)
    phi = np.empty((n, 27))
    dphi = np.empty((n, 3, 27))
    bad = ctypes.c_long(-1)
    rc = lib().orc_build_grad(*grid.args(), comp, kind, eps, R, n, _p(x), _p(y), _p(z), _p(home), _p(phi),
                              _p(dphi), ctypes.byref(bad))
    if rc != 0 and check:
        raise OracleError(rc, bad.value)
    return dict(home=home, phi=phi, dphi=dphi, rc=rc, bad=bad.value)


def interp_grad(grid: Grid, comp, x, y, z, q):
    """Value and gradient of the MLS approximation of field q (on the
    staggering of comp) at the markers: (U [N], G [N, 3])."""
    r = build_grad(grid, comp, x, y, z)
    U = interp(grid, comp, r["home"], r["phi"], q)
    G = np.stack([interp(grid, comp, r["home"], np.ascontiguousarray(r["dphi"][:, d, :]), q) for d in range(3)],
                 axis=1)
    return U, G


# ---------------------------------------------------------------------------
# Counter-based jitter of the batched time step (SplitMix64 output function,
# Steele, Lea & Flood, OOPSLA 2014), written here independently of the HIP
# library from the published definition.
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, ctr):
    """Output of a SplitMix64 stream started at `seed` after ctr+1 advances."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(ctr, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def jitter(x0, y0, z0, step, amp, seed):
    """x = x0 + (u - 1/2)(2 amp) per axis, u = top 24 bits of
    splitmix64(seed, (step n + l) 3 + axis) / 2^24, all in FP32."""
    n = len(x0)
    l = np.arange(n, dtype=np.uint64)
    out = []
    amp2 = np.float32(2.0) * np.float32(amp)
    for axis, a0 in enumerate((x0, y0, z0)):
        ctr = (np.uint64(step) * np.uint64(n) + l) * np.uint64(3) + np.uint64(axis)
        u = (splitmix64(seed, ctr) >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
        d = (u - np.float32(0.5)) * amp2
        out.append((np.asarray(a0, dtype=np.float32) + d).astype(np.float32))
    return out
