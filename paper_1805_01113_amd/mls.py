"""Thin ctypes binding of the C ABI in include/mls.h (argument marshalling only).

Every step of the transfer runs in the HIP library libmls_hip.so; torch
tensors are used only as device buffers and their streams.  The library is
loaded on first use and a missing library raises -- there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmls_hip.so")

MLS_EXACT, MLS_FAST, MLS_LEARNED, MLS_FAST_LINEAR = 0, 1, 2, 3
MLS_STEP_COMPACT = 1
SPREAD_NOALLOC_BYTES = 64 << 20   # MLS_SPREAD_NOALLOC_BYTES
MLS_OK, MLS_E_ARG, MLS_E_SUPPORT, MLS_E_SINGULAR, MLS_E_NONFINITE, MLS_E_HIP, MLS_E_NOMEM, MLS_E_RANGE = \
    0, -1, -2, -3, -4, -5, -6, -7
W_GAUSS_SHIFTED, W_GAUSS, W_CONST = 0, 1, 2
STATUS = {0: "MLS_OK", -1: "MLS_E_ARG", -2: "MLS_E_SUPPORT", -3: "MLS_E_SINGULAR", -4: "MLS_E_NONFINITE",
          -5: "MLS_E_HIP", -6: "MLS_E_NOMEM", -7: "MLS_E_RANGE"}

_lib = None


class MLSError(RuntimeError):
    def __init__(self, status: int, message: str, first_bad: int = -1):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status
        self.first_bad = first_bad


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("periodic", ctypes.c_int32 * 3),
                ("faces", ctypes.POINTER(ctypes.c_double) * 3)]


class _Weight(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("eps", ctypes.c_double), ("radius", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("kappa_tau", ctypes.c_double), ("n_sub", ctypes.c_int32), ("fallback_tol", ctypes.c_double),
                ("spread_tile", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("fp64_solves", ctypes.c_int64), ("fallbacks", ctypes.c_int64), ("learned", ctypes.c_int64),
                ("kappa_max", ctypes.c_double), ("spread_entries", ctypes.c_int64),
                ("spread_tiles", ctypes.c_int64)]


class _StepDesc(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("dt", ctypes.c_float), ("jitter", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_int32)]


class _StepBuf(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in (
        "x0", "y0", "z0", "x", "y", "z", "area", "vb", "home", "phi", "route", "u", "v", "w", "U", "F",
        "fx", "fy", "fz")]


MLP_PARAMS = 20891   # 6*128 + 128 + 128*128 + 128 + 128*27 + 27

class _Tune(ctypes.Structure):
    _fields_ = [("spread_tile", ctypes.c_int32), ("spread_blocks_per_cu", ctypes.c_int32),
                ("build_blocks_per_cu", ctypes.c_int32), ("interp_blocks_per_cu", ctypes.c_int32),
                ("spread_threads", ctypes.c_int32)]


class _TuneReport(ctypes.Structure):
    _fields_ = [("best", _Tune), ("ms_build", ctypes.c_double), ("ms_interp", ctypes.c_double),
                ("ms_spread", ctypes.c_double), ("from_cache", ctypes.c_int32), ("candidates", ctypes.c_int32)]


K_NAMES = ["build_exact", "build_fast", "build_learned", "interp", "spread_bin", "spread_tiles", "jitter", "force",
           "build_interp", "collide", "collide_clear", "refine", "build_grad", "interp_grad",
           "fast_interp"]


class _Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 16), ("launches", ctypes.c_int64 * 16)]


def load(path: str = LIB_PATH, need_torch: bool = True):
    """Load libmls_hip.so.  torch is imported first so that the library binds
    to the HIP runtime torch already uses."""
    global _lib
    if _lib is not None:
        return _lib
    if need_torch:
        import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError("libmls_hip.so is not built (%s); run __graft_entry__.build()" % path)
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.mls_version.restype = ctypes.c_char_p
    L.mls_ctx_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(_Grid), ctypes.POINTER(_Weight),
                                 ctypes.POINTER(_Opts)]
    L.mls_ctx_destroy.argtypes = [P]
    L.mls_ctx_destroy.restype = None
    L.mls_reserve.argtypes = [P, I64]
    L.mls_build.argtypes = [P, I64, P, P, P, I32, P, P, P, P]
    L.mls_interp.argtypes = [P, I64, P, P, P, P, P, P, P, P, P]
    L.mls_spread.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P]
    L.mls_spread_noalloc.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P]
    L.mls_collide.argtypes = [P, I64, P, P, P, P, P, P, P]
    L.mls_collide_clear.argtypes = [P, I64, P, P, P, P, P]
    L.mls_build_grad.argtypes = [P, I64, P, P, P, I32, P, P, P, P]
    L.mls_interp_grad.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P, P, P]
    L.mls_refine.argtypes = [P, I64, P, I64, P, P, P, ctypes.c_double, I32, I64, P, P, P, P, P, P, P, P, P]
    L.mls_sync.argtypes = [P, P, ctypes.POINTER(I64)]
    L.mls_last_error.argtypes = [P]
    L.mls_last_error.restype = ctypes.c_char_p
    L.mls_stats_get.argtypes = [P, ctypes.POINTER(_Stats)]
    L.mls_stats_reset.argtypes = [P]
    L.mls_fast_tables.argtypes = [P, P, ctypes.POINTER(I64), ctypes.POINTER(I32),
                                  ctypes.POINTER(I32), ctypes.POINTER(I32), P]
    L.mls_step.argtypes = [P, ctypes.POINTER(_StepDesc), ctypes.POINTER(_StepBuf), P]
    L.mls_step_counter_set.argtypes = [P, ctypes.c_uint64, P]
    L.mls_step_order.argtypes = [P, P, I64, P]
    L.mls_graph_create.argtypes = [P, ctypes.POINTER(_StepDesc), ctypes.POINTER(_StepBuf), ctypes.POINTER(P)]
    L.mls_graph_launch.argtypes = [P, I32, P]
    L.mls_graph_destroy.argtypes = [P]
    L.mls_graph_destroy.restype = None
    L.mls_timing_enable.argtypes = [P, I32]
    L.mls_timing_get.argtypes = [P, ctypes.POINTER(_Timing), I32]
    L.mls_tune_get.argtypes = [P, ctypes.POINTER(_Tune)]
    L.mls_tune_set.argtypes = [P, ctypes.POINTER(_Tune)]
    L.mls_autotune.argtypes = [P, I32, I32, ctypes.POINTER(_StepBuf), ctypes.c_char_p, ctypes.POINTER(_TuneReport),
                               P]
    L.mls_mlp_load.argtypes = [P, P, P]
    L.mls_mlp_get.argtypes = [P, P, P]
    L.mls_features.argtypes = [P, I64, P, P, P, P, P]
    L.mls_mlp_forward.argtypes = [P, I64, P, I64, P, P, P]
    L.mls_mlp_grad.argtypes = [P, I64, P, P, I64, P, ctypes.c_float, P, P, P]
    L.mls_mlp_train_step.argtypes = [P, I64, P, P, I64, P, ctypes.c_float, ctypes.c_float, P, P]
    for name in ("mls_tune_get", "mls_tune_set", "mls_autotune", "mls_mlp_load", "mls_mlp_get", "mls_features", "mls_mlp_forward", "mls_mlp_grad",
                 "mls_mlp_train_step","mls_ctx_create", "mls_reserve", "mls_build", "mls_interp", "mls_spread", "mls_spread_noalloc", "mls_sync",
                 "mls_stats_get", "mls_stats_reset", "mls_fast_tables", "mls_step", "mls_step_counter_set", "mls_step_order",
                 "mls_graph_create", "mls_graph_launch", "mls_timing_enable", "mls_timing_get"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check_dev(t, dtype, numel, name):
    import torch
    if t is None:
        raise ValueError("%s is required" % name)
    if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() != numel:
        raise ValueError("%s must be a contiguous CUDA %s tensor of %d elements (got %s %s %s)"
                         % (name, dtype, numel, t.device, t.dtype, tuple(t.shape)))


class Context:
    """One grid + weight + option set (mls_ctx)."""

    def __init__(self, faces: Sequence[np.ndarray], periodic: Sequence[bool], kind: int = W_GAUSS_SHIFTED,
                 eps: float = 1.0, radius: float = 1.5, kappa_tau: float = 1e6, n_sub: int = 9,
                 fallback_tol: float = 1e-4, spread_tile: int = 0):
        L = load()
        self._lib = L
        self.faces = [np.ascontiguousarray(f, dtype=np.float64) for f in faces]
        self.periodic = [bool(p) for p in periodic]
        self.n = [len(f) - 1 for f in self.faces]
        g = _Grid()
        for d in range(3):
            g.n[d] = self.n[d]
            g.periodic[d] = 1 if self.periodic[d] else 0
            g.faces[d] = self.faces[d].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        w = _Weight(kind, eps, radius)
        o = _Opts(kappa_tau, n_sub, fallback_tol, spread_tile)
        self.n_sub = n_sub
        self.mlp_loaded = False
        h = ctypes.c_void_p()
        st = L.mls_ctx_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(w), ctypes.byref(o))
        if st != 0:
            raise MLSError(st, "mls_ctx_create rejected the grid/weight/options")
        self.h = h

    @classmethod
    def from_grid(cls, grid, **kw):
        return cls(grid.faces, grid.periodic, **kw)

    def close(self):
        if getattr(self, "h", None):
            self._lib.mls_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st, what):
        if st != 0:
            raise MLSError(st, "%s: %s" % (what, self._lib.mls_last_error(self.h).decode()))

    def dims(self, comp: int):
        return tuple(self.n[d] + (1 if (d == comp and not self.periodic[d]) else 0) for d in range(3))

    def shape(self, comp: int):
        nx, ny, nz = self.dims(comp)
        return (nz, ny, nx)

    # ---- C ABI calls -------------------------------------------------------
    def reserve(self, n: int):
        self._raise(self._lib.mls_reserve(self.h, int(n)), "mls_reserve")

    def build(self, x, y, z, method: int = MLS_EXACT, home=None, phi=None, route=None, stream=None):
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dev(t, torch.float32, n, nm)
        dev = x.device
        m = npad(n)
        if home is None:
            home = torch.empty(3 * m, dtype=torch.int32, device=dev)
        if phi is None:
            phi = torch.empty(81 * m, dtype=torch.float32, device=dev)
        _check_dev(home, torch.int32, 3 * m, "home")
        _check_dev(phi, torch.float32, 81 * m, "phi")
        if route is not None:
            _check_dev(route, torch.uint8, 3 * m, "route")
        st = self._lib.mls_build(self.h, n, _ptr(x), _ptr(y), _ptr(z), int(method), _ptr(home), _ptr(phi),
                                 _ptr(route), _stream(stream))
        self._raise(st, "mls_build")
        return home, phi, route

    def interp(self, home, phi, u, v, w, n, out=None, stream=None):
        """U [3, n] = Phi^T q (eq. 6) for the n markers of home/phi."""
        import torch
        _check_dev(home, torch.int32, 3 * npad(n), "home")
        _check_dev(phi, torch.float32, 81 * npad(n), "phi")
        for c, q in enumerate((u, v, w)):
            _check_dev(q, torch.float32, int(np.prod(self.shape(c))), "field %d" % c)
        if out is None:
            out = torch.empty((3, n), dtype=torch.float32, device=home.device)
        _check_dev(out, torch.float32, 3 * n, "out")
        st = self._lib.mls_interp(self.h, n, _ptr(home), _ptr(phi), _ptr(u), _ptr(v), _ptr(w),
                                  _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _stream(stream))
        self._raise(st, "mls_interp")
        return out

    def spread(self, home, phi, area, F, fields, stream=None):
        """Adds the eq. 7-8 forcing of marker forces F [3, n] into fields (u, v, w grids)."""
        import torch
        n = area.numel()
        _check_dev(home, torch.int32, 3 * npad(n), "home")
        _check_dev(phi, torch.float32, 81 * npad(n), "phi")
        _check_dev(area, torch.float32, n, "area")
        _check_dev(F, torch.float32, 3 * n, "F")
        for c, q in enumerate(fields):
            _check_dev(q, torch.float32, int(np.prod(self.shape(c))), "force field %d" % c)
        st = self._lib.mls_spread(self.h, n, _ptr(home), _ptr(phi), _ptr(area), _ptr(F[0]), _ptr(F[1]),
                                  _ptr(F[2]), _ptr(fields[0]), _ptr(fields[1]), _ptr(fields[2]), _stream(stream))
        self._raise(st, "mls_spread")
        return fields

    def spread_noalloc(self, home, phi, area, F, fields, stream=None):
        """spread() through the allocation-free entry point: its scratch is the
        library's fixed per-GPU array (SPREAD_NOALLOC_BYTES), so calls that
        overlap on one GPU race."""
        import torch
        n = area.numel()
        _check_dev(home, torch.int32, 3 * npad(n), "home")
        _check_dev(phi, torch.float32, 81 * npad(n), "phi")
        _check_dev(area, torch.float32, n, "area")
        _check_dev(F, torch.float32, 3 * n, "F")
        for c, q in enumerate(fields):
            _check_dev(q, torch.float32, int(np.prod(self.shape(c))), "force field %d" % c)
        st = self._lib.mls_spread_noalloc(self.h, n, _ptr(home), _ptr(phi), _ptr(area), _ptr(F[0]), _ptr(F[1]),
                                          _ptr(F[2]), _ptr(fields[0]), _ptr(fields[1]), _ptr(fields[2]),
                                          _stream(stream))
        self._raise(st, "mls_spread_noalloc")
        return fields

    def cell_shape(self):
        """Shape (z, y, x) of the cell array of collision detection."""
        return tuple(int(v) for v in self.n[::-1])

    def collide(self, x, y, z, body, coll, flags=None, stream=None):
        """Coarse-grained collision detection (Sec. 4): enters the markers'
        body ids into the zeroed int32 cell array coll (0 empty, body + 1 one
        body, -1 several bodies) and, if given, sets flags [n] uint8 to 1 for
        markers in a cell holding -1."""
        import torch
        n = x.numel()
        for a, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dev(a, torch.float32, n, nm)
        _check_dev(body, torch.int32, n, "body")
        _check_dev(coll, torch.int32, int(np.prod(self.cell_shape())), "coll")
        if flags is not None:
            _check_dev(flags, torch.uint8, n, "flags")
        st = self._lib.mls_collide(self.h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(body), _ptr(coll), _ptr(flags),
                                   _stream(stream))
        self._raise(st, "mls_collide")
        return coll, flags

    def build_grad(self, x, y, z, stagger, home=None, phi=None, dphi=None, stream=None):
        """Exact shape functions and their derivatives in the marker position
        for one staggering (0, 1, 2: u, v, w grids; 3: cell centres), in the
        64-marker blocked layout: home [npad], phi [npad/64, 27, 64],
        dphi [npad/64, 3, 27, 64]."""
        import torch
        n = x.numel()
        for a, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dev(a, torch.float32, n, nm)
        npd = npad(n)
        dev = x.device
        if home is None:
            home = torch.empty(npd, dtype=torch.int32, device=dev)
        if phi is None:
            phi = torch.empty((npd // 64, 27, 64), dtype=torch.float32, device=dev)
        if dphi is None:
            dphi = torch.empty((npd // 64, 3, 27, 64), dtype=torch.float32, device=dev)
        _check_dev(home, torch.int32, npd, "home")
        _check_dev(phi, torch.float32, 27 * npd, "phi")
        _check_dev(dphi, torch.float32, 81 * npd, "dphi")
        st = self._lib.mls_build_grad(self.h, n, _ptr(x), _ptr(y), _ptr(z), int(stagger), _ptr(home), _ptr(phi),
                                      _ptr(dphi), _stream(stream))
        self._raise(st, "mls_build_grad")
        return home, phi, dphi

    def interp_grad(self, x, y, z, u, v, w, p=None, values=True, stream=None):
        """Velocities U [3, n] (if values), their gradients G [9, n]
        (G[3c + d] = d u_c / d x_d) and, for a cell-centred p, P [n] and
        GP [3, n] at the markers."""
        import torch
        n = x.numel()
        for a, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dev(a, torch.float32, n, nm)
        for c, q in enumerate((u, v, w)):
            _check_dev(q, torch.float32, int(np.prod(self.shape(c))), "field %d" % c)
        dev = x.device
        U = torch.empty((3, n), dtype=torch.float32, device=dev) if values else None
        G = torch.empty((9, n), dtype=torch.float32, device=dev)
        P = GP = None
        if p is not None:
            _check_dev(p, torch.float32, int(np.prod(self.cell_shape())), "p")
            P = torch.empty(n, dtype=torch.float32, device=dev)
            GP = torch.empty((3, n), dtype=torch.float32, device=dev)
        st = self._lib.mls_interp_grad(self.h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(u), _ptr(v), _ptr(w), _ptr(U),
                                       _ptr(G), _ptr(p), _ptr(P), _ptr(GP), _stream(stream))
        self._raise(st, "mls_interp_grad")
        return dict(U=U, G=G, P=P, GP=GP)

    def refine(self, tri, xv, yv, zv, ratio=1.0, level=-1, stream=None, sync=True):
        """Adaptive Lagrangian mesh refinement (Sec. 3): markers of the base
        triangles tri [T, 3] (int32) over vertices xv, yv, zv.  Returns a dict
        of device tensors x, y, z, area [M], normal [3, M], parent [M],
        level [T] and the marker count M (syncs the stream to read it)."""
        import torch
        T = tri.shape[0] if tri.dim() == 2 else tri.numel() // 3
        _check_dev(tri, torch.int32, 3 * T, "tri")
        nv = xv.numel()
        for a, nm in ((xv, "xv"), (yv, "yv"), (zv, "zv")):
            _check_dev(a, torch.float32, nv, nm)
        cap = max(4 * T, 1)
        dev = xv.device
        x, y, z, area = (torch.empty(cap, dtype=torch.float32, device=dev) for _ in range(4))
        normal = torch.empty((3, cap), dtype=torch.float32, device=dev)
        parent = torch.empty(cap, dtype=torch.int32, device=dev)
        lev = torch.empty(max(T, 1), dtype=torch.uint8, device=dev)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        st = self._lib.mls_refine(self.h, T, _ptr(tri), nv, _ptr(xv), _ptr(yv), _ptr(zv), float(ratio), int(level),
                                  cap, _ptr(x), _ptr(y), _ptr(z), _ptr(area), _ptr(normal), _ptr(parent), _ptr(lev),
                                  _ptr(count), _stream(stream))
        self._raise(st, "mls_refine")
        out = dict(x=x, y=y, z=z, area=area, normal=normal, parent=parent, level=lev[:T], count_dev=count,
                   capacity=cap)
        if sync:
            m = int(count.item())
            out.update(count=m, x=x[:m], y=y[:m], z=z[:m], area=area[:m], normal=normal[:, :m],
                       parent=parent[:m])
        return out

    def collide_clear(self, x, y, z, coll, stream=None):
        """Returns the cells of the markers at x, y, z to zero."""
        import torch
        n = x.numel()
        for a, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dev(a, torch.float32, n, nm)
        _check_dev(coll, torch.int32, int(np.prod(self.cell_shape())), "coll")
        st = self._lib.mls_collide_clear(self.h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(coll), _stream(stream))
        self._raise(st, "mls_collide_clear")
        return coll

    def sync(self, stream=None, raise_on_error=True):
        bad = ctypes.c_int64(-1)
        st = self._lib.mls_sync(self.h, _stream(stream), ctypes.byref(bad))
        if st != 0 and raise_on_error:
            raise MLSError(st, self._lib.mls_last_error(self.h).decode(), bad.value)
        return st, bad.value

    def stats(self):
        s = _Stats()
        self._raise(self._lib.mls_stats_get(self.h, ctypes.byref(s)), "mls_stats_get")
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def stats_reset(self):
        self._raise(self._lib.mls_stats_reset(self.h), "mls_stats_reset")

    def fast_tables(self, stream=None):
        """Copy of the fast-MLS tables: (array [count, n_sub^3, 27] on the device,
        first[2], stretched_axis)."""
        import torch
        cnt = ctypes.c_int64()
        stride = ctypes.c_int32()
        first = (ctypes.c_int32 * 2)()
        ax = ctypes.c_int32()
        st = self._lib.mls_fast_tables(self.h, None, ctypes.byref(cnt), ctypes.byref(stride), first,
                                       ctypes.byref(ax), _stream(stream))
        self._raise(st, "mls_fast_tables")
        rows = self.n_sub ** 3
        buf = torch.empty((cnt.value, rows, stride.value), dtype=torch.float32, device="cuda")
        st = self._lib.mls_fast_tables(self.h, ctypes.c_void_p(buf.data_ptr()), None, None, None, None,
                                       _stream(stream))
        self._raise(st, "mls_fast_tables")
        return buf[:, :, :27], (first[0], first[1]), ax.value

    # ---- launch shapes ---------------------------------------------------------
    def tune_get(self):
        t = _Tune()
        self._raise(self._lib.mls_tune_get(self.h, ctypes.byref(t)), "mls_tune_get")
        return {k: getattr(t, k) for k, _ in _Tune._fields_}

    def tune_set(self, **shape):
        cur = self.tune_get()
        cur.update(shape)
        t = _Tune(**cur)
        self._raise(self._lib.mls_tune_set(self.h, ctypes.byref(t)), "mls_tune_set")

    def autotune(self, bufs: "StepBuffers", method=MLS_EXACT, cache_path=None, stream=None, compact=False):
        """Time launch shapes on the step buffers and apply the fastest
        (mls_autotune); compact=True tunes the compact exact step.  Returns
        the report as a dict."""
        r = _TuneReport()
        b = bufs.struct()
        cp = None if cache_path is None else os.fsencode(cache_path)
        flags = MLS_STEP_COMPACT if compact else 0
        self._raise(self._lib.mls_autotune(self.h, int(method), flags, ctypes.byref(b), cp, ctypes.byref(r),
                                           _stream(stream)), "mls_autotune")
        out = {k: getattr(r.best, k) for k, _ in _Tune._fields_}
        out.update(ms_build=r.ms_build, ms_interp=r.ms_interp, ms_spread=r.ms_spread,
                   from_cache=bool(r.from_cache), candidates=r.candidates)
        return out

    # ---- learned surrogate ---------------------------------------------------
    def mlp_load(self, params: np.ndarray, norm: np.ndarray):
        """Load the network (MLP_PARAMS FP32 parameters, norm = shift[6], scale[6])."""
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        q = np.ascontiguousarray(norm, dtype=np.float32).ravel()
        if p.size != MLP_PARAMS or q.size != 12:
            raise ValueError("need %d parameters and 12 normalisation values" % MLP_PARAMS)
        self._raise(self._lib.mls_mlp_load(self.h, p.ctypes.data, q.ctypes.data), "mls_mlp_load")
        self.mlp_loaded = True

    def mlp_get(self):
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        q = np.empty(12, dtype=np.float32)
        self._raise(self._lib.mls_mlp_get(self.h, p.ctypes.data, q.ctypes.data), "mls_mlp_get")
        return p, q

    def features(self, x, y, z, out=None, stream=None):
        """Features [3, n, 6] (xi_x, xi_y, xi_z, rho_x, rho_y, rho_z per component)."""
        import torch
        n = x.numel()
        for t, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dev(t, torch.float32, n, nm)
        if out is None:
            out = torch.empty((3, n, 6), dtype=torch.float32, device=x.device)
        _check_dev(out, torch.float32, 18 * n, "out")
        self._raise(self._lib.mls_features(self.h, n, _ptr(x), _ptr(y), _ptr(z), _ptr(out), _stream(stream)),
                    "mls_features")
        return out

    def _rows(self, feat, idx):
        import torch
        if feat.dim() != 2 or feat.shape[1] != 6:
            feat = feat.reshape(-1, 6)
        _check_dev(feat, torch.float32, feat.shape[0] * 6, "feat")
        if idx is not None:
            _check_dev(idx, torch.int64, idx.numel(), "idx")
            return feat, idx.numel(), feat.shape[0]
        return feat, feat.shape[0], feat.shape[0]

    def mlp_forward(self, feat, idx=None, out=None, stream=None):
        """Network output [m, 27] for feature rows feat[idx] (or all rows)."""
        import torch
        feat, m, rows = self._rows(feat, idx)
        if out is None:
            out = torch.empty((m, 27), dtype=torch.float32, device=feat.device)
        _check_dev(out, torch.float32, 27 * m, "out")
        self._raise(self._lib.mls_mlp_forward(self.h, m, _ptr(feat), rows, _ptr(idx), _ptr(out), _stream(stream)),
                    "mls_mlp_forward")
        return out

    def mlp_grad(self, feat, target, mu=1.0, idx=None, stream=None):
        """(loss, gradient) of a batch; both device tensors."""
        import torch
        feat, m, rows = self._rows(feat, idx)
        target = target.reshape(-1, 27)
        _check_dev(target, torch.float32, rows * 27, "target")
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feat.device)
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        self._raise(self._lib.mls_mlp_grad(self.h, m, _ptr(feat), _ptr(target), rows, _ptr(idx), float(mu),
                                           _ptr(grad), _ptr(loss), _stream(stream)), "mls_mlp_grad")
        return loss, grad

    def mlp_train_step(self, feat, target, lr, mu=1.0, idx=None, loss=None, stream=None):
        import torch
        feat, m, rows = self._rows(feat, idx)
        target = target.reshape(-1, 27)
        _check_dev(target, torch.float32, rows * 27, "target")
        if loss is not None:
            _check_dev(loss, torch.float32, 1, "loss")
        self._raise(self._lib.mls_mlp_train_step(self.h, m, _ptr(feat), _ptr(target), rows, _ptr(idx), float(mu),
                                                 float(lr), _ptr(loss), _stream(stream)), "mls_mlp_train_step")


class StepBuffers:
    """Device buffers of one batched time step (all bodies back to back)."""

    def __init__(self, ctx: "Context", x0, y0, z0, area, fields, forcing, vb=None, route=False):
        import torch
        n = x0.numel()
        dev = x0.device
        self.n = n
        self.x0, self.y0, self.z0, self.area = x0, y0, z0, area
        self.x = torch.empty_like(x0)
        self.y = torch.empty_like(y0)
        self.z = torch.empty_like(z0)
        self.vb = vb
        self.home = torch.empty(3 * npad(n), dtype=torch.int32, device=dev)
        self.phi = torch.empty(81 * npad(n), dtype=torch.float32, device=dev)
        self.route = torch.zeros(3 * npad(n), dtype=torch.uint8, device=dev) if route else None
        self.fields = fields
        self.forcing = forcing
        self.U = torch.empty((3, n), dtype=torch.float32, device=dev)
        self.F = torch.empty((3, n), dtype=torch.float32, device=dev)
        for t, nm in ((x0, "x0"), (y0, "y0"), (z0, "z0"), (area, "area")):
            _check_dev(t, torch.float32, n, nm)
        for c in range(3):
            _check_dev(fields[c], torch.float32, int(np.prod(ctx.shape(c))), "field %d" % c)
            _check_dev(forcing[c], torch.float32, int(np.prod(ctx.shape(c))), "forcing %d" % c)
        if vb is not None:
            _check_dev(vb, torch.float32, 3 * n, "vb")

    def struct(self):
        b = _StepBuf()
        b.n = self.n
        for k in ("x0", "y0", "z0", "x", "y", "z", "area", "vb", "home", "phi", "route", "U", "F"):
            setattr(b, k, _ptr(getattr(self, k)))
        b.u, b.v, b.w = [t.data_ptr() for t in self.fields]
        b.fx, b.fy, b.fz = [t.data_ptr() for t in self.forcing]
        return b


def _desc(method, dt, jitter, seed, compact=False):
    return _StepDesc(int(method), float(dt), float(jitter), int(seed), MLS_STEP_COMPACT if compact else 0)


def step(ctx: "Context", bufs: StepBuffers, method=MLS_EXACT, dt=1.0, jitter=0.0, seed=0, stream=None,
         compact=False):
    """One time step (mls_step).  compact=True (exact MLS): the transfer
    functions stay in their compact form (MLS_STEP_COMPACT); bufs.phi then
    receives only the rows solved in FP64."""
    d = _desc(method, dt, jitter, seed, compact)
    b = bufs.struct()
    ctx._raise(ctx._lib.mls_step(ctx.h, ctypes.byref(d), ctypes.byref(b), _stream(stream)), "mls_step")


def step_order(ctx: "Context", n: int, stream=None):
    """Row order of the last exact step: row p of its home / phi holds marker order[p]."""
    import torch
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx._raise(ctx._lib.mls_step_order(ctx.h, _ptr(out), int(n), _stream(stream)), "mls_step_order")
    return out


def step_counter_set(ctx: "Context", value: int, stream=None):
    ctx._raise(ctx._lib.mls_step_counter_set(ctx.h, int(value), _stream(stream)), "mls_step_counter_set")


class StepGraph:
    """One step captured as a HIP graph (mls_graph_create) and replayed."""

    def __init__(self, ctx: "Context", bufs: StepBuffers, method=MLS_EXACT, dt=1.0, jitter=0.0, seed=0,
                 compact=False):
        self.ctx = ctx
        self.bufs = bufs      # keeps the baked-in buffers alive
        d = _desc(method, dt, jitter, seed, compact)
        b = bufs.struct()
        h = ctypes.c_void_p()
        ctx._raise(ctx._lib.mls_graph_create(ctx.h, ctypes.byref(d), ctypes.byref(b), ctypes.byref(h)),
                   "mls_graph_create")
        self.h = h

    def launch(self, n_steps=1, stream=None):
        self.ctx._raise(self.ctx._lib.mls_graph_launch(self.h, int(n_steps), _stream(stream)), "mls_graph_launch")

    def close(self):
        if getattr(self, "h", None):
            self.ctx._lib.mls_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(ctx: "Context", on=True):
    ctx._raise(ctx._lib.mls_timing_enable(ctx.h, 1 if on else 0), "mls_timing_enable")


def timing_get(ctx: "Context", reset=True):
    t = _Timing()
    ctx._raise(ctx._lib.mls_timing_get(ctx.h, ctypes.byref(t), 1 if reset else 0), "mls_timing_get")
    return {K_NAMES[i]: (t.ms[i], t.launches[i]) for i in range(len(K_NAMES)) if t.launches[i] > 0}


def version() -> str:
    """mls_version(): library version and the SHA-256 of the sources it was
    compiled from."""
    return load().mls_version().decode()


def npad(n: int) -> int:
    """Marker count rounded up to the 64-marker blocks of the phi/home layout."""
    return (int(n) + 63) // 64 * 64


def unblock(a, n: int, per: int = 1):
    """Blocked layout [npad/64][3][per][64] -> [3, n, per] (numpy or torch)."""
    m = npad(n)
    if hasattr(a, "permute"):
        return a.reshape(m // 64, 3, per, 64).permute(1, 0, 3, 2).reshape(3, m, per)[:, :n]
    return np.asarray(a).reshape(m // 64, 3, per, 64).transpose(1, 0, 3, 2).reshape(3, m, per)[:, :n]


def unpack_phi(phi, n: int):
    """phi (81 * npad) -> [3, n, 27] (component, marker, support node)."""
    return unblock(phi, n, 27)


def unpack_route(route, n: int):
    return unblock(route, n, 1)[:, :, 0]


def unpack_home(home, n: int) -> np.ndarray:
    """Packed home (3 * npad, uint32 bits) -> [3, n, 3] int (component, marker, axis)."""
    h = np.asarray(unblock(np.asarray(home), n, 1)[:, :, 0]).astype(np.int64) & 0xFFFFFFFF
    return np.stack([h & 0x7FF, (h >> 11) & 0x7FF, h >> 22], axis=-1)
