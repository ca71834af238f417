"""Seeded synthetic inputs shaped like the paper's immersed-boundary workloads.

This module only generates inputs (grids, surface markers, velocity fields,
marker forces).  It holds none of the transfer-function arithmetic; both the
HIP library and the CPU oracle receive its arrays.

Shapes follow the paper's workloads: triangulated closed surfaces with one
marker at each triangle centroid (Sec. 3: C = (V1+V2+V3)/3), marker area =
triangle area, Lagrangian edge length l about 0.8 of the Eulerian spacing h
(Sec. 1 and Sec. 3 give 0.7-0.9), O(10^3) markers per body and up to O(10^4)
bodies (Sec. 1), staggered Eulerian grids uniform or stretched in one direction
(Sec. 2).  Icosphere subdivisions 2/3/4 give 320/1280/5120 triangles (the
paper's spheres have 320 faces, Sec. 2; its base meshes have 162/642/2562
vertices, Table 1).  All randomness comes from numpy.random.SeedSequence(20180503).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED = 20180503

# children of the root SeedSequence, one per kind of randomness
_STREAMS = ("geometry", "placement", "rotation", "fields", "forces", "jitter", "training", "misc")


def rng(stream: str, config: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence([SEED, config])
    kids = ss.spawn(len(_STREAMS))
    return np.random.default_rng(kids[_STREAMS.index(stream)])


# ---------------------------------------------------------------------------
# Grids
# ---------------------------------------------------------------------------

def uniform_faces(n: int, length: float = 1.0, origin: float = 0.0) -> np.ndarray:
    """n + 1 equally spaced face coordinates (exact for power-of-two n, length 1)."""
    return origin + length * (np.arange(n + 1, dtype=np.float64) / n)


def tanh_faces(n: int, length: float, beta: float) -> np.ndarray:
    """Wall-clustered faces z_k = L/2 (1 + tanh(beta (2k/n - 1)) / tanh(beta))."""
    k = np.arange(n + 1, dtype=np.float64)
    f = 0.5 * length * (1.0 + np.tanh(beta * (2.0 * k / n - 1.0)) / math.tanh(beta))
    f[0] = 0.0
    f[-1] = length
    return f


@dataclass
class GridSpec:
    faces: List[np.ndarray]
    periodic: List[bool]

    @property
    def n(self):
        return [len(f) - 1 for f in self.faces]

    def dims(self, comp: int):
        return tuple(self.n[d] + (1 if (d == comp and not self.periodic[d]) else 0) for d in range(3))

    def shape(self, comp: int):
        nx, ny, nz = self.dims(comp)
        return (nz, ny, nx)

    def node_coords(self, comp: int, axis: int) -> np.ndarray:
        """Coordinates of the component's nodes along an axis (faces on its own
        axis, cell centres elsewhere), used to sample the input fields."""
        f = self.faces[axis]
        if axis == comp:
            return f[:-1].copy() if self.periodic[axis] else f.copy()
        return 0.5 * (f[:-1] + f[1:])

    @property
    def h_min(self) -> float:
        return min(float(np.min(np.diff(f))) for f in self.faces)

    def uniform_axis(self, axis: int) -> bool:
        """All cell widths along the axis equal (to 1e-9 relative)."""
        w = np.diff(np.asarray(self.faces[axis], dtype=np.float64))
        return bool(w.max() <= w.min() * (1.0 + 1e-9))


# ---------------------------------------------------------------------------
# Surfaces
# ---------------------------------------------------------------------------

def icosphere(subdiv: int):
    """Unit icosphere: icosahedron refined by 1 -> 4 midpoint splits, vertices
    projected to the sphere.  Returns (V [nv,3] float64, F [nf,3] int64)."""
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(subdiv):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                mid[key] = len(V) - 1
            return mid[key]

        F2 = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    return np.array(V), np.array(F, dtype=np.int64)


_ICO_CACHE = {}


def _ico(subdiv):
    if subdiv not in _ICO_CACHE:
        _ICO_CACHE[subdiv] = icosphere(subdiv)
    return _ICO_CACHE[subdiv]


def random_rotations(r: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from uniform unit quaternions."""
    q = r.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def surface_markers(subdiv, centres, axes, rots, chunk=256):
    """Markers of bodies sharing one icosphere template: each body's unit
    icosphere is scaled by its semi-axes, rotated, translated; a marker sits at
    each triangle centroid with the flat triangle's area and outward normal.
    Returns positions [nb*nf, 3] (float64), areas [nb*nf], normals [nb*nf, 3]."""
    V, F = _ico(subdiv)
    nb = len(centres)
    nf = len(F)
    pos = np.empty((nb * nf, 3))
    area = np.empty(nb * nf)
    nrm = np.empty((nb * nf, 3))
    for s in range(0, nb, chunk):
        e = min(nb, s + chunk)
        # scale, rotate, translate: x = R (axes * v) + c
        sv = V[None, :, :] * axes[s:e, None, :]
        Vb = np.einsum("bij,bvj->bvi", rots[s:e], sv) + centres[s:e, None, :]
        A, B, C = Vb[:, F[:, 0]], Vb[:, F[:, 1]], Vb[:, F[:, 2]]
        cen = (A + B + C) / 3.0
        cr = np.cross(B - A, C - A)
        ar = 0.5 * np.linalg.norm(cr, axis=2)
        nr = cr / (2.0 * ar[..., None])
        # orient outward (away from the body centre)
        sgn = np.sign(np.einsum("bfi,bfi->bf", nr, cen - centres[s:e, None, :]))
        nr *= sgn[..., None]
        pos[s * nf:e * nf] = cen.reshape(-1, 3)
        area[s * nf:e * nf] = ar.reshape(-1)
        nrm[s * nf:e * nf] = nr.reshape(-1, 3)
    return pos, area, nrm


def surface_mesh(subdiv, centres, axes, rots):
    """Triangle meshes of bodies sharing one icosphere template (the base
    Lagrangian meshes whose face centroids surface_markers returns): FP32
    vertices [nb*nv, 3] and int32 triangles [nb*nf, 3] indexing them, body
    after body, in the template's face order."""
    V, F = _ico(subdiv)
    nb = len(centres)
    sv = V[None, :, :] * np.asarray(axes)[:, None, :]
    Vb = np.einsum("bij,bvj->bvi", rots, sv) + np.asarray(centres)[:, None, :]
    tri = (F[None, :, :] + (np.arange(nb) * len(V))[:, None, None]).reshape(-1, 3)
    return Vb.reshape(-1, 3).astype(np.float32), tri.astype(np.int32)


def body_mesh(wl):
    """Base meshes of a workload's bodies (stored by the generators that keep
    their geometry): (vertices [nv, 3] FP32, triangles [nt, 3] int32), the
    triangles in the order of the workload's markers."""
    m = wl.meta
    if "centres" not in m:
        raise ValueError("workload %s keeps no body geometry" % wl.name)
    subdiv = np.asarray(m["subdivs"])
    verts, tris, base = [], [], 0
    # bodies are stored one after another; group runs of equal subdivision
    for b0 in range(len(subdiv)):
        v, t = surface_mesh(int(subdiv[b0]), m["centres"][b0:b0 + 1], m["axes"][b0:b0 + 1], m["rots"][b0:b0 + 1])
        verts.append(v)
        tris.append(t + base)
        base += len(v)
    return np.concatenate(verts), np.concatenate(tris)


def place_bodies(r: np.random.Generator, radii, lo, hi, periodic, gap, max_tries=2000000):
    """Random non-overlapping placement: bounding spheres of radius R_i keep a
    periodic distance >= R_i + R_j + gap.  lo/hi bound the centres per axis.
    Candidates are checked against a hash of equal cells no smaller than the
    largest exclusion distance, so only the 27 neighbouring cells matter."""
    radii = np.asarray(radii, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    L = np.asarray(hi, dtype=np.float64) - lo
    box = np.array([1.0 if periodic[d] else 0.0 for d in range(3)])
    need = 2.0 * radii.max() + gap
    nk = np.maximum(1, np.floor(L / need)).astype(int)
    cell = L / nk
    grid = {}
    centres = np.empty((len(radii), 3))
    order = np.argsort(-radii, kind="stable")
    tries = 0
    for i in order:
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("placement failed: domain too crowded")
            c = lo + r.random(3) * L
            key = np.minimum(((c - lo) // cell).astype(int), nk - 1)
            ok = True
            seen = set()
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        kk = key + np.array([dx, dy, dz])
                        kk = tuple(int(kk[d] % nk[d]) if periodic[d] else int(kk[d]) for d in range(3))
                        if kk in seen:
                            continue
                        seen.add(kk)
                        for j in grid.get(kk, ()):
                            dv = centres[j] - c
                            dv -= box * L * np.round(dv / L)
                            if np.linalg.norm(dv) < radii[i] + radii[j] + gap:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                centres[i] = c
                grid.setdefault(tuple(int(k) for k in key), []).append(i)
                break
    return centres


# ---------------------------------------------------------------------------
# Fields
# ---------------------------------------------------------------------------

def fourier_modes(r: np.random.Generator, n_modes: int, kmax: int = 4):
    """n_modes random modes: integer wave vectors in {-kmax..kmax}^3 \\ {0},
    amplitudes N(0,1), phases U[0, 2 pi)."""
    ks = []
    while len(ks) < n_modes:
        k = r.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    a = r.normal(size=n_modes)
    th = r.uniform(0.0, 2.0 * np.pi, size=n_modes)
    return np.array(ks, dtype=np.float64), a, th


def fourier_field(grid: GridSpec, comp: int, modes, lengths, device="cpu", out=None, slab=256):
    """q(x) = sum_m a_m cos(2 pi k_m . x / L + theta_m) sampled in FP64 at the
    component's nodes, stored FP32 [z][y][x].  Uses torch (CPU or GPU) so the
    large grids can be filled on the device in z-slabs."""
    import torch
    ks, a, th = modes
    xs = [torch.as_tensor(grid.node_coords(comp, d), dtype=torch.float64, device=device) for d in range(3)]
    nz, ny, nx = grid.shape(comp)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=device)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        acc = torch.zeros((z1 - z0, ny, nx), dtype=torch.float64, device=device)
        for m in range(len(a)):
            px = 2 * math.pi * ks[m, 0] / lengths[0] * xs[0]
            py = 2 * math.pi * ks[m, 1] / lengths[1] * xs[1]
            pz = 2 * math.pi * ks[m, 2] / lengths[2] * xs[2][z0:z1] + th[m]
            # cos(px + py + pz) expanded so that only plane-sized temporaries appear
            cA = torch.cos(py)[:, None] * torch.cos(px)[None, :] - torch.sin(py)[:, None] * torch.sin(px)[None, :]
            sA = torch.sin(py)[:, None] * torch.cos(px)[None, :] + torch.cos(py)[:, None] * torch.sin(px)[None, :]
            acc += a[m] * (torch.cos(pz)[:, None, None] * cA[None] - torch.sin(pz)[:, None, None] * sA[None])
        out[z0:z1] = acc.to(torch.float32)
    return out


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    grid: GridSpec
    lengths: List[float]
    x: np.ndarray          # FP32 marker positions
    y: np.ndarray
    z: np.ndarray
    area: np.ndarray       # FP32 marker areas A_l
    normal: np.ndarray     # [N,3] FP32 outward normals
    force: np.ndarray      # [3,N] FP32 marker forces F_l = f_l n_l
    body_offsets: np.ndarray  # CSR offsets of bodies into the marker arrays (int64, nb+1)
    modes: tuple           # Fourier modes of the velocity fields (one set per component)
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.x)

    def fields(self, device="cpu"):
        """u, v, w as FP32 torch tensors on `device`."""
        return [fourier_field(self.grid, c, self.modes[c], self.lengths, device=device) for c in range(3)]


def _finish(name, grid, lengths, pos, area, nrm, offsets, cfg_id, n_modes, kmax=4, meta=None):
    rf = rng("forces", cfg_id)
    fmag = rf.normal(size=len(area))
    force = (fmag[:, None] * nrm).T.astype(np.float32)
    rm = rng("fields", cfg_id)
    modes = tuple(fourier_modes(rm, n_modes, kmax) for _ in range(3))
    pos32 = pos.astype(np.float32)
    return Workload(name=name, grid=grid, lengths=list(lengths),
                    x=np.ascontiguousarray(pos32[:, 0]), y=np.ascontiguousarray(pos32[:, 1]),
                    z=np.ascontiguousarray(pos32[:, 2]), area=area.astype(np.float32),
                    normal=nrm.astype(np.float32), force=np.ascontiguousarray(force),
                    body_offsets=np.asarray(offsets, dtype=np.int64), modes=modes, meta=meta or {})


def single_sphere(n: int = 64, subdiv: int = 4, radius: float = 0.1, n_modes: int = 8, cfg_id: int = 1):
    """One icosphere (5120 centroid markers at subdiv 4), radius 0.1, centre
    U[0,1)^3, periodic unit cube with a uniform n^3 staggered grid."""
    g = GridSpec([uniform_faces(n)] * 3, [True] * 3)
    c = rng("placement", cfg_id).random((1, 3))
    axes = np.full((1, 3), radius)
    pos, area, nrm = surface_markers(subdiv, c, axes, np.eye(3)[None])
    return _finish("single_sphere_%d^3_sub%d" % (n, subdiv), g, [1.0] * 3, pos, area, nrm,
                   [0, len(area)], cfg_id, n_modes,
                   meta=dict(centres=c, axes=axes, rots=np.eye(3)[None], subdivs=np.array([subdiv])))


def ellipsoids(n_bodies: int = 1000, n: int = 512, subdiv: int = 3, r0_h: float = 5.31,
               n_modes: int = 16, cfg_id: int = 2):
    """n_bodies ellipsoids (icosphere subdiv 3: 1280 markers each), semi-axes
    r0 U(0.8,1.25)^3 with r0 = 5.31 h (l/h ~ 0.8), random rotations, random
    non-overlapping placement (gap 3h) in a periodic unit cube, uniform n^3."""
    h = 1.0 / n
    g = GridSpec([uniform_faces(n)] * 3, [True] * 3)
    rg = rng("geometry", cfg_id)
    axes = r0_h * h * rg.uniform(0.8, 1.25, size=(n_bodies, 3))
    rots = random_rotations(rng("rotation", cfg_id), n_bodies)
    cen = place_bodies(rng("placement", cfg_id), axes.max(axis=1), np.zeros(3), np.ones(3), [True] * 3, 3 * h)
    pos, area, nrm = surface_markers(subdiv, cen, axes, rots)
    nf = len(_ico(subdiv)[1])
    offs = np.arange(n_bodies + 1) * nf
    return _finish("ellipsoids_%d_%d^3_sub%d" % (n_bodies, n, subdiv), g, [1.0] * 3, pos, area, nrm,
                   offs, cfg_id, n_modes, meta=dict(n_bodies=n_bodies))


def uneven_bodies(n_bodies: int = 10000, n: int = 1024, n_modes: int = 16, cfg_id: int = 3,
                  subdivs=(2, 3, 4), radii_h=(2.72, 5.31, 10.6)):
    """n_bodies bodies with icosphere subdivision drawn uniformly from {2,3,4}
    (320/1280/5120 markers), radius 2.72h/5.31h/10.6h (l/h ~ 0.8), ellipsoidal
    stretch U(0.8,1.25)^3 and random rotation, non-overlapping placement in a
    periodic unit cube with a uniform n^3 grid.  Bodies are stored one after
    another (CSR offsets), in the order of the draw."""
    h = 1.0 / n
    g = GridSpec([uniform_faces(n)] * 3, [True] * 3)
    rg = rng("geometry", cfg_id)
    lvl = rg.integers(0, len(subdivs), size=n_bodies)
    base = np.array(radii_h)[lvl] * h
    axes = base[:, None] * rg.uniform(0.8, 1.25, size=(n_bodies, 3))
    rots = random_rotations(rng("rotation", cfg_id), n_bodies)
    cen = place_bodies(rng("placement", cfg_id), axes.max(axis=1), np.zeros(3), np.ones(3), [True] * 3, 3 * h)
    counts = np.array([len(_ico(subdivs[i])[1]) for i in lvl])
    offs = np.concatenate([[0], np.cumsum(counts)])
    N = int(offs[-1])
    pos = np.empty((N, 3)); area = np.empty(N); nrm = np.empty((N, 3))
    for li, sd in enumerate(subdivs):
        idx = np.nonzero(lvl == li)[0]
        if len(idx) == 0:
            continue
        p, a, nr = surface_markers(sd, cen[idx], axes[idx], rots[idx])
        nf = counts[idx[0]]
        dst = (offs[idx][:, None] + np.arange(nf)[None, :]).reshape(-1)
        pos[dst] = p; area[dst] = a; nrm[dst] = nr
    return _finish("uneven_%d_%d^3" % (n_bodies, n), g, [1.0] * 3, pos, area, nrm, offs, cfg_id, n_modes,
                   meta=dict(n_bodies=n_bodies, levels=lvl, centres=cen, axes=axes, rots=rots,
                             subdivs=np.array(subdivs)[lvl]))


def contact_pairs(n_pairs: int = 5000, n: int = 1024, n_modes: int = 16, cfg_id: int = 6,
                  subdivs=(2, 3, 4), radii_h=(2.72, 5.31, 10.6), gap_h=(-1.5, 0.5)):
    """Bodies in contact, for the collision detection of Sec. 4: n_pairs pairs
    of spheres (subdivision and radius drawn as in uneven_bodies, l/h ~ 0.8)
    whose surfaces are a gap U(gap_h) h apart along a random direction (a
    negative gap overlaps), pairs placed without overlapping each other in a
    periodic unit cube with a uniform n^3 grid.  Bodies 2p and 2p + 1 form
    pair p; markers are stored body after body."""
    h = 1.0 / n
    g = GridSpec([uniform_faces(n)] * 3, [True] * 3)
    rg = rng("geometry", cfg_id)
    nb = 2 * n_pairs
    lvl = rg.integers(0, len(subdivs), size=nb)
    rad = np.array(radii_h)[lvl] * h
    gap = rg.uniform(gap_h[0], gap_h[1], size=n_pairs) * h
    u = rg.normal(size=(n_pairs, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    ra, rb = rad[0::2], rad[1::2]
    bound = np.maximum(2 * ra, 2 * rb) + np.abs(gap)
    mid = place_bodies(rng("placement", cfg_id), bound, np.zeros(3), np.ones(3), [True] * 3, 3 * h)
    cen = np.empty((nb, 3))
    cen[0::2] = mid - u * (ra + 0.5 * gap)[:, None]
    cen[1::2] = mid + u * (rb + 0.5 * gap)[:, None]
    rots = random_rotations(rng("rotation", cfg_id), nb)
    counts = np.array([len(_ico(subdivs[i])[1]) for i in lvl])
    offs = np.concatenate([[0], np.cumsum(counts)])
    N = int(offs[-1])
    pos = np.empty((N, 3)); area = np.empty(N); nrm = np.empty((N, 3))
    for li, sd in enumerate(subdivs):
        idx = np.nonzero(lvl == li)[0]
        if len(idx) == 0:
            continue
        p, a, nr = surface_markers(sd, cen[idx], np.repeat(rad[idx][:, None], 3, axis=1), rots[idx])
        nf = counts[idx[0]]
        dst = (offs[idx][:, None] + np.arange(nf)[None, :]).reshape(-1)
        pos[dst] = p; area[dst] = a; nrm[dst] = nr
    return _finish("contact_%d_pairs_%d^3" % (n_pairs, n), g, [1.0] * 3, pos, area, nrm, offs, cfg_id, n_modes,
                   meta=dict(n_bodies=nb, levels=lvl, gap=gap))


def body_ids(offsets) -> np.ndarray:
    """Body index of every marker from CSR body offsets (int32)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    return np.repeat(np.arange(len(offsets) - 1, dtype=np.int32), np.diff(offsets))


def stretched_channel(n_bodies: int = 2000, nxy: int = 512, nz: int = 768, lz: float = 1.5, beta: float = 2.5,
                      subdiv: int = 3, r_h: float = 5.31, n_modes: int = 16, cfg_id: int = 4):
    """Spheres (subdiv 3) in an nxy x nxy x nz box: x, y periodic uniform on
    [0,1) (h = 1/nxy), z between walls on [0, lz] with tanh clustering
    (stretch factor beta).  Every sphere keeps its markers at least three
    cells away from the walls so that every 3x3x3 support is interior."""
    h = 1.0 / nxy
    fz = tanh_faces(nz, lz, beta)
    g = GridSpec([uniform_faces(nxy), uniform_faces(nxy), fz], [True, True, False])
    r = r_h * h
    zlo, zhi = fz[4] + r, fz[nz - 4] - r
    cen = place_bodies(rng("placement", cfg_id), np.full(n_bodies, r), np.array([0.0, 0.0, zlo]),
                       np.array([1.0, 1.0, zhi]), [True, True, False], 3 * h)
    rots = random_rotations(rng("rotation", cfg_id), n_bodies)
    pos, area, nrm = surface_markers(subdiv, cen, np.full((n_bodies, 3), r), rots)
    nf = len(_ico(subdiv)[1])
    offs = np.arange(n_bodies + 1) * nf
    dz = np.diff(fz)
    geo = dict(centres=cen, axes=np.full((n_bodies, 3), r), rots=rots, subdivs=np.full(n_bodies, subdiv))
    return _finish("stretched_%d_%dx%dx%d_beta%.2f" % (n_bodies, nxy, nxy, nz, beta), g, [1.0, 1.0, lz],
                   pos, area, nrm, offs, cfg_id, n_modes,
                   meta=dict(n_bodies=n_bodies, dz_min=float(dz.min()), dz_max=float(dz.max()),
                             dz_ratio=float(dz.min() / dz.max()), **geo))
