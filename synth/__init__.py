"""Seeded synthetic inputs for the elasticity solve: problem descriptions only.

This module builds the input data of a solve (grid, stiffness field,
eigenstrain, boundary data) for the workloads of the paper's examples and for
tests.  It holds none of the solver's arithmetic: no finite difference, no
operator, no transfer.  Both the CPU oracle and the GPU library consume what it
produces, so it must stay free of either's code.

Layout conventions (shared input format):
  * ``n``: nodes per axis including both ends, ``n[2] == 1`` in 2D.
  * A periodic axis stores ``n - 1`` unique nodes (node ``n-1`` is node 0).
  * Fields are float64 arrays ``[comp][z][y][x]`` over the stored nodes.
  * Isotropic moduli: 2 components (lambda, mu).  Anisotropic moduli: the
    upper triangle, row-major, of the symmetric Voigt matrix (21 in 3D with
    Voigt order 11,22,33,23,31,12; 6 in 2D with order 11,22,12) -- the layout
    of Sec. 4.3 (eq. for the cubic Voigt modulus and the Voigt vectors).
  * Eigenstrain: tensor components (not engineering shears) in Voigt order,
    6 in 3D, 3 in 2D.
  * Face data (face ``2*axis + side``): ``d`` components over the face's
    nodes, shaped like a field with the face's normal axis of extent 1;
    prescribed displacement on Dirichlet faces, prescribed traction on
    traction faces, prescribed normal derivative of the displacement on
    Neumann faces.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

DIRICHLET = "dirichlet"
TRACTION = "traction"
PERIODIC = "periodic"
NEUMANN = "neumann"


@dataclasses.dataclass
class Problem:
    dim: int
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    bc: Tuple[str, str, str, str, str, str]
    kind: str                      # "iso" or "aniso"
    C: np.ndarray                  # [nc][mz][my][mx]
    eps0: Optional[np.ndarray] = None
    b: Optional[np.ndarray] = None
    face: Dict[int, np.ndarray] = dataclasses.field(default_factory=dict)
    name: str = ""

    @property
    def periodic(self) -> Tuple[bool, bool, bool]:
        return tuple(a < self.dim and self.bc[2 * a] == PERIODIC for a in range(3))

    @property
    def m(self) -> Tuple[int, int, int]:
        """Stored (unique) nodes per axis."""
        return tuple((self.n[a] - 1 if self.periodic[a] else self.n[a]) if a < self.dim else 1
                     for a in range(3))

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple((self.hi[a] - self.lo[a]) / (self.n[a] - 1) if a < self.dim else 1.0 for a in range(3))

    @property
    def nodes(self) -> int:
        m = self.m
        return m[0] * m[1] * m[2]

    def coords(self):
        """Node coordinates (x, y, z) broadcastable to [mz][my][mx]."""
        m, h = self.m, self.h
        x = self.lo[0] + h[0] * np.arange(m[0])
        y = self.lo[1] + h[1] * np.arange(m[1])
        z = self.lo[2] + h[2] * np.arange(m[2]) if self.dim == 3 else np.zeros(1)
        return x[None, None, :], y[None, :, None], z[:, None, None]

    def face_shape(self, f: int) -> Tuple[int, int, int]:
        m = list(self.m)[::-1]          # [mz, my, mx]
        m[2 - f // 2] = 1
        return tuple(m)

    def dirichlet_count(self) -> int:
        """Stored nodes on at least one Dirichlet face."""
        m = self.m
        mask = np.zeros(m[::-1], dtype=bool)
        for f in range(2 * self.dim):
            if self.bc[f] != DIRICHLET:
                continue
            a = f // 2
            sl = [slice(None)] * 3
            sl[2 - a] = 0 if f % 2 == 0 else m[a] - 1
            mask[tuple(sl)] = True
        return int(mask.sum())

    def dofs(self) -> int:
        """Unknowns: d x stored nodes not on a Dirichlet face."""
        return self.dim * (self.nodes - self.dirichlet_count())


# --------------------------------------------------------------------------
# stiffness tensors (input construction only)
# --------------------------------------------------------------------------

_V3 = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3, (0, 2): 4, (2, 0): 4, (0, 1): 5, (1, 0): 5}


def cubic_voigt(c11: float, c12: float, c44: float) -> np.ndarray:
    """6x6 Voigt matrix of a cubic crystal in its own frame (Sec. 4.3)."""
    V = np.zeros((6, 6))
    V[:3, :3] = c12
    np.fill_diagonal(V[:3, :3], c11)
    V[3, 3] = V[4, 4] = V[5, 5] = c44
    return V


def voigt_to_tensor(V: np.ndarray) -> np.ndarray:
    T = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    T[i, j, k, l] = V[_V3[i, j], _V3[k, l]]
    return T


def tensor_to_voigt(T: np.ndarray) -> np.ndarray:
    V = np.zeros((6, 6))
    for (i, j), I in _V3.items():
        for (k, l), J in _V3.items():
            V[I, J] = T[i, j, k, l]
    return V


def rotate_voigt(V: np.ndarray, R: np.ndarray) -> np.ndarray:
    """C'_pqst = R_pi R_qj C_ijkl R_sk R_tl (Sec. 4.3, rotated modulus)."""
    T = voigt_to_tensor(V)
    return tensor_to_voigt(np.einsum("pi,qj,sk,tl,ijkl->pqst", R, R, R, R, T, optimize=True))


def upper21(V: np.ndarray) -> np.ndarray:
    n = V.shape[0]
    return np.array([V[I, J] for I in range(n) for J in range(I, n)])


def shoemake_rotation(u: Sequence[float]) -> np.ndarray:
    """Uniform random rotation from three U[0,1) numbers (Shoemake, Graphics Gems III, 1992)."""
    u1, u2, u3 = u
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


CUBIC = (1.68, 1.21, 0.75)   # C11, C12, C44 of the polycrystal example (Sec. 4.3)


def _tanh_step(s):
    return 0.5 * (1.0 - np.tanh(s))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def inclusion_2d(n: int = 65, width: float = 0.02, radius: float = 0.25, eigen: float = 1e-3) -> Problem:
    """2D plane strain, [0,1]^2: isotropic matrix (mu=1, lambda=1.5) with a
    circular inclusion (mu=2, lambda=3) blended by a tanh of the given width,
    isotropic in-plane eigenstrain inside, u=0 on the bottom face, the other
    faces traction-free."""
    p = Problem(dim=2, n=(n, n, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.0),
                bc=(TRACTION, TRACTION, DIRICHLET, TRACTION, TRACTION, TRACTION),
                kind="iso", C=np.zeros(0), name=f"inclusion2d_{n}")
    x, y, _ = p.coords()
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    eta = _tanh_step((r - radius) / width)               # [1][my][mx]
    lam = 1.5 + (3.0 - 1.5) * eta
    mu = 1.0 + (2.0 - 1.0) * eta
    p.C = np.stack([lam, mu]).astype(np.float64)
    p.eps0 = np.stack([eigen * eta, eigen * eta, np.zeros_like(eta)]).astype(np.float64)
    return p


def _voronoi_worker(args):
    """Process-pool entry: one BLAS thread per worker process."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return _voronoi_block(args)


def _voronoi_block(args):
    """Moduli of z-planes [z0, z1) of the Voronoi polycrystal (see
    ``_voronoi_moduli``)."""
    (z0, z1, zs, x, y, m, centers, periodic, Lper, hmin, width_cells, grainC) = args
    out = np.empty((21, z1 - z0, m[1], m[0]))
    chunk = max(1, int(2 ** 22 // (m[0] * m[1] * max(len(centers), 1))))
    for za in range(z0, z1, chunk):
        zb = min(z1, za + chunk)
        z = zs[za:zb][:, None, None]
        pos = [np.broadcast_to(x, (len(z), m[1], m[0])), np.broadcast_to(y, (len(z), m[1], m[0])),
               np.broadcast_to(z, (len(z), m[1], m[0]))]
        # per-seed displacement vectors with the minimum image on periodic axes
        dvec = []
        for a in range(3):
            dv = pos[a][None] - centers[:, a][:, None, None, None]
            if periodic[a]:
                dv = dv - Lper[a] * np.round(dv / Lper[a])
            dvec.append(dv)
        d2 = dvec[0] ** 2 + dvec[1] ** 2 + dvec[2] ** 2                       # [G][...]
        a_idx = np.argmin(d2, axis=0)
        d2a = np.take_along_axis(d2, a_idx[None], 0)[0]
        # image positions of the seeds relative to the node: x - dvec
        sep2 = np.zeros_like(d2)
        for a in range(3):
            pa = np.take_along_axis(dvec[a], a_idx[None], 0)[0]
            sep2 += (dvec[a] - pa[None]) ** 2
        sep = np.sqrt(np.maximum(sep2, 1e-300))
        delta = np.where(sep2 > 0, (d2 - d2a[None]) / (2.0 * sep), 0.0)
        g = _tanh_step(delta / (0.5 * width_cells * hmin))
        g = g / g.sum(axis=0, keepdims=True)
        out[:, za - z0:zb - z0] = np.einsum("g...,gc->c...", g, grainC, optimize=True)
    return out


def _voronoi_moduli(p: Problem, centers: np.ndarray, rots: Sequence[np.ndarray], width_cells: float,
                    base: np.ndarray, scale=None, workers: int = 0) -> np.ndarray:
    """Voronoi polycrystal, per-grain rotated moduli, grain boundaries
    smoothed by tanh of the distance to the bisector plane (transition about
    two cells), mixture rule C = sum g_n C_n / sum g_n (Sec. 4.3).  Large
    grids are split over z-planes across ``workers`` processes (0: up to 16
    for grids above 4 M nodes); every node's value is the same either way."""
    grainC = np.stack([upper21(rotate_voigt(base, R)) for R in rots])      # [G][21]
    m = p.m
    x, y, _ = p.coords()
    hmin = min(p.h[:p.dim])
    Lper = [p.hi[a] - p.lo[a] for a in range(3)]
    zs = p.lo[2] + p.h[2] * np.arange(m[2])
    if workers == 0:
        workers = min(16, os.cpu_count() or 1) if m[0] * m[1] * m[2] > 4_000_000 else 1
    common = (zs, x, y, m, np.asarray(centers), tuple(p.periodic), Lper, hmin, width_cells, grainC)
    if workers <= 1:
        out = _voronoi_block((0, m[2]) + common)
    else:
        import concurrent.futures
        import multiprocessing
        nj = min(m[2], 4 * workers)
        bounds = np.linspace(0, m[2], nj + 1).astype(int)
        jobs = [(int(bounds[i]), int(bounds[i + 1])) + common for i in range(nj) if bounds[i] < bounds[i + 1]]
        out = np.empty((21, m[2], m[1], m[0]))
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("fork")) as ex:
            for (z0, z1, *_), blk in zip(jobs, ex.map(_voronoi_worker, jobs)):
                out[:, z0:z1] = blk
    if scale is not None:
        out = out * scale[None]
    return out


def polycrystal_3d(n: int = 129, grains: int = 16, seed: int = 2002, strain: float = 1e-3,
                   inclusion: Optional[Tuple[float, float]] = None) -> Problem:
    """3D Voronoi polycrystal on [0,1]^3 with cubic grains (C11=1.68,
    C12=1.21, C44=0.75) rotated uniformly at random, periodic x and y faces,
    u = 0 on z = 0 and u = (0, 0, strain) on z = 1.

    ``inclusion=(stiffening, eigenstrain)`` adds a sphere of radius 0.25 at
    the centre: C = (1 + (stiffening-1) eta) C_poly and isotropic eigenstrain
    ``eigenstrain * eta`` with eta a tanh step of width 2 cells."""
    rng = np.random.default_rng(seed)
    centers = rng.random((grains, 3))
    rots = [shoemake_rotation(rng.random(3)) for _ in range(grains)]
    p = Problem(dim=3, n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC, DIRICHLET, DIRICHLET),
                kind="aniso", C=np.zeros(0), name=f"polycrystal_{n}_{grains}g")
    scale = None
    eta = None
    if inclusion is not None:
        x, y, z = p.coords()
        r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2)
        eta = _tanh_step((r - 0.25) / (2.0 * p.h[0]))
        scale = 1.0 + (inclusion[0] - 1.0) * eta
        p.name += "_sphere"
    p.C = _voronoi_moduli(p, centers, rots, 2.0, cubic_voigt(*CUBIC), scale)
    if eta is not None:
        e = inclusion[1] * eta
        z0 = np.zeros_like(e)
        p.eps0 = np.stack([e, e, e, z0, z0, z0])
    top = np.zeros((3,) + p.face_shape(5))
    top[2] = strain
    p.face[5] = top
    return p


def iso_from_lame(lam: np.ndarray, mu: np.ndarray) -> np.ndarray:
    return np.stack([lam, mu]).astype(np.float64)


def random_problem(dim: int, n: Sequence[int], bc: Sequence[str], kind: str, seed: int,
                   with_eps0: bool = True, with_body: bool = False, with_face_data: bool = True,
                   smooth: bool = True, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> Problem:
    """Random but well-posed test problem: smooth positive-definite moduli
    (rotated cubic plus isotropic background, modulated by low-order
    trigonometric fields, or independent per node when ``smooth`` is false),
    random smooth eigenstrain, body force and face data."""
    rng = np.random.default_rng(seed)
    n3 = tuple(n) + (1,) * (3 - len(n))
    hi3 = tuple(hi[a] if a < dim else lo[a] for a in range(3))
    p = Problem(dim=dim, n=n3, lo=tuple(lo), hi=hi3, bc=tuple(bc), kind=kind, C=np.zeros(0),
                name=f"random{dim}d_{kind}_{seed}")
    x, y, z = p.coords()
    m = p.m
    shape = (m[2], m[1], m[0])

    def field(amp):
        if not smooth:
            return amp * rng.uniform(-1, 1, size=shape)
        k = rng.uniform(0.5, 2.5, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        f = np.sin(2 * np.pi * k[0] * x + ph[0]) * np.cos(2 * np.pi * k[1] * y + ph[1])
        if dim == 3:
            f = f * np.cos(2 * np.pi * k[2] * z + ph[2])
        return amp * np.broadcast_to(f, shape)

    if kind == "iso":
        mu = 1.0 + 0.5 * (1 + field(1.0))
        lam = 1.5 + 0.7 * field(1.0)
        p.C = iso_from_lame(lam, mu)
    else:
        R = shoemake_rotation(rng.random(3))
        if dim == 3:
            V = rotate_voigt(cubic_voigt(*CUBIC), R)
            comps = upper21(V)
        else:
            c = rng.uniform(-0.2, 0.2)
            V2 = np.array([[1.8, 1.1, c], [1.1, 1.6, -0.5 * c], [c, -0.5 * c, 0.7]])
            comps = np.array([V2[I, J] for I in range(3) for J in range(I, 3)])
        s = 1.0 + 0.4 * field(1.0)               # positive scale keeps it SPD
        p.C = np.stack([comps[c] * s for c in range(len(comps))]).astype(np.float64)
        # add a small SPD isotropic part with its own variation
        lam_mu = (0.2 + 0.1 * field(1.0), 0.3 + 0.1 * field(1.0))
        if dim == 3:
            iso = [(0, lam_mu[0] + 2 * lam_mu[1]), (1, lam_mu[0]), (2, lam_mu[0]), (6, lam_mu[0] + 2 * lam_mu[1]),
                   (7, lam_mu[0]), (11, lam_mu[0] + 2 * lam_mu[1]), (15, lam_mu[1]), (18, lam_mu[1]), (20, lam_mu[1])]
        else:
            iso = [(0, lam_mu[0] + 2 * lam_mu[1]), (1, lam_mu[0]), (3, lam_mu[0] + 2 * lam_mu[1]), (5, lam_mu[1])]
        for c, v in iso:
            p.C[c] = p.C[c] + v
    ne = 6 if dim == 3 else 3
    if with_eps0:
        p.eps0 = np.stack([field(1e-3) for _ in range(ne)]).astype(np.float64)
    if with_body:
        p.b = np.stack([field(1e-2) for _ in range(dim)]).astype(np.float64)
    if with_face_data:
        for f in range(2 * dim):
            if bc[f] == PERIODIC:
                continue
            shp = (dim,) + p.face_shape(f)
            p.face[f] = (1e-3 * rng.uniform(-1, 1, size=shp)).astype(np.float64)
    return p


def plane_strain_voigt(V6: np.ndarray) -> np.ndarray:
    """3x3 Voigt matrix (order 11, 22, 12) of the in-plane restriction of a 3D
    stiffness given as its 6x6 Voigt matrix."""
    sel = [0, 1, 5]
    return V6[np.ix_(sel, sel)]


def upper_tri(V: np.ndarray) -> np.ndarray:
    """Row-major upper triangle of a symmetric matrix (the stored moduli layout)."""
    return upper21(V)


# --------------------------------------------------------------------------
# block-structured AMR inputs: a base problem plus nested boxes
# --------------------------------------------------------------------------

@dataclasses.dataclass
class AmrProblem:
    """Base grid plus refined levels (ratio 2).  Level k >= 1 is a list of
    boxes of nodes [lo, hi] (inclusive, even) of level k's index space
    (``boxlists[k-1]``; one box if ``boxlists`` is None); ``boxes[k-1]`` is
    the bounding box of that list, and the level's fields are sampled on the
    bounding box grown by one node per side."""
    base: Problem
    boxes: list
    C: list
    eps0: list
    b: list
    name: str = ""
    boxlists: Optional[list] = None

    def level_boxes(self, k):
        """The boxes of refined level k (k >= 1)."""
        if self.boxlists is None:
            return [self.boxes[k - 1]]
        return list(self.boxlists[k - 1])

    def valid_mask(self, k):
        """Valid nodes of level k over its ghosted bounding box, [z][y][x]."""
        lo, hi = self.boxes[k - 1]
        d = self.base.dim
        shp = [hi[a] - lo[a] + 3 if a < d else 1 for a in range(3)]
        m = np.zeros((shp[2], shp[1], shp[0]), dtype=bool)
        for bl, bh in self.level_boxes(k):
            m[tuple(slice(bl[a] - lo[a] + 1, bh[a] - lo[a] + 2) if a < d else slice(None) for a in (2, 1, 0))] = True
        return m

    def level_h(self, k):
        return tuple(self.base.h[a] / 2 ** k if a < self.base.dim else 1.0 for a in range(3))

    def box_coords(self, k):
        lo, hi = self.boxes[k - 1]
        h = self.level_h(k)
        out = []
        for a in range(3):
            if a < self.base.dim:
                out.append(self.base.lo[a] + h[a] * np.arange(lo[a] - 1, hi[a] + 2))
            else:
                out.append(np.zeros(1))
        return out[0][None, None, :], out[1][None, :, None], out[2][:, None, None]

    def composite_nodes(self):
        """Valid nodes of every level minus the coarse nodes they cover."""
        n = self.base.nodes
        d = self.base.dim
        for k in range(1, len(self.boxes) + 1):
            m = self.valid_mask(k)
            lo = self.boxes[k - 1][0]
            even = m.copy()
            for a in range(d):
                ax = 2 - a
                idx = np.arange(m.shape[ax])
                shp = [1, 1, 1]
                shp[ax] = -1
                even &= ((lo[a] - 1 + idx) % 2 == 0).reshape(shp)
            n += int(m.sum()) - int(even.sum())
        return n


def _even_floor(v):
    return int(np.floor(v / 2.0)) * 2


def _even_ceil(v):
    return int(np.ceil(v / 2.0)) * 2


def blocks_from_tags(tagged: np.ndarray, origin, dim: int, parent_valid, parent_origin, domain_m=None,
                     block: int = 16, max_cells: int = 32, buffer: int = 2):
    """Boxes of the next finer level covering tagged coarse nodes, the way a
    block-structured hierarchy is built (Sec. 1): tags grown by `buffer`
    coarse cells, mapped to fine nodes, covered by blocks of `block` cells
    on a lattice of `block` cells, merged 2^dim at a time into blocks of
    `max_cells` (= 2 block) where all of them are selected.  A block is kept
    only if, grown by two coarse cells, it consists of valid coarse nodes
    (proper nesting); for the base grid (parent_valid None) it must lie two
    coarse cells inside the domain of `domain_m` nodes per axis.

    tagged: bool array [z][y][x] over coarse array indices, origin = coarse
    index of array index 0; parent_valid: bool array of the coarse level's
    valid nodes (same layout, parent_origin) or None.
    Returns (lo, hi) boxes of fine node indices, 2D boxes with lo[2] = hi[2] = 0."""
    idx = np.argwhere(tagged)                      # (z, y, x) rows
    origin = tuple(int(v) for v in origin)
    parent_origin = tuple(int(v) for v in parent_origin)
    if idx.size == 0:
        return []
    sel = set()
    r = range(-buffer, buffer + 1)
    for z, y, x in idx:
        J = (x + origin[0], y + origin[1], z + origin[2])
        for dz in (r if dim == 3 else (0,)):
            for dy in r:
                for dx in r:
                    q = (2 * (J[0] + dx), 2 * (J[1] + dy), 2 * (J[2] + dz) if dim == 3 else 0)
                    sel.add(tuple(q[a] // block if a < dim else 0 for a in range(3)))
    def nested(lo, hi):
        c0 = [lo[a] // 2 - 2 for a in range(dim)]
        c1 = [hi[a] // 2 + 2 for a in range(dim)]
        if parent_valid is None:
            return all(c0[a] >= 0 and c1[a] <= domain_m[a] - 1 for a in range(dim))
        sl = []
        for a in (2, 1, 0):
            if a >= dim:
                sl.append(slice(None))
                continue
            i0, i1 = c0[a] - parent_origin[a], c1[a] - parent_origin[a]
            if i0 < 0 or i1 >= parent_valid.shape[2 - a]:
                return False
            sl.append(slice(i0, i1 + 1))
        return bool(parent_valid[tuple(sl)].all())

    def box_of(b, size):
        return (tuple(int(b[a] * size) if a < dim else 0 for a in range(3)),
                tuple(int((b[a] + 1) * size) if a < dim else 0 for a in range(3)))

    ratio = max_cells // block
    boxes = []
    merged = set()
    for bk in sorted(sel):
        sup = tuple(bk[a] // ratio if a < dim else 0 for a in range(3))
        if sup in merged:
            continue
        subs = [tuple(sup[a] * ratio + ((o // ratio ** a) % ratio) if a < dim else 0 for a in range(3))
                for o in range(ratio ** dim)]
        if all(sb in sel for sb in subs) and nested(*box_of(sup, max_cells)):
            merged.add(sup)
            boxes.append(box_of(sup, max_cells))
    for bk in sorted(sel):
        sup = tuple(bk[a] // ratio if a < dim else 0 for a in range(3))
        if sup not in merged and nested(*box_of(bk, block)):
            boxes.append(box_of(bk, block))
    return boxes


def _bbox(boxes, dim):
    lo = tuple(min(b[0][a] for b in boxes) if a < dim else 0 for a in range(3))
    hi = tuple(max(b[1][a] for b in boxes) if a < dim else 0 for a in range(3))
    return lo, hi


def penny_crack(n: int = 65, levels: int = 3, radius: float = 0.2, width: float = 0.01, floor: float = 1e-4,
                opening: float = 1e-3, tag: float = 0.1, blocks: bool = True, block: int = 16,
                max_cells: int = 32) -> AmrProblem:
    """Diffuse penny crack in an isotropic matrix (mu=1, lambda=1.5) on
    [0,1]^3: moduli scaled by 1 - (1 - floor) eta, eta = sech^2(d / width),
    d the distance to the disc (centre (0.5,0.5,0.5), normal z); opening
    displacement +-opening/2 in z on the z faces, x/y faces traction-free.
    Level k >= 1 refines the level-(k-1) nodes where |grad eta| h > tag
    (Sec. 4.2 tagging on the gradient of the crack field).  blocks=True: the
    tags (grown by two coarse cells) are covered by blocks of `block` cells
    on a `block`-cell lattice, merged into `max_cells` blocks where possible
    (blocks_from_tags); blocks=False: one box, the tags' bounding box grown by
    two coarse cells, clipped to nest in level k-1."""
    def eta_of(x, y, z):
        rho = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
        d = np.sqrt(np.maximum(rho - radius, 0.0) ** 2 + (z - 0.5) ** 2)
        return 1.0 / np.cosh(d / width) ** 2

    def grad_eta(x, y, z, h):
        g = 0.0
        for a, (dx, dy, dz) in enumerate(((h, 0, 0), (0, h, 0), (0, 0, h))):
            g = g + ((eta_of(x + dx, y + dy, z + dz) - eta_of(x - dx, y - dy, z - dz)) / (2 * h)) ** 2
        return np.sqrt(g)

    base = Problem(dim=3, n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                   bc=(TRACTION, TRACTION, TRACTION, TRACTION, DIRICHLET, DIRICHLET), kind="iso", C=np.zeros(0),
                   name=f"penny_{n}_{levels}L" + ("_blocks" if blocks else ""))

    def moduli(x, y, z):
        s = 1.0 - (1.0 - floor) * eta_of(x, y, z)
        s = np.broadcast_to(s, np.broadcast(x, y, z).shape)
        return np.stack([1.5 * s, 1.0 * s])

    x, y, z = base.coords()
    base.C = moduli(x, y, z)
    for f, v in ((4, -0.5 * opening), (5, 0.5 * opening)):
        a = np.zeros((3,) + base.face_shape(f))
        a[2] = v
        base.face[f] = a
    amr = AmrProblem(base=base, boxes=[], C=[], eps0=[], b=[], name=base.name, boxlists=[] if blocks else None)
    prev = (tuple([0, 0, 0]), tuple(m - 1 for m in base.m))
    for k in range(1, levels):
        h_prev = amr.level_h(k - 1)[0]
        if k == 1:
            origin = (0, 0, 0)
            idx = [np.arange(0, base.m[a]) for a in range(3)]
            pvalid = None
        else:
            plo, phi = amr.boxes[k - 2]
            origin = tuple(plo[a] - 1 for a in range(3))
            idx = [np.arange(plo[a] - 1, phi[a] + 2) for a in range(3)]
            pvalid = amr.valid_mask(k - 1)
        X = base.lo[0] + h_prev * idx[0][None, None, :]
        Y = base.lo[1] + h_prev * idx[1][None, :, None]
        Z = base.lo[2] + h_prev * idx[2][:, None, None]
        tagged = grad_eta(X, Y, Z, h_prev) * h_prev > tag
        if pvalid is not None:
            tagged &= pvalid
        if not tagged.any():
            break
        if blocks:
            bl = blocks_from_tags(tagged, origin, 3, pvalid, origin, base.m, block, max_cells)
            if not bl:
                break
            amr.boxlists.append(bl)
            amr.boxes.append(_bbox(bl, 3))
        else:
            zz, yy, xx = np.nonzero(tagged)
            t_lo = [idx[0][xx.min()], idx[1][yy.min()], idx[2][zz.min()]]
            t_hi = [idx[0][xx.max()], idx[1][yy.max()], idx[2][zz.max()]]
            lo_p, hi_p = prev
            lo, hi = [], []
            for a in range(3):
                # tagged bounding box grown by two coarse cells, refined
                l_f = _even_floor(2 * (t_lo[a] - 2))
                h_f = _even_ceil(2 * (t_hi[a] + 2))
                l_f = max(l_f, 2 * (lo_p[a] + 2))
                h_f = min(h_f, 2 * (hi_p[a] - 2))
                lo.append(l_f)
                hi.append(h_f)
            amr.boxes.append((tuple(lo), tuple(hi)))
            prev = (tuple(lo), tuple(hi))
        Xf, Yf, Zf = amr.box_coords(k)
        amr.C.append(np.ascontiguousarray(moduli(Xf, Yf, Zf)))
        amr.eps0.append(None)
        amr.b.append(None)
    return amr


# L-shaped refined levels of smooth_amr(..., shape="L") for a 17-node base:
# level 1 is two boxes meeting along y = 14, level 2 two boxes meeting along
# y = 24 (each box grown by two coarse cells lies in the level above).
L_SHAPE_BOXES = {
    1: [((6, 6, 6), (26, 14, 26)), ((6, 14, 6), (14, 26, 26))],
    2: [((16, 16, 16), (48, 24, 48)), ((16, 24, 16), (24, 48, 48))],
}


def smooth_amr(dim: int = 2, levels: int = 2, n: int = 17, seed: int = 2, kind: str = "iso",
               shape: str = "box") -> AmrProblem:
    """Small composite test problem: smooth moduli (analytic, sampled on
    every level), body force, mixed Dirichlet/traction faces, and centred
    nested boxes (each half the previous box's width).  kind "iso": (lambda,
    mu) fields; kind "aniso": the Voigt matrix of those fields plus a smoothly
    varying multiple of a fixed rotated cubic crystal (SPD everywhere),
    stored as the 21 (3D) or 6 (2D, plane strain) upper-triangle constants."""
    rng = np.random.default_rng(seed)
    k = rng.uniform(1.0, 3.0, size=4)
    R = shoemake_rotation(rng.random(3))
    cub = rotate_voigt(cubic_voigt(1.68, 1.21, 0.75), R)
    liso = np.zeros((6, 6))
    liso[:3, :3] = 1.0
    miso = np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])
    if dim == 2:
        liso, miso, cub = plane_strain_voigt(liso), plane_strain_voigt(miso), plane_strain_voigt(cub)
    lu, mu_, cu = upper_tri(liso), upper_tri(miso), upper_tri(cub)

    def fields(x, y, z):
        lam = 1.5 + 0.8 * np.sin(k[0] * x + 0.3) * np.cos(k[1] * y) * np.cos(k[2] * z)
        mu = 1.0 + 0.5 * np.cos(k[3] * x + y - 0.5 * z)
        if kind == "iso":
            return np.stack([lam + 0 * x * y * z, mu + 0 * x * y * z])
        s = 0.3 * (1.0 + 0.4 * np.sin(k[1] * x - k[2] * y + 0.7 * z))
        return np.stack([lu[c] * lam + mu_[c] * mu + cu[c] * s + 0 * x * y * z for c in range(len(lu))])

    def body(x, y, z):
        g = np.exp(-((x - 0.45) ** 2 + (y - 0.55) ** 2 + (z - 0.5) ** 2) / 0.05)
        return np.stack([1e-2 * g, -2e-2 * g, 1.5e-2 * g][:dim])

    n3 = (n,) * dim + (1,) * (3 - dim)
    hi = (1.0,) * dim + (0.0,) * (3 - dim)
    bc = ("dirichlet", "traction", "traction", "traction", "dirichlet", "traction") if dim == 3 else \
        ("dirichlet", "traction", "dirichlet", "traction", PERIODIC, PERIODIC)
    base = Problem(dim=dim, n=n3, lo=(0.0, 0.0, 0.0), hi=hi, bc=bc, kind=kind, C=np.zeros(0),
                   name=f"smooth_amr_{dim}d_{levels}L_{kind}")
    x, y, z = base.coords()
    shp = (base.m[2], base.m[1], base.m[0])
    nc = 2 if kind == "iso" else len(lu)
    base.C = np.ascontiguousarray(np.broadcast_to(fields(x, y, z), (nc,) + shp))
    base.b = np.ascontiguousarray(np.broadcast_to(body(x, y, z), (dim,) + shp))
    amr = AmrProblem(base=base, boxes=[], C=[], eps0=[], b=[], name=base.name,
                     boxlists=[] if shape == "L" else None)
    if shape == "L":
        assert n == 17 and levels <= 3
        amr.name += "_L"
    lo_p, hi_p = [0] * 3, [m - 1 for m in base.m]
    for lev in range(1, levels):
        if shape == "L":
            bl = [(tuple(lo[a] if a < dim else 0 for a in range(3)), tuple(hi[a] if a < dim else 0 for a in range(3)))
                  for lo, hi in L_SHAPE_BOXES[lev]]
            amr.boxlists.append(bl)
            amr.boxes.append(_bbox(bl, dim))
            X, Y, Z = amr.box_coords(lev)
            mshape = tuple(len(v.ravel()) for v in (Z, Y, X))
            amr.C.append(np.ascontiguousarray(np.broadcast_to(fields(X, Y, Z), (nc,) + mshape)))
            amr.eps0.append(None)
            amr.b.append(np.ascontiguousarray(np.broadcast_to(body(X, Y, Z), (dim,) + mshape)))
            continue
        lo, hi = [0, 0, 0], [0, 0, 0]
        for a in range(dim):
            span = hi_p[a] - lo_p[a]
            c0 = lo_p[a] + span // 4
            c1 = hi_p[a] - span // 4
            lo[a] = 2 * max(c0, lo_p[a] + 2)
            hi[a] = 2 * min(c1, hi_p[a] - 2)
        amr.boxes.append((tuple(lo), tuple(hi)))
        X, Y, Z = amr.box_coords(lev)
        mshape = tuple(len(v.ravel()) for v in (Z, Y, X))
        amr.C.append(np.ascontiguousarray(np.broadcast_to(fields(X, Y, Z), (nc,) + mshape)))
        amr.eps0.append(None)
        amr.b.append(np.ascontiguousarray(np.broadcast_to(body(X, Y, Z), (dim,) + mshape)))
        lo_p, hi_p = lo, hi
    return amr


def _disc_fields(radius, width, eigen, center=(0.5, 0.5)):
    """Moduli (lambda, mu) and eigenstrain of the plane-strain inclusion disc:
    matrix mu=1, lambda=1.5, inclusion mu=2, lambda=3, blended by a tanh
    profile of the given width, isotropic eigenstrain `eigen` inside."""
    def fields(x, y, z):
        r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2) + 0 * z
        eta = _tanh_step((r - radius) / width)
        C = np.stack([1.5 + 1.5 * eta, 1.0 + 1.0 * eta])
        e = eigen * eta
        return C, np.stack([e, e, np.zeros_like(e)])
    return fields


def eshelby_amr_2d(n0: int = 129, levels: int = 3, radius: float = 0.1, width_cells: float = 2.0,
                   eigen: float = 1e-3) -> AmrProblem:
    """AMR-efficiency input (the paper's 2D Eshelby example, Sec. 4.1 / the
    AMR performance study of Sec. 5): the inclusion_2d disc moduli (radius `radius`,
    centre (0.5, 0.5)) on [0,1]^2 with a base grid of n0 nodes per axis and
    levels - 1 refined boxes around the disc (one per level, ratio 2).  The
    tanh width is width_cells cells of the finest level, so the finest level
    resolves the interface; box k spans the disc plus a margin of two widths
    and 4 cells of level k, which nests it in box k-1 with 2 coarse cells to
    spare.  y = 0 clamped, other faces traction-free."""
    h0 = 1.0 / (n0 - 1)
    hf = h0 / 2 ** (levels - 1)
    fields = _disc_fields(radius, width_cells * hf, eigen)
    base = Problem(dim=2, n=(n0, n0, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.0),
                   bc=(TRACTION, TRACTION, DIRICHLET, TRACTION, PERIODIC, PERIODIC), kind="iso", C=np.zeros(0),
                   name=f"eshelby_amr_2d_{n0}_{levels}L")
    x, y, z = base.coords()
    shp = (base.m[2], base.m[1], base.m[0])
    C, e = fields(x, y, z)
    base.C = np.ascontiguousarray(np.broadcast_to(C, (2,) + shp)).astype(np.float64)
    base.eps0 = np.ascontiguousarray(np.broadcast_to(e, (3,) + shp)).astype(np.float64)
    amr = AmrProblem(base=base, boxes=[], C=[], eps0=[], b=[], name=base.name)
    for k in range(1, levels):
        hk = h0 / 2 ** k
        margin = 2.0 * width_cells * hf + 4.0 * hk
        lo = _even_floor((0.5 - radius - margin) / hk)
        hi = _even_ceil((0.5 + radius + margin) / hk)
        amr.boxes.append(((lo, lo, 0), (hi, hi, 0)))
        X, Y, Z = amr.box_coords(k)
        mshape = (1, Y.size, X.size)
        Ck, ek = fields(X, Y, Z)
        amr.C.append(np.ascontiguousarray(np.broadcast_to(Ck, (2,) + mshape)).astype(np.float64))
        amr.eps0.append(np.ascontiguousarray(np.broadcast_to(ek, (3,) + mshape)).astype(np.float64))
        amr.b.append(None)
    return amr


class Microstructure2D:
    """2D polycrystal of the AMR performance study (Sec. 5.1 "AMR
    performance", phase-field microstructure case): `grains` Voronoi grains
    in [0,1]^2 (seeds U[0,1]^2 from default_rng(seed)), each a cubic crystal
    (C11=1.68, C12=1.21, C44=0.75) rotated about z by a uniform angle, plane
    strain.  Order parameters eta_n = g_n / sum g, g_n = tanh step of the
    distance to the bisector between the node's nearest seed and seed n,
    diffuse over `width` (physical); moduli C = sum eta_n C_n (mixture rule,
    Sec. 4.3).  Evaluated at any points."""

    def __init__(self, grains: int = 10, seed: int = 2010, width: float = 0.01):
        rng = np.random.default_rng(seed)
        self.centers = rng.random((grains, 2))
        th = 2.0 * np.pi * rng.random(grains)
        cub = cubic_voigt(*CUBIC)
        Cs = []
        for t in th:
            R = np.array([[np.cos(t), -np.sin(t), 0.0], [np.sin(t), np.cos(t), 0.0], [0.0, 0.0, 1.0]])
            Cs.append(upper_tri(plane_strain_voigt(rotate_voigt(cub, R))))
        self.grainC = np.stack(Cs)          # [G][6]
        self.width = width

    def eta(self, x, y):
        """Order parameters [G][...] at points (x, y) (broadcast arrays)."""
        x, y = np.broadcast_arrays(x, y)
        cx = self.centers[:, 0].reshape((-1,) + (1,) * x.ndim)
        cy = self.centers[:, 1].reshape((-1,) + (1,) * x.ndim)
        dx, dy = x[None] - cx, y[None] - cy
        d2 = dx * dx + dy * dy
        a = np.argmin(d2, axis=0)
        d2a = np.take_along_axis(d2, a[None], 0)[0]
        pax, pay = self.centers[a, 0], self.centers[a, 1]
        sep = np.sqrt((cx - pax[None]) ** 2 + (cy - pay[None]) ** 2)
        delta = np.where(sep > 0, (d2 - d2a[None]) / (2.0 * np.maximum(sep, 1e-300)), -np.inf)
        g = _tanh_step(delta / (0.5 * self.width))
        return g / g.sum(axis=0, keepdims=True)

    def moduli(self, x, y):
        e = self.eta(x, y)
        return np.einsum("g...,gc->c...", e, self.grainC)

    def tags(self, x, y, h, tag=0.1):
        """|grad eta_n| h > tag for some n (central differences of width h)."""
        gx = (self.eta(x + h, y) - self.eta(x - h, y)) / (2 * h)
        gy = (self.eta(x, y + h) - self.eta(x, y - h)) / (2 * h)
        return (np.sqrt(gx * gx + gy * gy) * h > tag).any(axis=0)


def _microstructure_base(n0, ms, shear, name):
    base = Problem(dim=2, n=(n0, n0, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.0),
                   bc=(TRACTION, TRACTION, DIRICHLET, DIRICHLET, PERIODIC, PERIODIC), kind="aniso", C=np.zeros(0),
                   name=name)
    x, y, _ = base.coords()
    base.C = np.ascontiguousarray(ms.moduli(np.broadcast_to(x, (1, n0, n0)), np.broadcast_to(y, (1, n0, n0))))
    top = np.zeros((2,) + base.face_shape(3))
    top[0] = shear
    base.face[3] = top
    return base


def microstructure_amr_2d(n_finest: int = 513, levels: int = 3, grains: int = 10, seed: int = 2010,
                          width_cells: float = 4.0, shear: float = 1e-3, tag: float = 0.1) -> AmrProblem:
    """The AMR performance study's microstructure case at a fixed finest
    resolution: base grid of (n_finest - 1) / 2^(levels-1) + 1 nodes per axis,
    levels - 1 refined levels of 16/32-cell blocks covering the nodes where
    some |grad eta_n| |dx| > tag (Sec. 4.3 tagging criterion), grown by two
    cells and properly nested.  Diffuse width `width_cells` finest cells.
    Bottom clamped, top sheared by `shear` in x, sides traction-free."""
    nf = n_finest - 1
    n0 = nf // 2 ** (levels - 1) + 1
    assert (n0 - 1) * 2 ** (levels - 1) == nf
    ms = Microstructure2D(grains, seed, width_cells / nf)
    base = _microstructure_base(n0, ms, shear, f"microstructure_amr_{n_finest}_{levels}L")
    amr = AmrProblem(base=base, boxes=[], C=[], eps0=[], b=[], name=base.name, boxlists=[])
    for k in range(1, levels):
        h_prev = amr.level_h(k - 1)[0]
        if k == 1:
            origin = (0, 0, 0)
            idx = [np.arange(0, base.m[a]) for a in range(2)]
            pvalid = None
        else:
            plo, phi = amr.boxes[k - 2]
            origin = (plo[0] - 1, plo[1] - 1, 0)
            idx = [np.arange(plo[a] - 1, phi[a] + 2) for a in range(2)]
            pvalid = amr.valid_mask(k - 1)
        X = (h_prev * idx[0])[None, None, :]
        Y = (h_prev * idx[1])[None, :, None]
        tagged = ms.tags(X, Y, h_prev, tag)
        if pvalid is not None:
            tagged &= pvalid
        bl = blocks_from_tags(tagged, origin, 2, pvalid, origin, base.m) if tagged.any() else []
        if not bl:
            break
        amr.boxlists.append(bl)
        amr.boxes.append(_bbox(bl, 2))
        Xk, Yk, _ = amr.box_coords(k)
        shp = (1, Yk.size, Xk.size)
        amr.C.append(np.ascontiguousarray(ms.moduli(np.broadcast_to(Xk, shp), np.broadcast_to(Yk, shp))))
        amr.eps0.append(None)
        amr.b.append(None)
    return amr


def microstructure_uniform_2d(n_finest: int = 513, grains: int = 10, seed: int = 2010, width_cells: float = 4.0,
                              shear: float = 1e-3) -> Problem:
    """The same microstructure on one uniform grid of n_finest nodes per axis."""
    ms = Microstructure2D(grains, seed, width_cells / (n_finest - 1))
    return _microstructure_base(n_finest, ms, shear, f"microstructure_uniform_{n_finest}")


def eshelby_uniform_2d(n0: int = 129, levels: int = 3, **kw) -> Problem:
    """The same disc on one uniform grid at the finest resolution of
    eshelby_amr_2d(n0, levels): (n0 - 1) 2^(levels - 1) + 1 nodes per axis."""
    amr = eshelby_amr_2d(n0, 1, **kw) if levels == 1 else None
    radius = kw.get("radius", 0.1)
    width_cells = kw.get("width_cells", 2.0)
    eigen = kw.get("eigen", 1e-3)
    n = (n0 - 1) * 2 ** (levels - 1) + 1
    hf = 1.0 / (n - 1)
    fields = _disc_fields(radius, width_cells * hf, eigen)
    p = Problem(dim=2, n=(n, n, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.0),
                bc=(TRACTION, TRACTION, DIRICHLET, TRACTION, PERIODIC, PERIODIC), kind="iso", C=np.zeros(0),
                name=f"eshelby_uniform_2d_{n}")
    x, y, z = p.coords()
    shp = (p.m[2], p.m[1], p.m[0])
    C, e = fields(x, y, z)
    p.C = np.ascontiguousarray(np.broadcast_to(C, (2,) + shp)).astype(np.float64)
    p.eps0 = np.ascontiguousarray(np.broadcast_to(e, (3,) + shp)).astype(np.float64)
    del amr
    return p


def ellipsoid_eta(x, y, z, axes, width):
    """Diffuse indicator of the ellipsoid x^T A x <= 1, A = diag(a_i^-2), for
    the Eshelby example of Sec. 4.1 (its error-function mollification):
    eta = (1 - erf((x^T A x - 1) / (2 width |A x|))) / 2, 1 inside and 0
    outside.  Readings: A holds the inverse squared semi-axes and the
    argument carries the "- 1" that puts the transition on the surface;
    eta = 1 marks the eigenstrained interior."""
    from scipy.special import erf
    a = [float(v) for v in axes]
    q = (x / a[0]) ** 2 + (y / a[1]) ** 2 + (z / a[2]) ** 2
    g = np.sqrt((x / a[0] ** 2) ** 2 + (y / a[1] ** 2) ** 2 + (z / a[2] ** 2) ** 2)
    g = np.maximum(g, 1e-300)
    return 0.5 * (1.0 - erf((q - 1.0) / (2.0 * width * g)))


def eshelby_ellipsoid_amr(n0: int = 33, levels: int = 5, L: float = 4.0, axes=(1.0, 0.75, 0.5), E: float = 210.0,
                          nu: float = 0.3, eigen: float = 1e-3, width: float = 0.1, tag: float = 0.01,
                          far_field: bool = True, phys_boxes=None) -> AmrProblem:
    """The Eshelby inclusion of Sec. 4.1: an ellipsoid with semi-axes `axes`
    centred in [-L, L]^3, one isotropic material (E, nu) everywhere and the
    dilatational eigenstrain eigen * eta * I with eta from ellipsoid_eta
    (diffuse width `width`).  Base grid n0 nodes per axis, levels - 1 boxes
    (ratio 2): box k is the bounding box of the level-(k-1) nodes tagged by
    |grad eta| |dx| > tag (|dx| the length of the vector of grid spacings,
    sqrt(3) h), grown by two coarse cells and kept two coarse cells inside
    box k-1 (with phys_boxes, a list of ((xlo, ylo, zlo), (xhi, yhi, zhi)),
    box k is instead the given region, whose bounds must fall on even nodes
    of level k).  Every face is Dirichlet: with far_field the displacement of
    the equivalent centre of dilatation, u = (1+nu)/(1-nu) eigen V x /
    (4 pi r^3) with V the ellipsoid's volume (the exterior field's leading
    term at large r), else zero."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    base = Problem(dim=3, n=(n0, n0, n0), lo=(-L, -L, -L), hi=(L, L, L), bc=(DIRICHLET,) * 6, kind="iso",
                   C=np.zeros(0), name=f"eshelby_ellipsoid_{n0}_{levels}L_w{width:g}")

    def fields(X, Y, Z):
        eta = ellipsoid_eta(X, Y, Z, axes, width)
        shp = eta.shape
        C = np.stack([np.full(shp, lam), np.full(shp, mu)])
        e = eigen * eta
        return C, np.stack([e, e, e, np.zeros(shp), np.zeros(shp), np.zeros(shp)])

    x, y, z = base.coords()
    X, Y, Z = np.broadcast_arrays(x, y, z)
    base.C, base.eps0 = (np.ascontiguousarray(v) for v in fields(X, Y, Z))
    vol = 4.0 / 3.0 * np.pi * float(np.prod(axes))
    amp = (1.0 + nu) / (1.0 - nu) * eigen * vol / (4.0 * np.pi) if far_field else 0.0
    for f in range(6):
        sl = [slice(None)] * 3
        sl[2 - f // 2] = slice(0, 1) if f % 2 == 0 else slice(base.m[2 - f // 2] - 1, base.m[2 - f // 2])
        Xf, Yf, Zf = X[tuple(sl)], Y[tuple(sl)], Z[tuple(sl)]
        r3 = np.sqrt(Xf ** 2 + Yf ** 2 + Zf ** 2) ** 3
        base.face[f] = np.ascontiguousarray(np.stack([amp * Xf / r3, amp * Yf / r3, amp * Zf / r3]))

    def grad_eta(X, Y, Z, h):
        g = 0.0
        for dx, dy, dz in ((h, 0, 0), (0, h, 0), (0, 0, h)):
            g = g + ((ellipsoid_eta(X + dx, Y + dy, Z + dz, axes, width)
                      - ellipsoid_eta(X - dx, Y - dy, Z - dz, axes, width)) / (2 * h)) ** 2
        return np.sqrt(g)

    amr = AmrProblem(base=base, boxes=[], C=[], eps0=[], b=[], name=base.name)
    prev = ((0, 0, 0), tuple(m - 1 for m in base.m))
    nlev = levels if phys_boxes is None else len(phys_boxes) + 1
    for k in range(1, nlev):
        if phys_boxes is not None:
            hk = amr.level_h(k)[0]
            lo = [int(round((phys_boxes[k - 1][0][a] - base.lo[a]) / hk)) for a in range(3)]
            hi = [int(round((phys_boxes[k - 1][1][a] - base.lo[a]) / hk)) for a in range(3)]
            if any(v % 2 for v in lo + hi):
                raise ValueError("box bounds must fall on even nodes of their level")
        else:
            h_prev = amr.level_h(k - 1)[0]
            lo_p, hi_p = prev
            idx = [np.arange(lo_p[a], hi_p[a] + 1) for a in range(3)]
            Xc = base.lo[0] + h_prev * idx[0][None, None, :]
            Yc = base.lo[1] + h_prev * idx[1][None, :, None]
            Zc = base.lo[2] + h_prev * idx[2][:, None, None]
            tagged = grad_eta(Xc, Yc, Zc, h_prev) * np.sqrt(3.0) * h_prev > tag
            if not tagged.any():
                break
            zz, yy, xx = np.nonzero(tagged)
            t_lo = [idx[0][xx.min()], idx[1][yy.min()], idx[2][zz.min()]]
            t_hi = [idx[0][xx.max()], idx[1][yy.max()], idx[2][zz.max()]]
            lo, hi = [], []
            for a in range(3):
                lo.append(max(_even_floor(2 * (t_lo[a] - 2)), 2 * (lo_p[a] + 2)))
                hi.append(min(_even_ceil(2 * (t_hi[a] + 2)), 2 * (hi_p[a] - 2)))
        amr.boxes.append((tuple(lo), tuple(hi)))
        Xk, Yk, Zk = np.broadcast_arrays(*amr.box_coords(k))
        Ck, ek = fields(Xk, Yk, Zk)
        amr.C.append(np.ascontiguousarray(Ck))
        amr.eps0.append(np.ascontiguousarray(ek))
        amr.b.append(None)
        prev = (tuple(lo), tuple(hi))
    return amr


def inclusion_3d(n: int = 33, seed: int = 0, radius: float = 0.25, eigen: float = 1e-3) -> Problem:
    """3D spherical inclusion in an isotropic matrix (matrix mu=1, lambda=1.5;
    inclusion mu=2, lambda=3), centre jittered by up to 0.05 per axis, tanh
    blend of width max(0.02, 1.5 h), isotropic eigenstrain inside; z = 0
    clamped, the other faces traction-free."""
    rng = np.random.default_rng(seed)
    c = 0.5 + rng.uniform(-0.05, 0.05, size=3)
    p = Problem(dim=3, n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                bc=(TRACTION, TRACTION, TRACTION, TRACTION, DIRICHLET, TRACTION), kind="iso", C=np.zeros(0),
                name=f"inclusion3d_{n}_{seed}")
    x, y, z = p.coords()
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    w = max(0.02, 1.5 * p.h[0])
    eta = _tanh_step((r - radius) / w)
    p.C = np.stack([1.5 + 1.5 * eta, 1.0 + 1.0 * eta]).astype(np.float64)
    e = eigen * eta
    zz = np.zeros_like(e)
    p.eps0 = np.stack([e, e, e, zz, zz, zz]).astype(np.float64)
    return p


def precipitate_step(base: Problem, t: int, steps: int = 6, r0: float = 0.12, r1: float = 0.3, stiff: float = 3.0,
                     eigen: float = 2e-3, center=(0.5, 0.5, 0.5)) -> Problem:
    """Step t of a phase-field coupling loop: a stiff, eigenstrained spherical
    precipitate (moduli x stiff, isotropic eigenstrain `eigen` inside, tanh
    profile of width 2h) of radius r0 + (r1 - r0) t / (steps - 1) inside the
    moduli of `base` (3D); grid, boundary conditions and face data are base's."""
    assert base.dim == 3
    x, y, z = base.coords()
    r = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    rad = r0 + (r1 - r0) * t / max(1, steps - 1)
    eta = _tanh_step((r - rad) / (2.0 * base.h[0]))
    q = dataclasses.replace(base, name=f"{base.name}_precipitate{t}")
    q.C = (base.C * (1.0 + (stiff - 1.0) * eta)[None]).astype(np.float64)
    e = eigen * eta
    zz = np.zeros_like(e)
    eps = np.stack([e, e, e, zz, zz, zz]).astype(np.float64)
    q.eps0 = eps if base.eps0 is None else base.eps0 + eps
    return q


def growing_precipitate(base: Problem, steps: int = 6, **kw):
    """All steps of the growing-precipitate loop (see precipitate_step)."""
    return [precipitate_step(base, t, steps, **kw) for t in range(steps)]


SERVE_SIZES = (33, 49, 65, 97, 129)


@dataclasses.dataclass(frozen=True)
class ServeRequest:
    """One request of a served stream: arrival time (s), problem type
    ("inclusion" or "polycrystal"), nodes per axis, and the pooled input
    variant it draws (inputs are pre-generated per (type, n, variant))."""
    t: float
    kind: str
    n: int
    variant: int


def serving_trace(count: int = 512, seed: int = 2005, rate: float = 200.0, variants: int = 2):
    """Poisson stream of independent solve requests: exponential gaps of mean
    1/rate; size log-uniform in [33, 129] nodes per axis rounded in log space
    to the nearest of 33, 49, 65, 97, 129; even ids are 3D spherical
    inclusions, odd ids polycrystals; each request draws one of ``variants``
    inputs of its type and size, or (variants = 0) an input of its own,
    seeded from its id."""
    rng = np.random.default_rng(seed)
    logs = np.log(np.array(SERVE_SIZES, dtype=np.float64))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        s = rng.uniform(logs[0], logs[-1])
        n = SERVE_SIZES[int(np.argmin(np.abs(logs - s)))]
        v = int(rng.integers(variants)) if variants > 0 else i
        out.append(ServeRequest(t, "inclusion" if i % 2 == 0 else "polycrystal", n, v))
    return out


def _serving_worker(key):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        return key, serving_problem(*key)


def serving_inputs(trace, workers: int = 16):
    """The inputs of a trace's distinct (type, n, variant) keys, generated in
    `workers` processes (each key's input is the same however it is made);
    yields (key, Problem) as they complete."""
    import concurrent.futures
    import multiprocessing
    keys = sorted({(r.kind, r.n, r.variant) for r in trace}, key=lambda k: -k[1])
    if workers <= 1:
        for k in keys:
            yield k, serving_problem(*k)
        return
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("fork")) as ex:
        for k, p in ex.map(_serving_worker, keys, chunksize=2):
            yield k, p


def serving_problem(kind: str, n: int, variant: int, seed: int = 2005) -> Problem:
    """Input of a served request type: a spherical inclusion (isotropic, as
    ``inclusion_3d``) or a polycrystal with 8 to 32 grains (as
    ``polycrystal_3d``), seeded by (seed, type, n, variant)."""
    key = seed * 1000003 + (0 if kind == "inclusion" else 1) * 1009 * 1013 + n * 1013 + variant
    if kind == "inclusion":
        return inclusion_3d(n=n, seed=key)
    rng = np.random.default_rng(key)
    return polycrystal_3d(n=n, grains=int(rng.integers(8, 33)), seed=int(rng.integers(2 ** 31)))
