"""Oracle of the reflux-free coarse/fine coupling on block-structured AMR
(Sec. 3.2 "Reflux-free BSAMR extension" and App. A).  TEST INFRASTRUCTURE ONLY.

Levels: level 0 is the base grid (a plain ``Grid``); level k >= 1 (spacing
h_{k-1}/2) is a list of boxes of nodes [lo, hi] (inclusive, even bounds) in
its own index space.  The level's valid nodes are the union of its boxes;
its fields are stored over the bounding box of the union grown by one node
per side (array extent hi - lo + 3 per axis of the bounding box).  Every box
grown by two coarse cells lies inside the valid nodes of level k-1 (for
k = 1: inside the domain, off its boundary), so no fine node touches the
domain boundary and every ghost is interpolated from valid coarse nodes.

Composite system (the reading of Sec. 3.2 and App. A):
  * unknowns: every valid node of every refined level, plus the level-0 (and
    intermediate-level) nodes not covered by valid nodes of the next level;
  * a covered coarse node takes the value of the coincident fine node
    (App. A: phi_c2 = phi_f4);
  * a fine node that is not valid takes the bi/trilinear interpolation of
    the next coarser level (Sec. 3.2: interpolation operator; App. A:
    phi_f3 = (phi_c1 + phi_c2)/2); those next to valid nodes are the ghosts
    the fine rows read;
  * rows: fine valid nodes use the fine operator with those ghosts (the
    coarse/fine boundary layer is relaxed like any fine node, Sec. 3.2);
    uncovered coarse nodes use the coarse operator with injected
    neighbours; domain-boundary rows as on a single level.  Where two boxes
    of a level meet, their nodes are simply valid nodes: the union, not the
    box list, defines the rows.
A refined level is handled as a grid whose faces are all Dirichlet and whose
non-valid nodes are Dirichlet rows as well (their value is the right-hand
side: zero or the interpolated ghost value), so the single-level primitives
apply with that one override.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import (DIRICHLET, Grid, Hierarchy, ROW_DIRICHLET, apply, dirichlet_mask, jacobi, norm, residual, restrict,
               rhs, row_class, vcycle, fcycle)


class FineLevel:
    """One refined level: the union of boxes of nodes [lo, hi] of its level's
    index space, stored over their bounding box grown by one node."""

    def __init__(self, parent_h, dim, kind, lo, hi, C, eps0=None, b=None, boxes=None):
        self.dim = dim
        if boxes is None:
            boxes = [(lo, hi)]
        self.boxes = [(tuple(int(v) for v in bl), tuple(int(v) for v in bh)) for bl, bh in boxes]
        self.lo = tuple(min(bl[a] for bl, _ in self.boxes) if a < dim else 0 for a in range(3))
        self.hi = tuple(max(bh[a] for _, bh in self.boxes) if a < dim else 0 for a in range(3))
        assert tuple(int(v) for v in lo)[:dim] == self.lo[:dim] and tuple(int(v) for v in hi)[:dim] == self.hi[:dim], \
            "lo, hi must be the bounding box of the boxes"
        m = [1, 1, 1]
        h = [1.0, 1.0, 1.0]
        for a in range(dim):
            for bl, bh in self.boxes:
                assert bl[a] % 2 == 0 and bh[a] % 2 == 0 and bh[a] > bl[a]
            m[a] = self.hi[a] - self.lo[a] + 3
            h[a] = parent_h[a] / 2.0
        bc = [DIRICHLET] * (2 * dim) + [2] * (6 - 2 * dim)
        self.grid = Grid(dim, m, h, bc, kind)
        self.C = np.array(C, dtype=np.float64, order="C", copy=True)
        self.eps0 = None if eps0 is None else np.array(eps0, dtype=np.float64, order="C", copy=True)
        self.b = None if b is None else np.array(b, dtype=np.float64, order="C", copy=True)
        assert self.C.shape[1:] == (m[2], m[1], m[0])
        # valid nodes: the union of the boxes, in array coordinates [z][y][x]
        self.valid_mask = np.zeros((m[2], m[1], m[0]), dtype=bool)
        for bl, bh in self.boxes:
            sl = tuple(slice(bl[a] - self.lo[a] + 1, bh[a] - self.lo[a] + 2) if a < dim else slice(None)
                       for a in (2, 1, 0))
            self.valid_mask[sl] = True

    @property
    def shape(self):
        return self.grid.shape(self.dim)

    def valid_full(self):
        """Valid-node mask broadcast over the vector components."""
        return np.broadcast_to(self.valid_mask, self.shape)

    def global_index(self, a, i):
        """Level index along axis a of array index i."""
        return self.lo[a] - 1 + i


def _axis_interp(lo_f, n_f, coarse_index_of):
    """Per fine index i (ghosted array index 0..n_f-1, fine global index
    lo_f - 1 + i): coarse indices (a, b) and weights (wa, wb)."""
    ia, ib, wa, wb = [], [], [], []
    for i in range(n_f):
        I = lo_f - 1 + i
        c = coarse_index_of(I // 2)
        if I % 2 == 0:
            ia.append(c); ib.append(c); wa.append(1.0); wb.append(0.0)
        else:
            ia.append(c); ib.append(coarse_index_of(I // 2 + 1)); wa.append(0.5); wb.append(0.5)
    return np.array(ia), np.array(ib), np.array(wa), np.array(wb)


def interp_to_box(uc: np.ndarray, coarse_origin, fine: FineLevel) -> np.ndarray:
    """Bi/trilinear interpolation of a coarse field (array whose index 0 is
    coarse global index ``coarse_origin`` per axis) at every node of the
    fine ghosted box."""
    d = fine.dim
    out = uc
    # axes in array order: comp, z, y, x -> fine axes a = 2, 1, 0
    res = uc
    for a in range(d):
        arr_ax = 3 - a
        n_f = fine.grid.m[a]
        ia, ib, wa, wb = _axis_interp(fine.lo[a], n_f, lambda c: c - coarse_origin[a])
        A = np.take(res, ia, axis=arr_ax)
        B = np.take(res, ib, axis=arr_ax)
        shp = [1] * res.ndim
        shp[arr_ax] = n_f
        res = A * wa.reshape(shp) + B * wb.reshape(shp)
    out = res
    return np.ascontiguousarray(out)


def covered_index(fine: FineLevel, coarse_origin):
    """Index arrays ([z][y][x], with a leading component slice) of the
    coarse nodes coincident with valid fine nodes, in the coarse array
    (whose index 0 is coarse index ``coarse_origin``), and of those fine
    nodes in the fine array; in storage order of the fine array."""
    sel = fine.valid_mask.copy()
    for a in range(fine.dim):
        ax = 2 - a
        idx = np.arange(sel.shape[ax])
        even = (fine.lo[a] - 1 + idx) % 2 == 0
        shp = [1, 1, 1]
        shp[ax] = -1
        sel &= even.reshape(shp)
    fz, fy, fx = np.nonzero(sel)
    f = (fz, fy, fx)
    c = []
    for ax, a in ((0, 2), (1, 1), (2, 0)):
        if a < fine.dim:
            c.append((fine.lo[a] - 1 + f[ax]) // 2 - coarse_origin[a])
        else:
            c.append(f[ax])
    return (slice(None),) + tuple(c), (slice(None),) + f


def covered_slices(fine: FineLevel, coarse_origin):
    """Same as covered_index (kept for callers of the one-box form)."""
    return covered_index(fine, coarse_origin)


def average_to_coarse(fl: FineLevel, field: np.ndarray) -> np.ndarray:
    """Full weighting (tensor product of [1/4, 1/2, 1/4]) of a field given on
    the ghosted fine array, at the fine nodes coincident with the coarse
    nodes the level covers (order of covered_index)."""
    res = np.asarray(field, dtype=np.float64)
    for a in range(fl.dim):
        ax = 3 - a
        n = res.shape[ax]
        centre = np.take(res, np.arange(1, n - 1), axis=ax)
        lo = np.take(res, np.arange(0, n - 2), axis=ax)
        hi = np.take(res, np.arange(2, n), axis=ax)
        full = 0.5 * centre + 0.25 * (lo + hi)          # index i-1 of `full` is fine array index i
        pad = [(0, 0)] * res.ndim
        pad[ax] = (1, 1)
        res = np.pad(full, pad)
    _, fs = covered_index(fl, (0, 0, 0))
    return res[fs]


def relax(fl: FineLevel, e: np.ndarray, f: np.ndarray, omega: float) -> np.ndarray:
    """One damped Jacobi sweep on a refined level: the fine operator's sweep
    at valid nodes, the Dirichlet row (value f) at every other node."""
    out = jacobi(fl.grid, fl.C, e, f, omega)
    return np.where(fl.valid_full(), out, f)


class Composite:
    """Base grid plus nested fine boxes."""

    def __init__(self, base_prob, fines: Sequence[FineLevel]):
        self.base = base_prob
        self.g0 = Grid.of(base_prob)
        self.fines = list(fines)
        self.dim = base_prob.dim
        for k, fl in enumerate(self.fines, start=1):
            for bl, bh in fl.boxes:
                # the box grown by two coarse cells lies inside the valid nodes of level k-1
                rng = [range(bl[a] // 2 - 2, bh[a] // 2 + 3) if a < self.dim else range(1) for a in range(3)]
                if k == 1:
                    for a in range(self.dim):
                        assert rng[a][0] >= 0 and rng[a][-1] <= self.g0.m[a] - 1, "improper nesting"
                else:
                    par = self.fines[k - 2]
                    o = self.origin(k - 1)
                    sl = tuple(slice(rng[a][0] - o[a], rng[a][-1] - o[a] + 1) if a < self.dim else slice(None)
                               for a in (2, 1, 0))
                    for a in range(self.dim):
                        assert rng[a][0] - o[a] >= 0 and rng[a][-1] - o[a] < par.grid.m[a], "improper nesting"
                    assert par.valid_mask[sl].all(), "improper nesting"
        # coarse levels take the average of the finer level where it exists
        # (Sec. 1: coarse levels are updated from fine levels by averaging):
        # moduli and eigenstrain at covered nodes <- full weighting of the
        # next finer level's values (its ghost layer completes the stencil)
        self.C0 = np.array(base_prob.C, dtype=np.float64)
        self.E0 = None if base_prob.eps0 is None else np.array(base_prob.eps0, dtype=np.float64)
        for k in range(len(self.fines), 0, -1):
            fl = self.fines[k - 1]
            cs, _ = covered_index(fl, self.origin(k - 1))
            tgtC = self.C0 if k == 1 else self.fines[k - 2].C
            tgtC[cs] = average_to_coarse(fl, fl.C)
            if fl.eps0 is not None:
                tgtE = self.E0 if k == 1 else self.fines[k - 2].eps0
                if tgtE is not None:
                    tgtE[cs] = average_to_coarse(fl, fl.eps0)
        self.H = Hierarchy(self.g0, self.C0)
        self.f = [rhs(self.g0, self.C0, self.E0, base_prob.b, base_prob.face)]
        for fl in self.fines:
            self.f.append(rhs(fl.grid, fl.C, fl.eps0, fl.b, None))

    def origin(self, k):
        """Global index of array index 0 of level k."""
        if k == 0:
            return (0, 0, 0)
        fl = self.fines[k - 1]
        return tuple(fl.lo[a] - 1 if a < self.dim else 0 for a in range(3))

    def grid(self, k):
        return self.g0 if k == 0 else self.fines[k - 1].grid

    def C(self, k):
        return self.H.C[0] if k == 0 else self.fines[k - 1].C

    # ---- composite state: injection and ghosts ----
    def sync(self, u: List[np.ndarray]) -> List[np.ndarray]:
        """Covered coarse nodes <- coincident fine values (finest first),
        then fine ghosts <- interpolation of the next coarser level."""
        u = [x.copy() for x in u]
        for k in range(len(self.fines), 0, -1):
            cs, fs = covered_index(self.fines[k - 1], self.origin(k - 1))
            u[k - 1][cs] = u[k][fs]
        for k in range(1, len(self.fines) + 1):
            fl = self.fines[k - 1]
            gi = interp_to_box(u[k - 1], self.origin(k - 1), fl)
            u[k] = np.where(fl.valid_full(), u[k], gi)
        return u

    def unknown_masks(self) -> List[np.ndarray]:
        """Rows that are composite unknowns (True) per level."""
        masks = []
        for k in range(len(self.fines) + 1):
            g = self.grid(k)
            if k == 0:
                mk = ~dirichlet_mask(g).copy()
            else:
                mk = self.fines[k - 1].valid_full().copy()
            if k < len(self.fines):
                cs, _ = covered_index(self.fines[k], self.origin(k))
                mk = np.array(mk)
                mk[cs] = False
            masks.append(np.array(mk))
        return masks

    def residual(self, u: List[np.ndarray]) -> List[np.ndarray]:
        """Composite residual (zero outside the composite rows)."""
        us = self.sync(u)
        masks = self.unknown_masks()
        out = []
        for k in range(len(us)):
            r = residual(self.grid(k), self.C(k), us[k], self.f[k])
            out.append(np.where(masks[k], r, 0.0))
        return out

    def norm(self, r: List[np.ndarray]) -> float:
        return float(np.sqrt(sum(float(np.sum(x * x)) for x in r)))

    def initial(self) -> List[np.ndarray]:
        """Dirichlet lift on the base grid; fine levels interpolated from it."""
        u0 = np.where(dirichlet_mask(self.g0), self.f[0], 0.0)
        u = [u0]
        for k in range(1, len(self.fines) + 1):
            u.append(interp_to_box(u[k - 1], self.origin(k - 1), self.fines[k - 1]))
        return self.sync(u)

    # ---- dense composite system (tiny cases) ----
    def dense_solve(self) -> List[np.ndarray]:
        masks = self.unknown_masks()
        shapes = [self.grid(k).shape(self.dim) for k in range(len(masks))]
        base = self.initial()
        # composite rows are affine in the unknowns: A x = r(0-state) - r(x)
        idx = [np.flatnonzero(m.ravel()) for m in masks]
        n = sum(len(i) for i in idx)

        def pack(fields):
            return np.concatenate([f.ravel()[i] for f, i in zip(fields, idx)])

        def unpack(x, template):
            out = [t.copy() for t in template]
            o = 0
            for k, i in enumerate(idx):
                flat = out[k].ravel()
                flat[i] = x[o:o + len(i)]
                out[k] = flat.reshape(shapes[k])
                o += len(i)
            return out

        zero = [np.where(masks[k], 0.0, base[k]) for k in range(len(masks))]
        r0 = pack(self.residual(zero))
        A = np.empty((n, n))
        e = np.zeros(n)
        for q in range(n):
            e[q] = 1.0
            A[:, q] = r0 - pack(self.residual(unpack(e, zero)))
            e[q] = 0.0
        x = np.linalg.solve(A, r0)
        return self.sync(unpack(x, zero))

    # ---- composite correction cycle ----
    def cycle(self, u: List[np.ndarray], nu1=2, nu2=2, omega=2.0 / 3.0, base="V") -> List[np.ndarray]:
        """One composite correction cycle (Sec. 3.2): fine corrections relaxed
        with zero ghosts (the coarse/fine boundary acting as Dirichlet), fine
        residual restricted onto the covered coarse nodes, coarse residual at
        uncovered nodes updated for the injected fine correction, V-cycle (or
        F-cycle, base="F") on the base grid, then interpolation back to the
        fine nodes and ghosts and relaxation with the interpolated ghosts as
        Dirichlet values."""
        L = len(self.fines)
        u = self.sync(u)
        r = self.residual(u)
        masks = self.unknown_masks()
        e = [None] * (L + 1)
        rr = [x.copy() for x in r]
        for k in range(L, 0, -1):
            fl = self.fines[k - 1]
            g, C = fl.grid, fl.C
            ek = np.zeros(fl.shape)
            for _ in range(nu1):
                ek = relax(fl, ek, rr[k], omega)          # non-valid rows: rhs 0 -> stay 0
            e[k] = ek
            rk = residual(g, C, ek, rr[k])
            rk[~fl.valid_full()] = 0.0
            # coarse residual at uncovered nodes: minus the coarse operator of the injected fine correction
            gc, Cc = self.grid(k - 1), self.C(k - 1)
            cs, fs = covered_index(fl, self.origin(k - 1))
            inj = np.zeros(gc.shape(self.dim))
            inj[cs] = ek[fs]
            Ainj = apply(gc, Cc, inj)
            rc = np.where(masks[k - 1], rr[k - 1] - Ainj, 0.0)
            rc[cs] = self._restrict_valid(fl, rk)
            rr[k - 1] = rc
        # base grid: one V- (or F-) cycle for the correction
        step = {"V": vcycle, "F": fcycle}[base]
        e[0] = step(self.H, 0, np.zeros(self.g0.shape(self.dim)), rr[0], nu1, nu2, omega)
        for k in range(1, L + 1):
            fl = self.fines[k - 1]
            g, C = fl.grid, fl.C
            ec = e[k - 1].copy()
            pe = interp_to_box(ec, self.origin(k - 1), fl)
            valid = fl.valid_full()
            ek = np.where(valid, e[k] + pe, pe)
            fk = np.where(valid, rr[k], pe)
            for _ in range(nu2):
                ek = relax(fl, ek, fk, omega)
            e[k] = ek
        return self.sync([u[k] + e[k] for k in range(L + 1)])

    def _restrict_valid(self, fl: FineLevel, rk: np.ndarray) -> np.ndarray:
        """Full weighting of a fine residual onto the coarse nodes coincident
        with the level's valid nodes, over valid fine nodes only, the weights
        renormalised to sum to one where the stencil would reach a non-valid
        node."""
        d = fl.dim
        valid = fl.valid_mask.astype(float)
        num = rk.copy()
        den = valid.copy()
        for a in range(d):
            ax = 2 - a
            def fw(x, axis):
                y = 0.5 * x
                y[(slice(None),) * axis + (slice(1, None),)] += 0.25 * x[(slice(None),) * axis + (slice(None, -1),)]
                y[(slice(None),) * axis + (slice(None, -1),)] += 0.25 * x[(slice(None),) * axis + (slice(1, None),)]
                return y
            num = fw(num, ax + 1)
            den = fw(den, ax)
        _, fs = covered_index(fl, (0, 0, 0))
        return num[fs] / den[fs[1:]]

    def solve(self, tol=1e-12, max_cycles=300, nu1=2, nu2=2, omega=2.0 / 3.0, base="V"):
        u = self.initial()
        r0 = self.norm(self.residual(u))
        hist = [1.0]
        for c in range(max_cycles):
            u = self.cycle(u, nu1, nu2, omega, base)
            rel = self.norm(self.residual(u)) / r0
            hist.append(rel)
            if rel <= tol:
                break
            if rel < 1e-11 and len(hist) > 3 and hist[-1] > 0.95 * hist[-4]:
                break
        return u, hist


def from_problem(ap) -> Composite:
    """Composite system of an AMR problem description (``synth.AmrProblem``)."""
    from . import ANISO, ISO
    kind = ISO if ap.base.kind == "iso" else ANISO
    fines = []
    for k, (lo, hi) in enumerate(ap.boxes, start=1):
        fines.append(FineLevel(ap.level_h(k - 1), ap.base.dim, kind, lo, hi, ap.C[k - 1], ap.eps0[k - 1],
                               ap.b[k - 1], boxes=ap.level_boxes(k)))
    return Composite(ap.base, fines)
