"""ctypes binding of ``libemg.so``: the C ABI of ``include/emg.h`` under the
same names, plus a small ``Problem`` wrapper that marshals numpy arrays (host)
and torch tensors (device) into the ABI's pointers.  No arithmetic of the
solve happens here."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EMG_LIB") or os.path.join(_HERE, "libemg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2001_04789_amd.build` "
                      "(or __graft_entry__.build()) first")

lib = ctypes.CDLL(LIB_PATH)

c_int, c_int64, c_double, c_size_t, c_void_p = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p

EMG_OK, EMG_EINVAL, EMG_ENOMEM, EMG_EDEVICE, EMG_ENOTCONV, EMG_EDIVERGED, EMG_ESTATE, EMG_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
EMG_NOALLOC_SCRATCH_BYTES = 8 << 20
EMG_BC_DIRICHLET, EMG_BC_TRACTION, EMG_BC_PERIODIC, EMG_BC_NEUMANN = 0, 1, 2, 3
EMG_MOD_ISO, EMG_MOD_ANISO = 0, 1
EMG_FP64, EMG_MIXED = 0, 1
EMG_VCYCLE, EMG_FCYCLE = 0, 1

_BC = {"dirichlet": EMG_BC_DIRICHLET, "traction": EMG_BC_TRACTION, "periodic": EMG_BC_PERIODIC,
       "neumann": EMG_BC_NEUMANN}
_CYCLE = {"V": EMG_VCYCLE, "F": EMG_FCYCLE, EMG_VCYCLE: EMG_VCYCLE, EMG_FCYCLE: EMG_FCYCLE}
_KIND = {"iso": EMG_MOD_ISO, "aniso": EMG_MOD_ANISO}
_PREC = {"fp64": EMG_FP64, "mixed": EMG_MIXED, EMG_FP64: EMG_FP64, EMG_MIXED: EMG_MIXED}


class emg_domain(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int64 * 3), ("lo", c_double * 3), ("hi", c_double * 3),
                ("bc", c_int * 6), ("kind", c_int)]


class emg_box(ctypes.Structure):
    _fields_ = [("lo", c_int64 * 3), ("hi", c_int64 * 3)]


class emg_solve_opts(ctypes.Structure):
    _fields_ = [("rtol", c_double), ("max_cycles", c_int), ("precision", c_int), ("nu1", c_int), ("nu2", c_int),
                ("omega", c_double), ("warm_start", c_int), ("check_every", c_int), ("use_graph", c_int),
                ("cycle", c_int), ("stall_iters", c_int), ("stall_factor", c_double),
                ("inner_cycles", c_int)]


class emg_solve_stats(ctypes.Structure):
    _fields_ = [("cycles", c_int), ("converged", c_int), ("rel_res", c_double), ("conv_factor", c_double),
                ("solve_seconds", c_double), ("setup_seconds", c_double), ("dofs", c_int64),
                ("fp64_fallback", c_int)]


class emg_request(ctypes.Structure):
    _fields_ = [("dom", emg_domain), ("C", c_void_p), ("eps0", c_void_p), ("body", c_void_p),
                ("face", c_void_p * 6), ("u_out", c_void_p), ("flags", c_int)]


class emg_ticket_info(ctypes.Structure):
    _fields_ = [("done", c_int), ("status", c_int), ("stats", emg_solve_stats), ("t_submit", c_double),
                ("t_admit", c_double), ("t_ready", c_double), ("t_done", c_double)]


P = ctypes.POINTER
_SIGS = {
    "emg_last_error": ([], ctypes.c_char_p),
    "emg_default_opts": ([P(emg_solve_opts)], None),
    "emg_ctx_create": ([c_int, c_size_t, P(c_void_p)], c_int),
    "emg_ctx_destroy": ([c_void_p], c_int),
    "emg_problem_create": ([c_void_p, P(emg_domain), P(c_void_p)], c_int),
    "emg_problem_destroy": ([c_void_p], c_int),
    "emg_set_stream": ([c_void_p, c_void_p], c_int),
    "emg_footprint": ([c_void_p, P(c_size_t)], c_int),
    "emg_set_moduli": ([c_void_p, c_void_p, c_int], c_int),
    "emg_set_eigenstrain": ([c_void_p, c_void_p, c_int], c_int),
    "emg_set_body_force": ([c_void_p, c_void_p, c_int], c_int),
    "emg_set_face": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_solve": ([c_void_p, P(emg_solve_opts), P(emg_solve_stats)], c_int),
    "emg_get_displacement": ([c_void_p, c_void_p, c_int], c_int),
    "emg_set_displacement": ([c_void_p, c_void_p, c_int], c_int),
    "emg_get_stress": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_get_von_mises": ([c_void_p, c_void_p, c_int], c_int),
    "emg_level_zmarch": ([c_void_p, c_int, c_int, P(c_int)], c_int),
    "emg_get_rhs": ([c_void_p, c_void_p, c_int], c_int),
    "emg_num_levels": ([c_void_p, P(c_int)], c_int),
    "emg_level_shape": ([c_void_p, c_int, P(c_int64), P(c_double)], c_int),
    "emg_level_moduli": ([c_void_p, c_int, c_void_p], c_int),
    "emg_level_apply": ([c_void_p, c_int, c_int, c_void_p, c_void_p], c_int),
    "emg_level_residual": ([c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p], c_int),
    "emg_level_jacobi": ([c_void_p, c_int, c_int, c_double, c_void_p, c_void_p, c_void_p], c_int),
    "emg_level_restrict": ([c_void_p, c_int, c_int, c_void_p, c_void_p], c_int),
    "emg_level_prolong_add": ([c_void_p, c_int, c_int, c_void_p, c_void_p], c_int),
    "emg_level_bottom_solve": ([c_void_p, c_int, c_void_p, c_void_p], c_int),
    "emg_kernel_time": ([c_void_p, c_int, c_int, c_int, c_int, P(c_double)], c_int),
    "emg_autotune": ([c_void_p, c_int, c_int, c_int, P(c_int)], c_int),
    "emg_autotune_reset": ([], c_int),
    "emg_solve_batch": ([P(c_void_p), c_int, P(emg_solve_opts), P(emg_solve_stats)], c_int),
    "emg_solve_batch_noalloc": ([P(c_void_p), c_int, P(emg_solve_opts), P(emg_solve_stats)], c_int),
    "emg_server_create": ([c_void_p, c_int, P(emg_solve_opts), P(c_void_p)], c_int),
    "emg_server_submit": ([c_void_p, P(emg_request), P(ctypes.c_uint64)], c_int),
    "emg_server_poll": ([c_void_p, ctypes.c_uint64, P(emg_ticket_info)], c_int),
    "emg_server_wait": ([c_void_p, ctypes.c_uint64, P(emg_ticket_info)], c_int),
    "emg_server_now": ([c_void_p, P(c_double)], c_int),
    "emg_server_destroy": ([c_void_p], c_int),
    "emg_amr_add_level": ([c_void_p, P(c_int64), P(c_int64)], c_int),
    "emg_level_tiles": ([c_void_p, c_int, c_int, P(c_int), P(c_int), P(c_int)], c_int),
    "emg_tail_levels": ([c_void_p, c_int, P(c_int)], c_int),
    "emg_set_level_boxes": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_amr_level_valid": ([c_void_p, c_int, c_void_p, P(c_int64)], c_int),
    "emg_amr_num_levels": ([c_void_p, P(c_int)], c_int),
    "emg_amr_level_shape": ([c_void_p, c_int, P(c_int64)], c_int),
    "emg_amr_set_moduli": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_amr_set_eigenstrain": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_amr_set_body_force": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_amr_get_displacement": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_amr_set_displacement": ([c_void_p, c_int, c_void_p, c_int], c_int),
    "emg_amr_residual": ([c_void_p, c_int, c_void_p, P(c_double)], c_int),
}
SYMBOLS = tuple(_SIGS)

for _name, (_args, _ret) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = _ret
    globals()[_name] = _fn


class EmgError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib.emg_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def check(status: int, where: str = "emg") -> int:
    if status != EMG_OK:
        raise EmgError(status, where)
    return status


def _ready(t):
    """Device buffers handed to the library must hold their final contents
    when the call is made: the problem's stream does not wait on torch's, so
    torch's work queued on its current stream of the tensor's device (fills,
    copies, kernels producing the tensor) is finished first."""
    import torch
    torch.cuda.current_stream(t.device).synchronize()


def _host_or_device(a, dtype=np.float64):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if a is None:
        return None, 0, None
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if a.is_cuda:
            assert a.is_contiguous(), "device tensors must be contiguous"
            _ready(a)
            return c_void_p(a.data_ptr()), 1, a
        a = a.numpy()
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(c_void_p), 0, arr


def _dev(t):
    """Device pointer of a contiguous torch tensor on the GPU (after _ready)."""
    assert hasattr(t, "is_cuda") and t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    _ready(t)
    return c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = c_void_p()
        check(lib.emg_ctx_create(device, hbm_budget_bytes, ctypes.byref(h)), "emg_ctx_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib.emg_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_opts(**kw) -> emg_solve_opts:
    o = emg_solve_opts()
    lib.emg_default_opts(ctypes.byref(o))
    names = {f[0] for f in emg_solve_opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solve option {k!r}")
        if k == "precision":
            v = _PREC[v]
        elif k == "cycle":
            v = _CYCLE[v]
        setattr(o, k, v)
    return o


def _batch(fn, name, problems, raise_on_error, opts):
    n = len(problems)
    arr = (c_void_p * n)(*[p.handle for p in problems])
    o = default_opts(**opts)
    st = (emg_solve_stats * n)()
    s = fn(arr, n, ctypes.byref(o), st)
    out = [dict({k: getattr(x, k) for k, _ in emg_solve_stats._fields_}, status=s) for x in st]
    if raise_on_error and s != EMG_OK:
        check(s, name)
    return out


def solve_batch(problems, raise_on_error: bool = True, **opts):
    """Solve several problems together (emg_solve_batch); per-problem stats."""
    return _batch(lib.emg_solve_batch, "emg_solve_batch", problems, raise_on_error, opts)


def solve_batch_noalloc(problems, raise_on_error: bool = True, **opts):
    """emg_solve_batch_noalloc: the batch without device allocation (work
    lists in the library's fixed per-GPU scratch, direct launches); every
    problem must have been solved since its moduli were last set."""
    return _batch(lib.emg_solve_batch_noalloc, "emg_solve_batch_noalloc", problems, raise_on_error, opts)


def _domain(dim: int, n, lo, hi, bc, kind) -> emg_domain:
    d = emg_domain()
    d.dim = dim
    for a in range(3):
        d.n[a] = int(n[a])
        d.lo[a] = float(lo[a])
        d.hi[a] = float(hi[a]) if a < dim else float(lo[a]) + 1.0
    for f in range(6):
        d.bc[f] = _BC[bc[f]] if isinstance(bc[f], str) else int(bc[f])
    d.kind = _KIND[kind] if isinstance(kind, str) else int(kind)
    return d


class Server:
    """Continuous-batching solve server (emg_server_*): submit host problems,
    collect displacements and per-request timing."""

    def __init__(self, ctx: Context, max_slots: int = 8, **opts):
        o = default_opts(**opts)
        h = c_void_p()
        check(lib.emg_server_create(ctx.handle, max_slots, ctypes.byref(o), ctypes.byref(h)), "emg_server_create")
        self.handle, self.ctx = h, ctx
        self._keep = {}

    def submit(self, spec, out=None) -> int:
        """Queue ``spec`` (attributes as for Problem.from_spec: numpy arrays,
        copied at submit, or contiguous float64 device tensors, borrowed until
        the request is done); returns a ticket.  ``out`` is an optional
        device tensor for the displacement (required with device inputs)."""
        r = emg_request()
        r.dom = _domain(spec.dim, spec.n, spec.lo, spec.hi, spec.bc, spec.kind)
        dev = hasattr(spec.C, "is_cuda") and spec.C.is_cuda
        keep = []

        def arr(a):
            if a is None:
                return None
            if dev:
                assert a.is_cuda and a.is_contiguous() and str(a.dtype) == "torch.float64"
                keep.append(a)
                return _dev(a)
            x = np.ascontiguousarray(a, dtype=np.float64)
            keep.append(x)
            return x.ctypes.data_as(c_void_p)

        r.C, r.eps0, r.body = arr(spec.C), arr(spec.eps0), arr(spec.b)
        for f in range(6):
            r.face[f] = arr(spec.face.get(f)) if spec.face and f < 2 * spec.dim else None
        if dev:
            assert out is not None, "device inputs need a device output tensor"
            u = out
            r.u_out = _dev(out)
            r.flags = 1
        else:
            u = np.empty((spec.dim,) + tuple(spec.m[::-1]), dtype=np.float64)
            r.u_out = u.ctypes.data_as(c_void_p)
        t = ctypes.c_uint64()
        check(lib.emg_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "emg_server_submit")
        # the output (and, for device requests, the borrowed inputs) must outlive the request
        self._keep[t.value] = (u, keep if dev else None)
        return t.value

    @staticmethod
    def _info(i: emg_ticket_info) -> dict:
        return {"done": bool(i.done), "status": i.status, "t_submit": i.t_submit, "t_admit": i.t_admit,
                "t_ready": i.t_ready, "t_done": i.t_done, **{k: getattr(i.stats, k) for k, _ in emg_solve_stats._fields_}}

    def poll(self, ticket: int) -> dict:
        i = emg_ticket_info()
        check(lib.emg_server_poll(self.handle, ticket, ctypes.byref(i)), "emg_server_poll")
        return self._info(i)

    def wait(self, ticket: int):
        """Block until the request is done; returns (displacement, info)."""
        i = emg_ticket_info()
        check(lib.emg_server_wait(self.handle, ticket, ctypes.byref(i)), "emg_server_wait")
        u = self._keep.pop(ticket, (None, None))[0]
        return u, self._info(i)

    def now(self) -> float:
        t = c_double()
        check(lib.emg_server_now(self.handle, ctypes.byref(t)), "emg_server_now")
        return t.value

    def close(self):
        if self.handle:
            lib.emg_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """One solve problem on the GPU (owns its hierarchy and stream)."""

    def __init__(self, ctx: Context, dim: int, n, lo, hi, bc, kind: str):
        d = _domain(dim, n, lo, hi, bc, kind)
        h = c_void_p()
        check(lib.emg_problem_create(ctx.handle, ctypes.byref(d), ctypes.byref(h)), "emg_problem_create")
        self.handle, self.ctx, self.dim = h, ctx, dim
        self.ncomp_moduli = 2 if d.kind == EMG_MOD_ISO else (21 if dim == 3 else 6)
        m = (c_int64 * 3)()
        check(lib.emg_level_shape(h, 0, m, None), "emg_level_shape")
        self.m = tuple(int(x) for x in m)

    @classmethod
    def from_spec(cls, ctx: Context, spec) -> "Problem":
        """Create from a problem description with attributes dim, n, lo, hi,
        bc, kind, C, eps0, b, face (e.g. ``synth.Problem``) and upload its data."""
        p = cls(ctx, spec.dim, spec.n, spec.lo, spec.hi, spec.bc, spec.kind)
        p.set_moduli(spec.C)
        p.set_eigenstrain(spec.eps0)
        p.set_body_force(spec.b)
        for f in range(2 * spec.dim):
            if spec.bc[f] != "periodic":
                p.set_face(f, spec.face.get(f) if spec.face else None)
        return p

    @property
    def N(self) -> int:
        return self.m[0] * self.m[1] * self.m[2]

    def close(self):
        if self.handle:
            lib.emg_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inputs ----
    def set_stream(self, stream_handle: Optional[int]):
        check(lib.emg_set_stream(self.handle, c_void_p(stream_handle) if stream_handle else None), "emg_set_stream")

    def set_moduli(self, C):
        ptr, dev, keep = _host_or_device(C)
        check(lib.emg_set_moduli(self.handle, ptr, dev), "emg_set_moduli")

    def set_eigenstrain(self, e):
        ptr, dev, keep = _host_or_device(e)
        check(lib.emg_set_eigenstrain(self.handle, ptr, dev), "emg_set_eigenstrain")

    def set_body_force(self, b):
        ptr, dev, keep = _host_or_device(b)
        check(lib.emg_set_body_force(self.handle, ptr, dev), "emg_set_body_force")

    def set_face(self, f: int, v):
        ptr, dev, keep = _host_or_device(v)
        check(lib.emg_set_face(self.handle, f, ptr, dev), "emg_set_face")

    def footprint(self) -> int:
        b = c_size_t()
        check(lib.emg_footprint(self.handle, ctypes.byref(b)), "emg_footprint")
        return int(b.value)

    # ---- solve ----
    def solve(self, raise_on_error: bool = True, **opts) -> dict:
        o = default_opts(**opts)
        st = emg_solve_stats()
        s = lib.emg_solve(self.handle, ctypes.byref(o), ctypes.byref(st))
        out = {k: getattr(st, k) for k, _ in emg_solve_stats._fields_}
        out["status"] = s
        if raise_on_error and s != EMG_OK:
            check(s, "emg_solve")
        return out

    # ---- outputs ----
    def _get(self, fn, comps, out=None):
        if out is not None:
            check(fn(self.handle, _dev(out), 1), fn.__name__)
            return out
        a = np.empty((comps, self.m[2], self.m[1], self.m[0]))
        check(fn(self.handle, a.ctypes.data_as(c_void_p), 0), fn.__name__)
        return a

    def displacement(self, out=None):
        return self._get(lib.emg_get_displacement, self.dim, out)

    def set_displacement(self, u):
        ptr, dev, keep = _host_or_device(u)
        check(lib.emg_set_displacement(self.handle, ptr, dev), "emg_set_displacement")

    def stress(self, out=None, level: int = 0):
        """Voigt stress on the base grid (level 0) or on refined level k (its
        bounding array, valid after a solve)."""
        comps = 6 if self.dim == 3 else 3
        if out is not None:
            check(lib.emg_get_stress(self.handle, level, _dev(out), 1), "emg_get_stress")
            return out
        m = self.m if level == 0 else self.amr_level_shape(level)
        a = np.empty((comps, m[2], m[1], m[0]))
        check(lib.emg_get_stress(self.handle, level, a.ctypes.data_as(c_void_p), 0), "emg_get_stress")
        return a

    def von_mises(self, out=None):
        """Von Mises stress per node (3D), shape (1, mz, my, mx) on the host."""
        return self._get(lib.emg_get_von_mises, 1, out)

    def rhs(self, out=None):
        return self._get(lib.emg_get_rhs, self.dim, out)

    # ---- level-wise steps (device tensors) ----
    def level_zmarch(self, level: int = 0, precision="fp64") -> int:
        """Plane runs per column of the z-marching pass on a level (0: tile kernel)."""
        c = c_int()
        check(lib.emg_level_zmarch(self.handle, level, _PREC[precision], ctypes.byref(c)), "emg_level_zmarch")
        return c.value

    def level_tiles(self, level: int = 0, precision="fp64"):
        """(stencil, restriction, interpolation) tile shapes of a level:
        0 = 64x4, 1 = 64x2, 2 = 128x2, 3 = 32x8 (-1: none)."""
        a, b, c = c_int(), c_int(), c_int()
        check(lib.emg_level_tiles(self.handle, level, _PREC[precision], ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(c)), "emg_level_tiles")
        return a.value, b.value, c.value

    def tail_levels(self, precision="fp64") -> int:
        """Coarsest levels whose cycle runs as one fused launch (0: none)."""
        c = c_int()
        check(lib.emg_tail_levels(self.handle, _PREC[precision], ctypes.byref(c)), "emg_tail_levels")
        return c.value

    def num_levels(self) -> int:
        n = c_int()
        check(lib.emg_num_levels(self.handle, ctypes.byref(n)), "emg_num_levels")
        return n.value

    def level_shape(self, level: int):
        m = (c_int64 * 3)()
        h = (c_double * 3)()
        check(lib.emg_level_shape(self.handle, level, m, h), "emg_level_shape")
        return tuple(int(x) for x in m), tuple(float(x) for x in h)

    def level_moduli(self, level: int, out):
        check(lib.emg_level_moduli(self.handle, level, _dev(out)), "emg_level_moduli")
        return out

    def level_apply(self, level, u, out, precision="fp64"):
        check(lib.emg_level_apply(self.handle, level, _PREC[precision], _dev(u), _dev(out)), "emg_level_apply")
        return out

    def level_residual(self, level, u, f, out, precision="fp64"):
        check(lib.emg_level_residual(self.handle, level, _PREC[precision], _dev(u), _dev(f), _dev(out)),
              "emg_level_residual")
        return out

    def level_jacobi(self, level, u, f, out, omega=2.0 / 3.0, precision="fp64"):
        check(lib.emg_level_jacobi(self.handle, level, _PREC[precision], float(omega), _dev(u), _dev(f), _dev(out)),
              "emg_level_jacobi")
        return out

    def level_restrict(self, level, r, fc, precision="fp64"):
        check(lib.emg_level_restrict(self.handle, level, _PREC[precision], _dev(r), _dev(fc)), "emg_level_restrict")
        return fc

    def level_prolong_add(self, level, ec, uf, precision="fp64"):
        check(lib.emg_level_prolong_add(self.handle, level, _PREC[precision], _dev(ec), _dev(uf)),
              "emg_level_prolong_add")
        return uf

    def level_bottom_solve(self, f, e, precision="fp64"):
        check(lib.emg_level_bottom_solve(self.handle, _PREC[precision], _dev(f), _dev(e)), "emg_level_bottom_solve")
        return e

    # ---- block-structured AMR ----
    @classmethod
    def from_amr(cls, ctx: Context, amr) -> "Problem":
        """Create from an AMR description (base problem + nested boxes with
        fields on the ghosted boxes, e.g. ``synth.AmrProblem``)."""
        p = cls.from_spec(ctx, amr.base)
        for k in range(1, len(amr.boxes) + 1):
            boxes = amr.level_boxes(k) if hasattr(amr, "level_boxes") else [amr.boxes[k - 1]]
            p.set_level_boxes(k, boxes)
            p.amr_set_moduli(k, amr.C[k - 1])
            if amr.eps0[k - 1] is not None:
                p.amr_set_eigenstrain(k, amr.eps0[k - 1])
            if amr.b[k - 1] is not None:
                p.amr_set_body_force(k, amr.b[k - 1])
        return p

    def set_level_boxes(self, level, boxes):
        """Refined level `level` (the next one) as the union of boxes, each
        ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z)) in that level's index space."""
        arr = (emg_box * len(boxes))()
        for i, (lo, hi) in enumerate(boxes):
            for a in range(3):
                arr[i].lo[a] = int(lo[a]) if a < len(lo) else 0
                arr[i].hi[a] = int(hi[a]) if a < len(hi) else 0
        check(lib.emg_set_level_boxes(self.handle, int(level), ctypes.cast(arr, c_void_p), len(boxes)),
              "emg_set_level_boxes")

    def amr_level_valid(self, level):
        """Valid-node mask (bool, [z][y][x]) of a refined level's array and its count."""
        m = self.amr_level_shape(level)
        mask = np.zeros((m[2], m[1], m[0]), dtype=np.uint8)
        n = c_int64()
        check(lib.emg_amr_level_valid(self.handle, level, mask.ctypes.data_as(c_void_p), ctypes.byref(n)),
              "emg_amr_level_valid")
        return mask.astype(bool), int(n.value)

    def amr_add_level(self, lo, hi):
        l3 = (c_int64 * 3)(*[int(v) for v in lo])
        h3 = (c_int64 * 3)(*[int(v) for v in hi])
        check(lib.emg_amr_add_level(self.handle, l3, h3), "emg_amr_add_level")

    def amr_num_levels(self) -> int:
        n = c_int()
        check(lib.emg_amr_num_levels(self.handle, ctypes.byref(n)), "emg_amr_num_levels")
        return n.value

    def amr_level_shape(self, level):
        m = (c_int64 * 3)()
        check(lib.emg_amr_level_shape(self.handle, level, m), "emg_amr_level_shape")
        return tuple(int(x) for x in m)

    def amr_set_moduli(self, level, C):
        ptr, dev, keep = _host_or_device(C)
        check(lib.emg_amr_set_moduli(self.handle, level, ptr, dev), "emg_amr_set_moduli")

    def amr_set_eigenstrain(self, level, e):
        ptr, dev, keep = _host_or_device(e)
        check(lib.emg_amr_set_eigenstrain(self.handle, level, ptr, dev), "emg_amr_set_eigenstrain")

    def amr_set_body_force(self, level, b):
        ptr, dev, keep = _host_or_device(b)
        check(lib.emg_amr_set_body_force(self.handle, level, ptr, dev), "emg_amr_set_body_force")

    def amr_displacement(self, level, out=None):
        m = self.amr_level_shape(level)
        if out is not None:
            check(lib.emg_amr_get_displacement(self.handle, level, _dev(out), 1), "emg_amr_get_displacement")
            return out
        a = np.empty((self.dim, m[2], m[1], m[0]))
        check(lib.emg_amr_get_displacement(self.handle, level, a.ctypes.data_as(c_void_p), 0),
              "emg_amr_get_displacement")
        return a

    def amr_set_displacement(self, level, u):
        ptr, dev, keep = _host_or_device(u)
        check(lib.emg_amr_set_displacement(self.handle, level, ptr, dev), "emg_amr_set_displacement")

    def amr_residual(self, level, out):
        nrm = c_double()
        check(lib.emg_amr_residual(self.handle, level, _dev(out), ctypes.byref(nrm)), "emg_amr_residual")
        return nrm.value

    def kernel_time(self, kernel: int, level: int = 0, precision="fp64", reps: int = 20) -> float:
        ms = c_double()
        check(lib.emg_kernel_time(self.handle, kernel, level, _PREC[precision], reps, ctypes.byref(ms)),
              "emg_kernel_time")
        return ms.value

    def autotune(self, precision="fp64", reps: int = 10, retune: bool = False) -> int:
        """Measure the stencil-pass variants of this problem's levels and
        record the fastest process-wide (emg_autotune); returns the number of
        levels measured."""
        n = c_int()
        check(lib.emg_autotune(self.handle, _PREC[precision], reps, int(bool(retune)), ctypes.byref(n)),
              "emg_autotune")
        return n.value


def autotune_reset():
    """Empty the process-wide autotuner table (emg_autotune_reset)."""
    check(lib.emg_autotune_reset(), "emg_autotune_reset")


__all__ = ["lib", "LIB_PATH", "SYMBOLS", "Context", "Problem", "Server", "EmgError", "check", "default_opts", "solve_batch", "solve_batch_noalloc",
           "autotune_reset",
           "emg_domain", "emg_box", "emg_solve_opts", "emg_solve_stats", "emg_request", "emg_ticket_info",
           "EMG_OK", "EMG_EINVAL", "EMG_ENOMEM", "EMG_EDEVICE", "EMG_ENOTCONV", "EMG_EDIVERGED", "EMG_ESTATE", "EMG_EBUSY", "EMG_NOALLOC_SCRATCH_BYTES",
           "EMG_BC_DIRICHLET", "EMG_BC_TRACTION", "EMG_BC_PERIODIC", "EMG_BC_NEUMANN", "EMG_VCYCLE", "EMG_FCYCLE",
           "EMG_MOD_ISO", "EMG_MOD_ANISO",
           "EMG_FP64", "EMG_MIXED"] + list(SYMBOLS)
