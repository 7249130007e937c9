"""Thin ctypes binding of libcteno.so (the C ABI declared in include/cteno.h).

Argument marshalling only: every step of the finite-volume path runs in the
library's HIP kernels.  PyTorch provides device memory (torch tensors passed
as device pointers) and the stream.  Importing this module fails loudly when
the built library is missing.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcteno.so")

OK, ERR_INVALID, ERR_MESH, ERR_STENCIL, ERR_NOMEM, ERR_DEVICE, ERR_NONPHYSICAL, ERR_BUSY = range(8)
PERIODIC, WALL, TRANSMISSIVE, INFLOW = 0, 1, 2, 3
ADVECTION, EULER = 0, 1
CTENO, CTENOZ, CWENO, TENO = 0, 1, 2, 3
CONSERVED, CHARACTERISTIC = 0, 1
GAMMA_PAPER, GAMMA_LAMBDA, GAMMA_SCALED = 0, 1, 2
FP64, MIXED, BOTH = 1, 2, 3
KERNEL_RECONSTRUCT, KERNEL_FLUX, KERNEL_PRECOMPUTE = 0, 1, 2


class CtenoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[status {status}] {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xy", C.c_void_p), ("n_cells", C.c_int32), ("tri", C.c_void_p),
                ("box", C.c_double * 4), ("bc", C.c_int32 * 4),
                ("behind", C.c_double * 4), ("ahead", C.c_double * 4), ("line", C.c_double * 3),
                ("split_kind", C.c_int32 * 4), ("split_at", C.c_double * 4)]


def mesh_desc(xy, tri, box, bc, boundary=None) -> MeshDesc:
    """Descriptor of contiguous xy (float64) and tri (int32) arrays, which
    the caller keeps alive.  boundary: an object with behind, ahead, line,
    split_kind and split_at (prescribed inflow states and side switches), or
    None."""
    d = MeshDesc(xy.shape[0], _np_ptr(xy), tri.shape[0], _np_ptr(tri), (C.c_double * 4)(*box),
                 (C.c_int32 * 4)(*bc))
    if boundary is not None:
        pad = lambda v: list(v) + [0.0] * (4 - len(v))
        d.behind = (C.c_double * 4)(*pad(boundary.behind))
        d.ahead = (C.c_double * 4)(*pad(boundary.ahead))
        d.line = (C.c_double * 3)(*boundary.line)
        d.split_kind = (C.c_int32 * 4)(*boundary.split_kind)
        d.split_at = (C.c_double * 4)(*boundary.split_at)
    return d


class Scheme(C.Structure):
    _fields_ = [("physics", C.c_int32), ("ax", C.c_double), ("ay", C.c_double), ("gamma", C.c_double),
                ("scheme", C.c_int32), ("degree", C.c_int32), ("lambda1_prime", C.c_double), ("c_t", C.c_double),
                ("eps", C.c_double), ("gamma_form", C.c_int32), ("precision", C.c_int32), ("reorder", C.c_int32),
                ("variables", C.c_int32), ("positivity", C.c_int32)]


class MeshInfo(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_faces", C.c_int64), ("n_boundary_faces", C.c_int64),
                ("K", C.c_int32), ("M", C.c_int32), ("slots", C.c_int32), ("nv", C.c_int32), ("nq", C.c_int32),
                ("n_inadmissible", C.c_int32), ("Kd", C.c_int32), ("Md", C.c_int32), ("device_bytes", C.c_int64),
                ("n_cross_cells", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("finished", C.c_int64), ("active", C.c_int32), ("peak_active", C.c_int32),
                ("ticks", C.c_int64), ("cell_stages", C.c_int64), ("bytes_in_use", C.c_int64),
                ("peak_bytes", C.c_int64), ("budget_bytes", C.c_int64), ("fallbacks", C.c_int64)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("n_cells", C.c_int64), ("steps_done", C.c_int64),
                ("fallbacks", C.c_int64), ("latency_s", C.c_double), ("build_s", C.c_double),
                ("queue_s", C.c_double), ("admit_s", C.c_double), ("run_s", C.c_double)]


REQ_QUEUED, REQ_READY, REQ_RUNNING, REQ_DONE, REQ_FAILED = range(5)

_lib = None

# exported symbols and their argument types (restype is cteno_status unless listed)
_SIGS = {
    "cteno_ctx_create": [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)],
    "cteno_ctx_destroy": [C.c_void_p],
    "cteno_ctx_set_stream": [C.c_void_p, C.c_void_p],
    "cteno_ctx_synchronize": [C.c_void_p],
    "cteno_last_error": [],
    "cteno_ctx_set_timing": [C.c_void_p, C.c_int32],
    "cteno_ctx_set_fused_stage": [C.c_void_p, C.c_int32],
    "cteno_ctx_kernel_stats": [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)],
    "cteno_ctx_reset_stats": [C.c_void_p],
    "cteno_mesh_upload": [C.c_void_p, C.POINTER(MeshDesc), C.POINTER(Scheme), C.POINTER(C.c_void_p)],
    "cteno_mesh_info_get": [C.c_void_p, C.POINTER(MeshInfo)],
    "cteno_mesh_stencils": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "cteno_mesh_pinv": [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "cteno_mesh_destroy": [C.c_void_p],
    "cteno_stencils_host": [C.POINTER(MeshDesc), C.POINTER(Scheme), C.c_void_p, C.c_void_p, C.c_void_p],
    "cteno_sol_create": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_void_p)],
    "cteno_sol_set": [C.c_void_p, C.c_void_p, C.c_double],
    "cteno_sol_download": [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)],
    "cteno_sol_destroy": [C.c_void_p],
    "cteno_sol_fallbacks": [C.c_void_p, C.POINTER(C.c_int64)],
    "cteno_reconstruct": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "cteno_flux": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_void_p],
    "cteno_flux_noalloc": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_void_p],
    "cteno_residual": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "cteno_rk_stage": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_double],
    "cteno_solve": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int64, C.c_double, C.c_int32,
                    C.POINTER(C.c_int64)],
    "cteno_count_flips": [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)],
    "cteno_util_copy": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t],
    "cteno_server_create": [C.c_void_p, C.POINTER(Scheme), C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)],
    "cteno_server_submit": [C.c_void_p, C.POINTER(MeshDesc), C.c_void_p, C.c_int32, C.c_double,
                            C.POINTER(C.c_uint64)],
    "cteno_server_poll": [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.c_void_p, C.POINTER(C.c_int64),
                          C.POINTER(C.c_double)],
    "cteno_server_drain": [C.c_void_p],
    "cteno_server_get_stats": [C.c_void_p, C.c_void_p],
    "cteno_server_request_info": [C.c_void_p, C.c_uint64, C.POINTER(RequestInfo)],
    "cteno_server_destroy": [C.c_void_p],
}
_VOID = {"cteno_ctx_destroy", "cteno_mesh_destroy", "cteno_sol_destroy", "cteno_server_destroy"}


def lib():
    """Loads the built library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2312_17042_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None if name in _VOID else C.c_int
        L.cteno_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != OK:
        raise CtenoError(rc, lib().cteno_last_error().decode())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t):
    import torch
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return C.c_void_p(t.data_ptr())


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """Allocator hooks of cteno_ctx_create backed by torch's caching
    allocator, so that the library's device memory (meshes, states, serving
    slots) is accounted by torch.  Counts the calls it served."""

    def __init__(self, device: int, stream: int):
        import torch
        self.device = device
        self.stream = stream
        self.allocs = 0
        self.frees = 0

        def alloc(nbytes, user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:           # out of memory: the library reports CTENO_ERR_NOMEM
                return None
            self.allocs += 1
            return ptr

        def free(ptr, user):
            self.frees += 1
            torch.cuda.caching_allocator_delete(ptr)

        self.alloc_fn = _ALLOC_FN(alloc)
        self.free_fn = _FREE_FN(free)


# every open context, closed (children first) before the interpreter shuts
# down, while the HIP runtime and torch are still whole
_live_contexts = weakref.WeakSet()


def _close_all():
    for ctx in list(_live_contexts):
        ctx.close()


atexit.register(_close_all)


class Context:
    """A library context on one device.  allocator="torch" (default) routes
    every device allocation of the library through torch's caching
    allocator; None uses hipMalloc."""

    def __init__(self, device: int = 0, stream=None, allocator: str | None = "torch"):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.allocator = TorchAllocator(device, stream) if allocator == "torch" else None
        a = self.allocator
        h = C.c_void_p()
        _check(lib().cteno_ctx_create(device, C.c_void_p(stream), a.alloc_fn if a else None,
                                      a.free_fn if a else None, None, C.byref(h)))
        self.h = h
        self.device = device
        self._children = weakref.WeakSet()   # servers, meshes and solutions, closed before the context
        _live_contexts.add(self)

    def close(self):
        """Destroys the children (servers, solutions, then meshes) and the
        context; idempotent."""
        if getattr(self, "h", None):
            rank = {Server: 0, Solution: 1, Mesh: 2}
            for ch in sorted(list(self._children), key=lambda o: rank.get(type(o), 3)):
                ch.close()
            lib().cteno_ctx_destroy(self.h)
            self.h = None
        _live_contexts.discard(self)

    def __del__(self, _is_finalizing=sys.is_finalizing):
        # (the default argument keeps the check reachable once interpreter
        # shutdown has cleared this module's globals; the exit handler has
        # closed every live handle by then)
        if getattr(self, "h", None) and not _is_finalizing():
            self.close()

    def synchronize(self):
        _check(lib().cteno_ctx_synchronize(self.h))

    def set_timing(self, on: bool):
        _check(lib().cteno_ctx_set_timing(self.h, int(bool(on))))

    def set_fused_stage(self, on: bool):
        """degree <= 3 RK stages: fused kernels (default) or reconstruction + flux"""
        _check(lib().cteno_ctx_set_fused_stage(self.h, int(bool(on))))

    def kernel_stats(self, kernel: int):
        n = C.c_int64()
        ms = C.c_double()
        _check(lib().cteno_ctx_kernel_stats(self.h, kernel, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def reset_stats(self):
        _check(lib().cteno_ctx_reset_stats(self.h))

    def copy(self, dst, src, nbytes: int):
        _check(lib().cteno_util_copy(self.h, _dev_ptr(dst), _dev_ptr(src), int(nbytes)))


def make_scheme(physics=EULER, scheme=CTENOZ, degree=3, lambda1_prime=1e4, c_t=1e-6, eps=1e-12, gamma=1.4,
                ax=1.0, ay=1.0, gamma_form=GAMMA_PAPER, precision=FP64, reorder=1, variables=0,
                positivity=0) -> Scheme:
    return Scheme(physics, ax, ay, gamma, scheme, degree, lambda1_prime, c_t, eps, gamma_form, precision, reorder,
                  variables, positivity)


class Mesh:
    def __init__(self, ctx: Context, xy, tri, box, bc, scheme: Scheme, boundary=None):
        self.ctx = ctx
        self._xy = np.ascontiguousarray(xy, np.float64)
        self._tri = np.ascontiguousarray(tri, np.int32)
        d = mesh_desc(self._xy, self._tri, box, bc, boundary)
        h = C.c_void_p()
        _check(lib().cteno_mesh_upload(ctx.h, C.byref(d), C.byref(scheme), C.byref(h)))
        self.h = h
        self._sols = weakref.WeakSet()
        ctx._children.add(self)
        self.scheme = scheme
        info = MeshInfo()
        _check(lib().cteno_mesh_info_get(h, C.byref(info)))
        self.info = info
        self.N = int(info.n_cells)
        self.nv = int(info.nv)
        self.K = int(info.K)
        self.M = int(info.M)
        self.nq = int(info.nq)
        self.Kd = int(info.Kd)
        self.Md = int(info.Md)

    @classmethod
    def from_workload(cls, ctx, mesh, **scheme_kw):
        return cls(ctx, mesh.xy, mesh.tri, mesh.box, mesh.bc, make_scheme(**scheme_kw),
                   getattr(mesh, "boundary", None))

    def close(self):
        if getattr(self, "h", None):
            for sol in list(self._sols):
                sol.close()
            if self.ctx.h:
                lib().cteno_mesh_destroy(self.h)
            self.h = None

    def __del__(self, _is_finalizing=sys.is_finalizing):
        # (the default argument keeps the check reachable once interpreter
        # shutdown has cleared this module's globals; the exit handler has
        # closed every live handle by then)
        if getattr(self, "h", None) and not _is_finalizing():
            self.close()

    def stencils(self):
        cen = np.empty((self.N, self.M), np.int32)
        dr = np.empty((self.N, 3, self.Md), np.int32)
        dn = np.empty((self.N, 3), np.int32)
        _check(lib().cteno_mesh_stencils(self.h, _np_ptr(cen), _np_ptr(dr), _np_ptr(dn)))
        return cen, dr, dn

    def pinv(self, cells, which=FP64):
        cells = np.ascontiguousarray(cells, np.int32)
        n = cells.shape[0]
        pc = np.empty((n, self.K, self.M))
        pd = np.empty((n, 3, self.Kd, self.Md))
        _check(lib().cteno_mesh_pinv(self.ctx.h, self.h, which, n, _np_ptr(cells), _np_ptr(pc), _np_ptr(pd)))
        return pc, pd


def stencils_host(xy, tri, box, bc, scheme: Scheme, boundary=None):
    """Host-only stencil construction (no GPU needed)."""
    xy = np.ascontiguousarray(xy, np.float64)
    tri = np.ascontiguousarray(tri, np.int32)
    d = mesh_desc(xy, tri, box, bc, boundary)
    N = tri.shape[0]
    r = scheme.degree
    K = (r + 1) * (r + 2) // 2 - 1
    rd = 1 if r <= 3 else (r + 1) // 2
    Md = 2 * ((rd + 1) * (rd + 2) // 2 - 1)
    cen = np.empty((N, 2 * K), np.int32)
    dr = np.empty((N, 3, Md), np.int32)
    dn = np.empty((N, 3), np.int32)
    _check(lib().cteno_stencils_host(C.byref(d), C.byref(scheme), _np_ptr(cen), _np_ptr(dr), _np_ptr(dn)))
    return cen, dr, dn


class Solution:
    def __init__(self, mesh: Mesh, u0, t0: float = 0.0):
        self.mesh = mesh
        self.ctx = mesh.ctx
        u0 = np.ascontiguousarray(u0, np.float64).reshape(mesh.nv, mesh.N)
        h = C.c_void_p()
        _check(lib().cteno_sol_create(self.ctx.h, mesh.h, _np_ptr(u0), float(t0), C.byref(h)))
        self.h = h
        mesh._sols.add(self)
        self.ctx._children.add(self)

    def close(self):
        if getattr(self, "h", None):
            if self.ctx.h and self.mesh.h:
                lib().cteno_sol_destroy(self.h)
            self.h = None

    def __del__(self, _is_finalizing=sys.is_finalizing):
        # (the default argument keeps the check reachable once interpreter
        # shutdown has cleared this module's globals; the exit handler has
        # closed every live handle by then)
        if getattr(self, "h", None) and not _is_finalizing():
            self.close()

    def set(self, u, t=0.0):
        u = np.ascontiguousarray(u, np.float64).reshape(self.mesh.nv, self.mesh.N)
        _check(lib().cteno_sol_set(self.h, _np_ptr(u), float(t)))

    def download(self):
        u = np.empty((self.mesh.nv, self.mesh.N))
        t = C.c_double()
        _check(lib().cteno_sol_download(self.h, _np_ptr(u), C.byref(t)))
        return u, t.value

    # ---- stage calls (torch device buffers) ----
    def reconstruct(self, precision=FP64, forced=None, want_delta=True):
        import torch
        m = self.mesh
        dt = torch.float64 if precision == FP64 else torch.float32
        fv = torch.empty((m.N, 3, m.nq, m.nv), dtype=dt, device=f"cuda:{self.ctx.device}")
        dshape = (m.N, 3, m.nv) if m.scheme.variables == CHARACTERISTIC else (m.N, m.nv)
        dl = torch.empty(dshape, dtype=torch.uint8, device=fv.device) if want_delta else None
        fr = None
        if forced is not None:
            fr = torch.as_tensor(np.ascontiguousarray(forced, np.uint8)).to(fv.device)
        torch.cuda.synchronize()
        _check(lib().cteno_reconstruct(self.ctx.h, m.h, self.h, precision, _dev_ptr(fv),
                                       _dev_ptr(dl) if dl is not None else None,
                                       _dev_ptr(fr) if fr is not None else None))
        return fv, dl

    def residual(self, precision=FP64):
        import torch
        m = self.mesh
        r = torch.empty((m.nv, m.N), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        torch.cuda.synchronize()
        _check(lib().cteno_residual(self.ctx.h, m.h, self.h, precision, _dev_ptr(r)))
        return r

    def rk_stage(self, stage: int, dt: float, precision=FP64):
        _check(lib().cteno_rk_stage(self.ctx.h, self.mesh.h, self.h, precision, int(stage), float(dt)))

    def solve(self, t_final=float("inf"), max_steps=(1 << 62), cfl=0.3, precision=FP64, use_graph=True):
        n = C.c_int64()
        _check(lib().cteno_solve(self.ctx.h, self.mesh.h, self.h, precision, float(t_final), int(max_steps),
                                 float(cfl), int(bool(use_graph)), C.byref(n)))
        return n.value

    def count_flips(self):
        n = C.c_int64()
        _check(lib().cteno_count_flips(self.ctx.h, self.mesh.h, self.h, C.byref(n)))
        return n.value

    def fallbacks(self):
        """cells x stages that took the positivity fallback since create / set"""
        n = C.c_int64()
        _check(lib().cteno_sol_fallbacks(self.h, C.byref(n)))
        return n.value


def flux(mesh: Mesh, face_vals, precision=FP64, t=0.0, out=None, noalloc=False):
    """Outward face fluxes times |A_f|; t is the time of prescribed inflow
    states.  noalloc=True calls cteno_flux_noalloc (staging in the library's
    fixed device scratch); out: a preallocated [N][3][nv] tensor."""
    import torch
    dt = torch.float64 if precision == FP64 else torch.float32
    fo = torch.empty((mesh.N, 3, mesh.nv), dtype=dt, device=face_vals.device) if out is None else out
    torch.cuda.synchronize()
    fn = lib().cteno_flux_noalloc if noalloc else lib().cteno_flux
    _check(fn(mesh.ctx.h, mesh.h, precision, _dev_ptr(face_vals.contiguous()), float(t), _dev_ptr(fo)))
    return fo


class Server:
    """Continuous-batching server of independent 2-D Euler solves (FP32-mixed)."""

    def __init__(self, ctx: Context, scheme: Scheme, budget_bytes: int, max_slots: int = 64):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().cteno_server_create(ctx.h, C.byref(scheme), int(budget_bytes), int(max_slots), C.byref(h)))
        self.h = h
        self._cells = {}
        ctx._children.add(self)

    def close(self):
        if getattr(self, "h", None):
            if self.ctx.h:
                lib().cteno_server_destroy(self.h)
            self.h = None

    def __del__(self, _is_finalizing=sys.is_finalizing):
        # (the default argument keeps the check reachable once interpreter
        # shutdown has cleared this module's globals; the exit handler has
        # closed every live handle by then)
        if getattr(self, "h", None) and not _is_finalizing():
            self.close()

    def submit(self, mesh, u0, n_steps: int, cfl: float = 0.3) -> int:
        xy = np.ascontiguousarray(mesh.xy, np.float64)
        tri = np.ascontiguousarray(mesh.tri, np.int32)
        u0 = np.ascontiguousarray(u0, np.float64).reshape(4, tri.shape[0])
        d = mesh_desc(xy, tri, mesh.box, mesh.bc, getattr(mesh, "boundary", None))
        t = C.c_uint64()
        _check(lib().cteno_server_submit(self.h, C.byref(d), _np_ptr(u0), int(n_steps), float(cfl), C.byref(t)))
        self._cells[t.value] = tri.shape[0]
        return t.value

    def poll(self, ticket: int, take: bool = False):
        """(state, result or None, steps, latency_s).  take=True fetches and releases a finished result."""
        st = C.c_int32()
        steps = C.c_int64()
        lat = C.c_double()
        out = np.empty((4, self._cells[ticket])) if take else None
        rc = lib().cteno_server_poll(self.h, int(ticket), C.byref(st), _np_ptr(out) if take else None,
                                     C.byref(steps), C.byref(lat))
        if rc != OK:
            if take:
                self._cells.pop(ticket, None)
            raise CtenoError(rc, lib().cteno_last_error().decode())
        done = st.value == REQ_DONE
        if take and done:
            self._cells.pop(ticket, None)
        return st.value, (out if (take and done) else None), steps.value, lat.value

    def drain(self):
        _check(lib().cteno_server_drain(self.h))

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().cteno_server_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def info(self, ticket: int) -> dict:
        """state, counts and latency split (build, queue, admit, run) of an unreleased request"""
        r = RequestInfo()
        _check(lib().cteno_server_request_info(self.h, int(ticket), C.byref(r)))
        return {f: getattr(r, f) for f, _ in RequestInfo._fields_}
