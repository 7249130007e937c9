"""Python handle on the plain-C FP64 oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcteno_oracle.so")
SRC_PATH = os.path.join(HERE, "cteno_oracle.c")

PERIODIC, WALL, TRANSMISSIVE, INFLOW = 0, 1, 2, 3
ADVECTION, EULER = 0, 1
CTENO, CTENOZ, CWENO, TENO = 0, 1, 2, 3
GAMMA_PAPER, GAMMA_LAMBDA, GAMMA_SCALED = 0, 1, 2
CONSERVED, CHARACTERISTIC = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Scheme(C.Structure):
    _fields_ = [("physics", C.c_int), ("ax", C.c_double), ("ay", C.c_double), ("gamma", C.c_double),
                ("scheme", C.c_int), ("degree", C.c_int), ("gamma_form", C.c_int),
                ("lambda1_prime", C.c_double), ("c_t", C.c_double), ("eps", C.c_double),
                ("variables", C.c_int), ("positivity", C.c_int)]


class _Boundary(C.Structure):
    _fields_ = [("behind", C.c_double * 4), ("ahead", C.c_double * 4), ("line", C.c_double * 3),
                ("split_kind", C.c_int * 4), ("split_at", C.c_double * 4)]


def _boundary(b):
    """ctypes copy of an object with behind, ahead, line, split_kind and
    split_at (None: no inflow sides, no switches)."""
    if b is None:
        return None
    pad = lambda v, n: list(v) + [0.0] * (n - len(v))
    return _Boundary((C.c_double * 4)(*pad(b.behind, 4)), (C.c_double * 4)(*pad(b.ahead, 4)),
                     (C.c_double * 3)(*b.line), (C.c_int * 4)(*b.split_kind), (C.c_double * 4)(*b.split_at))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_create.restype = P
        L.or_create.argtypes = [C.c_int, P, C.c_int, P, P, P, C.POINTER(_Scheme), C.POINTER(_Boundary)]
        L.or_destroy.argtypes = [P]
        L.or_last_error.restype = C.c_char_p
        L.or_dims.argtypes = [P] + [C.POINTER(C.c_int)] * 6
        L.or_prepare.argtypes = [P]
        L.or_geometry.argtypes = [P, P, P, P, P, P]
        L.or_stencils.argtypes = [P, C.c_int, P, P, P, P]
        L.or_pinv.argtypes = [P, C.c_int, P, P, P]
        L.or_ls_matrix.argtypes = [P, C.c_int, P, P]
        L.or_smoothness.restype = C.c_double
        L.or_smoothness.argtypes = [P, P, C.c_int, C.c_int]
        L.or_select.argtypes = [P, P, P]
        L.or_char_vectors.argtypes = [C.c_double, P, C.c_double, C.c_double, P, P]
        L.or_cweno_weights.argtypes = [P, P, P, P]
        L.or_hllc.argtypes = [C.c_double, P, P, C.c_double, C.c_double, P]
        L.or_euler_flux.argtypes = [C.c_double, P, C.c_double, C.c_double, P]
        L.or_wall_flux.argtypes = [C.c_double, P, C.c_double, C.c_double, P]
        L.or_reconstruct.argtypes = [P, P, P, P, P, P]
        L.or_reconstruct_cells.argtypes = [P, P, C.c_int, P, P, P]
        L.or_face_fluxes.argtypes = [P, P, C.c_double, P]
        L.or_residual_cells.argtypes = [P, P, C.c_double, C.c_int, P, P]
        L.or_residual.argtypes = [P, P, C.c_double, P]
        L.or_dt_bound.restype = C.c_double
        L.or_dt_bound.argtypes = [P, P]
        L.or_rk3_step.argtypes = [P, P, C.c_double, C.c_double]
        L.or_solve.argtypes = [P, P, C.c_double, C.c_double, C.c_int, C.c_double,
                               C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_fallbacks.restype = C.c_longlong
        L.or_fallbacks.argtypes = [P]
        L.or_reset_fallbacks.argtypes = [P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    pass


class Oracle:
    """One mesh + scheme in the oracle.  Arrays follow the input cell order."""

    def __init__(self, xy, tri, box, bc, physics=EULER, scheme=CTENOZ, degree=3,
                 lambda1_prime=1e4, c_t=1e-6, eps=1e-12, gamma=1.4, ax=1.0, ay=1.0,
                 gamma_form=GAMMA_PAPER, variables=CONSERVED, boundary=None, positivity=0):
        L = lib()
        self._xy = np.ascontiguousarray(xy, dtype=np.float64)
        self._tri = np.ascontiguousarray(tri, dtype=np.int32)
        box = np.ascontiguousarray(box, dtype=np.float64)
        bc = np.ascontiguousarray(bc, dtype=np.int32)
        s = _Scheme(physics, ax, ay, gamma, scheme, degree, gamma_form, lambda1_prime, c_t, eps, variables,
                    int(bool(positivity)))
        bnd = _boundary(boundary)
        h = L.or_create(self._xy.shape[0], _p(self._xy), self._tri.shape[0], _p(self._tri), _p(box), _p(bc),
                        C.byref(s), C.byref(bnd) if bnd is not None else None)
        if not h:
            raise OracleError(L.or_last_error().decode())
        self.h = h
        self.N = int(self._tri.shape[0])
        d = [C.c_int() for _ in range(6)]
        L.or_dims(h, *[C.byref(x) for x in d])
        self.K, self.M, self.Kd, self.Md, self.Nq, self.nv = [x.value for x in d]
        self.physics, self.scheme, self.degree = physics, scheme, degree
        self.variables = variables
        # selection bytes: per variable, or per face and characteristic field
        self.dshape = (3, self.nv) if variables == CHARACTERISTIC else (self.nv,)

    @classmethod
    def from_mesh(cls, mesh, **kw):
        kw.setdefault("boundary", getattr(mesh, "boundary", None))
        return cls(mesh.xy, mesh.tri, mesh.box, mesh.bc, **kw)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().or_destroy(h)
            self.h = None

    def _check(self, rc):
        if rc:
            raise OracleError(f"{lib().or_last_error().decode()} [rc={rc}]")

    def prepare(self):
        self._check(lib().or_prepare(self.h))

    def geometry(self):
        N = self.N
        cxy = np.empty((N, 2)); area = np.empty(N)
        fnb = np.empty((N, 3), np.int32); fnbf = np.empty((N, 3), np.int32); fn = np.empty((N, 3, 3))
        lib().or_geometry(self.h, _p(cxy), _p(area), _p(fnb), _p(fnbf), _p(fn))
        return dict(centroid=cxy, area=area, nbr=fnb, nbr_face=fnbf, normal=fn[..., :2], length=fn[..., 2])

    def stencils(self, cells=None):
        cells = np.arange(self.N, dtype=np.int32) if cells is None else np.ascontiguousarray(cells, np.int32)
        n = cells.shape[0]
        cen = np.empty((n, self.M), np.int32)
        dr = np.empty((n, 3, self.Md), np.int32)
        dn = np.empty((n, 3), np.int32)
        self._check(lib().or_stencils(self.h, n, _p(cells), _p(cen), _p(dr), _p(dn)))
        return cen, dr, dn

    def pinv(self, cells):
        cells = np.ascontiguousarray(cells, np.int32)
        n = cells.shape[0]
        pc = np.empty((n, self.K, self.M))
        pd = np.empty((n, 3, self.Kd, self.Md))
        self._check(lib().or_pinv(self.h, n, _p(cells), _p(pc), _p(pd)))
        return pc, pd

    def ls_matrix(self, i):
        A = np.empty((self.K, self.M))
        w = np.empty(self.M)
        self._check(lib().or_ls_matrix(self.h, int(i), _p(A), _p(w)))
        return A.T.copy(), w

    def smoothness(self, a, r):
        a = np.ascontiguousarray(a, np.float64)
        return lib().or_smoothness(self.h, _p(a), a.shape[0], r)

    @staticmethod
    def char_vectors(U, nx, ny, gamma=1.4):
        """Right eigenvectors R (columns) of the Euler flux Jacobian along
        (nx, ny) at the conserved state U, and L = R^-1."""
        U = np.ascontiguousarray(U, np.float64)
        R = np.empty((4, 4)); Lm = np.empty((4, 4))
        if lib().or_char_vectors(gamma, _p(U), nx, ny, _p(R), _p(Lm)):
            raise OracleError("singular eigenvector matrix")
        return R, Lm

    def select(self, si, adm=(1, 1, 1, 1)):
        si = np.ascontiguousarray(si, np.float64)
        adm = np.ascontiguousarray(adm, np.int32)
        return lib().or_select(self.h, _p(si), _p(adm))

    def cweno_weights(self, si, adm=(1, 1, 1, 1)):
        si = np.ascontiguousarray(si, np.float64)
        adm = np.ascontiguousarray(adm, np.int32)
        w = np.empty(4)
        lib().or_cweno_weights(self.h, _p(si), _p(adm), _p(w))
        return w

    def reconstruct(self, U, forced=None, want_coef=False):
        U = np.ascontiguousarray(U, np.float64).reshape(self.nv, self.N)
        fv = np.empty((self.N, 3, self.Nq, self.nv))
        dl = np.empty((self.N,) + self.dshape, np.uint8)
        coef = np.empty((self.N, self.nv, self.K)) if want_coef else None
        f = None if forced is None else np.ascontiguousarray(forced, np.uint8)
        self._check(lib().or_reconstruct(self.h, _p(U), _p(f), _p(fv), _p(dl), _p(coef)))
        return (fv, dl, coef) if want_coef else (fv, dl)

    def reconstruct_cells(self, U, cells):
        U = np.ascontiguousarray(U, np.float64).reshape(self.nv, self.N)
        cells = np.ascontiguousarray(cells, np.int32)
        n = cells.shape[0]
        fv = np.empty((n, 3, self.Nq, self.nv))
        dl = np.empty((n,) + self.dshape, np.uint8)
        self._check(lib().or_reconstruct_cells(self.h, _p(U), n, _p(cells), _p(fv), _p(dl)))
        return fv, dl

    def residual_cells(self, U, cells, t=0.0):
        """Residual of selected cells only at time t (the time of inflow
        boundary states), R[n][nv] (reconstructs only what it needs)."""
        U = np.ascontiguousarray(U, np.float64).reshape(self.nv, self.N)
        cells = np.ascontiguousarray(cells, np.int32)
        R = np.empty((cells.shape[0], self.nv))
        self._check(lib().or_residual_cells(self.h, _p(U), float(t), cells.shape[0], _p(cells), _p(R)))
        return R

    def face_fluxes(self, fv, t=0.0):
        fv = np.ascontiguousarray(fv, np.float64)
        fo = np.empty((self.N, 3, self.nv))
        self._check(lib().or_face_fluxes(self.h, _p(fv), float(t), _p(fo)))
        return fo

    def residual(self, U, t=0.0):
        U = np.ascontiguousarray(U, np.float64).reshape(self.nv, self.N)
        R = np.empty((self.nv, self.N))
        self._check(lib().or_residual(self.h, _p(U), float(t), _p(R)))
        return R

    def fallbacks(self, reset=False):
        """cell reconstructions that took the positivity fallback (positivity=1)
        since creation or the last reset"""
        n = int(lib().or_fallbacks(self.h))
        if reset:
            lib().or_reset_fallbacks(self.h)
        return n

    def dt_bound(self, U):
        U = np.ascontiguousarray(U, np.float64).reshape(self.nv, self.N)
        return lib().or_dt_bound(self.h, _p(U))

    def rk3_step(self, U, dt, t=0.0):
        U = np.array(U, dtype=np.float64, order="C").reshape(self.nv, self.N)
        self._check(lib().or_rk3_step(self.h, _p(U), float(t), float(dt)))
        return U

    def solve(self, U, t_final, cfl=0.3, t0=0.0, max_steps=1 << 30):
        U = np.array(U, dtype=np.float64, order="C").reshape(self.nv, self.N)
        steps = C.c_int()
        t = C.c_double()
        self._check(lib().or_solve(self.h, _p(U), float(t0), float(t_final), int(max_steps), float(cfl),
                                   C.byref(steps), C.byref(t)))
        return U, steps.value, t.value


def hllc(UL, UR, n, gamma=1.4):
    UL = np.ascontiguousarray(UL, np.float64)
    UR = np.ascontiguousarray(UR, np.float64)
    F = np.empty(4)
    rc = lib().or_hllc(gamma, _p(UL), _p(UR), float(n[0]), float(n[1]), _p(F))
    if rc:
        raise OracleError("non-physical state")
    return F


def wall_flux(U, n, gamma=1.4):
    """HLLC flux through a wall (against the mirror image of U), written out
    with its zero contact speed."""
    U = np.ascontiguousarray(U, np.float64)
    F = np.empty(4)
    if lib().or_wall_flux(gamma, _p(U), float(n[0]), float(n[1]), _p(F)):
        raise OracleError("non-physical state")
    return F


def euler_flux(U, n, gamma=1.4):
    U = np.ascontiguousarray(U, np.float64)
    F = np.empty(4)
    lib().or_euler_flux(gamma, _p(U), float(n[0]), float(n[1]), _p(F))
    return F


def threads() -> int:
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of oracle contexts created afterwards (results are
    bitwise independent of the count)."""
    lib().or_set_threads.argtypes = [C.c_int]
    lib().or_set_threads(int(n))
