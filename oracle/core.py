"""ctypes binding of the FP64 C oracle (``mrt_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

NQ = 16
KINDS = {"periodic": 0, "dirichlet": 1, "reflect": 2, "extrapolate": 3, "wall": 4}
SIDES = ("west", "east", "south", "north")

_dp = C.POINTER(C.c_double)


class OrcSide(C.Structure):
    _fields_ = [
        ("kind_lo", C.c_int32), ("kind_hi", C.c_int32),
        ("state_lo", C.c_double * 4), ("state_hi", C.c_double * 4),
        ("split0", C.c_double), ("split_rate", C.c_double),
    ]


class OrcParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dt", C.c_double),
        ("s", C.c_double * NQ),
        ("side", OrcSide * 4),
    ]


class OrcModel(C.Structure):
    _fields_ = [("v", C.c_double * 32), ("M", C.c_double * 256), ("Minv", C.c_double * 256)]


_lib = None


def lib():
    """Load liboracle.so, compiling it first when it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        L = C.CDLL(build_oracle.LIB)
        P, M = C.POINTER(OrcParams), C.POINTER(OrcModel)
        L.orc_model_init.argtypes = [M]
        L.orc_model_init.restype = C.c_int
        L.orc_invert.argtypes = [C.c_int, _dp, _dp]
        L.orc_invert.restype = C.c_int
        L.orc_feq_moments.argtypes = [C.c_double] * 4 + [_dp]
        L.orc_feq_velocity.argtypes = [M] + [C.c_double] * 4 + [_dp]
        L.orc_moments.argtypes = [M, _dp, _dp]
        L.orc_macro_of.argtypes = [M, _dp, _dp]
        L.orc_collision.argtypes = [M, _dp, _dp, _dp]
        L.orc_cell_update.argtypes = [M, P] + [_dp] * 6
        L.orc_init_macro.argtypes = [M, P] + [_dp] * 5
        L.orc_read_macro.argtypes = [M, P] + [_dp] * 6
        L.orc_sums.argtypes = [M, P, _dp, _dp]
        L.orc_fill_ghosts.argtypes = [M, P, _dp, C.c_double]
        L.orc_face_outflow.argtypes = [M, P, _dp, _dp]
        L.orc_step.argtypes = [M, P, _dp, _dp, C.c_double, C.c_int, _dp]
        L.orc_run.argtypes = [M, P, _dp, _dp, C.c_int64, C.c_int64, C.c_int, _dp]
        _lib = L
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


class Model:
    """Velocity set (Eq. 4), M (Eq. 5) and the oracle's own inverse of M."""

    def __init__(self):
        self._m = OrcModel()
        if lib().orc_model_init(C.byref(self._m)) != 0:
            raise RuntimeError("oracle: M is singular")
        self.v = np.ctypeslib.as_array(self._m.v).reshape(NQ, 2).copy()
        self.M = np.ctypeslib.as_array(self._m.M).reshape(NQ, NQ).copy()
        self.Minv = np.ctypeslib.as_array(self._m.Minv).reshape(NQ, NQ).copy()

    @property
    def ref(self):
        return C.byref(self._m)


_model = None


def model() -> Model:
    global _model
    if _model is None:
        _model = Model()
    return _model


def invert(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    out = np.empty_like(A)
    if lib().orc_invert(n, _ptr(A), _ptr(out)) != 0:
        raise np.linalg.LinAlgError("oracle: singular matrix")
    return out


def feq_moments(rho, jx, jy, e):
    out = np.empty(NQ)
    lib().orc_feq_moments(rho, jx, jy, e, _ptr(out))
    return out


def feq_velocity(rho, ux, uy, T):
    out = np.empty(NQ)
    lib().orc_feq_velocity(model().ref, rho, ux, uy, T, _ptr(out))
    return out


def moments(f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(NQ)
    lib().orc_moments(model().ref, _ptr(f), _ptr(out))
    return out


def macro_of(f):
    """(rho, u1, u2, T, p) of one node's 16 populations."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(5)
    lib().orc_macro_of(model().ref, _ptr(f), _ptr(out))
    return out


def collision(f, s):
    f = np.ascontiguousarray(f, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    out = np.empty(NQ)
    lib().orc_collision(model().ref, _ptr(s), _ptr(f), _ptr(out))
    return out


def make_params(problem) -> OrcParams:
    """Translate a problem description (see the ``synth`` package) into the
    oracle's own parameter struct."""
    p = OrcParams()
    p.nx, p.ny = int(problem.nx), int(problem.ny)
    p.dx, p.dy, p.dt = float(problem.dx), float(problem.dy), float(problem.dt)
    for k in range(NQ):
        p.s[k] = float(problem.s[k])
    for k, name in enumerate(SIDES):
        sd = problem.sides[name]
        p.side[k].kind_lo = KINDS[sd["kind_lo"]]
        p.side[k].kind_hi = KINDS[sd["kind_hi"]]
        for q in range(4):
            p.side[k].state_lo[q] = float(sd["state_lo"][q])
            p.side[k].state_hi[q] = float(sd["state_hi"][q])
        p.side[k].split0 = float(sd["split0"])
        p.side[k].split_rate = float(sd["split_rate"])
    return p


def cell_update(problem, fc, fE, fW, fN, fS):
    p = make_params(problem)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (fc, fE, fW, fN, fS)]
    out = np.empty(NQ)
    lib().orc_cell_update(model().ref, C.byref(p), *[_ptr(a) for a in arrs], _ptr(out))
    return out


class Grid:
    """An nx*ny grid with one ghost layer; f is stored [ny+2][nx+2][16]."""

    def __init__(self, problem, nthreads: int = 1):
        self.problem = problem
        self.p = make_params(problem)
        self.nx, self.ny = self.p.nx, self.p.ny
        self.f = np.zeros((self.ny + 2, self.nx + 2, NQ))
        self.work = np.zeros_like(self.f)
        self.step_index = 0
        # ORACLE_MAX_THREADS caps the thread count where parallel test
        # workers share the host's cores; the results do not depend on it
        # (one static parallel loop over nodes per step)
        cap = os.environ.get("ORACLE_MAX_THREADS")
        self.nthreads = max(1, min(int(nthreads), int(cap))) if cap else int(nthreads)
        # outflow of (rho, j1, j2, e) node sums through west, east, south,
        # north since the last init_macro / set_f
        self.outflow = np.zeros((4, 4))

    @property
    def t(self):
        return self.step_index * self.p.dt

    def init_macro(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx)
                for a in (rho, ux, uy, T)]
        lib().orc_init_macro(model().ref, C.byref(self.p), *[_ptr(a) for a in arrs],
                             _ptr(self.f))
        self.step_index = 0
        self.outflow = np.zeros((4, 4))
        lib().orc_fill_ghosts(model().ref, C.byref(self.p), _ptr(self.f), 0.0)

    def init_problem(self):
        ic = self.problem.ic
        self.init_macro(ic["rho"], ic["ux"], ic["uy"], ic["T"])

    def set_f(self, f_packed):
        """Set the interior from a packed [16][ny][nx] array."""
        f_packed = np.asarray(f_packed, dtype=np.float64)
        self.f[1:-1, 1:-1, :] = np.moveaxis(f_packed, 0, -1)
        self.outflow = np.zeros((4, 4))
        lib().orc_fill_ghosts(model().ref, C.byref(self.p), _ptr(self.f), self.t)

    def get_f(self):
        """Interior as a packed [16][ny][nx] array."""
        return np.ascontiguousarray(np.moveaxis(self.f[1:-1, 1:-1, :], -1, 0))

    def run(self, nsteps: int):
        lib().orc_run(model().ref, C.byref(self.p), _ptr(self.f), _ptr(self.work),
                      self.step_index, int(nsteps), self.nthreads, _ptr(self.outflow))
        self.step_index += int(nsteps)

    def macro(self):
        """dict of rho, ux, uy, T, p as [ny][nx] arrays."""
        outs = [np.empty((self.ny, self.nx)) for _ in range(5)]
        lib().orc_read_macro(model().ref, C.byref(self.p), _ptr(self.f), *[_ptr(o) for o in outs])
        return dict(zip(("rho", "ux", "uy", "T", "p"), outs))

    def sums(self):
        out = np.empty(4)
        lib().orc_sums(model().ref, C.byref(self.p), _ptr(self.f), _ptr(out))
        return out
