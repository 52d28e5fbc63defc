"""Thin Python front end of libmrtfd: torch provides device memory and the
stream; every step of the computation runs in the library's HIP kernels."""
import ctypes as C
import math

import numpy as np

from . import _abi
from ._abi import check, lib

SIDES = ("west", "east", "south", "north")
KERNELS = {"auto": _abi.MRTFD_KERNEL_AUTO, "simple": _abi.MRTFD_KERNEL_SIMPLE,
           "rows": _abi.MRTFD_KERNEL_ROWS}
KERNEL_NAMES = {_abi.MRTFD_KERNEL_SIMPLE: "simple", _abi.MRTFD_KERNEL_ROWS: "rows",
                _abi.MRTFD_KERNEL_MFMA: "mfma"}
PRECISIONS = {"fp32": _abi.MRTFD_FP32, "bf16x3": _abi.MRTFD_BF16X3, "fp64": _abi.MRTFD_FP64}


COLLISIONS = {"mrt": _abi.MRTFD_COLLISION_MRT, "srt": _abi.MRTFD_COLLISION_SRT}


LAYOUTS = {"rows": _abi.MRTFD_LAYOUT_ROWS, "planes": _abi.MRTFD_LAYOUT_PLANES,
           "tiles": _abi.MRTFD_LAYOUT_TILES}


def make_params(nx, ny, dx, dy, dt, s, sides, precision="fp32", kernel="auto", rows=0,
                graph_steps=0, collision="mrt", layout="rows", flux_budget=False, ref=None):
    """Fill the C parameter struct.  sides: dict west/east/south/north of
    dicts with kind_lo, kind_hi (rule names), state_lo, state_hi
    (rho, u1, u2, T), split0, split_rate.  ref: (rho0, T0) of the reference
    state at rest whose equilibrium the library subtracts from the stored
    populations, or None."""
    p = _abi.mrtfd_params()
    p.nx, p.ny = int(nx), int(ny)
    p.dx, p.dy, p.dt = float(dx), float(dy), float(dt)
    if len(s) != 16:
        raise ValueError("s must hold the 16 rates s_1..s_16")
    for k in range(16):
        p.s[k] = float(s[k])
    for k, name in enumerate(SIDES):
        sd = sides[name]
        p.side[k].kind_lo = _abi.BC_KINDS[sd["kind_lo"]]
        p.side[k].kind_hi = _abi.BC_KINDS[sd["kind_hi"]]
        for q in range(4):
            p.side[k].state_lo[q] = float(sd["state_lo"][q])
            p.side[k].state_hi[q] = float(sd["state_hi"][q])
        p.side[k].split0 = float(sd.get("split0", math.inf))
        p.side[k].split_rate = float(sd.get("split_rate", 0.0))
    p.precision = PRECISIONS[precision]
    p.kernel = KERNELS[kernel]
    p.rows = int(rows)
    p.graph_steps = int(graph_steps)
    p.collision = COLLISIONS[collision]
    p.layout = LAYOUTS[layout]
    p.flux_budget = 1 if flux_budget else 0
    if ref is not None:
        p.ref_rho, p.ref_T = float(ref[0]), float(ref[1])
    return p


def ref_populations(p):
    """f_ref (FP64, 16 values) of a parameter struct; zeros without a
    reference state."""
    out = (C.c_double * 16)()
    st = lib().mrtfd_ref_populations(C.byref(p), out)
    if st != _abi.MRTFD_OK:
        raise _abi.MrtfdError(st, "ref_populations")
    return np.array(out[:])


def check_params(p):
    """(status, message) of the library's validation; needs no GPU."""
    buf = C.create_string_buffer(256)
    st = lib().mrtfd_check_params(C.byref(p), buf, len(buf))
    return st, buf.value.decode()


class MRT2D:
    """One 2D grid on one GPU."""

    def __init__(self, nx, ny, dx, dy, dt, s, sides, precision="fp32", kernel="auto",
                 rows=0, graph_steps=0, collision="mrt", layout="rows", flux_budget=False,
                 ref=None, device=None, stream=None):
        import torch

        self.torch = torch
        self.p = make_params(nx, ny, dx, dy, dt, s, sides, precision, kernel, rows, graph_steps,
                             collision, layout, flux_budget, ref)
        st, msg = check_params(self.p)
        if st != _abi.MRTFD_OK:
            raise _abi.MrtfdError(st, msg)
        self.nx, self.ny = int(nx), int(ny)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = lib().mrtfd_workspace_bytes(C.byref(self.p))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().mrtfd_create(C.byref(self.p), C.c_void_p(self.workspace.data_ptr()), nbytes,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx)))
        self._keep = []

    @classmethod
    def from_problem(cls, problem, **kw):
        """Build from any object with nx, ny, dx, dy, dt, s and sides
        attributes (the seeded problem descriptions used by tests/bench)."""
        return cls(problem.nx, problem.ny, problem.dx, problem.dy, problem.dt, problem.s,
                   problem.sides, **kw)

    # ------------------------------------------------------------ helpers
    def _dev(self, a):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
        a = a.to(device=self.device, dtype=t.float32).contiguous()
        return a

    def _ptr(self, a):
        return C.c_void_p(a.data_ptr()) if a is not None else None

    # ------------------------------------------------------------- C ABI
    def init_macro(self, rho, ux, uy, T):
        arrs = [self._dev(a).reshape(self.ny, self.nx) for a in (rho, ux, uy, T)]
        self._keep = arrs
        check(lib().mrtfd_init_macro(self._ctx, *[self._ptr(a) for a in arrs]), self._ctx)

    def init_problem(self, problem):
        ic = problem.ic
        self.init_macro(ic["rho"], ic["ux"], ic["uy"], ic["T"])

    def step(self, nsteps=1):
        check(lib().mrtfd_step(self._ctx, int(nsteps)), self._ctx)

    def read_macro(self):
        t = self.torch
        out = {k: t.empty((self.ny, self.nx), dtype=t.float32, device=self.device)
               for k in ("rho", "ux", "uy", "T", "p")}
        check(lib().mrtfd_read_macro(self._ctx, *[self._ptr(out[k]) for k in ("rho", "ux", "uy", "T", "p")]),
              self._ctx)
        return out

    def macro_numpy(self):
        out = self.read_macro()
        self.stream.synchronize()
        return {k: v.cpu().numpy().astype(np.float64) for k, v in out.items()}

    def sums(self):
        out = (C.c_double * 4)()
        check(lib().mrtfd_sums(self._ctx, out), self._ctx)
        return np.array(out[:])

    def outflow(self):
        """[side][k] FP64 outflow of (rho, j1, j2, e) through west, east,
        south, north since the last init / set_f (needs flux_budget=True)."""
        out = (C.c_double * 16)()
        check(lib().mrtfd_outflow(self._ctx, out), self._ctx)
        return np.array(out[:]).reshape(4, 4)

    def get_f(self):
        t = self.torch
        f = t.empty((16, self.ny, self.nx), dtype=t.float32, device=self.device)
        check(lib().mrtfd_get_f(self._ctx, self._ptr(f)), self._ctx)
        return f

    def get_f_numpy(self):
        """The stored populations (g = f - f_ref with a reference state)."""
        f = self.get_f()
        self.stream.synchronize()
        return f.cpu().numpy()

    def get_f64(self):
        """The stored values as a device FP64 tensor (exact in the FP64 mode)."""
        t = self.torch
        f = t.empty((16, self.ny, self.nx), dtype=t.float64, device=self.device)
        check(lib().mrtfd_get_f64(self._ctx, self._ptr(f)), self._ctx)
        return f

    def get_f64_numpy(self):
        f = self.get_f64()
        self.stream.synchronize()
        return f.cpu().numpy()

    def set_f64(self, f):
        t = self.torch
        if isinstance(f, np.ndarray):
            f = t.from_numpy(np.ascontiguousarray(f, dtype=np.float64))
        a = f.to(device=self.device, dtype=t.float64).contiguous().reshape(16, self.ny, self.nx)
        self._keep = [a]
        check(lib().mrtfd_set_f64(self._ctx, self._ptr(a)), self._ctx)

    def ref_populations(self):
        return ref_populations(self.p)

    def populations_numpy(self):
        """f = g + f_ref in FP64, [16][ny][nx]."""
        return self.get_f64_numpy() + self.ref_populations()[:, None, None]

    def set_f(self, f):
        a = self._dev(f).reshape(16, self.ny, self.nx)
        self._keep = [a]
        check(lib().mrtfd_set_f(self._ctx, self._ptr(a)), self._ctx)

    def time(self):
        step = C.c_int64()
        t = C.c_double()
        check(lib().mrtfd_time(self._ctx, C.byref(step), C.byref(t)), self._ctx)
        return step.value, t.value

    def set_step(self, step):
        check(lib().mrtfd_set_step(self._ctx, int(step)), self._ctx)

    def kernel_info(self):
        """(kernel name, rows per wave) of the step kernel in use."""
        return self.kernel_details()[:2]

    def kernel_details(self):
        """(kernel name, rows per wave, streaming stores) of the step kernel."""
        return self.kernel_variant()[:3]

    def kernel_variant(self):
        """(kernel name, rows per wave, streaming stores, tile order)."""
        k, s, st, o = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().mrtfd_kernel_info(self._ctx, C.byref(k), C.byref(s), C.byref(st), C.byref(o)),
              self._ctx)
        return KERNEL_NAMES.get(k.value, "none"), s.value, bool(st.value), o.value

    def close(self):
        if self._ctx:
            lib().mrtfd_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TubeBatch:
    """Many independent shock tubes (4 rows, periodic in y, f^eq of the end
    states beyond both ends) advanced together, each to its own step count."""

    ROWS = 4

    def __init__(self, n, steps, left, right, dx, dt, s, seg_cols=0, round_steps=0,
                 use_graph=False, device=None, stream=None):
        import torch

        self.torch = torch
        self.n = [int(v) for v in n]
        nt = len(self.n)
        p = _abi.mrtfd_batch_params()
        p.ntubes = nt
        p.dx, p.dt = float(dx), float(dt)
        for k in range(16):
            p.s[k] = float(s[k])
        p.seg_cols, p.round_steps, p.use_graph = int(seg_cols), int(round_steps), int(bool(use_graph))
        self.p = p
        self._n = (C.c_int32 * nt)(*self.n)
        self._steps = (C.c_int64 * nt)(*[int(v) for v in steps])
        lf = np.ascontiguousarray(left, dtype=np.float64).reshape(nt, 4)
        rt = np.ascontiguousarray(right, dtype=np.float64).reshape(nt, 4)
        self._left = (C.c_double * (4 * nt))(*lf.ravel().tolist())
        self._right = (C.c_double * (4 * nt))(*rt.ravel().tolist())
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = lib().mrtfd_batch_workspace_bytes(C.byref(p), self._n)
        if nbytes == 0:
            raise _abi.MrtfdError(_abi.MRTFD_ERR_ARG, "invalid batch parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._b = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().mrtfd_batch_create(C.byref(p), self._n, self._steps, self._left, self._right,
                                           C.c_void_p(self.workspace.data_ptr()), nbytes,
                                           C.c_void_p(self.stream.cuda_stream), C.byref(self._b)))

    @classmethod
    def from_description(cls, batch, **kw):
        """From a dict with tubes (n, left, right as (rho, u, p), steps), dx,
        dt, s -- the seeded batch descriptions used by tests and bench."""
        left = [(r, u, 0.0, p / r) for (r, u, p) in (t["left"] for t in batch["tubes"])]
        right = [(r, u, 0.0, p / r) for (r, u, p) in (t["right"] for t in batch["tubes"])]
        return cls([t["n"] for t in batch["tubes"]], [t["steps"] for t in batch["tubes"]], left, right,
                   batch["dx"], batch["dt"], batch["s"], **kw)

    def init(self):
        check(lib().mrtfd_batch_init(self._b), batch=self._b)

    def run(self):
        check(lib().mrtfd_batch_run(self._b), batch=self._b)

    def info(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().mrtfd_batch_info(self._b, C.byref(a), C.byref(b), C.byref(c)), batch=self._b)
        return a.value, b.value, c.value

    def read_macro(self, k):
        t = self.torch
        out = {key: t.empty((self.ROWS, self.n[k]), dtype=t.float32, device=self.device)
               for key in ("rho", "ux", "uy", "T", "p")}
        check(lib().mrtfd_batch_read_macro(self._b, int(k), *[C.c_void_p(out[key].data_ptr())
                                                             for key in ("rho", "ux", "uy", "T", "p")]),
              batch=self._b)
        return out

    def macro_numpy(self, k):
        out = self.read_macro(k)
        self.stream.synchronize()
        return {key: v.cpu().numpy().astype(np.float64) for key, v in out.items()}

    def get_f_numpy(self, k):
        t = self.torch
        f = t.empty((16, self.ROWS, self.n[k]), dtype=t.float32, device=self.device)
        check(lib().mrtfd_batch_get_f(self._b, int(k), C.c_void_p(f.data_ptr())), batch=self._b)
        self.stream.synchronize()
        return f.cpu().numpy()

    def close(self):
        if self._b:
            lib().mrtfd_batch_destroy(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
