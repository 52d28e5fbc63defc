"""Von Neumann screen of Sect. IV on the GPU: the eigenvalues of the
amplification matrix of one Fourier mode around a uniform state, per phase
pair (mrtfd_screen in include/mrtfd.h), and max |omega| for many parameter
sets at once (mrtfd_screen_sets).  Argument marshalling, plus a bisection
over the time step that calls the screen (largest_stable_dt); the screen's
arithmetic runs in the library's kernels."""
import ctypes as C
import math

import numpy as np

from ._abi import check, lib
from .solver import make_params

_PERIODIC = {"kind_lo": "periodic", "kind_hi": "periodic", "state_lo": (1.0, 0.0, 0.0, 1.0),
             "state_hi": (1.0, 0.0, 0.0, 1.0), "split0": math.inf, "split_rate": 0.0}


def screen_into(state, s, dx, dy, dt, d_theta, d_rho=None, d_eig=None, stream=None):
    """Enqueue the screen on torch device tensors without synchronising:
    d_theta (n, 2) float64 phase pairs, d_rho (n,) and/or d_eig (n, 16, 2)
    float64 outputs; stream = a torch stream (default: the current one)."""
    import torch

    n = int(d_theta.shape[0])
    for t in (d_theta, d_rho, d_eig):
        assert t is None or (t.dtype == torch.float64 and t.is_contiguous() and t.is_cuda)
    p = make_params(3, 3, dx, dy, dt, s, {k: dict(_PERIODIC) for k in ("west", "east", "south", "north")})
    st = (C.c_double * 4)(*[float(v) for v in state])
    stream = stream if stream is not None else torch.cuda.current_stream(d_theta.device)
    check(lib().mrtfd_screen(C.byref(p), st, C.c_void_p(d_theta.data_ptr()), n,
                             C.c_void_p(d_eig.data_ptr() if d_eig is not None else 0),
                             C.c_void_p(d_rho.data_ptr() if d_rho is not None else 0),
                             C.c_void_p(stream.cuda_stream)))


def _screen(state, s, dx, dy, dt, theta, device, want_eig):
    import torch

    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, 2))
    n = th.shape[0]
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    d_th = torch.from_numpy(th).to(dev)
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    eig = torch.empty((n, 16, 2), dtype=torch.float64, device=dev) if want_eig else None
    stream = torch.cuda.current_stream(dev)
    screen_into(state, s, dx, dy, dt, d_th, rho, eig, stream)
    stream.synchronize()
    r = rho.cpu().numpy()
    if not want_eig:
        return r
    e = eig.cpu().numpy()
    return e[..., 0] + 1j * e[..., 1], r


def eigenvalues(state, s, dx, dy, dt, theta, device=None):
    """The 16 eigenvalues omega of G, largest modulus first, for each phase
    pair theta[p] = (k_x dx, k_y dy) of an (n, 2) array; state = (rho, u1,
    u2, T), s = the 16 rates.  Returns an (n, 16) complex array."""
    return _screen(state, s, dx, dy, dt, theta, device, True)[0]


def spectral_radius(state, s, dx, dy, dt, theta, device=None):
    """max |omega| of G for each phase pair (as eigenvalues()): an array of n
    values."""
    return _screen(state, s, dx, dy, dt, theta, device, False)


def screen_sets(states, rates, dx, dy, dt, theta, per_phase=False, device=None):
    """max |omega| over the phase pairs theta (an (n, 2) array) for each of
    many parameter sets: states (nsets, 4) = (rho, u1, u2, T), rates (nsets,
    16); numpy arrays or torch tensors.  Returns the (nsets,) maxima as a
    numpy array, and with per_phase=True also the (nsets, n) values."""
    import torch

    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)

    def on_dev(x, cols):
        t = x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
        return t.to(device=dev, dtype=torch.float64).reshape(-1, cols).contiguous()

    d_st, d_s, d_th = on_dev(states, 4), on_dev(rates, 16), on_dev(theta, 2)
    nsets, n = d_st.shape[0], d_th.shape[0]
    if d_s.shape[0] != nsets:
        raise ValueError(f"{nsets} states but {d_s.shape[0]} rate sets")
    d_max = torch.empty(nsets, dtype=torch.float64, device=dev)
    d_rho = torch.empty((nsets, n), dtype=torch.float64, device=dev) if per_phase else None
    p = make_params(3, 3, dx, dy, dt, [0.0] * 16, {k: dict(_PERIODIC) for k in ("west", "east", "south", "north")})
    stream = torch.cuda.current_stream(dev)
    check(lib().mrtfd_screen_sets(C.byref(p), nsets, C.c_void_p(d_st.data_ptr()), C.c_void_p(d_s.data_ptr()),
                                  C.c_void_p(d_th.data_ptr()), n,
                                  C.c_void_p(d_rho.data_ptr() if per_phase else 0), C.c_void_p(d_max.data_ptr()),
                                  C.c_void_p(stream.cuda_stream)))
    stream.synchronize()
    if per_phase:
        return d_max.cpu().numpy(), d_rho.cpu().numpy()
    return d_max.cpu().numpy()


def largest_stable_dt(states, rates, dx, dy, dt_lo, dt_hi, n=16, tol=1e-9, rel=1e-3, device=None):
    """Bisection for the largest time step in [dt_lo, dt_hi] at which every
    state (rows of `states`, (rho, u1, u2, T)) with the 16 `rates` has max
    |omega| <= 1 + tol over phase_grid(n), to a relative width `rel`.
    Assumes that the stable time steps in the interval are those below some
    dt*; raises ValueError when dt_lo is unstable.  Returns (dt, dt_next):
    the largest stable time step found and the smallest unstable one (None
    when dt_hi is stable)."""
    st = np.atleast_2d(np.asarray(states, dtype=np.float64))
    R = np.tile(np.asarray(rates, dtype=np.float64).reshape(1, 16), (st.shape[0], 1))
    th = phase_grid(n)

    def stable(dt):
        return bool(np.max(screen_sets(st, R, dx, dy, dt, th, device=device)) <= 1.0 + tol)

    if not stable(dt_lo):
        raise ValueError(f"unstable already at dt = {dt_lo}")
    if stable(dt_hi):
        return dt_hi, None
    lo, hi = dt_lo, dt_hi
    while hi - lo > rel * lo:
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo, hi


def phase_grid(n):
    """(n + 1) x (2 n + 1) phase pairs over [0, pi] x [-pi, pi] (the other
    half follows by the symmetry of real data), as an (m, 2) array."""
    tx = np.linspace(0.0, math.pi, n + 1)
    ty = np.linspace(-math.pi, math.pi, 2 * n + 1)
    return np.array([(a, b) for a in tx for b in ty])


def max_growth(state, s, dx, dy, dt, n=32, device=None):
    """(max |omega|, (theta_x, theta_y)) over phase_grid(n)."""
    th = phase_grid(n)
    w = spectral_radius(state, s, dx, dy, dt, th, device)
    i = int(np.argmax(w))
    return float(w[i]), (float(th[i, 0]), float(th[i, 1]))
