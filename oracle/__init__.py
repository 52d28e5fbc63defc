"""FP64 CPU oracle for the MRT finite-difference lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import, call, link or execute
anything in this package.  The product library never does, and it shares no
code with this package.

* ``core``     -- ctypes binding of ``mrt_oracle.c``: velocity set, M, M^-1,
                  equilibria, collision, Lax-Wendroff/Euler update, boundary
                  rules, whole-grid runs (FP64).
* ``riemann``  -- exact Riemann solver (gamma is a parameter; the model's is 2).
* ``analytic`` -- Couette series, transport coefficients, Fourier
                  amplification of the difference scheme.
* ``metrics``  -- the paper's relative error E, L1/Linf, shock location.
* ``stability`` -- the von Neumann screen of Sect. IV in numpy (eigenvalues
                  of the amplification matrix), the reference of the GPU one.
"""
from . import analytic, core, metrics, riemann, stability  # noqa: F401
from .core import Grid, model  # noqa: F401
