"""MI355X (gfx950) implementation of the MRT finite-difference lattice
Boltzmann step of Chen, Xu, Zhang and Li (arXiv:0908.3749).

The computation lives in ``libmrtfd.so`` (HIP kernels + C ABI, see
include/mrtfd.h); this package only marshals arguments.  Importing it does
not need a GPU; using a grid does.
"""
from . import _abi  # noqa: F401
from ._abi import MrtfdError, lib  # noqa: F401
from .solver import MRT2D, TubeBatch, check_params, make_params, ref_populations  # noqa: F401
