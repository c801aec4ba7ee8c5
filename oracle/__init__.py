"""FP64 CPU oracle for the time-stepped stencil sweep.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2309_08864_amd``) never imports, links or calls it, and this package
imports nothing from the product: the two share no code.

Contents:
  * ``so2dr_oracle.c`` - plain C loops in FP64 (OpenMP over the slowest axis):
    the in-core Jacobi sweep, its transpose, the adjoint gradient and a
    light-cone sub-box sweep for grids too large to sweep whole.
  * ``oracle.py`` - ctypes wrapper plus the stencil point sets (Fig. 1a of the
    paper: star = axis arms, box = full (2r+1)^dim cube).
  * ``emulator.py`` - a bit-exact NumPy model of the library's documented
    FP32 arithmetic (FMA chain order, per-step BF16/FP16 rounding).

Every function below is pinned in ``tests/test_oracle_pins.py`` against
mathematics that does not go through this code: exact rational arithmetic,
library correlation / convolution routines, closed-form Fourier decay,
conservation laws, the adjoint dot-product identity and finite differences.
"""
from .oracle import (  # noqa: F401
    stencil_offsets, sweep, transpose_step, adjoint, sweep_box, build, lib_path,
    extract_window, sweep_box_from_field, sweep_box_window, reach_of,
)
from . import emulator  # noqa: F401
