"""Seeded synthetic inputs for the Wilson-Dirac path.

This module is shared by the CPU oracle and by the GPU path's tests and
benchmark.  It only draws random numbers and arranges them into the
canonical host layout; it holds none of the operator's arithmetic.

Canonical host layout (numpy, C order):

* site index   idx = x1 + L1*(x2 + L2*(x3 + L3*x4)), i.e. arrays are shaped
  (L4, L3, L2, L1, ...) with x1 fastest;  x4 is the time direction.
* spinor field (L4, L3, L2, L1, 4, 3) complex128: [site][spin][colour].
* gauge field  (L4, L3, L2, L1, 4, 3, 3) complex128: [site][mu][row][col],
  mu = 0..3 standing for the directions x1..x4.
"""
from .fields import (  # noqa: F401
    lattice_shape,
    volume,
    rng_for,
    random_traceless_hermitian,
    gauge_field,
    unit_gauge,
    random_su3,
    gaussian_spinor,
    point_source,
    point_sources,
    batch_lattices,
    CONFIG_SEEDS,
)
