"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This package only draws random numbers and shapes them into lattice fields:
SU(3) gauge links, random gauge transformations and Gaussian right-hand
sides.  It holds none of the solver's arithmetic (no Dirac operator, no CG,
no eigCG, no deflation), so that both sides of every parity test can start
from byte-identical inputs without sharing any of the method.

Conventions (fixed here once for every consumer):

* a lattice is ``dims = (Lx, Ly, Lz, Lt)``, periodic in all four directions;
* site arrays are shaped ``(Lt, Lz, Ly, Lx, ...)`` so x runs fastest;
* spinor fields are complex128 ``(Lt, Lz, Ly, Lx, 4 spin, 3 colour)``;
* gauge fields are complex128 ``(Lt, Lz, Ly, Lx, 4 mu, 3, 3)`` with
  ``mu = 0, 1, 2, 3`` the x, y, z, t directions and ``U[..., mu, a, b]``
  the row ``a`` / column ``b`` entry of the link matrix ``U_mu(x)``.
"""

from .fields import (  # noqa: F401
    site_shape,
    n_sites,
    n_dof,
    gauge_field,
    unit_gauge_field,
    random_su3_sites,
    gaussian_rhs,
    gaussian_rhs_block,
    gaussian_half_rhs,
)
