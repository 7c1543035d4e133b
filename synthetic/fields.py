"""Seeded random lattice fields (gauge links, gauge transforms, right-hand sides).

Nothing here knows about the Dirac operator or the solvers; see the package
docstring for the array conventions.

Link recipe: draw ``G = (N(0,1) + i N(0,1)) / sqrt(2)`` for every link with
``numpy.random.default_rng(seed)`` (the whole real-part array first, then the
whole imaginary-part array), make it traceless Hermitian,
``H = (G + G^H)/2 - tr(.)/3 I``, and exponentiate ``U = exp(i eps H)`` through
the eigendecomposition ``H = W diag(h) W^H``, so ``U = W diag(exp(i eps h)) W^H``.
Because ``tr H = 0``, ``det U = 1`` up to rounding and ``U`` is in SU(3).

Right-hand sides: complex Gaussian with real and imaginary parts each
``N(0, 1/2)``, one generator per right-hand side seeded with ``seed``.
"""

from __future__ import annotations

import numpy as np

_CHUNK = 1 << 18  # links per eigendecomposition batch (bounds peak memory)


def site_shape(dims):
    """Array shape of the site index for ``dims = (Lx, Ly, Lz, Lt)``."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def n_sites(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def n_dof(dims) -> int:
    """Complex unknowns per spinor field: 4 spins x 3 colours per site."""
    return 12 * n_sites(dims)


def _expm_i_hermitian(g: np.ndarray, eps: float) -> np.ndarray:
    """``exp(i eps H)`` with ``H`` the traceless Hermitian part of ``g`` (..., 3, 3)."""
    h = 0.5 * (g + np.conj(np.swapaxes(g, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1)
    h = h - (tr / 3.0)[..., None, None] * np.eye(3)
    out = np.empty_like(h)
    flat_h = h.reshape(-1, 3, 3)
    flat_o = out.reshape(-1, 3, 3)
    for s in range(0, flat_h.shape[0], _CHUNK):
        e = slice(s, min(s + _CHUNK, flat_h.shape[0]))
        w, v = np.linalg.eigh(flat_h[e])
        ph = np.exp(1j * eps * w)
        flat_o[e] = np.einsum("nab,nb,ncb->nac", v, ph, np.conj(v))
    return out


def _complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    z = np.empty(shape, dtype=np.complex128)
    z.real = re
    z.imag = im
    z *= np.sqrt(0.5)
    return z


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links ``exp(i eps H)``; complex128 ``(Lt,Lz,Ly,Lx,4,3,3)``.

    ``eps = 0`` gives the unit (free) field.
    """
    shape = site_shape(dims) + (4, 3, 3)
    rng = np.random.default_rng(seed)
    g = _complex_gaussian(rng, shape)
    return np.ascontiguousarray(_expm_i_hermitian(g, float(eps)))


def unit_gauge_field(dims) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    u = np.zeros(site_shape(dims) + (4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = 1.0
    u[..., 1, 1] = 1.0
    u[..., 2, 2] = 1.0
    return u


def random_su3_sites(dims, seed: int, eps: float = 1.0) -> np.ndarray:
    """One random SU(3) matrix per site, ``(Lt,Lz,Ly,Lx,3,3)`` (gauge transforms)."""
    shape = site_shape(dims) + (3, 3)
    rng = np.random.default_rng(seed)
    g = _complex_gaussian(rng, shape)
    return np.ascontiguousarray(_expm_i_hermitian(g, float(eps)))


def gaussian_rhs(dims, seed: int) -> np.ndarray:
    """One complex Gaussian spinor field ``(Lt,Lz,Ly,Lx,4,3)``."""
    rng = np.random.default_rng(seed)
    return _complex_gaussian(rng, site_shape(dims) + (4, 3))


def gaussian_rhs_block(dims, seeds) -> np.ndarray:
    """Several right-hand sides stacked on a leading axis, one seed each."""
    return np.stack([gaussian_rhs(dims, s) for s in seeds], axis=0)


def gaussian_half_rhs(dims, seed: int) -> np.ndarray:
    """One complex Gaussian field on half of the sites, ``(V/2, 4, 3)``: a
    vector of the odd-even preconditioned system (one entry per even site, in
    lexicographic order)."""
    rng = np.random.default_rng(seed)
    return _complex_gaussian(rng, (n_sites(dims) // 2, 4, 3))
