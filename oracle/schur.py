"""Odd-even (Schur complement) preconditioned Wilson operator, plain NumPy FP64
(test infrastructure only).

The paper's lattice runs (the comparisons of Section 3.1 and the QCD tests of
Section 5.1) solve the odd-even preconditioned normal equations, a
system of half the size; the paper does not write the preconditioned operator
out.  The reading used here is the exact Schur complement of the even-site
block of M.

Sites split by parity (x + y + z + t) mod 2 into even (e) and odd (o); every
dimension is even so that the split is consistent with the periodic wrap.  The
Wilson hopping term D (``dirac.hopping``) only connects sites of opposite
parity, so with d = 4 + m_q

    M = [[ d I,        -1/2 D_eo ],
         [ -1/2 D_oe,   d I      ]]

and eliminating the odd sites gives, on the even sites,

    Mhat   = M_ee - M_eo M_oo^{-1} M_oe = d I - 1/(4 d) D_eo D_oe
    M x = b   <=>   Mhat x_e = bhat_e = b_e + 1/(2 d) D_eo b_o,
                    x_o = (b_o + 1/2 D_oe x_e) / d.

Mhat^H has the same form with the hopping term of M^H (the adjoint of the
block D_eo D_oe is the product of the adjoint hopping blocks).  CG, eigCG and
init-CG run unchanged on Ahat = Mhat^H Mhat with the right-hand side
Mhat^H bhat_e (Section 1: the normal equations).

Even-site vectors list the even sites in lexicographic order (x fastest), so
the even site s = x + Lx (y + Ly (z + Lz t)) is entry s // 2; odd-site vectors
likewise.  Each entry is a (spin, colour) block of 12 complex numbers.
"""

from __future__ import annotations

import numpy as np

from .dirac import WilsonOperator, apply_gamma5, hopping


class SchurOperator:
    """Mhat, Mhat^H and Ahat = Mhat^H Mhat on flat even-site vectors of length
    6 V, plus the maps between the full system M x = b and the even-site one."""

    def __init__(self, U, mass):
        self.full = WilsonOperator(U, mass)
        if any(L % 2 for L in self.full.dims):
            raise ValueError("odd-even preconditioning needs every lattice extent even")
        self.U = self.full.U
        self.site_shape = self.full.site_shape
        self.d = 4.0 + float(mass)
        t, z, y, x = np.indices(self.site_shape)
        parity = ((x + y + z + t) % 2).reshape(-1)
        self.even = np.flatnonzero(parity == 0)
        self.odd = np.flatnonzero(parity == 1)
        self.volume = parity.size
        self.n = 12 * self.even.size

    # -- parity embedding --------------------------------------------------
    def _embed(self, v, sites):
        f = np.zeros((self.volume, 4, 3), dtype=np.complex128)
        f[sites] = np.asarray(v, dtype=np.complex128).reshape(-1, 4, 3)
        return f.reshape(self.site_shape + (4, 3))

    def _restrict(self, field, sites):
        return np.asarray(field).reshape(self.volume, 4, 3)[sites].reshape(-1)

    def split(self, v_full):
        """(even part, odd part) of a full-lattice vector."""
        return self._restrict(v_full, self.even), self._restrict(v_full, self.odd)

    def join(self, v_e, v_o):
        f = self._embed(v_e, self.even).reshape(self.volume, 4, 3)
        f[self.odd] = np.asarray(v_o, dtype=np.complex128).reshape(-1, 4, 3)
        return f.reshape(-1)

    def hop(self, v, src, dst, sign):
        """Block D_{dst,src} of the hopping sum (sign -1: that of M, +1: of M^H)
        applied to a vector living on the sites ``src``."""
        return self._restrict(hopping(self.U, self._embed(v, src), sign), dst)

    # -- the preconditioned operator ------------------------------------------
    def Mhat(self, v):
        t = self.hop(v, self.even, self.odd, -1.0)
        return self.d * np.asarray(v) - self.hop(t, self.odd, self.even, -1.0) / (4.0 * self.d)

    def Mhat_dag(self, v):
        t = self.hop(v, self.even, self.odd, +1.0)
        return self.d * np.asarray(v) - self.hop(t, self.odd, self.even, +1.0) / (4.0 * self.d)

    def A(self, v):
        """``Ahat v = Mhat^H (Mhat v)``."""
        return self.Mhat_dag(self.Mhat(v))

    def gamma5(self, v):
        return apply_gamma5(np.asarray(v, dtype=np.complex128).reshape(-1, 4, 3)).reshape(-1)

    # -- full system <-> even-site system -------------------------------------
    def bhat(self, b_full):
        """``bhat_e = b_e + D_eo b_o / (2 d)``, so that ``Mhat x_e = bhat_e``."""
        b_e, b_o = self.split(b_full)
        return b_e + self.hop(b_o, self.odd, self.even, -1.0) / (2.0 * self.d)

    def rhs(self, b_full):
        """Right-hand side of the normal equations: ``Mhat^H bhat_e``."""
        return self.Mhat_dag(self.bhat(b_full))

    def reconstruct(self, b_full, x_e):
        """Full solution from the even part: ``x_o = (b_o + D_oe x_e / 2) / d``."""
        _, b_o = self.split(b_full)
        x_o = (b_o + 0.5 * self.hop(x_e, self.even, self.odd, -1.0)) / self.d
        return self.join(x_e, x_o)
