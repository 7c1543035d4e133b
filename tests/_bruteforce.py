"""Brute-force dense Wilson matrix built with explicit site loops.

Independent of the oracle's ``np.roll`` stencil: every matrix element is
placed from the operator's definition (Kronecker deltas over explicit site
coordinates), so a wrong shift direction, a misplaced link or a missing
dagger in the stencil shows up as a mismatch.
"""

import itertools

import numpy as np


def site_index(coord, dims):
    x, y, z, t = coord
    lx, ly, lz, lt = dims
    return ((t * lz + z) * ly + y) * lx + x


def shifted(coord, mu, step, dims):
    c = list(coord)
    c[mu] = (c[mu] + step) % dims[mu]
    return tuple(c)


def wilson_dense(U, mass, gammas, dims):
    """M[(x,s,a),(y,t,b)] of M = (4+m) - 1/2 sum_mu [(1-g_mu) U_mu(x) d_{y,x+mu}
    + (1+g_mu) U_mu(x-mu)^dag d_{y,x-mu}]."""
    lx, ly, lz, lt = dims
    nsite = lx * ly * lz * lt
    Mat = np.zeros((12 * nsite, 12 * nsite), dtype=np.complex128)
    eye4 = np.eye(4)
    for coord in itertools.product(range(lx), range(ly), range(lz), range(lt)):
        xs = site_index(coord, dims)
        x, y, z, t = coord
        for k in range(12):
            Mat[12 * xs + k, 12 * xs + k] += 4.0 + mass
        for mu in range(4):
            fwd = shifted(coord, mu, +1, dims)
            bwd = shifted(coord, mu, -1, dims)
            ys_f = site_index(fwd, dims)
            ys_b = site_index(bwd, dims)
            bx, by, bz, bt = bwd
            link_here = U[t, z, y, x, mu]
            link_back = U[bt, bz, by, bx, mu]
            pf = eye4 - gammas[mu]
            pb = eye4 + gammas[mu]
            for s in range(4):
                for tt in range(4):
                    for a in range(3):
                        for b in range(3):
                            Mat[12 * xs + 3 * s + a, 12 * ys_f + 3 * tt + b] += \
                                -0.5 * pf[s, tt] * link_here[a, b]
                            Mat[12 * xs + 3 * s + a, 12 * ys_b + 3 * tt + b] += \
                                -0.5 * pb[s, tt] * np.conj(link_back[b, a])
    return Mat
