"""Integrated Legendre shape functions on the reference interval [-1, 1].

Section 2.1 (and the p-FEM basis it refers to): the trial space is spanned by
the two linear "vertex" modes and, for j = 2..p, the integrated Legendre
bubble modes.  The normalisation is the Szabo-Babuska one:

    N_0(xi) = (1 - xi) / 2                 (left vertex)
    N_1(xi) = (1 + xi) / 2                 (right vertex)
    N_j(xi) = (L_j(xi) - L_{j-2}(xi)) / sqrt(2 (2j - 1)),   j = 2..p

so that the bubble derivatives sqrt((2j-1)/2) L_{j-1} are orthonormal.  Mode
index j >= 2 is also the mode's polynomial degree; vertex modes have degree 1.
The set of order p contains every mode of order q < p (hierarchical basis,
eq. hierarchicalFunctions).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def legendre(j: int, xi):
    """Legendre polynomial L_j evaluated with numpy's Legendre series."""
    coeff = np.zeros(j + 1)
    coeff[j] = 1.0
    return npleg.legval(np.asarray(xi, dtype=np.float64), coeff)


def modes_1d(p: int, xi):
    """Values of the p+1 modes at points xi: array (p+1, len(xi))."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    out = np.empty((p + 1, xi.size))
    out[0] = 0.5 * (1.0 - xi)
    out[1] = 0.5 * (1.0 + xi)
    for j in range(2, p + 1):
        out[j] = (legendre(j, xi) - legendre(j - 2, xi)) / np.sqrt(2.0 * (2 * j - 1))
    return out


def dmodes_1d(p: int, xi):
    """Derivatives d/dxi of the p+1 modes: array (p+1, len(xi))."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    out = np.empty((p + 1, xi.size))
    out[0] = -0.5
    out[1] = 0.5
    for j in range(2, p + 1):
        # d/dxi (L_j - L_{j-2}) = (2j-1) L_{j-1}
        out[j] = (2 * j - 1) * legendre(j - 1, xi) / np.sqrt(2.0 * (2 * j - 1))
    return out


def mode_degree(j: int) -> int:
    """Polynomial degree of 1D mode j (vertex modes 0,1 have degree 1)."""
    return 1 if j < 2 else j


def gauss(npts: int):
    """Gauss-Legendre rule on [-1, 1] (numpy's leggauss)."""
    x, w = npleg.leggauss(npts)
    return x.astype(np.float64), w.astype(np.float64)
