"""Zeroth-order prolate spheroidal wave function psi_0(c, x) on [-1, 1].

Test infrastructure only (see the oracle package docstring).

psi_0 is the eigenfunction of the prolate operator
    L f = -d/dx[(1 - x^2) df/dx] + c^2 x^2 f
with the smallest eigenvalue.  Expanding in normalised Legendre polynomials
Pbar_n = sqrt(n + 1/2) P_n, the even functions couple only even degrees and the
operator becomes a symmetric tridiagonal matrix (Xiao, Rokhlin & Yarvin 2001):
    A[n, n]     = n(n+1) + c^2 (2n(n+1) - 1) / ((2n+3)(2n-1))
    A[n, n+2]   = c^2 (n+1)(n+2) / ((2n+3) sqrt((2n+1)(2n+5)))
The first follows from x^2 P_n = a P_{n+2} + b P_n + g P_{n-2} with
b = (n+1)^2/((2n+1)(2n+3)) + n^2/((2n-1)(2n+1)); the second is a rescaled by the
normalisation ratio.  The coefficients decay faster than geometrically once
the degree passes c, so a modest truncation is exact to rounding.

The imaging taper is psi(nu) = psi_0(c, nu) / psi_0(c, 0) for |nu| <= 1 and 0
outside, with c = pi * S / 2 for full support S cells: with that bandwidth the
Fourier transform of the taper is itself proportional to psi_0 squeezed into
|offset| <= S/2 cells (the finite Fourier transform eigen-relation), so an
S-cell kernel holds it.
"""

import math

import numpy as np
from numpy.polynomial import legendre as npleg


def prolate_matrix(c: float, k_terms: int) -> np.ndarray:
    """Symmetric tridiagonal matrix of the prolate operator on Pbar_0, Pbar_2, ..."""
    n = 2.0 * np.arange(k_terms)
    diag = n * (n + 1.0) + c * c * (2.0 * n * (n + 1.0) - 1.0) / ((2.0 * n + 3.0) * (2.0 * n - 1.0))
    nn = n[:-1]
    off = c * c * (nn + 1.0) * (nn + 2.0) / ((2.0 * nn + 3.0) * np.sqrt((2.0 * nn + 1.0) * (2.0 * nn + 5.0)))
    return np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)


def legendre_coeffs(c: float, k_terms: int = 0):
    """(chi_0, coefficients of psi_0 in the ordinary Legendre basis P_0..P_{2K-2}).

    The eigenvector is scaled so that psi_0(0) > 0; the overall scale is
    irrelevant because the taper is normalised to psi(0) = 1.
    """
    if k_terms <= 0:
        k_terms = int(c) + 40
    evals, evecs = np.linalg.eigh(prolate_matrix(c, k_terms))
    beta = evecs[:, 0]
    coef = np.zeros(2 * k_terms - 1)
    coef[0::2] = beta * np.sqrt(2.0 * np.arange(k_terms) + 0.5)
    if npleg.legval(0.0, coef) < 0:
        coef = -coef
    return evals[0], coef


def psi0(c: float, x) -> np.ndarray:
    """psi_0(c, x) with the eigenvector's own (arbitrary) scale, |x| <= 1."""
    _, coef = legendre_coeffs(c)
    return npleg.legval(np.asarray(x, dtype=np.float64), coef)


def taper(support: int, nu) -> np.ndarray:
    """psi(nu) = psi_0(c, nu)/psi_0(c, 0) inside |nu| <= 1, zero outside; c = pi S / 2."""
    c = math.pi * support / 2.0
    _, coef = legendre_coeffs(c)
    nu = np.asarray(nu, dtype=np.float64)
    val = npleg.legval(nu, coef) / npleg.legval(0.0, coef)
    return np.where(np.abs(nu) <= 1.0, val, 0.0)
