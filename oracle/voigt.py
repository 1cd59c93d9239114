"""Voigt function for the oracle.  TEST INFRASTRUCTURE ONLY.

H(x, a) = Re w(x + i a), with w the Faddeeva function, normalised so that
H(0, 0) = 1 and the integral of H over x equals sqrt(pi).  This is the line
profile H(dnu / dnu_D, gamma / (4 pi dnu_D)) of the line absorption
coefficient (Sec. 2.1, eq. l_nu_line).  The library routine scipy.special.wofz
is the step used here; the tests pin it against closed forms, mpmath and a
brute-force quadrature of the defining convolution integral.
"""
import numpy as np
from scipy.special import wofz


def voigt_h(x, a):
    """Voigt H(x, a) for real x and a >= 0 (broadcasting)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    return wofz(x + 1j * a).real
