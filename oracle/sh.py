"""View-dependent colour from real spherical harmonics.  Test infrastructure
only.

Sec. 4.1 lists spherical-harmonics coefficients among the optimised Gaussian
parameters; the basis, sign convention, offset and clamp are not stated and are
read as follows: orthonormal real SH with the Condon-Shortley phase, coefficient
index k = l^2 + l + m, colour = max(0, sum_k c_k Y_k(v) + 1/2) per channel, with
v the unit direction from the eye centre to the mean (world frame).

The basis is built from its definition: Legendre polynomials by Rodrigues'
formula, associated Legendre functions by differentiation (with the
(-1)^m phase), and the usual normalisation -- no table of constants.
"""
import math

import numpy as np
from numpy.polynomial import polynomial as P


def legendre_assoc(l, m, x):
    """P_l^m(x) = (-1)^m (1 - x^2)^(m/2) d^m/dx^m P_l(x), with
    P_l(x) = 1/(2^l l!) d^l/dx^l (x^2 - 1)^l.  m >= 0."""
    base = P.polypow([-1.0, 0.0, 1.0], l)                 # (x^2 - 1)^l
    pl = P.polyder(base, l) / (2.0 ** l * math.factorial(l)) if l > 0 else np.array([1.0])
    dm = P.polyder(pl, m) if m > 0 else pl
    x = np.asarray(x, np.float64)
    return ((-1.0) ** m) * (1.0 - x * x) ** (m / 2.0) * P.polyval(x, dm)


def real_sh(l, m, v):
    """Orthonormal real spherical harmonic Y_lm at unit vectors v (..., 3)."""
    v = np.asarray(v, np.float64)
    ct = np.clip(v[..., 2], -1.0, 1.0)
    phi = np.arctan2(v[..., 1], v[..., 0])
    am = abs(m)
    K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    plm = legendre_assoc(l, am, ct)
    if m == 0:
        return K * plm
    if m > 0:
        return math.sqrt(2.0) * K * np.cos(am * phi) * plm
    return math.sqrt(2.0) * K * np.sin(am * phi) * plm


def sh_basis(degree, v):
    """All Y_k(v), k = l^2 + l + m for l <= degree; returns (..., K)."""
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            out.append(real_sh(l, m, v))
    return np.stack(out, axis=-1)


def sh_color(sh, degree, v):
    """Colour per Gaussian: sh is (K, 3, N), v unit directions (N, 3).
    Returns (N, 3) = max(0, sum_k sh[k, c] Y_k(v) + 0.5)."""
    sh = np.asarray(sh, np.float64)
    K = (degree + 1) ** 2
    Y = sh_basis(degree, v)                    # (N, K)
    raw = np.einsum("nk,kcn->nc", Y, sh[:K])
    return np.maximum(raw + 0.5, 0.0), raw + 0.5
