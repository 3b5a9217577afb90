"""Depth along a view ray (Sec. 4.1: StopThePop re-sorts splats per pixel by
depth along the view rays).  Test infrastructure only.

Reading: the depth of Gaussian (mu, Sigma) on the unit ray d from the eye is the
ray parameter of maximum density along the ray,
    t*(d) = (d^T Sigma^-1 mu) / (d^T Sigma^-1 d),
obtained by setting the derivative of the exponent of Eq. 1 along the ray to
zero -- the same computation Eq. 4 performs along a tile edge, done in 3D.
"""
import numpy as np


def tstar(d, mu_c, B):
    """t*(d) for unit ray directions d (..., 3); mu_c (3,), B = Sigma_c^-1."""
    Bd = d @ B
    return (Bd @ mu_c) / np.einsum("...i,...i->...", Bd, d)
