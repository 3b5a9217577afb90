"""Projection of 3D Gaussians to 2D splats.  Test infrastructure only.

* ``optimal_projection`` follows Optimal Projection as used by the paper
  (end of Sec. 3 and Sec. 4.2): each Gaussian is projected onto the plane
  tangent to the unit sphere around the camera centre o, perpendicular to the
  line from o to the mean.  Coordinates on that plane are scaled by the focal
  length f so that, for a Gaussian straight ahead, they coincide with image
  pixels (this is a reading; the paper gives no formula).
* ``ewa_projection`` is the local-affine projection of Eq. 3
  (Sigma' = J W Sigma W^T J^T, top-left 2x2), which the paper notes is exact
  only at the image centre.  It is kept solely as a test reference.

Both add the same isotropic dilation delta (px^2) to the 2D covariance
(App. D mentions the dilation that keeps splats at least a pixel wide; its
value, 0.3 px^2, is a reading).
"""
import numpy as np


def tangent_basis(u):
    """Orthonormal basis (e1, e2) of the plane perpendicular to the unit vector
    u (N, 3): the images of the camera x and y axes under the minimal rotation
    taking +z to u.  Undefined only at u = -z, which the near-plane cull
    excludes.  Returns E of shape (N, 3, 2).  Any other orthonormal basis gives
    the same splat (the density is basis independent)."""
    ux, uy, uz = u[:, 0], u[:, 1], u[:, 2]
    k = 1.0 / (1.0 + uz)
    e1 = np.stack([1.0 - ux * ux * k, -ux * uy * k, -ux], axis=1)
    e2 = np.stack([-ux * uy * k, 1.0 - uy * uy * k, -uy], axis=1)
    return np.stack([e1, e2], axis=2)


def optimal_projection(mu_c, Sigma_c, f, dilation):
    """Optimal Projection of camera-frame means mu_c (N, 3) and covariances
    Sigma_c (N, 3, 3).

    r = |mu_c|, u = mu_c / r, E = tangent_basis(u);
    Sigma_2D = (f^2 / r^2) E^T Sigma_c E + delta I  (2x2 on the tangent plane
    at unit distance, in pixel units).  Returns dict with r, u, E, Sigma2D and
    the conic C = Sigma2D^-1.
    """
    r = np.linalg.norm(mu_c, axis=1)
    u = mu_c / r[:, None]
    E = tangent_basis(u)
    Et = np.transpose(E, (0, 2, 1))
    S2 = (f * f / (r * r))[:, None, None] * (Et @ Sigma_c @ E)
    S2 = S2 + dilation * np.eye(2)[None]
    C = np.linalg.inv(S2)
    return dict(r=r, u=u, E=E, Sigma2D=S2, conic=C)


def tangent_coords(d, u, E, f):
    """Tangent-plane coordinate of camera-frame ray directions d (..., 3):
    q(d) = f E^T d / (u . d), the central projection of the ray onto the plane
    through u perpendicular to u, scaled by f.  Valid only where u . d > 0;
    returns (q, h) with h = u . d (any positive scaling of d gives the same q)."""
    h = d @ u
    q = f * (d @ E) / h[..., None]
    return q, h


def ewa_projection(mu_c, Sigma_c, f, dilation):
    """Eq. 3: J = (f/z) [[1, 0, -x/z], [0, 1, -y/z]] evaluated at the mean,
    Sigma' = J Sigma_c J^T (the camera rotation W is already applied), plus the
    dilation.  Returns the 2x2 covariance in pixels (N, 2, 2)."""
    x, y, z = mu_c[:, 0], mu_c[:, 1], mu_c[:, 2]
    J = np.zeros((mu_c.shape[0], 2, 3))
    J[:, 0, 0] = f / z
    J[:, 0, 2] = -f * x / (z * z)
    J[:, 1, 1] = f / z
    J[:, 1, 2] = -f * y / (z * z)
    S2 = J @ Sigma_c @ np.transpose(J, (0, 2, 1))
    return S2 + dilation * np.eye(2)[None]
