"""3D Gaussian primitives (Sec. 3, Eq. 1 and the covariance built from a
rotation R and a diagonal scale S as R S S^T R^T).  Test infrastructure only.

Stored parameters (Sec. 4.1 lists them as the optimised quantities): a mean, a
quaternion (w, x, y, z) of any non-zero length, a per-axis log standard
deviation and an opacity logit.
"""
import numpy as np


def quat_to_rotmat(q):
    """Rotation matrix of the unit quaternion q/|q|; q has shape (4, N) as
    (w, x, y, z).  Returns (N, 3, 3).  Standard Hamilton convention: the
    matrix rotates a vector v to q v q^*."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=0, keepdims=True)
    w, x, y, z = q
    R = np.empty((q.shape[1], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def scales(log_scales):
    """Per-axis standard deviations s = exp(l); (3, N) -> (N, 3)."""
    return np.exp(np.asarray(log_scales, np.float64)).T


def covariance(quats, log_scales):
    """Sigma = R S S^T R^T (Sec. 3).  Returns (N, 3, 3)."""
    R = quat_to_rotmat(quats)
    s = scales(log_scales)
    RS = R * s[:, None, :]
    return RS @ np.transpose(RS, (0, 2, 1))


def opacity(opacity_logits):
    """sigma = 1 / (1 + exp(-o)): the opacity that scales the 2D Gaussian in
    the blending weight alpha_i = sigma_i G_2D (Eq. 2)."""
    o = np.asarray(opacity_logits, np.float64)
    return 1.0 / (1.0 + np.exp(-o))


def density(x, mean, Sigma):
    """G(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)) (Eq. 1); x is (..., 3)."""
    d = np.asarray(x, np.float64) - mean
    return np.exp(-0.5 * np.einsum("...i,ij,...j->...", d, np.linalg.inv(Sigma), d))
