"""Pins for the oracle's per-Gaussian geometry: each test checks the oracle
against something other than itself -- a second textbook construction, a
closed form, an invariant or brute force."""
import math

import numpy as np
import pytest

from oracle import camera as cam_mod
from oracle import depth as depth_mod
from oracle import gaussian as g_mod
from oracle import projection as proj_mod
from oracle import sh as sh_mod
import synth


def rodrigues(axis, angle):
    axis = axis / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def test_quaternion_matches_axis_angle():
    rng = np.random.default_rng(0)
    for _ in range(20):
        axis = rng.standard_normal(3)
        ang = rng.uniform(-math.pi, math.pi)
        n = axis / np.linalg.norm(axis)
        q = np.r_[math.cos(ang / 2), math.sin(ang / 2) * n] * rng.uniform(0.3, 3.0)
        R = g_mod.quat_to_rotmat(q[:, None])[0]
        np.testing.assert_allclose(R, rodrigues(axis, ang), atol=1e-12)
        np.testing.assert_allclose(g_mod.quat_to_rotmat(-q[:, None])[0], R, atol=1e-12)


def test_covariance_eigen_are_scales_squared():
    s = synth.uniform_scene(1, 50)
    Sig = g_mod.covariance(s.quats, s.log_scales)
    for i in range(50):
        ev = np.sort(np.linalg.eigvalsh(Sig[i]))
        np.testing.assert_allclose(ev, np.sort(np.exp(2 * s.log_scales[:, i].astype(np.float64))), rtol=1e-10)


def test_density_and_opacity():
    assert g_mod.opacity(np.array([0.0]))[0] == 0.5
    Sig = np.diag([1.0, 4.0, 9.0])
    x = np.array([1.0, 2.0, 3.0])
    # (1^2/1 + 2^2/4 + 3^2/9) = 3
    assert abs(g_mod.density(x, np.zeros(3), Sig) - math.exp(-1.5)) < 1e-15


def test_focal_and_principal_ray():
    cam = synth.camera_translate((0, 0, -3), 90.0, 256, 256)
    assert abs(cam_mod.focal(cam) - 128.0) < 1e-9
    d = cam_mod.ray_dirs(cam, 128.0, 128.0)
    np.testing.assert_allclose(d, [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(cam_mod.eye_center(cam), [0, 0, -3], atol=1e-6)


def _random_cov(rng, n, lo=-3.0, hi=-1.0):
    q = rng.standard_normal((4, n))
    ls = rng.uniform(lo, hi, (3, n))
    return g_mod.covariance(q, ls)


def test_op_equals_ewa_at_image_centre():
    """Eq. 3 is exact at the image centre: for a mean on the optical axis the
    tangent plane is the image plane and OP's conic equals EWA's."""
    rng = np.random.default_rng(2)
    n = 64
    z = rng.uniform(0.5, 10.0, n)
    mu = np.stack([np.zeros(n), np.zeros(n), z], axis=1)
    Sig = _random_cov(rng, n)
    f = 700.0
    op = proj_mod.optimal_projection(mu, Sig, f, 0.3)
    ewa = proj_mod.ewa_projection(mu, Sig, f, 0.3)
    np.testing.assert_allclose(op["Sigma2D"], ewa, rtol=1e-12, atol=1e-12)


def test_op_departs_from_ewa_off_axis():
    """The local-affine error grows with the off-axis angle (Sec. 3)."""
    rng = np.random.default_rng(3)
    Sig = _random_cov(rng, 1, -1.5, -1.0)
    f = 700.0
    errs = []
    for ang in (0.0, 15.0, 30.0, 45.0, 60.0):
        a = math.radians(ang)
        mu = np.array([[3 * math.sin(a), 0.0, 3 * math.cos(a)]])
        op = proj_mod.optimal_projection(mu, Sig, f, 0.0)
        ewa = proj_mod.ewa_projection(mu, Sig, f, 0.0)
        # Compare the splat areas (determinants), which differ once off axis.
        errs.append(abs(np.linalg.det(op["Sigma2D"][0]) - np.linalg.det(ewa[0])))
    assert errs[0] < 1e-6 * abs(np.linalg.det(ewa[0]) + 1)
    assert all(b > a for a, b in zip(errs[1:], errs[2:]))


def test_tangent_basis_orthonormal_and_density_basis_independent():
    rng = np.random.default_rng(4)
    n = 40
    u = rng.standard_normal((n, 3))
    u[:, 2] = np.abs(u[:, 2]) + 0.2
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    E = proj_mod.tangent_basis(u)
    for i in range(n):
        np.testing.assert_allclose(E[i].T @ E[i], np.eye(2), atol=1e-12)
        np.testing.assert_allclose(E[i].T @ u[i], 0, atol=1e-12)
    # Rotating the basis within the plane leaves q^T C q unchanged.
    mu = u * rng.uniform(1, 5, n)[:, None]
    Sig = _random_cov(rng, n)
    f = 500.0
    op = proj_mod.optimal_projection(mu, Sig, f, 0.3)
    d = u + 0.05 * rng.standard_normal((n, 3))
    for i in range(n):
        q, _ = proj_mod.tangent_coords(d[i], u[i], E[i], f)
        D2 = q @ op["conic"][i] @ q
        th = rng.uniform(0, 2 * math.pi)
        Rt = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        E2 = E[i] @ Rt
        S2 = (f * f / np.sum(mu[i] ** 2)) * E2.T @ Sig[i] @ E2 + 0.3 * np.eye(2)
        q2, _ = proj_mod.tangent_coords(d[i], u[i], E2, f)
        assert abs(q2 @ np.linalg.inv(S2) @ q2 - D2) < 1e-9 * max(1.0, D2)


def test_isotropic_closed_form_alpha():
    """An isotropic Gaussian (scale s, distance r) has, on the ray at angle
    theta from its mean direction, D^2 = f^2 tan^2(theta) / (f^2 s^2 / r^2 + delta)."""
    rng = np.random.default_rng(5)
    f, delta = 600.0, 0.3
    for _ in range(20):
        s = math.exp(rng.uniform(-4, -1))
        r = rng.uniform(1, 6)
        u = rng.standard_normal(3); u[2] = abs(u[2]) + 0.5; u /= np.linalg.norm(u)
        mu = r * u
        Sig = (s * s) * np.eye(3)
        op = proj_mod.optimal_projection(mu[None], Sig[None], f, delta)
        w = rng.standard_normal(3); w -= (w @ u) * u; w /= np.linalg.norm(w)
        th = rng.uniform(0, 0.3)
        d = math.cos(th) * u + math.sin(th) * w
        q, _ = proj_mod.tangent_coords(d, u, op["E"][0], f)
        D2 = q @ op["conic"][0] @ q
        expect = f * f * math.tan(th) ** 2 / (f * f * s * s / (r * r) + delta)
        assert abs(D2 - expect) <= 1e-9 * max(1.0, expect)


def test_sh_low_order_closed_forms_and_phase():
    rng = np.random.default_rng(6)
    v = rng.standard_normal((100, 3)); v /= np.linalg.norm(v, axis=1, keepdims=True)
    c0 = 1.0 / (2.0 * math.sqrt(math.pi))
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    Y = sh_mod.sh_basis(1, v)
    np.testing.assert_allclose(Y[:, 0], c0, rtol=1e-14)
    np.testing.assert_allclose(Y[:, 1], -c1 * v[:, 1], atol=1e-14)   # m = -1
    np.testing.assert_allclose(Y[:, 2], c1 * v[:, 2], atol=1e-14)    # m = 0
    np.testing.assert_allclose(Y[:, 3], -c1 * v[:, 0], atol=1e-14)   # m = +1 (Condon-Shortley sign)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 exactly.
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = 2 * math.pi * np.arange(nphi) / nphi
    ct = np.repeat(xg, nphi)
    ph = np.tile(phi, len(xg))
    st = np.sqrt(1 - ct ** 2)
    v = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    w = np.repeat(wg, nphi) * (2 * math.pi / nphi)
    Y = sh_mod.sh_basis(3, v)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_addition_theorem():
    rng = np.random.default_rng(7)
    v = rng.standard_normal((50, 3)); v /= np.linalg.norm(v, axis=1, keepdims=True)
    Y = sh_mod.sh_basis(3, v)
    for l in range(4):
        s = (Y[:, l * l:(l + 1) ** 2] ** 2).sum(axis=1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-12)


def test_sh_color_offset_and_clamp():
    sh = np.zeros((16, 3, 2))
    sh[0, :, 0] = 1.0
    sh[0, :, 1] = -10.0
    v = np.array([[0, 0, 1.0], [1.0, 0, 0]])
    col, raw = sh_mod.sh_color(sh, 3, v)
    np.testing.assert_allclose(col[0], 0.5 + 1.0 / (2 * math.sqrt(math.pi)))
    np.testing.assert_allclose(col[1], 0.0)


def test_tstar_isotropic_and_mean_direction():
    rng = np.random.default_rng(8)
    for _ in range(10):
        mu = rng.standard_normal(3); mu[2] = abs(mu[2]) + 1
        B = np.linalg.inv(_random_cov(rng, 1)[0])
        u = mu / np.linalg.norm(mu)
        assert abs(depth_mod.tstar(u, mu, B) - np.linalg.norm(mu)) < 1e-9
        d = u + 0.1 * rng.standard_normal(3); d /= np.linalg.norm(d)
        assert abs(depth_mod.tstar(d, mu, np.eye(3)) - d @ mu) < 1e-12


def test_tstar_is_argmax_of_density_along_ray():
    rng = np.random.default_rng(9)
    for _ in range(10):
        mu = rng.standard_normal(3); mu[2] = abs(mu[2]) + 2
        Sig = _random_cov(rng, 1, -1.0, 0.0)[0]
        d = mu / np.linalg.norm(mu) + 0.05 * rng.standard_normal(3)
        d /= np.linalg.norm(d)
        ts = np.linspace(0, 2 * np.linalg.norm(mu), 200001)
        dens = g_mod.density(ts[:, None] * d[None], mu, Sig)
        tb = ts[np.argmax(dens)]
        assert abs(depth_mod.tstar(d, mu, np.linalg.inv(Sig)) - tb) <= 2 * (ts[1] - ts[0])
