"""Pins for tile culling (Sec. 4.2, Eq. 4, Fig. 4), per-tile depth, keys and
ranges in the oracle."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from oracle import camera as cam_mod
from oracle import projection as proj_mod
from oracle import tiles as tiles_mod
from oracle.render import OracleOptions, instances_view, preprocess_view
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pixel_D2(cam, f, u, E, C, px, py):
    d = cam_mod.ray_dirs(cam, px, py, normalize=False)
    q, h = proj_mod.tangent_coords(d, u, E, f)
    D2 = np.einsum("...i,ij,...j->...", q, C, q)
    return np.where(h > 0, D2, np.inf)


def _brute_min(cam, f, u, E, C, box, n=161):
    x0, y0, x1, y1 = box
    xs = np.linspace(x0, x1, n)
    ys = np.linspace(y0, y1, n)
    X, Y = np.meshgrid(xs, ys)
    D = _pixel_D2(cam, f, u, E, C, X, Y)
    k = np.argmin(D)
    best = D.flat[k]
    if not np.isfinite(best):
        return best
    fun = lambda p: float(_pixel_D2(cam, f, u, E, C, np.array(p[0]), np.array(p[1])))
    r = minimize(fun, [X.flat[k], Y.flat[k]], method="L-BFGS-B",
                 bounds=[(x0, x1), (y0, y1)], options=dict(ftol=1e-15, gtol=1e-12, maxiter=500))
    return min(best, r.fun)


def _random_pairs(seed, fov=100.0, size=256, n=60, T=16):
    rng = np.random.default_rng(seed)
    cam = synth.camera_translate((0, 0, 0), fov, size, size)
    f = cam_mod.focal(cam)
    grid = tiles_mod.TileGrid(size, size, T)
    out = []
    for _ in range(n):
        z = rng.uniform(0.5, 4)
        tanx = math.tan(math.radians(fov / 2))
        x = rng.uniform(-1.3, 1.3) * tanx * z
        y = rng.uniform(-1.3, 1.3) * tanx * z
        mu = np.array([x, y, z])
        q = rng.standard_normal((4, 1))
        ls = rng.uniform(-3.5, -1.0, (3, 1))
        from oracle import gaussian as g_mod
        Sig = g_mod.covariance(q, ls)
        op = proj_mod.optimal_projection(mu[None], Sig, f, 0.3)
        x0 = cam.cx + f * x / z
        y0 = cam.cy + f * y / z
        tile = int(rng.integers(0, grid.n))
        out.append((cam, f, op["u"], op["E"], op["conic"], x0, y0, grid.boxes(np.array([tile]))))
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quad_test_matches_brute_force(seed):
    for cam, f, u, E, C, x0, y0, box in _random_pairs(seed):
        res = tiles_mod.quad_test(cam, f, u, E, C, np.array([x0]), np.array([y0]), *box)
        D2 = res["D2min"][0]
        bm = _brute_min(cam, f, u[0], E[0], C[0], tuple(b[0] for b in box))
        # Exact minimum: never above the brute-force estimate, and reached by it.
        assert D2 <= bm * (1 + 1e-9) + 1e-12
        assert bm <= D2 * (1 + 1e-6) + 1e-9
        # alpha at qhat equals the maximum (qhat is the arg-min on the plane).
        q = res["qhat"][0]
        assert abs(q @ C[0] @ q - D2) <= 1e-9 * max(1, D2)


def test_quad_test_partially_hidden_tiles():
    """Very wide view: Gaussians near one border see tiles on the far side
    partly behind their tangent plane; brute force over visible points."""
    hidden_cases = 0
    for seed in range(4):
        for cam, f, u, E, C, x0, y0, box in _random_pairs(100 + seed, fov=160.0, size=128, T=16):
            res = tiles_mod.quad_test(cam, f, u, E, C, np.array([x0]), np.array([y0]), *box)
            if res["front"].all():
                continue
            hidden_cases += 1
            D2 = res["D2min"][0]
            bm = _brute_min(cam, f, u[0], E[0], C[0], tuple(b[0] for b in box), n=401)
            if not np.isfinite(bm):
                assert not np.isfinite(D2) or D2 > 1e6
                continue
            assert D2 <= bm * (1 + 1e-9) + 1e-12
            assert bm <= D2 * (1 + 1e-5) + 1e-6
    assert hidden_cases > 5


def test_at_most_two_reachable_edges():
    """Sec. 4.2: with the mean outside the quad, at most two neighbouring
    edges face it, and the minimum over them equals the minimum over all."""
    n_out = 0
    for seed in range(5):
        for cam, f, u, E, C, x0, y0, box in _random_pairs(200 + seed):
            res = tiles_mod.quad_test(cam, f, u, E, C, np.array([x0]), np.array([y0]), *box)
            if res["inside"][0] or not res["front"].all():
                continue
            n_out += 1
            P = res["Pq"][0]
            area = sum(P[k, 0] * P[(k + 1) % 4, 1] - P[(k + 1) % 4, 0] * P[k, 1] for k in range(4))
            facing = []
            for k in range(4):
                a, b = P[k], P[(k + 1) % 4]
                cr = (b[0] - a[0]) * (-a[1]) - (b[1] - a[1]) * (-a[0])
                facing.append(cr * area < 0)
            assert sum(facing) <= 2
            if sum(facing) == 2:
                k = [i for i in range(4) if facing[i]]
                assert (k[1] - k[0]) % 4 in (1, 3)      # neighbouring edges
            m = min(res["edge_D2"][0][k] for k in range(4) if facing[k])
            assert abs(m - res["D2min"][0]) <= 1e-12 * max(1, m)
    assert n_out > 50


def test_inside_tile_gives_mean_and_depth_r():
    cam = synth.camera_translate((0, 0, 0), 90.0, 64, 64)
    f = cam_mod.focal(cam)
    rng = np.random.default_rng(3)
    from oracle import gaussian as g_mod
    for _ in range(10):
        mu = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(1, 3)])
        Sig = g_mod.covariance(rng.standard_normal((4, 1)), rng.uniform(-3, -1, (3, 1)))
        op = proj_mod.optimal_projection(mu[None], Sig, f, 0.3)
        x0 = cam.cx + f * mu[0] / mu[2]
        y0 = cam.cy + f * mu[1] / mu[2]
        tx, ty = int(x0 // 16), int(y0 // 16)
        box = tuple(np.array([v], float) for v in (tx * 16, ty * 16, tx * 16 + 16, ty * 16 + 16))
        res = tiles_mod.quad_test(cam, f, op["u"], op["E"], op["conic"], np.array([x0]), np.array([y0]), *box)
        assert res["inside"][0] and res["D2min"][0] == 0.0
        dep = tiles_mod.tile_depth(op["u"], op["E"], f, res["qhat"], mu[None], np.linalg.inv(Sig))
        assert abs(dep[0] - np.linalg.norm(mu)) < 1e-12


@pytest.mark.parametrize("fov,size,T", [(90.0, 128, 16), (150.0, 96, 16), (110.0, 160, 32)])
def test_cone_bound_is_conservative(fov, size, T):
    """The bounded instance set equals the exhaustive one (every tile tested)."""
    scene = synth.uniform_scene(11, 400, lo=-1.5, hi=1.5, log_scale=(-3.0, 0.8))
    cam = synth.camera_translate((0.1, -0.05, -2.2), fov, size, size - 16)
    params = synth.default_params(tile=T)
    pre = preprocess_view(scene, cam, params)
    grid = tiles_mod.TileGrid(cam.width, cam.height, T)
    a = instances_view(pre, cam, grid, params, OracleOptions())
    b = instances_view(pre, cam, grid, params, OracleOptions(exhaustive_tiles=True))
    ka = sorted(zip(a["tile"].tolist(), a["gid"].tolist()))
    kb = sorted(zip(b["tile"].tolist(), b["gid"].tolist()))
    assert ka == kb and len(ka) > 100


def test_tile_counts_match_paper():
    """Sec. 5.4: 2064x2272 gives 4615 tiles of 32x32."""
    with open(os.path.join(GOLDEN, "tile_counts.json")) as fh:
        g = json.load(fh)
    for case in g["cases"]:
        grid = tiles_mod.TileGrid(case["width"], case["height"], case["tile"])
        assert grid.n == case["tiles"], case


def test_ord_f32_monotone():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(2000) * 10, [0.0, -0.0, 1e-30, -1e-30, 3e38, -3e38]]).astype(np.float32)
    o = tiles_mod.ord_f32(x)
    xs = np.sort(x)
    os_ = np.sort(o)
    np.testing.assert_array_equal(tiles_mod.ord_f32(xs)[np.argsort(tiles_mod.ord_f32(xs), kind="stable")], os_)
    ordx = tiles_mod.ord_f32(xs)
    assert np.all(np.diff(ordx.astype(np.float64)) >= 0)


def test_keys_sort_and_ranges_against_python():
    rng = np.random.default_rng(6)
    n = 3000
    tiles = rng.integers(0, 50, n)
    dep = rng.normal(3, 1, n).astype(np.float32)
    dep[::7] = dep[3]  # ties in depth
    gid = rng.permutation(n)
    keys = tiles_mod.make_keys(tiles, dep)
    sk, sg = tiles_mod.sort_instances(keys, gid)
    ref = sorted(zip(tiles.tolist(), dep.astype(np.float64).tolist(), gid.tolist()))
    assert [(int(k >> np.uint64(32))) for k in sk] == [r[0] for r in ref]
    assert sg.tolist() == [r[2] for r in ref]
    rg = tiles_mod.tile_ranges(sk, 60)
    for t in range(60):
        idx = [i for i, r in enumerate(ref) if r[0] == t]
        if idx:
            assert tuple(rg[t]) == (idx[0], idx[-1] + 1)
        else:
            assert tuple(rg[t]) == (0, 0)


def _edge_argmin(cam, f, u, E, C, box):
    """Brute force over the tile's four boundary edges in pixel space: the
    pixel point with the smallest tangent-plane D^2 (dense sampling, then a
    bounded scalar refinement on the best edge)."""
    from scipy.optimize import minimize_scalar
    x0, y0, x1, y1 = box
    edges = [((x0, y0), (x1, y0)), ((x1, y0), (x1, y1)), ((x1, y1), (x0, y1)), ((x0, y1), (x0, y0))]
    best = (np.inf, None)
    for (ax, ay), (bx, by) in edges:
        s = np.linspace(0.0, 1.0, 4001)
        D = _pixel_D2(cam, f, u, E, C, ax + s * (bx - ax), ay + s * (by - ay))
        k = int(np.argmin(D))
        if not np.isfinite(D[k]):
            continue
        lo, hi = s[max(k - 1, 0)], s[min(k + 1, len(s) - 1)]
        fun = lambda t: float(_pixel_D2(cam, f, u, E, C, np.array(ax + t * (bx - ax)), np.array(ay + t * (by - ay))))
        r = minimize_scalar(fun, bounds=(lo, hi), method="bounded", options=dict(xatol=1e-13))
        t, val = (r.x, r.fun) if r.fun <= D[k] else (s[k], D[k])
        if val < best[0]:
            best = (val, (ax + t * (bx - ax), ay + t * (by - ay)))
    return best


def _ray_argmax_depth(d, mu, Sig):
    """1-D brute force: the ray parameter of maximum 3D Gaussian density along
    the unit ray d (dense scan, then a bounded refinement)."""
    from scipy.optimize import minimize_scalar
    r = np.linalg.norm(mu)
    # Far off the mean's direction the maximum can lie far along the ray, or
    # behind the eye: scan a wide interval on the negative log-density.
    ts = np.linspace(-200.0 * r, 200.0 * r, 400001)
    Binv = np.linalg.inv(Sig)
    x = ts[:, None] * d[None] - mu[None]
    k = int(np.argmin(np.einsum("ki,ij,kj->k", x, Binv, x)))
    nll = lambda t: float(0.5 * (t * d - mu) @ Binv @ (t * d - mu))
    res = minimize_scalar(nll, bounds=(ts[max(k - 1, 0)], ts[min(k + 1, len(ts) - 1)]),
                          method="bounded", options=dict(xatol=1e-13))
    return res.x


@pytest.mark.parametrize("fov,size,seed", [(100.0, 256, 300), (160.0, 128, 301)])
def test_tile_depth_off_the_mean_is_depth_on_the_max_boundary_ray(fov, size, seed):
    """Per-tile depth when the mean lies outside the tile (Sec. 4.2: the
    depth is evaluated at the point of maximum density found by Eq. 4).

    Independent of the tangent-plane back-projection: the pixel point of
    maximum density on the tile boundary is found by brute force in image
    space, and the depth is the 1-D argmax of the 3D density along that
    point's unit ray.  The back-projected ray must also map back to qhat.
    A sign or focal-length mistake in the back-projection fails both."""
    from oracle import gaussian as g_mod
    rng = np.random.default_rng(seed)
    cam = synth.camera_translate((0, 0, 0), fov, size, size)
    f = cam_mod.focal(cam)
    grid = tiles_mod.TileGrid(size, size, 16)
    checked, half_line, wrong_sign_caught, wrong_scale_caught = 0, 0, 0, 0
    tanx = math.tan(math.radians(fov / 2))
    for it in range(600):
        if fov > 150 and it % 2:
            # Large splats close to the eye, just outside the view: their
            # far tiles cross the tangent plane's horizon (half-line edges).
            z = rng.uniform(0.05, 0.4)
            mu = np.array([rng.choice([-1, 1]) * rng.uniform(1.0, 3.0) * tanx * z,
                           rng.uniform(-0.5, 0.5) * tanx * z, z])
            Sig = g_mod.covariance(rng.standard_normal((4, 1)), rng.uniform(-1.5, 0.0, (3, 1)))[0]
        else:
            z = rng.uniform(0.5, 4)
            mu = np.array([rng.uniform(-1.3, 1.3) * tanx * z, rng.uniform(-1.3, 1.3) * tanx * z, z])
            Sig = g_mod.covariance(rng.standard_normal((4, 1)), rng.uniform(-3.5, -1.0, (3, 1)))[0]
        op = proj_mod.optimal_projection(mu[None], Sig[None], f, 0.3)
        x0 = cam.cx + f * mu[0] / mu[2]
        y0 = cam.cy + f * mu[1] / mu[2]
        tile = int(rng.integers(0, grid.n))
        box = grid.boxes(np.array([tile]))
        res = tiles_mod.quad_test(cam, f, op["u"], op["E"], op["conic"], np.array([x0]), np.array([y0]), *box)
        D2 = res["D2min"][0]
        if res["inside"][0] or not np.isfinite(D2) or D2 > 40.0:
            continue
        val, pt = _edge_argmin(cam, f, op["u"][0], op["E"][0], op["conic"][0], tuple(b[0] for b in box))
        assert pt is not None and abs(val - D2) <= 1e-7 * max(1.0, D2)
        half_line += int(not res["front"][0].all())
        B = np.linalg.inv(Sig)
        dep = tiles_mod.tile_depth(op["u"], op["E"], f, res["qhat"], mu[None], B[None])[0]
        d_bf = cam_mod.ray_dirs(cam, pt[0], pt[1])
        t_bf = _ray_argmax_depth(d_bf, mu, Sig)
        rr = np.linalg.norm(mu)
        assert abs(dep - t_bf) <= 1e-7 * rr, (dep, t_bf)
        # Round trip: the back-projected ray has tangent coordinate qhat.
        dd = op["u"][0] + op["E"][0] @ res["qhat"][0] / f
        q_rt, h_rt = proj_mod.tangent_coords(dd / np.linalg.norm(dd), op["u"][0], op["E"][0], f)
        assert h_rt > 0 and np.allclose(q_rt, res["qhat"][0], rtol=1e-10, atol=1e-9)
        # The test has teeth: deliberately wrong back-projections disagree.
        for wrong, counter in (((op["u"][0] - op["E"][0] @ res["qhat"][0] / f), "sign"),
                               ((op["u"][0] + op["E"][0] @ res["qhat"][0]), "scale")):
            w = wrong / np.linalg.norm(wrong)
            tw = float((w @ B @ mu) / (w @ B @ w))
            if abs(tw - t_bf) > 1e-5 * rr:
                if counter == "sign":
                    wrong_sign_caught += 1
                else:
                    wrong_scale_caught += 1
        checked += 1
    assert checked >= 40
    assert wrong_sign_caught >= 0.8 * checked and wrong_scale_caught >= 0.8 * checked
    if fov > 150:
        assert half_line >= 3
