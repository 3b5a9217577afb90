"""FP64 CPU oracle for the VRSplat rendering path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never calls into it, and the two share
no code: this package re-derives every quantity from the paper's definitions in
plain NumPy float64 so that the GPU kernels can be checked against it.

Module map (each function cites the passage it follows):

* ``gaussian``   -- Sec. 3, Eq. 1: rotation, scale, covariance, opacity.
* ``camera``     -- pinhole rays for the cameras of Sec. 5 / App. D.
* ``projection`` -- Optimal Projection onto the per-Gaussian tangent plane
                    (Sec. 3 end, Sec. 4.2) and the EWA local-affine projection
                    of Eq. 3 (kept only as a test reference).
* ``sh``         -- view-dependent colour from real spherical harmonics built
                    from the associated-Legendre definition (no constant table).
* ``depth``      -- depth along a view ray (per-pixel resorting, Sec. 4.1).
* ``tiles``      -- tile grid, the tile-culling test on tangent-plane
                    quadrilaterals (Sec. 4.2, Eq. 4, Fig. 4), per-tile depth,
                    sort keys and tile ranges (Sec. 3 tile binning).
* ``blend``      -- front-to-back compositing (Eq. 2) with a per-sample resort
                    window, and the exhaustive per-pixel sort.
* ``fovea``      -- single-pass foveation classes, hybrid blending and the
                    periphery reconstruction (Sec. 4.3, Fig. 5a).
* ``render``     -- the whole forward pass, plus borderline-decision flags.

Parity status: every function here is pinned by a CPU test in ``tests/``
against a closed form, an invariant, brute force or a worked count from the
paper, except where a header says "parity unpinned".
"""
from . import gaussian, camera, projection, sh, depth, tiles, blend, fovea  # noqa: F401
from .render import render, preprocess_view, OracleOptions  # noqa: F401
