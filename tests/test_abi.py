"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and host-side argument validation rejects bad input before
any device work."""
import ctypes
import os
import re

import pytest

import synth
from paper_2505_10144_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrs.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vrs_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    # The binding wraps exactly the declared functions.
    assert sorted(L.SIGNATURES) == names


def test_version_and_status_strings():
    assert L.load().vrs_version().decode().startswith("vrs ")
    assert L.status_string(0) == "VRS_OK"
    assert L.status_string(-2) == "VRS_ERR_CAPACITY"
    assert L.status_string(-99) == "VRS_ERR_UNKNOWN"


def _sizes(n, cams, fovs, params, cap=0):
    s = L.vrs_sizes()
    rc = L.load().vrs_workspace_size(n, L.camera_array(cams), L.fovea_array(fovs), len(cams),
                                     ctypes.byref(L.make_params(params)), cap, ctypes.byref(s))
    return rc, s


def test_workspace_size_stereo_layout():
    scene, cams, fovs, params = synth.config_stereo(0, n=1000)
    rc, s = _sizes(500_000, cams, fovs, params, 2_000_000)
    assert rc == 0
    assert s.tiles_total == 2 * 65 * 69                     # 32x32 sort tiles per eye
    assert s.items_max == 2 * 4 * 65 * 69
    assert s.proj_bytes == 2 * 500_000 * (128 + 16 + 16)  # record, tile rectangle, colour
    assert s.counts_bytes == 2 * 500_000 * 4
    pre = 2 * 4 * 2064 * 2208 * 4                            # pre-compose images
    # ... then the longest-first ordering of the work items: a 256-byte
    # counter and the ordered items (u32)
    assert pre + 256 + 4 * s.items_max <= s.render_ws_bytes <= pre + 4 * s.items_max + 1024
    assert s.sort_ws_bytes >= 2_000_000 * 12


def test_workspace_size_plain_and_tile32():
    cam = synth.camera_translate((0, 0, -3), 90, 250, 170)
    rc, s = _sizes(10, [cam], [synth.fovea_off()], synth.default_params(tile=16))
    assert rc == 0 and s.tiles_total == 16 * 11 and s.items_max == 16 * 11
    assert 256 + 4 * s.items_max <= s.render_ws_bytes <= 4 * s.items_max + 1024  # work-item ordering only
    rc, s = _sizes(10, [cam], [synth.fovea_off()], synth.default_params(tile=32))
    assert rc == 0 and s.tiles_total == 8 * 6 and s.items_max == 4 * 8 * 6


@pytest.mark.parametrize("bad", [
    dict(tile=8), dict(window=-1), dict(window=33), dict(alpha_min=0.0), dict(alpha_min=1.0),
    dict(depth=3), dict(depth=-1),
    dict(schedule=2), dict(schedule=-1),
    dict(t_min=0.0), dict(z_near=0.0), dict(dilation=-1.0), dict(alpha_max=0.001),
])
def test_invalid_params_rejected(bad):
    cam = synth.camera_translate((0, 0, -3), 90, 64, 64)
    p = synth.default_params()
    for k, v in bad.items():
        setattr(p, k, v)
    rc, _ = _sizes(10, [cam], [synth.fovea_off()], p)
    assert rc == L.VRS_ERR_INVALID_ARG


def test_every_window_accepted_and_unsupported_batch():
    cam = synth.camera_translate((0, 0, -3), 90, 64, 64)
    for w in range(0, 33):
        rc, _ = _sizes(10, [cam], [synth.fovea_off()], synth.default_params(window=w))
        assert rc == L.VRS_OK, w
    rc, _ = _sizes(10, [cam], [synth.fovea_off()], synth.default_params(blend_batch=96))
    assert rc == L.VRS_ERR_UNSUPPORTED


def test_invalid_cameras_and_views_rejected():
    cam = synth.camera_translate((0, 0, -3), 90, 64, 64)
    p = synth.default_params()
    for w, h, fov in [(0, 64, 90), (64, 0, 90), (64, 64, 0), (64, 64, 180)]:
        c = synth.Camera(cam.world_to_cam, fov, 32, 32, w, h)
        assert _sizes(10, [c], [synth.fovea_off()], p)[0] == L.VRS_ERR_INVALID_ARG
    assert _sizes(-1, [cam], [synth.fovea_off()], p)[0] == L.VRS_ERR_INVALID_ARG
    many = [cam] * (L.VRS_MAX_VIEWS + 1)
    assert _sizes(10, many, [synth.fovea_off()] * len(many), p)[0] == L.VRS_ERR_INVALID_ARG
    bad_fov = synth.Fovea(True, (32.0, 32.0), -1.0, 0.1)
    assert _sizes(10, [cam], [bad_fov], p)[0] == L.VRS_ERR_INVALID_ARG


def test_entry_points_validate_before_device_work():
    lib = L.load()
    cam = L.camera_array([synth.camera_translate((0, 0, -3), 90, 64, 64)])
    fov = L.fovea_array([synth.fovea_off()])
    p = L.make_params(synth.default_params())
    g = L.vrs_gaussians()
    g.n = 5
    g.sh_degree = 4  # invalid
    null = ctypes.c_void_p(0)
    assert lib.vrs_preprocess(ctypes.byref(g), cam, fov, 1, ctypes.byref(p), null, null, null, null, null) == L.VRS_ERR_INVALID_ARG
    g.sh_degree = 3  # valid degree but NULL parameter pointers
    assert lib.vrs_preprocess(ctypes.byref(g), cam, fov, 1, ctypes.byref(p), null, null, null, null, null) == L.VRS_ERR_INVALID_ARG
    assert lib.vrs_sort_pairs(null, null, null, 10, 40, null, 0, null, null) == L.VRS_ERR_INVALID_ARG
    assert lib.vrs_sort_pairs(null, null, null, 10, 65, null, 0, null, null) == L.VRS_ERR_INVALID_ARG
    assert lib.vrs_fovea_plan(cam, fov, 1, ctypes.byref(p), None, null, 0, None, null) == L.VRS_ERR_INVALID_ARG
    imgs = (ctypes.c_void_p * 1)(0)
    assert lib.vrs_render_foveated(null, -1, null, null, cam, fov, 1, ctypes.byref(p), null, 0, imgs, null, 0,
                                   null, null) == L.VRS_ERR_INVALID_ARG
    assert L.load().vrs_sort_pairs_workspace_size(0) > 0


def test_noalloc_sort_rejects_requests_beyond_its_scratch():
    """The no-allocation sort refuses capacities beyond its fixed scratch
    array on the host, before any device call, and checks its arguments."""
    lib = L.load()
    big = L.VRS_SORT_NOALLOC_MAX_PAIRS + 1
    assert lib.vrs_sort_pairs_noalloc(None, None, ctypes.c_void_p(16), big, 40, None, None) == L.VRS_ERR_SCRATCH
    assert L.status_string(L.VRS_ERR_SCRATCH) == "VRS_ERR_SCRATCH"
    assert lib.vrs_sort_pairs_noalloc(None, None, None, 10, 40, None, None) == L.VRS_ERR_INVALID_ARG
    assert lib.vrs_sort_pairs_noalloc(None, None, ctypes.c_void_p(16), 10, 65, None, None) == L.VRS_ERR_INVALID_ARG
    assert lib.vrs_sort_pairs_noalloc(None, None, ctypes.c_void_p(16), 10, 40, None, None) == L.VRS_ERR_INVALID_ARG
    # The scratch holds the workspace of the largest request.
    assert lib.vrs_sort_pairs_workspace_size(L.VRS_SORT_NOALLOC_MAX_PAIRS) < 40 << 20


def test_training_and_two_pass_entry_points_validate_arguments():
    """The two-pass, loss, Adam and backward entry points reject bad
    arguments on the host, before any device work."""
    lib = L.load()
    bad = L.VRS_ERR_INVALID_ARG
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    cam = L.camera_array([synth.camera_translate((0, 0, -3), 90, 64, 64)])
    fov = L.fovea_array([synth.fovea_off()])
    p = L.make_params(synth.default_params())
    ptrs = (ctypes.c_void_p * 1)(256)
    nulls = (ctypes.c_void_p * 1)(0)
    # Two-pass: a plan is required; the centre box must lie in the image.
    ccam, lcam = (L.vrs_camera * 1)(), (L.vrs_camera * 1)()
    boxes = (ctypes.c_int32 * 4)()
    assert lib.vrs_two_pass_views(cam, fov, 1, ctypes.byref(p), null, ccam, boxes, lcam, null) == bad
    assert lib.vrs_two_pass_views(cam, fov, 0, ctypes.byref(p), fake, ccam, boxes, lcam, null) == bad
    assert lib.vrs_two_pass_compose(cam, fov, 1, boxes, nulls, nulls, nulls, null) == bad
    outside = (ctypes.c_int32 * 4)(0, 0, 65, 64)
    assert lib.vrs_two_pass_compose(cam, fov, 1, outside, ptrs, ptrs, ptrs, null) == bad
    # Loss: workspace of one FP64 partial per block, 8-byte aligned.
    assert lib.vrs_loss_workspace_size(0) == 0
    need = lib.vrs_loss_workspace_size(1)
    assert need > 0 and lib.vrs_loss_workspace_size(3) == 3 * need
    assert lib.vrs_loss_l1l2(cam, 1, ptrs, ptrs, ptrs, fake, null, need, null) == bad
    assert lib.vrs_loss_l1l2(cam, 1, ptrs, ptrs, ptrs, fake, ctypes.c_void_p(260), need, null) == bad
    assert lib.vrs_loss_l1l2(cam, 1, ptrs, ptrs, ptrs, fake, fake, need - 8, null) == bad
    assert lib.vrs_loss_l1l2(cam, 0, ptrs, ptrs, ptrs, fake, fake, need, null) == bad
    # Adam: an empty update is a no-op; hyper-parameters are checked.
    assert lib.vrs_adam_step(null, null, null, null, 0, 1e-3, 0.9, 0.999, 1e-15, 1, null) == L.VRS_OK
    ok_args = dict(lr=1e-3, b1=0.9, b2=0.999, eps=1e-15, step=1)
    for change in (dict(b1=1.0), dict(b2=-0.1), dict(eps=0.0), dict(step=0), dict(lr=float("nan"))):
        a = dict(ok_args, **change)
        assert lib.vrs_adam_step(fake, fake, fake, fake, 10, a["lr"], a["b1"], a["b2"], a["eps"], a["step"],
                                 null) == bad, change
    assert lib.vrs_adam_step(null, fake, fake, fake, 10, 1e-3, 0.9, 0.999, 1e-15, 1, null) == bad
    # Backward: Gaussian parameters and buffers are checked first.
    assert lib.vrs_backward_workspace_size(10, cam, fov, 1, ctypes.byref(p)) > 0
    g = L.vrs_gaussians()
    g.n = 5
    g.sh_degree = 3
    grads = L.vrs_gaussian_grads()
    assert lib.vrs_render_backward(ctypes.byref(g), null, null, null, cam, fov, 1, ctypes.byref(p), null, 0, ptrs,
                                   ptrs, ctypes.byref(grads), null, 0, null, null) == bad
