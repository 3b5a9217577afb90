"""ctypes binding of ``libvrs.so`` (include/vrs.h), with the same entry-point
names.  Argument marshalling only: every step of the rendering path runs in
the library's HIP kernels.  Loading fails loudly when the library is missing.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrs.so")

VRS_OK = 0
VRS_ERR_INVALID_ARG = -1
VRS_ERR_CAPACITY = -2
VRS_ERR_HIP = -3
VRS_ERR_UNSUPPORTED = -4
VRS_ERR_SCRATCH = -5
VRS_ERR_NONFINITE = -6
VRS_SORT_NOALLOC_MAX_PAIRS = 2097152
VRS_MAX_VIEWS = 32
VRS_MAX_WINDOW = 32
VRS_RECORD_FLOATS = 32
TILERECT_BYTES = 16  # candidate tile rectangle per (view, Gaussian), after the render records
VRS_CLASS_LOW, VRS_CLASS_HIGH, VRS_CLASS_HYBRID, VRS_CLASS_PLAIN = 0, 1, 2, 3
VRS_SCHEDULE_ONESHOT, VRS_SCHEDULE_PERSISTENT = 0, 1
PLAN_ITEMS_OFFSET = 256

c_float_p = ctypes.POINTER(ctypes.c_float)
c_u32_p = ctypes.POINTER(ctypes.c_uint32)
c_u64_p = ctypes.POINTER(ctypes.c_uint64)
c_i32_p = ctypes.POINTER(ctypes.c_int32)


class vrs_gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class vrs_camera(ctypes.Structure):
    _fields_ = [("world_to_cam", ctypes.c_float * 12), ("fov_x_deg", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class vrs_fovea(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int32), ("center_px", ctypes.c_float * 2),
                ("radius_deg", ctypes.c_float), ("band_frac", ctypes.c_float),
                ("shape", ctypes.c_int32), ("half_px", ctypes.c_float * 2)]


class vrs_params(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("window", ctypes.c_int32),
                ("blend_batch", ctypes.c_int32), ("schedule", ctypes.c_int32), ("z_near", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float),
                ("background", ctypes.c_float * 3), ("depth_mode", ctypes.c_int32)]


class vrs_sizes(ctypes.Structure):
    _fields_ = [("proj_bytes", ctypes.c_size_t), ("counts_bytes", ctypes.c_size_t),
                ("tiles_total", ctypes.c_uint32), ("items_max", ctypes.c_uint32),
                ("plan_bytes", ctypes.c_size_t), ("sort_ws_bytes", ctypes.c_size_t),
                ("render_ws_bytes", ctypes.c_size_t)]


class vrs_gaussian_grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacity_logits", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


# Every function the header declares, with its ctypes signature.
_P = ctypes.c_void_p
_I = ctypes.c_int32
_S = ctypes.c_size_t
_U = ctypes.c_uint32
SIGNATURES = {
    "vrs_workspace_size": (_I, [_I, ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                                ctypes.POINTER(vrs_params), _S, ctypes.POINTER(vrs_sizes)]),
    "vrs_fovea_plan": (_I, [ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                            ctypes.POINTER(vrs_params), ctypes.POINTER(ctypes.c_void_p), _P, _S, c_u32_p, _P]),
    "vrs_preprocess": (_I, [ctypes.POINTER(vrs_gaussians), ctypes.POINTER(vrs_camera),
                            ctypes.POINTER(vrs_fovea), _I, ctypes.POINTER(vrs_params), _P, _P, _P, _P, _P]),
    "vrs_duplicate": (_I, [ctypes.POINTER(vrs_gaussians), ctypes.POINTER(vrs_camera),
                           ctypes.POINTER(vrs_fovea), _I, ctypes.POINTER(vrs_params), _P, _P, _P, _P, _P, _S,
                           _P, _P, _S, _P, _P]),
    "vrs_sort_pairs": (_I, [_P, _P, _P, _S, _I, _P, _S, _P, _P]),
    "vrs_sort_pairs_workspace_size": (_S, [_S]),
    "vrs_sort_pairs_noalloc": (_I, [_P, _P, _P, _S, _I, _P, _P]),
    "vrs_tile_ranges": (_I, [_P, _P, _S, _U, _P, _P]),
    "vrs_sort": (_I, [ctypes.POINTER(vrs_gaussians), ctypes.POINTER(vrs_camera),
                      ctypes.POINTER(vrs_fovea), _I, ctypes.POINTER(vrs_params), _P, _P, _P, _P, _P, _S,
                      _P, _P, _P, _S, _P, _P]),
    "vrs_render_foveated": (_I, [_P, _I, _P, _P, ctypes.POINTER(vrs_camera),
                                 ctypes.POINTER(vrs_fovea), _I, ctypes.POINTER(vrs_params), _P, _U,
                                 ctypes.POINTER(ctypes.c_void_p), _P, _S, _P, _P]),
    "vrs_blend": (_I, [_P, _I, _P, _P, ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                       ctypes.POINTER(vrs_params), _P, _U, ctypes.POINTER(ctypes.c_void_p), _P, _S, _P, _P]),
    "vrs_blend_stats": (_I, [_P, _I, _P, _P, ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                             ctypes.POINTER(vrs_params), _P, _U, ctypes.POINTER(ctypes.c_void_p), _P, _S, _P,
                             _P]),
    "vrs_compose": (_I, [ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I, ctypes.POINTER(vrs_params),
                         _P, ctypes.POINTER(ctypes.c_void_p), _P, _S, _P]),
    "vrs_backward_workspace_size": (_S, [_I, ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                                         ctypes.POINTER(vrs_params)]),
    "vrs_render_backward": (_I, [ctypes.POINTER(vrs_gaussians), _P, _P, _P, ctypes.POINTER(vrs_camera),
                                 ctypes.POINTER(vrs_fovea), _I, ctypes.POINTER(vrs_params), _P, _U,
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                 ctypes.POINTER(vrs_gaussian_grads), _P, _S, _P, _P]),
    "vrs_two_pass_views": (_I, [ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                                ctypes.POINTER(vrs_params), _P, ctypes.POINTER(vrs_camera),
                                ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vrs_camera), _P]),
    "vrs_two_pass_compose": (_I, [ctypes.POINTER(vrs_camera), ctypes.POINTER(vrs_fovea), _I,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _P]),
    "vrs_loss_workspace_size": (_S, [_I]),
    "vrs_loss_l1l2": (_I, [ctypes.POINTER(vrs_camera), _I, ctypes.POINTER(ctypes.c_void_p),
                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), _P, _P, _S, _P]),
    "vrs_adam_step": (_I, [_P, _P, _P, _P, _S, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           _I, _P]),
    "vrs_status_string": (ctypes.c_char_p, [_I]),
    "vrs_version": (ctypes.c_char_p, []),
}

_lib = None


class VrsError(RuntimeError):
    def __init__(self, fn, code):
        self.code = code
        name = status_string(code) if _lib is not None else str(code)
        super().__init__(f"{fn} failed: {name} ({code})")


def load(path=None):
    """Load the library once.  Raises if it is missing: there is no fallback.

    PyTorch is imported first.  Its wheel ships its own HIP runtime, which
    its libraries name by a different file name than the runtime's soname:
    loaded before torch, the library would bind the system runtime and torch
    would then load a second one, and device pointers and streams of one
    runtime are invalid in the other.  Loaded after torch, the library binds
    the runtime torch already holds (same soname)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (binds the HIP runtime the tensors live in)
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with paper_2505_10144_amd.build.build() "
            "(hipcc --offload-arch=gfx950); the renderer has no non-HIP path")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code):
    return load().vrs_status_string(int(code)).decode()


def check(fn, code):
    if code != VRS_OK:
        raise VrsError(fn, code)


def call(name, *args):
    """Call ``name`` and raise VrsError on a non-zero status."""
    rc = getattr(load(), name)(*args)
    check(name, rc)
    return rc


# -- struct builders from the synth dataclasses ---------------------------------

def make_camera(cam) -> vrs_camera:
    c = vrs_camera()
    m = [float(x) for x in cam.world_to_cam.reshape(-1)]
    c.world_to_cam = (ctypes.c_float * 12)(*m)
    c.fov_x_deg = float(cam.fov_x_deg)
    c.cx = float(cam.cx)
    c.cy = float(cam.cy)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


def make_fovea(f) -> vrs_fovea:
    o = vrs_fovea()
    o.enabled = 1 if f.enabled else 0
    o.center_px = (ctypes.c_float * 2)(float(f.center_px[0]), float(f.center_px[1]))
    o.radius_deg = float(f.radius_deg)
    o.band_frac = float(f.band_frac)
    o.shape = int(getattr(f, "shape", 0))
    hp = getattr(f, "half_px", (0.0, 0.0))
    o.half_px = (ctypes.c_float * 2)(float(hp[0]), float(hp[1]))
    return o


def make_params(p) -> vrs_params:
    o = vrs_params()
    o.tile = int(p.tile)
    o.window = int(p.window)
    o.blend_batch = int(p.blend_batch) if p.blend_batch else 64
    o.schedule = int(getattr(p, "schedule", VRS_SCHEDULE_ONESHOT))
    o.z_near = float(p.z_near)
    o.alpha_min = float(p.alpha_min)
    o.alpha_max = float(p.alpha_max)
    o.t_min = float(p.t_min)
    o.dilation = float(p.dilation)
    o.background = (ctypes.c_float * 3)(*[float(b) for b in p.background])
    o.depth_mode = int(getattr(p, "depth", 0))
    return o


def camera_array(cams):
    arr = (vrs_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = make_camera(c)
    return arr


def fovea_array(foveas):
    arr = (vrs_fovea * len(foveas))()
    for i, f in enumerate(foveas):
        arr[i] = make_fovea(f)
    return arr
