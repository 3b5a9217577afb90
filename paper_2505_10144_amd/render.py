"""Torch glue over the C ABI: device buffers and streams come from PyTorch,
every computation runs in libvrs's HIP kernels.

Typical use::

    r = Renderer(cams, foveas, params, n_gaussians)
    g = r.upload(scene)               # SoA float32 tensors on the GPU
    images = r.render(g)              # list of (4, H, W) float32 tensors

``Renderer`` owns every buffer of one configuration (cameras, foveae, knobs,
Gaussian count), builds the foveation plan once (the paper precomputes the
tile mapping per eye and reuses it across frames, Sec. 4.3) and sizes the
instance buffers from an exact count on first use.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Gaussians:
    """Device-resident Gaussian parameters in the library's SoA layout."""

    def __init__(self, means, log_scales, quats, opacity_logits, sh, sh_degree=3):
        self.means = means.contiguous()
        self.log_scales = log_scales.contiguous()
        self.quats = quats.contiguous()
        self.opacity_logits = opacity_logits.contiguous()
        self.sh = sh.contiguous()
        self.sh_degree = int(sh_degree)
        for t in (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh):
            if t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError("Gaussian parameters must be float32 CUDA tensors")

    @property
    def n(self):
        return int(self.means.shape[1])

    def struct(self) -> L.vrs_gaussians:
        g = L.vrs_gaussians()
        g.n = self.n
        g.sh_degree = self.sh_degree
        g.means = self.means.data_ptr()
        g.log_scales = self.log_scales.data_ptr()
        g.quats = self.quats.data_ptr()
        g.opacity_logits = self.opacity_logits.data_ptr()
        g.sh = self.sh.data_ptr()
        return g


def upload(scene, device="cuda") -> Gaussians:
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return Gaussians(t(scene.means), t(scene.log_scales), t(scene.quats),
                     t(scene.opacity_logits), t(scene.sh), scene.sh_degree)


class Renderer:
    def __init__(self, cams: Sequence, foveas, params, n: int, device="cuda",
                 capacity: Optional[int] = None, stream=None, masks=None):
        """``masks``: optional per-view headset visibility masks (uint8
        arrays or tensors [H][W], nonzero = visible, or None) for
        visibility culling; they are copied to the device and consumed by
        the plan."""
        if not isinstance(foveas, (list, tuple)):
            foveas = [foveas] * len(cams)
        if len(cams) != len(foveas):
            raise ValueError("one fovea per camera")
        self.cams, self.foveas, self.params = list(cams), list(foveas), params
        self.n = int(n)
        self.device = torch.device(device)
        self.stream = stream
        self.c_cams = L.camera_array(self.cams)
        self.c_fovs = L.fovea_array(self.foveas)
        self.c_params = L.make_params(params)
        self.V = len(self.cams)
        sizes = self._sizes(0)
        self.tiles_total = sizes.tiles_total
        dev = self.device
        u8 = lambda nbytes: torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
        self.proj = u8(sizes.proj_bytes)
        self.counts = torch.empty(max(self.V * self.n, 1), dtype=torch.int32, device=dev)
        self.ranges = torch.empty(max(2 * self.tiles_total, 2), dtype=torch.int32, device=dev)
        self.n_inst = torch.zeros(2, dtype=torch.int32, device=dev)  # [candidates, kept]
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.plan = u8(sizes.plan_bytes)
        self.render_ws = u8(sizes.render_ws_bytes)
        self.images = [torch.empty((4, c.height, c.width), dtype=torch.float32, device=dev)
                       for c in self.cams]
        self._img_ptrs = (ctypes.c_void_p * self.V)(*[im.data_ptr() for im in self.images])
        self.capacity = 0
        self.keys = self.gids = self.sort_ws = None
        if capacity is not None:
            self._alloc_instances(int(capacity))
        n_items = ctypes.c_uint32(0)
        mask_t = [None] * self.V
        if masks is not None:
            for v, m in enumerate(masks):
                if m is None:
                    continue
                m = torch.as_tensor(np.asarray(m.cpu() if torch.is_tensor(m) else m, dtype=np.uint8))
                if tuple(m.shape) != (self.cams[v].height, self.cams[v].width):
                    raise ValueError("a visibility mask is [height][width]")
                mask_t[v] = m.contiguous().to(dev)
        self.masks = mask_t
        mask_ptrs = (ctypes.c_void_p * self.V)(*[(m.data_ptr() if m is not None else 0) for m in mask_t])
        L.call("vrs_fovea_plan", self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), mask_ptrs,
               _ptr(self.plan), ctypes.c_size_t(self.plan.numel()), ctypes.byref(n_items),
               _stream(self.stream))
        self.n_items = int(n_items.value)
        self.items_max = sizes.items_max
        self.generation = 0  # forward passes run (the backward replays the latest)

    # -- sizes / buffers --------------------------------------------------------
    def _sizes(self, capacity):
        s = L.vrs_sizes()
        L.call("vrs_workspace_size", self.n, self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), ctypes.c_size_t(capacity), ctypes.byref(s))
        return s

    def _alloc_instances(self, capacity):
        s = self._sizes(capacity)
        self.capacity = capacity
        dev = self.device
        self.keys = torch.empty(max(capacity, 1), dtype=torch.int64, device=dev)
        self.gids = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
        self.sort_ws = torch.empty(max(int(s.sort_ws_bytes), 256), dtype=torch.uint8, device=dev)

    def ensure_capacity(self, g: Gaussians, headroom=1.25):
        """Exact instance count of the current scene/cameras (one sync), and
        instance buffers of at least that size times ``headroom``."""
        if self.sort_ws is None:
            self._alloc_instances(0)
        self.preprocess(g)
        self.status.zero_()
        L.call("vrs_duplicate", ctypes.byref(g.struct()), self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), _ptr(self.plan), _ptr(self.proj), _ptr(self.counts), _ptr(self.keys),
               _ptr(self.gids), ctypes.c_size_t(0), _ptr(self.n_inst), _ptr(self.sort_ws),
               ctypes.c_size_t(self.sort_ws.numel()), _ptr(self.status), _stream(self.stream))
        need = int(self.n_inst[0].item())
        if need > self.capacity:
            self._alloc_instances(max(int(need * headroom), 1024))
        self.status.zero_()
        return need

    # -- stages -------------------------------------------------------------------
    def preprocess(self, g: Gaussians):
        L.call("vrs_preprocess", ctypes.byref(g.struct()), self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), _ptr(self.plan), _ptr(self.proj), _ptr(self.counts),
               _ptr(self.status), _stream(self.stream))

    def duplicate(self, g: Gaussians):
        L.call("vrs_duplicate", ctypes.byref(g.struct()), self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), _ptr(self.plan), _ptr(self.proj), _ptr(self.counts), _ptr(self.keys),
               _ptr(self.gids), ctypes.c_size_t(self.capacity), _ptr(self.n_inst), _ptr(self.sort_ws),
               ctypes.c_size_t(self.sort_ws.numel()), _ptr(self.status), _stream(self.stream))

    def key_bits(self):
        b = 0
        while (1 << b) < self.tiles_total:
            b += 1
        return 32 + b

    def sort(self, g: Gaussians):
        L.call("vrs_sort", ctypes.byref(g.struct()), self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), _ptr(self.plan), _ptr(self.proj), _ptr(self.counts), _ptr(self.keys),
               _ptr(self.gids),
               ctypes.c_size_t(self.capacity), _ptr(self.n_inst), _ptr(self.ranges),
               _ptr(self.sort_ws), ctypes.c_size_t(self.sort_ws.numel()), _ptr(self.status),
               _stream(self.stream))

    def blend_only(self):
        L.call("vrs_blend", _ptr(self.proj), self.n, _ptr(self.gids), _ptr(self.ranges),
               self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), _ptr(self.plan),
               ctypes.c_uint32(self.n_items), self._img_ptrs, _ptr(self.render_ws),
               ctypes.c_size_t(self.render_ws.numel()), _ptr(self.status), _stream(self.stream))

    def compose(self):
        L.call("vrs_compose", self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), _ptr(self.plan),
               self._img_ptrs, _ptr(self.render_ws), ctypes.c_size_t(self.render_ws.numel()),
               _stream(self.stream))

    def blend_stats(self):
        """Instrumented blend: returns dict of work counters (one sync)."""
        c = torch.zeros(6, dtype=torch.int64, device=self.device)
        L.call("vrs_blend_stats", _ptr(self.proj), self.n, _ptr(self.gids), _ptr(self.ranges),
               self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), _ptr(self.plan),
               ctypes.c_uint32(self.n_items), self._img_ptrs, _ptr(self.render_ws),
               ctypes.c_size_t(self.render_ws.numel()), _ptr(c), _stream(self.stream))
        v = c.cpu().tolist()
        return dict(pairs=v[0], contrib=v[1], samples=v[2], stopped=v[3], staged=v[4], push_steps=v[5])

    def blend(self):
        L.call("vrs_render_foveated", _ptr(self.proj), self.n, _ptr(self.gids), _ptr(self.ranges),
               self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), _ptr(self.plan),
               ctypes.c_uint32(self.n_items), self._img_ptrs, _ptr(self.render_ws),
               ctypes.c_size_t(self.render_ws.numel()), _ptr(self.status), _stream(self.stream))

    def render(self, g: Gaussians) -> List[torch.Tensor]:
        """One frame for every view: preprocess, sort, blend (and compose)."""
        if g.n != self.n:
            raise ValueError("Gaussian count differs from the renderer's")
        if self.sort_ws is None:
            self.ensure_capacity(g)
        self.preprocess(g)
        self.sort(g)
        self.blend()
        self.generation += 1
        return self.images

    def backward(self, g: Gaussians, grad_images: Sequence[torch.Tensor],
                 images: Optional[Sequence[torch.Tensor]] = None) -> dict:
        """Gradients of sum_v <grad_images[v], images[v]> with respect to the
        Gaussian parameters, for the forward pass whose state (records,
        sorted instances, ranges) this renderer currently holds.  ``images``
        defaults to the renderer's own output buffers (plain views; a
        foveated view's backward re-renders its samples instead)."""
        if g.n != self.n:
            raise ValueError("Gaussian count differs from the renderer's")
        images = list(images) if images is not None else self.images
        if len(grad_images) != self.V or len(images) != self.V:
            raise ValueError("one image and one gradient per view")
        grads = [gi.contiguous().to(torch.float32) for gi in grad_images]
        for gi, c in zip(grads, self.cams):
            if tuple(gi.shape) != (4, c.height, c.width) or not gi.is_cuda:
                raise ValueError("gradients must be (4, H, W) CUDA tensors")
        imgs = [im.contiguous() for im in images]
        need = int(L.load().vrs_backward_workspace_size(self.n, self.c_cams, self.c_fovs, self.V,
                                                        ctypes.byref(self.c_params)))
        if getattr(self, "bwd_ws", None) is None or self.bwd_ws.numel() < max(need, 256):
            self.bwd_ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        dev = self.device
        out = dict(means=torch.empty_like(g.means), log_scales=torch.empty_like(g.log_scales),
                   quats=torch.empty_like(g.quats), opacity_logits=torch.empty_like(g.opacity_logits),
                   sh=torch.zeros_like(g.sh))
        gs = L.vrs_gaussian_grads()
        gs.means = out["means"].data_ptr()
        gs.log_scales = out["log_scales"].data_ptr()
        gs.quats = out["quats"].data_ptr()
        gs.opacity_logits = out["opacity_logits"].data_ptr()
        gs.sh = out["sh"].data_ptr()
        img_ptrs = (ctypes.c_void_p * self.V)(*[im.data_ptr() for im in imgs])
        grad_ptrs = (ctypes.c_void_p * self.V)(*[gi.data_ptr() for gi in grads])
        L.call("vrs_render_backward", ctypes.byref(g.struct()), _ptr(self.proj), _ptr(self.gids),
               _ptr(self.ranges), self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), _ptr(self.plan),
               ctypes.c_uint32(self.n_items), img_ptrs,
               grad_ptrs, ctypes.byref(gs), _ptr(self.bwd_ws), ctypes.c_size_t(self.bwd_ws.numel()),
               _ptr(self.status), _stream(self.stream))
        # Keep the inputs alive until the kernels that read them are done.
        self._bwd_keep = (imgs, grads)
        return out

    def check(self):
        """Synchronise and raise if the device reported an error (capacity)."""
        st = int(self.status.item())
        if st != L.VRS_OK:
            raise L.VrsError("device", st)
        return int(self.n_inst[1].item())

    # -- views of the plan, for tests and tools -----------------------------------
    def plan_items(self) -> np.ndarray:
        off = L.PLAN_ITEMS_OFFSET
        raw = self.plan[off:off + 4 * self.n_items].cpu().numpy().view(np.uint32)
        return raw.copy()

    def plan_classes(self) -> bytes:
        off = L.PLAN_ITEMS_OFFSET + 4 * self.items_max
        return self.plan[off:].cpu().numpy()

    def pre_images(self) -> List[torch.Tensor]:
        """Per view, the blend's output before the periphery compose: for a
        foveated view the pre-compose image in the render workspace (LOW
        groups written to their 2x2 pixels, HYBRID pixels already mixed), for
        a plain view the output image itself."""
        out, off = [], 0
        for c, f, im in zip(self.cams, self.foveas, self.images):
            if f.enabled:
                n = 4 * c.width * c.height
                out.append(self.render_ws[4 * off:4 * (off + n)].view(torch.float32).view(4, c.height, c.width))
                off += n
            else:
                out.append(im)
        return out

    def records(self) -> torch.Tensor:
        return self.proj[: self.V * self.n * L.VRS_RECORD_FLOATS * 4].view(torch.float32).view(
            self.V, self.n, L.VRS_RECORD_FLOATS)

    def colours(self) -> torch.Tensor:
        """[V][n][4] float32: each Gaussian's colour (r, g, b, 0) per view,
        after the render records and tile rectangles in `proj`."""
        off = self.V * self.n * (L.VRS_RECORD_FLOATS * 4 + L.TILERECT_BYTES)
        return self.proj[off: off + self.V * self.n * 16].view(torch.float32).view(self.V, self.n, 4)


class _Cam:
    """A camera description read back from the library (the attributes
    ``_lib.make_camera`` reads)."""

    def __init__(self, c: L.vrs_camera):
        self.world_to_cam = np.array(list(c.world_to_cam), np.float32).reshape(3, 4)
        self.fov_x_deg = float(c.fov_x_deg)
        self.cx = float(c.cx)
        self.cy = float(c.cy)
        self.width = int(c.width)
        self.height = int(c.height)


class TwoPassRenderer:
    """The two-pass foveated baseline (App. A) over the same library: a
    centre pass at full resolution through the tight frustum of the centre
    region, a periphery pass at half resolution (both plain renders with
    16x16 tiles, all views of a pass in one call sequence), then
    vrs_two_pass_compose blends them into the output images."""

    def __init__(self, cams: Sequence, foveas, params, n: int, device="cuda", stream=None):
        if not isinstance(foveas, (list, tuple)):
            foveas = [foveas] * len(cams)
        self.cams, self.foveas, self.params = list(cams), list(foveas), params
        self.V = len(self.cams)
        self.stream = stream
        self.c_cams = L.camera_array(self.cams)
        self.c_fovs = L.fovea_array(self.foveas)
        # The single-pass plan of these views gives the centre region.
        plan_r = Renderer(self.cams, self.foveas, params, n, device=device, stream=stream)
        ccams = (L.vrs_camera * self.V)()
        lcams = (L.vrs_camera * self.V)()
        boxes = (ctypes.c_int32 * (4 * self.V))()
        L.call("vrs_two_pass_views", self.c_cams, self.c_fovs, self.V, ctypes.byref(plan_r.c_params),
               _ptr(plan_r.plan), ccams, boxes, lcams, _stream(stream))
        del plan_r
        self.boxes = boxes
        self.box_list = [tuple(boxes[4 * v:4 * v + 4]) for v in range(self.V)]
        self.centre_views = [v for v in range(self.V) if self.box_list[v][2] > self.box_list[v][0]]
        off = [synth_fovea_off() for _ in range(self.V)]
        p1 = params.replace(tile=16)
        p2 = params.replace(tile=16, dilation=float(np.float32(params.dilation) * np.float32(0.25)))
        self.centre_cams = [_Cam(ccams[v]) for v in self.centre_views]
        self.low_cams = [_Cam(lcams[v]) for v in range(self.V)]
        self.centre = (Renderer(self.centre_cams, off[:len(self.centre_cams)], p1, n, device=device, stream=stream)
                       if self.centre_views else None)
        self.low = Renderer(self.low_cams, off, p2, n, device=device, stream=stream)
        self.images = [torch.empty((4, c.height, c.width), dtype=torch.float32, device=device) for c in self.cams]
        self._out_ptrs = (ctypes.c_void_p * self.V)(*[im.data_ptr() for im in self.images])

    def ensure_capacity(self, g: Gaussians):
        if self.centre is not None:
            self.centre.ensure_capacity(g)
        self.low.ensure_capacity(g)

    def render(self, g: Gaussians) -> List[torch.Tensor]:
        """Both passes, then the blend."""
        cimgs = self.centre.render(g) if self.centre is not None else []
        limgs = self.low.render(g)
        self.compose(cimgs, limgs)
        return self.images

    def compose(self, cimgs=None, limgs=None):
        cimgs = self.centre.images if cimgs is None and self.centre is not None else (cimgs or [])
        limgs = self.low.images if limgs is None else limgs
        cptr = [0] * self.V
        for k, v in enumerate(self.centre_views):
            cptr[v] = cimgs[k].data_ptr()
        c_arr = (ctypes.c_void_p * self.V)(*cptr)
        l_arr = (ctypes.c_void_p * self.V)(*[im.data_ptr() for im in limgs])
        L.call("vrs_two_pass_compose", self.c_cams, self.c_fovs, self.V, self.boxes, c_arr, l_arr,
               self._out_ptrs, _stream(self.stream))

    def check(self):
        n = self.low.check()
        if self.centre is not None:
            n += self.centre.check()
        return n


def synth_fovea_off():
    """A disabled fovea (the attributes ``_lib.make_fovea`` reads)."""
    class _F:
        enabled = False
        center_px = (0.0, 0.0)
        radius_deg = 0.0
        band_frac = 0.0
        shape = 0
        half_px = (0.0, 0.0)
    return _F()
