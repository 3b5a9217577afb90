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
                 capacity: Optional[int] = None, stream=None):
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
        L.call("vrs_fovea_plan", self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params),
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
               ctypes.byref(self.c_params), _ptr(self.proj), _ptr(self.counts), _ptr(self.keys),
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
               ctypes.byref(self.c_params), _ptr(self.proj), _ptr(self.counts), _ptr(self.status),
               _stream(self.stream))

    def duplicate(self, g: Gaussians):
        L.call("vrs_duplicate", ctypes.byref(g.struct()), self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), _ptr(self.proj), _ptr(self.counts), _ptr(self.keys),
               _ptr(self.gids), ctypes.c_size_t(self.capacity), _ptr(self.n_inst), _ptr(self.sort_ws),
               ctypes.c_size_t(self.sort_ws.numel()), _ptr(self.status), _stream(self.stream))

    def key_bits(self):
        b = 0
        while (1 << b) < self.tiles_total:
            b += 1
        return 32 + b

    def sort(self, g: Gaussians):
        L.call("vrs_sort", ctypes.byref(g.struct()), self.c_cams, self.c_fovs, self.V,
               ctypes.byref(self.c_params), _ptr(self.proj), _ptr(self.counts), _ptr(self.keys),
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
        defaults to the renderer's own output buffers.  Plain views only."""
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
        need = int(L.load().vrs_backward_workspace_size(self.n, self.V))
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
               _ptr(self.ranges), self.c_cams, self.c_fovs, self.V, ctypes.byref(self.c_params), img_ptrs,
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

    def records(self) -> torch.Tensor:
        return self.proj[: self.V * self.n * L.VRS_RECORD_FLOATS * 4].view(torch.float32).view(
            self.V, self.n, L.VRS_RECORD_FLOATS)

    def colours(self) -> torch.Tensor:
        """[V][n][4] float32: each Gaussian's colour (r, g, b, 0) per view,
        after the render and tile-test records in `proj`."""
        off = self.V * self.n * (L.VRS_RECORD_FLOATS * 4 + L.TILEGEO_BYTES)
        return self.proj[off: off + self.V * self.n * 16].view(torch.float32).view(self.V, self.n, 4)
