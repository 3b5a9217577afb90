"""Fine-tuning by backpropagation through the renderer (Sec. 4.1: a
converged model is fine-tuned with StopThePop ordering and Optimal
Projection; Sec. 5 runs 5K further iterations): per iteration one forward
render of the training views, the L1 + L2 image loss and its gradient
(vrs_loss_l1l2), the backward pass (vrs_render_backward) and one Adam step
per parameter group (vrs_adam_step).  Argument marshalling only: every step
runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _lib as L
from .render import Gaussians, Renderer, _ptr, _stream

# Per-group learning rates of the 3DGS optimiser the fine-tuning continues
# (position, SH, opacity, scale, rotation), without its schedules.
DEFAULT_LR = dict(means=1.6e-4, sh=2.5e-3, opacity_logits=5e-2, log_scales=5e-3, quats=1e-3)
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


class FineTuner:
    def __init__(self, renderer: Renderer, g: Gaussians, targets: Sequence[torch.Tensor],
                 lr: Optional[Dict[str, float]] = None, betas=(0.9, 0.999), eps=1e-15):
        self.r, self.g = renderer, g
        self.targets = [t.contiguous() for t in targets]
        for t, c in zip(self.targets, renderer.cams):
            if tuple(t.shape) != (4, c.height, c.width) or t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError("targets are (4, H, W) float32 CUDA tensors")
        self.lr = dict(DEFAULT_LR, **(lr or {}))
        self.betas, self.eps = betas, eps
        self.t = 0
        self.m = {k: torch.zeros_like(getattr(g, k)) for k in GROUPS}
        self.v = {k: torch.zeros_like(getattr(g, k)) for k in GROUPS}
        dev = renderer.device
        self.grad_img = [torch.empty_like(t) for t in self.targets]
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=dev)
        self.loss_ws = torch.empty(max(int(L.load().vrs_loss_workspace_size(renderer.V)), 8),
                                   dtype=torch.uint8, device=dev)
        self._t_ptrs = (ctypes.c_void_p * renderer.V)(*[t.data_ptr() for t in self.targets])
        self._g_ptrs = (ctypes.c_void_p * renderer.V)(*[t.data_ptr() for t in self.grad_img])

    def loss_and_grad(self, images: Sequence[torch.Tensor]):
        imgs = (ctypes.c_void_p * self.r.V)(*[im.data_ptr() for im in images])
        L.call("vrs_loss_l1l2", self.r.c_cams, self.r.V, imgs, self._t_ptrs, self._g_ptrs, _ptr(self.loss_dev),
               _ptr(self.loss_ws), ctypes.c_size_t(self.loss_ws.numel()), _stream(self.r.stream))
        return self.loss_dev

    def step(self) -> torch.Tensor:
        """One iteration; returns the loss of the rendered state (a device
        scalar, FP64) before the update."""
        imgs = self.r.render(self.g)
        self.loss_and_grad(imgs)
        grads = self.r.backward(self.g, self.grad_img)
        self.t += 1
        b1, b2 = self.betas
        for k in GROUPS:
            p = getattr(self.g, k)
            L.call("vrs_adam_step", _ptr(p), _ptr(grads[k]), _ptr(self.m[k]), _ptr(self.v[k]),
                   ctypes.c_size_t(p.numel()), ctypes.c_float(self.lr[k]), ctypes.c_float(b1), ctypes.c_float(b2),
                   ctypes.c_float(self.eps), self.t, _stream(self.r.stream))
        self._keep = grads
        return self.loss_dev
