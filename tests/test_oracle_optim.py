"""Pins for the oracle's Adam step: against PyTorch's Adam in float64 (a
library routine), and the first step's closed form."""
import numpy as np
import torch

from oracle import optim


def test_adam_equals_library_adam():
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(6)]
    t = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad()
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = optim.adam_step(p, g, m, v, k, 3e-3, 0.9, 0.999, 1e-8)
        np.testing.assert_allclose(p, t.detach().numpy(), rtol=0, atol=1e-15)


def test_adam_first_step_is_a_signed_step_of_lr():
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p, _, _ = optim.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01, eps=1e-15)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-11)
