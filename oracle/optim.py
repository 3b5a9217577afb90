"""Adam, the optimiser of the fine-tuning (Sec. 4.1 fine-tunes a converged
model by backpropagation; the 3DGS training it continues uses Adam).  Test
infrastructure only.

Adam (Kingma and Ba, 2015) with bias correction, in float64:
    m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
    p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
at step t = 1, 2, ...
"""
import numpy as np


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One step; returns the new (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
