"""Adam, FP64 (test infrastructure only).

The training of Sec. 4.2 minimises the loss of Eq. 8 with Adam (Kingma and
Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015, Algorithm 1):
  m_t = b1 m_{t-1} + (1 - b1) g_t
  v_t = b2 v_{t-1} + (1 - b2) g_t^2
  p_t = p_{t-1} - lr * (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)

Lazy (sparse) Adam applies that update only to parameters whose gradient
is nonzero; every other parameter keeps its value and both moments, and t
stays the global step count.

Pins (tests): the first step moves every parameter with a nonzero gradient
by lr * g / (|g| + eps) (bias correction makes m/v^(1/2) exactly g/|g|); a
constant gradient keeps the step at lr * g / (|g| + eps) at every t; a zero
gradient from zero moments leaves the parameter unchanged; in lazy mode a
zero gradient leaves value and moments unchanged even with nonzero moments,
and a nonzero one gives the dense step exactly.
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float, lazy: bool = False):
    """Returns (p, m, v) after step t >= 1 (new arrays, FP64)."""
    p0 = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m0 = np.asarray(m, np.float64)
    v0 = np.asarray(v, np.float64)
    m1 = beta1 * m0 + (1.0 - beta1) * g
    v1 = beta2 * v0 + (1.0 - beta2) * g * g
    m_hat = m1 / (1.0 - beta1 ** t)
    v_hat = v1 / (1.0 - beta2 ** t)
    p1 = p0 - lr * m_hat / (np.sqrt(v_hat) + eps)
    if not lazy:
        return p1, m1, v1
    step = g != 0
    return np.where(step, p1, p0), np.where(step, m1, m0), np.where(step, v1, v0)


__all__ = ["adam_step"]
