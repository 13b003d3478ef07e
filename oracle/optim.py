"""Adam, FP64 (test infrastructure only).

The training of Sec. 4.2 minimises the loss of Eq. 8 with Adam (Kingma and
Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015, Algorithm 1):
  m_t = b1 m_{t-1} + (1 - b1) g_t
  v_t = b2 v_{t-1} + (1 - b2) g_t^2
  p_t = p_{t-1} - lr * (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)

Pins (tests): the first step moves every parameter with a nonzero gradient
by lr * g / (|g| + eps) (bias correction makes m/v^(1/2) exactly g/|g|); a
constant gradient keeps the step at lr * g / (|g| + eps) at every t; a zero
gradient from zero moments leaves the parameter unchanged.
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float):
    """Returns (p, m, v) after step t >= 1 (new arrays, FP64)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


__all__ = ["adam_step"]
