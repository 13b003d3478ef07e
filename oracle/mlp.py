"""The specular network F_s evaluated once per ray, FP64 (test infrastructure
only).

Sec. 4.2, Eq. 3: a shallow network maps the position encoding and the view
direction to colour and opacity.  Reading adopted: no biases; two hidden
layers with ReLU; four outputs (RGB, alpha) through a logistic sigmoid:
    h1 = relu(W1 in), h2 = relu(W2 h1), rgba = sigmoid(W3 h2),
weights row-major [out][in], computed with numpy FP64 matrix products.

Pins: all-zero weights give 0.5 exactly; hand-worked tiny networks.
"""
from __future__ import annotations

import numpy as np


def mlp_forward(inputs, weights) -> np.ndarray:
    h = np.asarray(inputs, np.float64)
    ws = [np.asarray(w, np.float64) for w in weights]
    for w in ws[:-1]:
        h = np.maximum(h @ w.T, 0.0)
    z = h @ ws[-1].T
    return 1.0 / (1.0 + np.exp(-z))
