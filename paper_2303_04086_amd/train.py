"""Training an i-NOLF object (Sec. 4.2): the per-ray path as a differentiable
function of the feature tables and the network weights, the MSE loss of
Eq. 8 on RGBA, and Adam.

Forward and backward are the library's kernels (inrf_forward,
inrf_backward, inrf_adam); PyTorch holds the tensors and forms the loss
gradient 2 (rgba - target) / n.
"""
from __future__ import annotations

from .model import Renderer, adam_step


def _torch():
    import torch
    return torch


class _RenderFunction:
    """Built lazily so that importing the package does not import torch."""
    cls = None

    @classmethod
    def get(cls):
        if cls.cls is None:
            torch = _torch()

            class RenderFunction(torch.autograd.Function):
                @staticmethod
                def forward(ctx, table, weights, o, d, R):
                    if table.data_ptr() != R.tables["f32"].data_ptr() or weights.data_ptr() != R.weights.data_ptr():
                        raise ValueError("table and weights must be the renderer's resident FP32 tensors")
                    o, d = o.contiguous(), d.contiguous()
                    ctx.R = R
                    ctx.save_for_backward(o, d)
                    return R.forward(o, d, "fp32", "f32")

                @staticmethod
                def backward(ctx, g):
                    o, d = ctx.saved_tensors
                    R = ctx.R
                    dt = torch.zeros_like(R.tables["f32"]) if ctx.needs_input_grad[0] else None
                    dw = torch.zeros_like(R.weights) if ctx.needs_input_grad[1] else None
                    R.backward(o, d, g.contiguous(), "f32", d_table=dt, d_weights=dw)
                    return dt, dw, None, None, None

            cls.cls = RenderFunction
        return cls.cls


def render_rays(R: Renderer, o, d, table=None, weights=None):
    """RGBA of rays o, d through the FP32 path, differentiable with respect to
    `table` and `weights` (the renderer's resident FP32 table and weights,
    which may be wrapped as leaves that require grad)."""
    fn = _RenderFunction.get()
    return fn.apply(R.tables["f32"] if table is None else table, R.weights if weights is None else weights, o, d, R)


class Trainer:
    """Adam (lr 1e-2, betas 0.9 / 0.99 by default) on a Renderer's FP32
    master table and weights, minimising the mean over rays of the squared
    RGBA error.  Gradients accumulate in persistent buffers that the Adam
    kernel clears; a resident FP16 table is refreshed by every step.
    lazy_table: step only the table entries the batch gave a nonzero
    gradient (the weights always take a dense step)."""

    def __init__(self, R: Renderer, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.99, eps: float = 1e-15,
                 lazy_table: bool = False):
        torch = _torch()
        self.R, self.lr, self.beta1, self.beta2, self.eps = R, lr, beta1, beta2, eps
        self.lazy_table = bool(lazy_table)
        t, w = R.tables["f32"], R.weights
        self.g_table, self.m_table, self.v_table = (torch.zeros_like(t) for _ in range(3))
        self.g_w, self.m_w, self.v_w = (torch.zeros_like(w) for _ in range(3))
        self.t = 0

    def step(self, o, d, target):
        """One step on a batch: forward, loss gradient, backward, Adam.
        Returns the batch loss before the update (a device scalar)."""
        R = self.R
        n = o.shape[0]
        rgba = R.forward(o, d, "fp32", "f32")
        diff = rgba - target
        loss = (diff * diff).sum() / max(n, 1)
        R.backward(o, d, diff.mul_(2.0 / max(n, 1)), "f32", d_table=self.g_table, d_weights=self.g_w)
        self.t += 1
        kw = dict(lr=self.lr, beta1=self.beta1, beta2=self.beta2, eps=self.eps, zero_grad=True)
        adam_step(R.tables["f32"].view(-1), self.g_table.view(-1), self.m_table.view(-1), self.v_table.view(-1),
                  self.t, param_f16=R.tables["f16"].view(-1) if "f16" in R.tables else None, lazy=self.lazy_table,
                  **kw)
        adam_step(R.weights, self.g_w, self.m_w, self.v_w, self.t, **kw)
        return loss
