"""Serving many clients from one resident i-NOLF object.

The paper's platform renders frames for many clients from resident models
and schedules the work per group of rays (Sec. 1, Sec. 5-6).  Here requests
(a camera and an arrival time) are admitted in arrival order while the batch
fits a pixel budget (which bounds the workspace the batch needs in HBM) and
a camera count, rendered together by inrf_render_batch — one trace launch
over all their tiles and one shading launch over all their hit rays, so rays
of different requests share waves — and retired when the batch completes.
The loop advances a clock by the measured device time of each batch, so a
request's latency is queueing plus service.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import _lib as L


@dataclass
class Request:
    client: int
    arrival_s: float
    camera: object

    @property
    def pixels(self) -> int:
        return int(self.camera.width) * int(self.camera.height)


def _pct(v, q):
    s = sorted(v)
    return s[min(len(s) - 1, int(round(q / 100.0 * (len(s) - 1))))] if s else 0.0


class Server:
    def __init__(self, renderer, precision: str = "fp16", table: str = "f16", pixel_budget: int = 2 * 3840 * 2160,
                 max_batch: int = L.MAX_CAMERAS):
        import torch
        self.R, self.precision, self.table = renderer, precision, table
        self.pixel_budget, self.max_batch = int(pixel_budget), int(min(max_batch, L.MAX_CAMERAS))
        self.torch = torch
        # one output buffer for the largest admissible batch, allocated once
        self.rgba = torch.empty((self.pixel_budget + 3840 * 2160, 4), dtype=torch.float32, device="cuda")

    def run(self, requests, on_batch=None) -> dict:
        """Serve `requests` (any order); `on_batch(batch, views)` may inspect
        each batch's images before the buffer is reused."""
        torch = self.torch
        todo = sorted(requests, key=lambda r: r.arrival_s)
        queue, lat, sizes = [], [], []
        clock, busy, pixels, i = 0.0, 0.0, 0, 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        while i < len(todo) or queue:
            while i < len(todo) and todo[i].arrival_s <= clock:
                queue.append(todo[i])
                i += 1
            if not queue:
                clock = todo[i].arrival_s
                continue
            batch, pix = [], 0
            while queue and len(batch) < self.max_batch and (not batch or pix + queue[0].pixels <= self.pixel_budget):
                pix += queue[0].pixels
                batch.append(queue.pop(0))
            if pix > self.rgba.shape[0]:
                raise ValueError("a request is larger than the server's output buffer")
            e0.record()
            _, views = self.R.render_batch([r.camera for r in batch], self.precision, self.table, rgba=self.rgba[:pix])
            e1.record()
            e1.synchronize()
            dt = e0.elapsed_time(e1) / 1e3
            if on_batch is not None:
                on_batch(batch, views)
            clock += dt
            busy += dt
            pixels += pix
            sizes.append(len(batch))
            lat.extend(clock - r.arrival_s for r in batch)
        return {"requests": len(lat), "batches": len(sizes), "mean_batch": round(sum(sizes) / max(1, len(sizes)), 2),
                "p50_latency_ms": round(_pct(lat, 50) * 1e3, 3), "p99_latency_ms": round(_pct(lat, 99) * 1e3, 3),
                "Mrays_per_s": round(pixels / max(busy, 1e-12) / 1e6, 1), "busy_s": round(busy, 4),
                "span_s": round(clock, 4)}
