"""Serving many clients from one resident i-NOLF object.

The paper's platform renders frames for many clients from resident models
and schedules the work per group of rays (Sec. 1, Sec. 5-6).  Here requests
(a camera and an arrival time) are admitted in arrival order while a batch
fits a pixel budget (which bounds the workspace the batch needs in HBM) and
a camera count, and each batch is rendered by inrf_render_batch: one trace
launch over all its tiles and one shading launch over all its hit rays, so
rays of different requests share waves.

The loop runs in real time.  Up to `in_flight` batches are on the device at
once, each on a stream (default priority) with its own workspace and output
buffer, so that a batch's trace (ALU-bound) overlaps the shading (bound by
HBM gathers) of the batch before it; a new batch is formed as soon as a
slot frees up.  A request's latency is the host time at which its batch was
seen complete minus its arrival time.
"""
from __future__ import annotations

import time
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
                 max_batch: int = L.MAX_CAMERAS, in_flight: int = 2, max_request_pixels: int = 3840 * 2160):
        import torch
        self.R, self.precision, self.table = renderer, precision, table
        self.pixel_budget, self.max_batch = int(pixel_budget), int(min(max_batch, L.MAX_CAMERAS))
        self.torch = torch
        # a batch holds at most pixel_budget pixels, or one request larger than that
        cap = max(self.pixel_budget, int(max_request_pixels))
        need = int(L.lib().inrf_batch_workspace_size(self.max_batch, cap))
        if need < 0:
            raise ValueError("invalid server limits")
        self.cap = cap
        # per slot: stream, output buffer and workspace, allocated once
        self.slots = [(torch.cuda.Stream(device=renderer.device),
                       torch.empty((cap, 4), dtype=torch.float32, device=renderer.device),
                       torch.empty(need, dtype=torch.uint8, device=renderer.device)) for _ in range(int(in_flight))]

    def run(self, requests, on_batch=None, time_scale: float = 1.0) -> dict:
        """Serve `requests` (any order); request r is released at
        r.arrival_s * time_scale seconds after the start (time_scale 0: all
        at once, the saturated case).  `on_batch(batch, views)` may inspect
        each batch's images when it completes, before its buffer is reused."""
        torch = self.torch
        todo = sorted(requests, key=lambda r: r.arrival_s)
        for r in todo:
            if r.pixels > self.cap:
                raise ValueError("a request is larger than the server's output buffer")
        free = list(range(len(self.slots)))
        queue, flight, lat, sizes = [], [], [], []
        pixels, busy, busy_from, i = 0, 0.0, None, 0
        torch.cuda.current_stream(self.R.device).synchronize()
        t0 = time.perf_counter()
        while i < len(todo) or queue or flight:
            now = time.perf_counter() - t0
            while i < len(todo) and todo[i].arrival_s * time_scale <= now:
                queue.append(todo[i])
                i += 1
            # retire batches in submission order
            while flight and flight[0][2].query():
                slot, batch, _, views = flight.pop(0)
                done = time.perf_counter() - t0
                if on_batch is not None:
                    on_batch(batch, views)
                lat.extend(done - r.arrival_s * time_scale for r in batch)
                free.append(slot)
                if not flight:
                    busy += done - busy_from
            if queue and free:
                batch, pix = [], 0
                while queue and len(batch) < self.max_batch and (not batch or pix + queue[0].pixels <= self.pixel_budget):
                    pix += queue[0].pixels
                    batch.append(queue.pop(0))
                slot = free.pop(0)
                stream, rgba, ws = self.slots[slot]
                if not flight:
                    busy_from = time.perf_counter() - t0
                _, views = self.R.render_batch([r.camera for r in batch], self.precision, self.table,
                                               rgba=rgba[:pix], stream=stream, ws=ws)
                ev = torch.cuda.Event()
                ev.record(stream)
                flight.append((slot, batch, ev, views))
                pixels += pix
                sizes.append(len(batch))
            elif not flight and i < len(todo):
                time.sleep(max(0.0, min(1e-3, todo[i].arrival_s * time_scale - now)))
        span = time.perf_counter() - t0
        return {"requests": len(lat), "batches": len(sizes), "mean_batch": round(sum(sizes) / max(1, len(sizes)), 2),
                "in_flight": len(self.slots),
                "p50_latency_ms": round(_pct(lat, 50) * 1e3, 3), "p99_latency_ms": round(_pct(lat, 99) * 1e3, 3),
                "Mrays_per_s": round(pixels / max(busy, 1e-12) / 1e6, 1), "busy_s": round(busy, 4),
                "span_s": round(span, 4)}
