"""Serving many clients from a resident object or scene.

The paper's platform renders frames for many clients from resident models
and schedules the work per group of rays (Sec. 1, Sec. 5-6).  Here requests
(a camera and an arrival time) are admitted in arrival order into batches
under an HBM budget: a batch grows while its workspace plus its output
images fit the budget of one in-flight slot (and at most
INRF_MAX_CAMERAS cameras).  Each batch is rendered in one pass over all its
rays -- inrf_render_batch for one object, inrf_render_scene_batch for a
scene (one trace launch over every camera's tiles, then the shading grouped
by object across the requests) -- so rays of different requests share
waves.

The loop runs in real time (continuous batching).  Up to `in_flight`
batches are on the device at once, each on a stream (default priority)
with its own workspace and output buffer, allocated once; a new batch is
formed from the queue as soon as a slot frees up, so requests that arrive
while others render are admitted as slots and memory free up, and their
work overlaps on the device.  With every slot busy the loop blocks on the
oldest batch's event; otherwise it polls, yielding the core between polls.
A request's latency is the host time at which its batch was seen complete
minus its arrival time.
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
    """target: a Renderer or a Scene (anything with render_batch and
    batch_workspace_bytes).  hbm_budget: bytes of device memory one batch
    may hold, its workspace followed by its FP32 RGBA images; the server
    allocates exactly that much per in-flight slot, once, and every batch it
    forms fits in it.  max_request_pixels, if given, is checked against the
    budget up front."""

    def __init__(self, target, precision: str = "fp16", table: str = "f16", hbm_budget: int = 1 << 30,
                 max_batch: int = L.MAX_CAMERAS, in_flight: int = 2, max_request_pixels: int | None = None):
        import torch
        self.T, self.precision, self.table = target, precision, table
        self.max_batch = int(min(max_batch, L.MAX_CAMERAS))
        self.budget = int(hbm_budget)
        self.torch = torch
        if max_request_pixels is not None and self.cost(1, int(max_request_pixels)) > self.budget:
            raise ValueError("the HBM budget cannot hold one request of the largest size")
        self.slots = [(torch.cuda.Stream(device=target.device),
                       torch.empty(self.budget, dtype=torch.uint8, device=target.device))
                      for _ in range(int(in_flight))]

    def cost(self, n_cameras: int, n_pixels: int) -> int:
        """HBM bytes a batch holds: its workspace and its RGBA images."""
        return self.T.batch_workspace_bytes(n_cameras, n_pixels) + 16 * int(n_pixels)

    def run(self, requests, on_batch=None, time_scale: float = 1.0) -> dict:
        """Serve `requests` (any order); request r is released at
        r.arrival_s * time_scale seconds after the start (time_scale 0: all
        at once, the saturated case).  `on_batch(batch, views)` may inspect
        each batch's images when it completes, before its buffer is reused."""
        torch = self.torch
        todo = sorted(requests, key=lambda r: r.arrival_s)
        for r in todo:
            if self.cost(1, r.pixels) > self.budget:
                raise ValueError("a request is larger than the HBM budget of one batch")
        free = list(range(len(self.slots)))
        queue, flight, lat, sizes, held = [], [], [], [], []
        pixels, busy, busy_from, i = 0, 0.0, None, 0
        torch.cuda.current_stream(self.T.device).synchronize()
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
                batch = [queue.pop(0)]
                pix = batch[0].pixels
                while (queue and len(batch) < self.max_batch
                       and self.cost(len(batch) + 1, pix + queue[0].pixels) <= self.budget):
                    pix += queue[0].pixels
                    batch.append(queue.pop(0))
                slot = free.pop(0)
                stream, buf = self.slots[slot]
                # the slot's bytes: workspace (a multiple of 256 bytes), then the images
                need = self.T.batch_workspace_bytes(len(batch), pix)
                rgba = buf[need:need + 16 * pix].view(torch.float32).view(pix, 4)
                if not flight:
                    busy_from = time.perf_counter() - t0
                _, views = self.T.render_batch([r.camera for r in batch], self.precision, self.table,
                                               rgba=rgba, stream=stream, ws=buf[:need])
                ev = torch.cuda.Event()
                ev.record(stream)
                flight.append((slot, batch, ev, views))
                pixels += pix
                sizes.append(len(batch))
                held.append(self.cost(len(batch), pix))
            elif flight and not free:
                # every slot is busy: nothing can start before the oldest batch completes
                flight[0][2].synchronize()
            elif not flight and i < len(todo):
                time.sleep(max(0.0, min(1e-3, todo[i].arrival_s * time_scale - now)))
            else:
                time.sleep(0)  # waiting on a completion or an arrival: yield the core between polls
        span = time.perf_counter() - t0
        return {"requests": len(lat), "batches": len(sizes), "mean_batch": round(sum(sizes) / max(1, len(sizes)), 2),
                "in_flight": len(self.slots), "hbm_budget_bytes": self.budget,
                "max_batch_bytes": max(held) if held else 0,
                "p50_latency_ms": round(_pct(lat, 50) * 1e3, 3), "p99_latency_ms": round(_pct(lat, 99) * 1e3, 3),
                "Mrays_per_s": round(pixels / max(busy, 1e-12) / 1e6, 1), "busy_s": round(busy, 4),
                "span_s": round(span, 4)}
