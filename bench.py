#!/usr/bin/env python
"""Benchmark of the i-NOLF one-query-per-ray render path on one MI355X.

Workload: one displaced-sphere object (100,820-triangle proxy, 16 PSH levels
16..2048, F=2, MLP 48-64-64-4) rendered at 3840x2160 from 8 cameras on a
sphere of radius 2 (synthetic stand-in for one trained object; see the design
notes).  A step is one full frame through the whole path: ray generation,
BVH closest hit, hit compaction, PSH gather + trilinear + SH16 + MLP, RGBA
output.  `value` is Mrays/s (all primary rays, hits and misses) of the
FP16-table / FP16-MFMA path over the timed region; the FP32 path is measured
the same way and reported beside it.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s at 3840x2160 one-object render (FP32 vs FP16-MFMA); p99 frame latency"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp32": 157.3}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def requested_bytes_per_hit(n_levels: int, table: str) -> int:
    """Gather bytes one hit ray asks for: per level 8 corners x (F features
    of the table type + one 4-byte offset entry)."""
    return 8 * n_levels * (2 * (4 if table == "f32" else 2) + 4)


def mlp_flops(d_in: int) -> int:
    return 2 * (d_in * 64 + 64 * 64 + 64 * 4)


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_04086_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def run_frames(torch, R, cams, prec, table, steps, warmup):
    """Timed frames (one inrf_render each, per-frame events on the caller's
    stream around each call), then the same frames through the stage-event
    entry point, which records trace start, shading start and end on the
    kernels' stream: the trace / shade breakdown and the shading launch time
    of the roofline object come from that pass."""
    rgba = torch.empty((cams[0].height, cams[0].width, 4), dtype=torch.float32, device="cuda")
    for i in range(warmup):
        R.render(cams[i % len(cams)], prec, table, rgba=rgba)
    torch.cuda.synchronize()
    hits = []
    for c in cams:
        R.render(c, prec, table, rgba=rgba)
        torch.cuda.synchronize()
        hits.append(R.hit_count())
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    fr = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    for trip in ev + fr:                 # create the underlying events before use
        for e in trip:
            e.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fr[i][0].record()
        R.render(cams[i % len(cams)], prec, table, rgba=rgba)
        fr[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frame = [fr[i][0].elapsed_time(fr[i][1]) for i in range(steps)]
    for i in range(steps):
        R.render(cams[i % len(cams)], prec, table, rgba=rgba, events=ev[i])
    torch.cuda.synchronize()
    trace = [ev[i][0].elapsed_time(ev[i][1]) for i in range(steps)]
    shade = [ev[i][1].elapsed_time(ev[i][2]) for i in range(steps)]
    shade_hits = [hits[i % len(cams)] for i in range(steps)]
    return {"wall_s": wall, "frame_ms": frame, "trace_ms": trace, "shade_ms": shade, "hits": shade_hits,
            "hits_per_camera": hits}


def pct(v, q):
    s = sorted(v)
    return s[min(len(s) - 1, int(round(q / 100.0 * (len(s) - 1))))]


def summarize(r, W, H, steps, n_levels, table):
    rays = W * H * steps
    shade_s = sum(r["shade_ms"]) / 1e3
    bytes_req = sum(r["hits"]) * requested_bytes_per_hit(n_levels, table)
    achieved = bytes_req / shade_s / 1e9
    return {
        "value": round(rays / r["wall_s"] / 1e6, 2),
        "ms_per_step": round(r["wall_s"] / steps * 1e3, 4),
        "p50_ms": round(pct(r["frame_ms"], 50), 4),
        "p99_ms": round(pct(r["frame_ms"], 99), 4),
        "trace_ms_avg": round(sum(r["trace_ms"]) / steps, 4),
        "shade_ms_avg": round(sum(r["shade_ms"]) / steps, 4),
        "hit_rays_per_frame_avg": round(sum(r["hits"]) / steps, 1),
        "hit_Mrays_per_s": round(sum(r["hits"]) / r["wall_s"] / 1e6, 2),
        "shade_requested_GBps": round(achieved, 1),
    }


def mlp_bench(torch, R, prec, n, reps=5, encoded=False):
    """The network alone on n rays: FP32 input rows [encoding, SH16]
    (inrf_mlp), or with `encoded` 16-bit encodings and FP32 directions
    (inrf_mlp_encoded, SH16 computed on the fly).  Useful FLOPs only."""
    d_in = 2 * R.n_levels + 16
    if encoded:
        dt = torch.float16 if prec == "fp16" else torch.bfloat16
        enc = (torch.randn((n, 2 * R.n_levels), device="cuda") * 0.1).to(dt)
        dirs = torch.randn((n, 3), device="cuda")
        run = lambda: R.mlp_encoded(enc, dirs, prec, out=out)
        in_bytes = n * (2 * 2 * R.n_levels + 12)
    else:
        x = torch.randn((n, d_in), device="cuda") * 0.1
        run = lambda: R.mlp(x, prec, out=out)
        in_bytes = n * 4 * d_in
    out = torch.empty((n, 4), device="cuda")
    run()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        run()
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    tf = n * mlp_flops(d_in) / (ms / 1e3) / 1e12
    return {"rays": n, "input": "16-bit encodings + FP32 directions" if encoded else "FP32 rows",
            "input_bytes": in_bytes, "ms": round(ms, 4), "TFLOPs": round(tf, 2), "peak": MFMA_PEAK_TFLOPS[prec],
            "utilisation": round(tf / MFMA_PEAK_TFLOPS[prec], 4),
            "input_GBps": round((in_bytes + 16 * n) / (ms / 1e3) / 1e9, 1)}


_ORACLE = {}


def _oracle_task(idx):
    """Worker of the multi-core oracle run: FP64 path on the listed rays."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        t0 = time.perf_counter()
        r = oracle.render_rays(_ORACLE["model"], _ORACLE["o"][idx], _ORACLE["d"][idx], eps_bary=1e-4)
        dt = time.perf_counter() - t0
    return idx, r["rgba"], r["tri"], r["ambiguous"], r["cos"], dt


def disc_pixels(cam, n_near, n_any, seed, centre=(0.5, 0.5, 0.5), radius=0.5):
    """n_near pixels whose FP64 ray passes within `radius` of the object's
    centre (the proxy lies in that ball, so most of them hit), then n_any
    uniform pixels: chosen from the camera geometry alone."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    pool = rng.integers(0, cam.width * cam.height, 12 * n_near + 1000)
    o, d = oracle.camera_rays(cam, pool // cam.width, pool % cam.width)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    v = np.asarray(centre) - o
    tca = np.sum(v * d, axis=1)
    near = pool[(np.sum(v * v, axis=1) - tca ** 2 < radius ** 2) & (tca > 0)][:n_near]
    return np.concatenate([near, rng.integers(0, cam.width * cam.height, n_any)])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, n_near, n_any, n_one, seed=11):
    """The FP64 oracle, as it stands, on the host cores, before anything
    touches the GPU: a seeded sample of pixels of camera 0 (n_near near the
    object, n_any uniform) split over worker processes (one BLAS thread
    each), the first n_one of them again on one core, and the tiny
    workload's full 64x64 frame on one core.  Its outputs are kept: they are
    the FP64 reference of the GPU frames' error figures."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    import synth
    from threadpoolctl import threadpool_limits
    cam = w.cameras[0]
    pix = disc_pixels(cam, n_near, n_any, seed)
    o, d = oracle.camera_rays(cam, pix // cam.width, pix % cam.width)
    _ORACLE.update(model=oracle.Model.from_workload(w, materialize=False, check_keys=False), o=o, d=d)
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    with threadpool_limits(1):
        t0 = time.perf_counter()
        _oracle_task(np.arange(n_one))
        dt1 = time.perf_counter() - t0
        ctx = mp.get_context("fork")
        with ctx.Pool(cores) as pool:
            pool.map(_oracle_task, [np.arange(0, 1)] * cores)  # workers up
            chunks = np.array_split(np.arange(len(pix)), 8 * cores)
            t0 = time.perf_counter()
            res = pool.map(_oracle_task, chunks)
            dtk = time.perf_counter() - t0
        wt = synth.workload_tiny()
        mt = oracle.Model.from_workload(wt)
        t0 = time.perf_counter()
        oracle.render_camera(mt, wt.cameras[0])
        dtw1 = time.perf_counter() - t0
    rgba = np.zeros((len(pix), 4))
    tri = np.zeros(len(pix), np.int64)
    amb = np.zeros(len(pix), bool)
    cos = np.zeros(len(pix))
    for idx, r, t, a, c, _ in res:
        rgba[idx], tri[idx], amb[idx], cos[idx] = r, t, a, c
    ref = {"pix": pix, "rgba": rgba, "tri": tri, "ambiguous": amb, "cos": cos}
    base = {"value": round(len(pix) / dtk / 1e6, 6), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{len(pix)} seeded pixels of camera 0 at {cam.width}x{cam.height} ({n_near} chosen near the "
                      f"object, {n_any} uniform; hit fraction {float((tri >= 0).mean()):.3f}), full path in FP64 "
                      f"over {cores} processes ({dtk:.1f} s)",
            "one_core": {"value": round(n_one / dt1 / 1e6, 6), "rays": n_one, "s": round(dt1, 2)},
            "full_frame_4k_extrapolated_s": round(cam.width * cam.height / (len(pix) / dtk), 1),
            "tiny_full_frame": {"workload": wt.name, "rays": 64 * 64, "s": round(dtw1, 2),
                                "Mrays_per_s": round(64 * 64 / dtw1 / 1e6, 6), "cores": 1}}
    return base, ref


GRAZING_COS = 0.01


def frame_errors(torch, R, cam, ref, cases):
    """Error of the GPU frames of camera 0 against the FP64 oracle on the
    sampled pixels: max abs over pixels whose hit/miss agrees (every
    disagreement must be a ray the oracle flags ambiguous), also without the
    grazing hits (|cos| of the incidence angle below 0.01, where an FP32
    ray fixes the hit point only to ~t 2^-23 / |cos|), and PSNR over the
    pixels hit by either side."""
    import numpy as np
    out = {}
    n = cam.width * cam.height
    for prec, table in cases:
        tri = torch.empty(n, dtype=torch.int32, device="cuda")
        rgba = R.render(cam, prec, table, tri=tri).reshape(-1, 4).cpu().numpy()[ref["pix"]]
        tri = tri.cpu().numpy()[ref["pix"]]
        agree = (tri >= 0) == (ref["tri"] >= 0)
        clear = ~ref["ambiguous"]
        hit = agree & ((tri >= 0) | (ref["tri"] >= 0))
        mse = float(np.mean((rgba[hit] - ref["rgba"][hit]) ** 2))
        steep = agree & ~(ref["cos"] < GRAZING_COS)
        out[prec] = {"max_abs": float(f"{np.abs(rgba[agree] - ref['rgba'][agree]).max():.3e}"),
                     "max_abs_not_grazing": float(f"{np.abs(rgba[steep] - ref['rgba'][steep]).max():.3e}"),
                     "grazing_pixels": int((agree & ~steep).sum()),
                     "psnr_db": float(round(10 * np.log10(1.0 / mse), 1)) if mse > 0 else None,
                     "pixels": int(len(tri)), "hit_pixels": int(hit.sum()),
                     "ids_bit_exact": bool(np.array_equal(tri[clear], ref["tri"][clear])),
                     "disagreements_all_ambiguous": bool(np.all(agree | ref["ambiguous"]))}
    return out


def load_traffic(kernel: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def sweep_bench(torch, R, w, frames):
    """The paper's speed-distance protocol: the same object from 8 directions
    at decreasing distance (hit fraction rising towards a full screen), FP16
    path; plus 1920x1080 at the headline distance."""
    import synth
    out = {}
    cases = [(f"d{d}", d, w.cameras[0].width, w.cameras[0].height) for d in (2.0, 1.4, 1.0, 0.7)]
    cases.append(("1080p_d2.0", 2.0, 1920, 1080))
    for name, dist, W, H in cases:
        cams = synth.fibonacci_cameras(8, dist, W, H)
        r = run_frames(torch, R, cams, "fp16", "f16", frames, 2)
        hits = sum(r["hits"]) / frames
        shade_s = sum(r["shade_ms"]) / frames / 1e3
        mlp_tf = hits * mlp_flops(2 * R.n_levels + 16) / shade_s / 1e12
        out[name] = {"width": W, "height": H, "distance": dist,
                     "Mrays_per_s": round(W * H * frames / (sum(r["frame_ms"]) / 1e3) / 1e6, 1),
                     "hit_fraction": round(hits / (W * H), 4),
                     "trace_ms_avg": round(sum(r["trace_ms"]) / frames, 4),
                     "shade_ms_avg": round(shade_s * 1e3, 4),
                     "shade_requested_GBps": round(hits * requested_bytes_per_hit(R.n_levels, "f16") / shade_s / 1e9, 1),
                     "shade_mlp_TFLOPs": round(mlp_tf, 2),
                     "shade_mlp_mfma_util": round(mlp_tf / MFMA_PEAK_TFLOPS["fp16"], 4)}
        log(f"sweep {name}: {out[name]}")
    return out


def train_bench(torch, P, R, w, steps, batch):
    """Training steps (Sec. 4.2, Eq. 8): batches of rays from 64 viewpoints,
    MSE on RGBA against the FP32 renders of a second seeded model on the same
    proxy (other features, other network), backward, Adam on the FP32 table
    (lazy: only the entries the batch touched) and the weights, FP16 table
    refreshed.  A few dense-Adam steps are timed beside it."""
    import numpy as np
    import synth
    from paper_2303_04086_amd.train import Trainer
    origins = np.stack([c.origin for c in synth.random_cameras(64, 7, 2.0, 64, 64)])
    R2 = P.Renderer(w.verts, w.tris, w.res, synth.xavier_mlp(33, w.d_in),
                    lambda l, lv: synth.feature_values(w.feature_seed + 17, l, lv.keys, F=w.F),
                    tables=("f32",), psh_levels=R.levels)
    batches = []
    for k in range(4):
        o, d = (torch.from_numpy(a).cuda() for a in synth.view_rays(origins, batch, 100 + k))
        batches.append((o, d, R2.forward(o, d, "fp32", "f32").clone()))
    torch.cuda.synchronize()
    del R2
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()

    def timed(tr, n):
        for k in range(2):
            tr.step(*batches[k % 4])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        losses = [tr.step(*batches[k % 4]) for k in range(n)]
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n, [float(x) for x in losses]

    ms, losses = timed(Trainer(R, lr=1e-2, beta1=0.9, beta2=0.99, lazy_table=True), steps)
    peak = torch.cuda.max_memory_allocated() / 1e9
    dense_ms, _ = timed(Trainer(R, lr=1e-2, beta1=0.9, beta2=0.99), max(2, steps // 3))
    return {"steps": steps, "batch_rays": batch, "ms_per_step": round(ms, 4), "steps_per_s": round(1e3 / ms, 2),
            "Mrays_per_s": round(batch / ms / 1e3, 2), "first_loss": round(losses[0], 6),
            "last_loss": round(losses[-1], 6), "peak_hbm_GB": round(peak, 3),
            "params": int(R.tables["f32"].numel() + R.weights.numel()),
            "dense_adam_ms_per_step": round(dense_ms, 4),
            "targets": "FP32 renders of a second seeded model on the same proxy (other features and network)",
            "note": "forward + backward + Adam each step: lazy on the table (entries with a nonzero gradient), "
                    "dense on the weights"}


def scene_bench(torch, P, frames, W, H):
    """Multi-object scene: 12 objects with their own tables and networks,
    merged per pixel by depth; FP16 and FP32 paths at W x H.  Returns the
    figures and the resident scene (served next)."""
    import synth
    sc = synth.scene_objects(12, W, H)
    t0 = time.time()
    rs = []
    keys = 0
    for o in sc.objects:
        w = o.workload
        R = P.Renderer(w.verts, w.tris, w.res, w.weights,
                       lambda l, lv, w=w: synth.feature_values(w.feature_seed, l, lv.keys, F=w.F),
                       tables=("f32", "f16"), dilate=w.dilate, seed=w.psh_seed)
        keys += sum(len(lv.keys) for lv in R.levels)
        rs.append(R)
    S = P.Scene(rs, [(o.scale, o.rotation, o.translation) for o in sc.objects])
    log(f"scene of {len(rs)} objects resident ({keys} keys) in {time.time() - t0:.1f} s")
    out = {"workload": sc.name, "objects": len(rs), "keys": keys,
           "triangles": int(sum(len(o.workload.tris) for o in sc.objects))}
    rgba = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    obj = torch.empty(H * W, dtype=torch.int32, device="cuda")
    for prec, table in (("fp16", "f16"), ("fp32", "f32")):
        for i in range(3):
            S.render(sc.cameras[i % len(sc.cameras)], prec, table, rgba=rgba)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(frames + 1)]
        ev[0].record()
        for i in range(frames):
            S.render(sc.cameras[i % len(sc.cameras)], prec, table, rgba=rgba)
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(frames)]
        S.render(sc.cameras[0], prec, table, rgba=rgba, obj=obj)
        torch.cuda.synchronize()
        hit = float((obj >= 0).float().mean())
        out[prec] = {"Mrays_per_s": round(W * H * frames / (sum(ms) / 1e3) / 1e6, 1),
                     "ms_per_frame": round(sum(ms) / frames, 4), "p99_ms": round(pct(ms, 99), 4),
                     "hit_fraction_camera0": round(hit, 4)}
        log(f"scene {prec}: {out[prec]}")
    return out, S


def single_level_bench(torch, P, frames, W, H, multi_ms):
    """The paper's single-resolution PSH (one level of N^3, Sec. 4.1) on the
    same proxy and cameras, FP16 path, against the 16-level shading time."""
    import synth
    out = {}
    for N in (128, 256, 512):
        w = synth.workload_object(W, H)
        w.res = [N]
        w.weights = synth.xavier_mlp(3, w.d_in)
        R1 = P.Renderer(w.verts, w.tris, w.res, w.weights,
                        lambda l, lv, w=w: synth.feature_values(w.feature_seed, l, lv.keys, F=w.F),
                        tables=("f16",), dilate=w.dilate, seed=w.psh_seed)
        r = run_frames(torch, R1, w.cameras, "fp16", "f16", frames, 3)
        shade = sum(r["shade_ms"]) / frames
        out[f"N{N}"] = {"keys": int(len(R1.levels[0].keys)),
                        "Mrays_per_s": round(W * H * frames / (sum(r["frame_ms"]) / 1e3) / 1e6, 1),
                        "shade_ms_avg": round(shade, 4),
                        "shade_vs_16_levels": round(shade / multi_ms, 3)}
        log(f"single level N={N}: {out[f'N{N}']}")
        del R1
    return out


def nolf_bench(torch, P, frames, W, H):
    """The paper's own i-NOLF form at W x H: density-cube march (b=64, r=8,
    the instant-NGP step), four PSH levels up to 512, the network with the
    coarse-opacity input, diffuse + tint composition; FP16 and FP32."""
    import synth
    t0 = time.time()
    w = synth.nolf_object(W, H)
    R = P.NolfRenderer.from_workload(w, tables=("f32", "f16"))
    out = {"workload": w.name, "cubes": int(len(w.density)), "levels": w.res, "keys": int(R.n_keys),
           "step": round(w.step, 7), "setup_s": round(time.time() - t0, 1)}
    rgba = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    for prec, table in (("fp16", "f16"), ("fp32", "f32")):
        hits = []
        for c in w.cameras:
            R.render(c, prec, table, rgba=rgba)
            torch.cuda.synchronize()
            hits.append(R.hit_count())
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(frames)]
        for i in range(frames):
            ev[i][0].record()
            R.render(w.cameras[i % len(w.cameras)], prec, table, rgba=rgba)
            ev[i][1].record()
        torch.cuda.synchronize()
        ms = [a.elapsed_time(b) for a, b in ev]
        out[prec] = {"Mrays_per_s": round(frames * W * H / (sum(ms) / 1e3) / 1e6, 1),
                     "ms_per_frame": round(sum(ms) / frames, 4), "p99_ms": round(pct(ms, 99), 4),
                     "hit_fraction": round(sum(hits) / len(hits) / (W * H), 4)}
        log(f"nolf {prec}: {out[prec]}")
    del R
    return out


def graph_bench(torch, P, R, frames=200):
    """One 1920x1080 camera at distance 2, FP16: eager renders (one
    library call each) against replays of the same render captured as a
    HIP graph; wall time over the frames between two synchronisations."""
    import synth
    cam = synth.fibonacci_cameras(8, 2.0, 1920, 1080)[0]
    n = cam.width * cam.height
    g = P.CapturedFrame(R, cam, "fp16", "f16")
    out = {"camera": "1920x1080, distance 2", "frames": frames}
    rgba = torch.empty((cam.height, cam.width, 4), device="cuda")
    for mode in ("eager", "graph"):
        for _ in range(5):
            g.replay() if mode == "graph" else R.render(cam, "fp16", "f16", rgba=rgba)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(frames):
            g.replay() if mode == "graph" else R.render(cam, "fp16", "f16", rgba=rgba)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[mode] = {"Mrays_per_s": round(frames * n / dt / 1e6, 1), "ms_per_frame": round(dt / frames * 1e3, 4)}
    torch.cuda.synchronize()
    same = bool(torch.equal(g.replay(), R.render(cam, "fp16", "f16")))
    torch.cuda.synchronize()
    out["replay_equals_eager"] = same
    log(f"graph: {out}")
    del g
    return out


def pipelined_bench(torch, P, R, cams, steps, warmup):
    """Frames of the headline workload with two in flight on two streams
    (FramePipeline): the trace of one frame overlaps the shading of the one
    before.  Whole-run throughput: all frames between two synchronizations."""
    W, H = cams[0].width, cams[0].height
    out = {"frames_in_flight": 2, "frames": steps}
    for prec, table in (("fp16", "f16"), ("fp32", "f32")):
        pipe = P.FramePipeline(R, depth=2)
        bufs = [torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for _ in range(2)]
        for i in range(warmup):
            pipe.submit(cams[i % len(cams)], prec, table, rgba=bufs[i % 2])
        pipe.wait()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            pipe.submit(cams[i % len(cams)], prec, table, rgba=bufs[i % 2])
        pipe.wait()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[prec] = {"Mrays_per_s": round(steps * W * H / dt / 1e6, 1), "ms_per_frame": round(dt / steps * 1e3, 4)}
        log(f"pipelined {prec}: {out[prec]}")
        del pipe
    return out


SERVE_BUDGET = 2 << 30  # HBM bytes per in-flight batch: workspace + FP32 RGBA images


def serve_bench(torch, P, S, center, distance, duration_s, clients=32, rate_hz=30.0):
    """Serving the resident 12-object scene: `clients` clients on seeded
    orbits ask for frames at Poisson times, each request's resolution drawn
    uniformly from 720p/1080p/1440p/4K; requests are admitted in arrival
    order into batches under an HBM budget per batch (workspace + output),
    each batch rendered by inrf_render_scene_batch, two batches in flight on
    their own streams.  Run in real time, then with every request released
    at once (saturated: aggregate throughput)."""
    import synth
    from paper_2303_04086_amd.serve import Request, Server
    reqs = [Request(k, t, c) for k, t, c in
            synth.orbit_requests(clients, duration_s, rate_hz, 13, distance=distance, center=center,
                                 resolutions=synth.SERVING_RESOLUTIONS, per_request=True)]
    offered = sum(r.pixels for r in reqs) / duration_s / 1e6
    out = {"target": "12-object scene (inrf_render_scene_batch)", "clients": clients,
           "rate_hz_per_client": rate_hz, "duration_s": duration_s, "requests": len(reqs),
           "offered_Mrays_per_s": round(offered, 1),
           "resolutions": "uniform per request over 1280x720, 1920x1080, 2560x1440, 3840x2160",
           "hbm_budget_bytes_per_batch": SERVE_BUDGET, "in_flight": 2,
           "graphs": "not used: the graph leg measures replay against eager launches of the same frame"}
    for prec, table in (("fp16", "f16"), ("fp32", "f32")):
        srv = Server(S, prec, table, hbm_budget=SERVE_BUDGET, in_flight=2, max_request_pixels=3840 * 2160)
        srv.run(reqs[: min(len(reqs), 16)], time_scale=0.0)  # warm-up
        out[prec] = srv.run(reqs)
        out[prec + "_saturated"] = srv.run(reqs, time_scale=0.0)
        log(f"serve {prec}: {out[prec]}; saturated {out[prec + '_saturated']}")
        del srv
        torch.cuda.empty_cache()
    return out


def views_bench(torch, R, cams, frames_label):
    """Frames over a list of cameras, FP16 path, one inrf_render each."""
    r = run_frames(torch, R, cams, "fp16", "f16", len(cams), 3)
    W, H = cams[0].width, cams[0].height
    hits = sum(r["hits"]) / len(cams)
    out = {"frames": len(cams), "width": W, "height": H, "protocol": frames_label,
           "Mrays_per_s": round(W * H * len(cams) / r["wall_s"] / 1e6, 1),
           "fps": round(len(cams) / r["wall_s"], 1),
           "p50_ms": round(pct(r["frame_ms"], 50), 4), "p99_ms": round(pct(r["frame_ms"], 99), 4),
           "hit_fraction": round(hits / (W * H), 4)}
    log(f"{frames_label}: {out}")
    return out


def compulsory_bench(torch, P, R, cam):
    """The gather's compulsory traffic on one 4K frame (FP16 tables): the
    distinct 128-byte lines of the feature table and of the offset table
    that the frame's hit rays touch, per level (each counted once, as if
    every later touch hit in cache), against the bytes the rays request."""
    import numpy as np
    n = cam.width * cam.height
    depth = torch.empty(n, device="cuda")
    R.render(cam, "fp16", "f16", depth=depth)
    o, d = P.camera_rays(cam)
    hit = torch.isfinite(depth)
    x = (o[hit] + depth[hit, None] * d[hit]).clamp(0.0, 1.0).contiguous()
    _, slots = R.encode(x, table="f16", slots=True)
    corners = torch.tensor([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], device="cuda")

    def lines(side, cx, cy, cz):
        # storage index of the brick layout (8 x 4 x 1 cells, inrf_brick_index), 32 four-byte entries per line
        row = 32 * ((side + 7) // 8)
        plane = row * ((side + 3) // 4)
        idx = cz * plane + (cy // 4) * row + (cx // 8) * 32 + (cy % 4) * 8 + cx % 8
        return int(torch.unique(idx // 32).numel())

    table_lines = phi_lines = 0
    for l, lv in enumerate(R.levels):
        m, rb, N = lv.mbar, lv.rbar, lv.res
        sl = slots[:, l, :].reshape(-1).long()
        table_lines += lines(m, sl % m, (sl // m) % m, sl // (m * m))
        p = torch.clamp(torch.floor(x * N), max=N - 1).long()
        v = (p[:, None, :] + corners[None]).reshape(-1, 3) % rb
        phi_lines += lines(rb, v[:, 0], v[:, 1], v[:, 2])
    hits = int(hit.sum().item())
    requested = hits * requested_bytes_per_hit(R.n_levels, "f16")
    out = {"hit_rays": hits, "requested_bytes": requested, "table_lines": table_lines, "offset_lines": phi_lines,
           "compulsory_bytes": 128 * (table_lines + phi_lines),
           "compulsory_over_requested": round(128 * (table_lines + phi_lines) / requested, 4)}
    log(f"compulsory: {out}")
    del slots, x
    return out


def peaks_bench(torch):
    """Measured ceilings (libinrf_peaks.so): streaming HBM read of a 4 GiB
    buffer and the network's matrix instructions in FP32, FP16 and BF16."""
    from paper_2303_04086_amd import peaks
    out = {"hbm_read": peaks.hbm_read(torch)}
    for prec in ("fp16", "bf16", "fp32"):
        out["mfma_" + prec] = peaks.mfma(torch, prec)
    log(f"peaks: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--distance", type=float, default=2.0,
                    help="camera distance from the object centre (the headline workload uses 2.0)")
    ap.add_argument("--width", type=int, default=3840)
    ap.add_argument("--height", type=int, default=2160)
    ap.add_argument("--cpu-sample", type=int, default=8192,
                    help="pixels of the oracle baseline (three quarters near the object)")
    ap.add_argument("--cpu-one-core", type=int, default=1024, help="of which timed again on one core")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--mlp-rays", type=int, default=1 << 24)
    ap.add_argument("--sweep-frames", type=int, default=8, help="frames per sweep case (0: no sweep)")
    ap.add_argument("--views", type=int, default=200,
                    help="seeded random 4K views of the paper's average-over-views protocol (0: none)")
    ap.add_argument("--no-peaks", dest="peaks", action="store_false", help="skip the measured-ceiling leg")
    ap.add_argument("--train-steps", type=int, default=10, help="timed training steps (0: none)")
    ap.add_argument("--train-batch", type=int, default=1 << 18)
    ap.add_argument("--scene-frames", type=int, default=16, help="timed frames of the 12-object scene (0: none)")
    ap.add_argument("--serve-seconds", type=float, default=0.25,
                    help="simulated client time of the serving leg (0: none)")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="skip the 1080p eager-versus-graph-replay leg")
    ap.add_argument("--nolf-frames", type=int, default=16,
                    help="timed frames of the paper's own i-NOLF form (0: none)")
    ap.add_argument("--pipelined-frames", type=int, default=100,
                    help="frames of the two-in-flight throughput leg (0: none)")
    ap.add_argument("--single-frames", type=int, default=16,
                    help="timed frames of the single-resolution PSH variants (0: none)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times), the reference "
                         "for scaling hardware byte counters, and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this path has no multi-GPU mode (rays are independent, "
              "so a frame would shard by tiles with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import synth

    W, H = args.width, args.height
    w = synth.workload_object(W, H)
    if args.distance != 2.0:
        w.cameras = synth.fibonacci_cameras(8, args.distance, W, H)
        w.name += f"_d{args.distance}"
    base = ref = None
    if not args.no_cpu_baseline:
        # on the host cores before anything touches the GPU (the workers are forked)
        log(f"timing the FP64 oracle on {args.cpu_sample} rays ...")
        base, ref = cpu_baseline(w, args.cpu_sample * 3 // 4, args.cpu_sample // 4, args.cpu_one_core)
        log(f"oracle: {base}")

    import torch
    import paper_2303_04086_amd as P
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    log(f"workload {w.name}: {len(w.tris)} triangles, levels {w.res}")
    t0 = time.time()
    levels = P.build_psh(w.verts, w.tris, w.res, dilate=w.dilate, seed=w.psh_seed)
    n_keys = sum(len(l.keys) for l in levels)
    log(f"PSH built: {n_keys} keys in {time.time() - t0:.1f} s")
    t0 = time.time()
    feats = lambda l, lv: synth.feature_values(w.feature_seed, l, lv.keys, F=w.F)
    R = P.Renderer(w.verts, w.tris, w.res, w.weights, feats, tables=("f32", "f16"), psh_levels=levels)
    del levels
    log(f"device model resident ({R.n_slots} slots/table) in {time.time() - t0:.1f} s")

    out = {}
    for prec, table in (("fp16", "f16"), ("fp32", "f32"), ("bf16", "f16")):
        r = run_frames(torch, R, w.cameras, prec, table, args.steps, args.warmup)
        out[prec] = (r, summarize(r, W, H, args.steps, R.n_levels, table))
        log(f"{prec}: {out[prec][1]['value']} Mrays/s, p50 {out[prec][1]['p50_ms']} ms, "
            f"p99 {out[prec][1]['p99_ms']} ms, trace {out[prec][1]['trace_ms_avg']} ms, "
            f"shade {out[prec][1]['shade_ms_avg']} ms")
    errors = None
    if ref is not None:
        errors = frame_errors(torch, R, w.cameras[0], ref, (("fp32", "f32"), ("fp16", "f16"), ("bf16", "f16")))
        log(f"errors against FP64: {errors}")
    mlp = {}
    if not args.no_mlp:
        for prec in ("fp16", "bf16"):
            mlp[prec] = mlp_bench(torch, R, prec, args.mlp_rays, encoded=True)
            mlp[prec + "_fp32_rows"] = mlp_bench(torch, R, prec, args.mlp_rays)
        mlp["fp32"] = mlp_bench(torch, R, "fp32", args.mlp_rays)
        for k, v in mlp.items():
            log(f"mlp {k}: {v}")
    # two frames in flight, measured before the legs that create more streams: with more than four
    # streams alive the runtime maps several onto one of its four hardware queues
    piped = (pipelined_bench(torch, P, R, w.cameras, args.pipelined_frames, args.warmup)
             if args.pipelined_frames > 0 else None)
    graph = graph_bench(torch, P, R) if args.graph else None
    sweep = sweep_bench(torch, R, w, args.sweep_frames) if args.sweep_frames > 0 else None
    views = None
    if args.views > 0:
        views = {"w2_200": views_bench(torch, R, synth.random_cameras(args.views, 21, 2.0, W, H),
                                       f"{args.views} seeded random views at distance 2"),
                 "w2_800": views_bench(torch, R, synth.fibonacci_cameras(8, 2.0, 800, 800) * 5,
                                       "800x800, the 8 cameras 5 times")}
    compulsory = compulsory_bench(torch, P, R, w.cameras[0])
    peaks = peaks_bench(torch) if args.peaks else None
    scene = serve = None
    if args.scene_frames > 0 or args.serve_seconds > 0:
        scene, S = scene_bench(torch, P, max(1, args.scene_frames), W, H)
        if args.serve_seconds > 0:
            serve = serve_bench(torch, P, S, (2.0, 2.0, 2.0), 6.0, args.serve_seconds)
        del S
        torch.cuda.empty_cache()
    nolf = nolf_bench(torch, P, args.nolf_frames, W, H) if args.nolf_frames > 0 else None
    single = (single_level_bench(torch, P, args.single_frames, W, H, out["fp16"][1]["shade_ms_avg"])
              if args.single_frames > 0 else None)
    train = None
    if args.train_steps > 0:
        train = train_bench(torch, P, R, w, args.train_steps, args.train_batch)
        log(f"train: {train}")

    head = out["fp16"][1]
    r16 = out["fp16"][0]
    shade_avg_s = sum(r16["shade_ms"]) / args.steps / 1e3
    bytes_launch = sum(r16["hits"]) / args.steps * requested_bytes_per_hit(R.n_levels, "f16")
    achieved = bytes_launch / shade_avg_s / 1e9
    traffic = load_traffic("k_shade_f16")
    roof = {"kernel": "k_shade (PSH gather + trilinear + SH16 + MLP)", "bound": "hbm",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "per_unit": f"{requested_bytes_per_hit(R.n_levels, 'f16')} B requested per hit ray",
            "units_per_launch": round(sum(r16["hits"]) / args.steps, 1),
            "avg_launch_ms": round(shade_avg_s * 1e3, 4)}
    if traffic:
        roof["traffic_GBps"] = round(traffic / shade_avg_s / 1e9, 1)
        roof["traffic_frac"] = round(traffic / shade_avg_s / 1e9 / HBM_PEAK_GBS, 4)
    if peaks:
        mp = peaks["hbm_read"]["GBps"]
        roof["measured_peak"] = mp
        roof["frac_of_measured_peak"] = round(achieved / mp, 4)
        if traffic:
            roof["traffic_frac_of_measured_peak"] = round(traffic / shade_avg_s / 1e9 / mp, 4)
        for k in mlp:
            pk = peaks["mfma_" + k.split("_")[0]]["TFLOPs"]
            mlp[k]["measured_peak"] = pk
            mlp[k]["utilisation_of_measured_peak"] = round(mlp[k]["TFLOPs"] / pk, 4)
    ratio = round(head["value"] / out["fp32"][1]["value"], 3)
    targets = {"gather_ge_0.60_of_hbm": {"value": roof["frac"], "met": bool(roof["frac"] >= 0.60)}}
    if mlp:
        targets["mlp_ge_0.40_of_mfma"] = {"value": mlp["fp16"]["utilisation"],
                                          "of_measured_peak": mlp["fp16"].get("utilisation_of_measured_peak"),
                                          "met": bool(mlp["fp16"]["utilisation"] >= 0.40)}
    if errors:
        targets["fp32_max_abs_le_1e-5"] = {"value": errors["fp32"]["max_abs_not_grazing"],
                                           "all_pixels": errors["fp32"]["max_abs"],
                                           "met": bool(errors["fp32"]["max_abs_not_grazing"] <= 1e-5)}
        targets["fp16_max_abs_le_2e-3_psnr_ge_50"] = {
            "value": [errors["fp16"]["max_abs"], errors["fp16"]["psnr_db"]],
            "met": bool(errors["fp16"]["max_abs"] <= 2e-3 and (errors["fp16"]["psnr_db"] or 1e9) >= 50.0)}
    targets["fp16_ge_2x_fp32"] = {"value": ratio, "met": bool(ratio >= 2.0)}
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": w.name, "width": W, "height": H, "levels": R.n_levels, "res_max": max(w.res),
                   "features": w.F, "mlp": "48-64-64-4", "cameras": len(w.cameras), "tables": "f16",
                   "network": "fp16 MFMA, fp32 accumulate", "keys": n_keys},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "fp16": head,
        "fp32": out["fp32"][1],
        "bf16": out["bf16"][1],
        "fp16_over_fp32": ratio,
        "errors_vs_fp64": errors,
        "targets": targets,
        "roofline": roof,
        "peaks": peaks,
        "compulsory": compulsory,
        "mlp": mlp or None,
        "sweep": sweep,
        "views": views,
        "scene": scene,
        "single_level": single,
        "serve": serve,
        "pipelined": piped,
        "graph": graph,
        "nolf": nolf,
        "train": train,
        "cpu_baseline": base,
        "source": source_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
