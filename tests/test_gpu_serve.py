"""Batched rendering of several cameras (inrf_render_batch) and the serving
loop built on it: every pixel of a batch equals the single-camera render bit
for bit (rays of different requests share waves but each ray's closest hit
and colour are its own), and the loop serves every request."""
import numpy as np
import pytest

import synth
from gpu_helpers import make_renderer

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R(tiny):
    return make_renderer(tiny, tables=("f32", "f16"), kind="uniform", sigma=0.5)


def _cams():
    from synth.camera import fibonacci_directions
    dirs = fibonacci_directions(8)
    sizes = [(64, 64), (37, 23), (17, 33), (1, 1), (100, 40)]
    return [synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 2.0 * d, (0.5, 0.5, 0.5), 40.0, w, h)
            for d, (w, h) in zip(dirs, sizes)]


@pytest.mark.parametrize("prec,table", [("fp32", "f32"), ("fp16", "f16")])
def test_batch_equals_single_renders(R, prec, table):
    cams = _cams()
    n = sum(c.width * c.height for c in cams)
    depth = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    _, views = R.render_batch(cams, prec, table, depth=depth, tri=tri)
    torch.cuda.synchronize()
    off = 0
    for c, v in zip(cams, views):
        k = c.width * c.height
        d1 = torch.empty(k, device="cuda")
        t1 = torch.empty(k, dtype=torch.int32, device="cuda")
        ref = R.render(c, prec, table, depth=d1, tri=t1)
        torch.cuda.synchronize()
        assert torch.equal(v, ref)
        assert torch.equal(depth[off:off + k], d1) and torch.equal(tri[off:off + k], t1)
        off += k


def test_server_serves_every_request(R):
    from paper_2303_04086_amd.serve import Request, Server
    # arrivals compressed 1000x so that requests queue behind a running batch
    reqs = [Request(k, t / 1000.0, c) for k, t, c in
            synth.orbit_requests(8, 0.02, 400.0, 3, resolutions=((64, 64), (48, 32), (33, 17)))]
    assert len(reqs) > 20
    S = Server(R, "fp32", "f32", pixel_budget=3 * 64 * 64, max_batch=6)
    checked = []

    def check(batch, views):
        if len(checked) < 3:
            for r, v in zip(batch, views):
                assert torch.equal(v, R.render(r.camera, "fp32", "f32"))
            checked.append(len(batch))

    out = S.run(reqs, on_batch=check)
    print("serve:", out)
    assert out["requests"] == len(reqs) and out["batches"] >= len(reqs) / 6
    assert 0 < out["p50_latency_ms"] <= out["p99_latency_ms"]
    assert max(checked) > 1  # batches of several requests were compared


def test_server_overlap_and_saturation(R):
    """Two batches in flight and all requests released at once (the
    saturated case): every request is served and its image equals a lone
    render; one batch in flight gives the same images."""
    from paper_2303_04086_amd.serve import Request, Server
    reqs = [Request(k, t, c) for k, t, c in
            synth.orbit_requests(6, 0.05, 200.0, 5, resolutions=((64, 64), (48, 32), (100, 40)))]
    for in_flight in (2, 1):
        S = Server(R, "fp16", "f16", pixel_budget=2 * 64 * 64, max_batch=4, in_flight=in_flight,
                   max_request_pixels=100 * 40)
        seen = []

        def check(batch, views):
            for r, v in zip(batch, views):
                assert torch.equal(v, R.render(r.camera, "fp16", "f16"))
            seen.extend(r.client for r in batch)

        out = S.run(reqs, on_batch=check, time_scale=0.0)
        assert out["requests"] == len(reqs) == len(seen) and out["in_flight"] == in_flight
        assert out["mean_batch"] > 1


def test_frame_pipeline_matches_lone_renders(R):
    import paper_2303_04086_amd as P
    cams = _cams()
    pipe = P.FramePipeline(R, depth=2)
    outs = []
    for c in cams + cams:
        k = c.width * c.height
        d = torch.empty(k, device="cuda")
        t = torch.empty(k, dtype=torch.int32, device="cuda")
        outs.append((c, pipe.submit(c, "fp16", "f16", depth=d, tri=t), d, t))
    rgbas = []
    pipe2 = P.FramePipeline(R, depth=2)
    for c in cams:
        rgbas.append(torch.empty((c.height, c.width, 4), device="cuda"))
        pipe2.submit(c, "fp32", "f32", rgba=rgbas[-1])
    pipe.wait()
    pipe2.wait()
    torch.cuda.synchronize()
    for c, x, d, t in outs:
        d1 = torch.empty_like(d)
        t1 = torch.empty_like(t)
        ref = R.render(c, "fp16", "f16", depth=d1, tri=t1)
        torch.cuda.synchronize()
        assert torch.equal(x, ref) and torch.equal(d, d1) and torch.equal(t, t1)
    for c, x in zip(cams, rgbas):
        assert torch.equal(x, R.render(c, "fp32", "f32"))


def test_batch_limits(R):
    import ctypes
    import paper_2303_04086_amd as P
    from paper_2303_04086_amd import _lib as L
    with pytest.raises(ValueError):
        R.render_batch(_cams() * 4)  # 20 cameras
    assert P.lib().inrf_batch_workspace_size(17, 100) == -1 and P.lib().inrf_batch_workspace_size(0, 100) == -1
    arr = (L.CameraDesc * 1)()
    st = P.lib().inrf_render_batch(ctypes.byref(R.desc("f32")), 0, arr, 17, None, None, None, None, 0, None)
    assert st == -1
