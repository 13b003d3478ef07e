"""Batched rendering of several cameras (inrf_render_batch for one object,
inrf_render_scene_batch for a scene) and the serving loop built on them:
every pixel of a batch equals the single-camera render bit for bit (rays of
different requests share waves but each ray's closest hit and colour are
its own), and the loop serves every request under its HBM budget, each
frame equal to the same frame rendered alone."""
import numpy as np
import pytest

import synth
from gpu_helpers import make_renderer

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R(tiny):
    return make_renderer(tiny, tables=("f32", "f16"), kind="uniform", sigma=0.5)


def _budget(T, n_cameras, n_pixels):
    """The HBM bytes of a batch of n_cameras cameras with n_pixels in all."""
    return T.batch_workspace_bytes(n_cameras, n_pixels) + 16 * n_pixels


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
    S = Server(R, "fp32", "f32", hbm_budget=_budget(R, 6, 3 * 64 * 64), max_batch=6, max_request_pixels=64 * 64)
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
        S = Server(R, "fp16", "f16", hbm_budget=_budget(R, 4, 2 * 64 * 64), max_batch=4, in_flight=in_flight,
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


def test_server_admission_by_hbm_bytes(R):
    """No batch holds more than the budget, and a request larger than the
    budget is refused before anything runs."""
    from paper_2303_04086_amd.serve import Request, Server
    reqs = [Request(k, t, c) for k, t, c in
            synth.orbit_requests(8, 0.05, 200.0, 11, resolutions=((64, 64), (48, 32), (100, 40)), per_request=True)]
    budget = _budget(R, 3, 2 * 64 * 64)
    S = Server(R, "fp16", "f16", hbm_budget=budget, in_flight=2, max_request_pixels=100 * 40)
    out = S.run(reqs, time_scale=0.0)
    assert out["requests"] == len(reqs) and 0 < out["max_batch_bytes"] <= budget
    big = synth.look_at_camera((0.5, 0.5, 2.5), (0.5, 0.5, 0.5), 40.0, 400, 400)
    with pytest.raises(ValueError):
        S.run([Request(0, 0.0, big)])
    with pytest.raises(ValueError):
        Server(R, "fp16", "f16", hbm_budget=_budget(R, 1, 64 * 64) - 1, max_request_pixels=64 * 64)


# -- scenes -----------------------------------------------------------------

@pytest.fixture(scope="module")
def scene():
    import paper_2303_04086_amd as P
    sc = synth.scene_tiny(3)
    rs = [make_renderer(o.workload, tables=("f32", "f16")) for o in sc.objects]
    return sc, P.Scene(rs, [(o.scale, o.rotation, o.translation) for o in sc.objects])


def _scene_cams(sc, sizes):
    from synth.camera import fibonacci_directions
    c = np.array([1.25, 1.25, 1.25])
    return [synth.look_at_camera(c + 4.5 * d, c, 40.0, w, h) for d, (w, h) in zip(fibonacci_directions(8), sizes)]


def _scene_alone(S, cam, prec, table):
    k = cam.width * cam.height
    d = torch.empty(k, device="cuda")
    t = torch.empty(k, dtype=torch.int32, device="cuda")
    o = torch.empty(k, dtype=torch.int32, device="cuda")
    rgba = S.render(cam, prec, table, depth=d, tri=t, obj=o)
    torch.cuda.synchronize()
    return rgba.clone(), d, t, o


@pytest.mark.parametrize("prec,table", [("fp32", "f32"), ("fp16", "f16"), ("bf16", "f16")])
def test_scene_batch_equals_single_renders(scene, prec, table):
    """inrf_render_scene_batch over cameras of different sizes (ragged
    tiles, a 1x1 frame) equals inrf_render_scene of each camera alone, in
    colour, depth, triangle and object ids, bit for bit."""
    sc, S = scene
    cams = _scene_cams(sc, [(64, 64), (37, 23), (1, 1), (100, 40), (17, 33)])
    n = sum(c.width * c.height for c in cams)
    depth = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    obj = torch.empty(n, dtype=torch.int32, device="cuda")
    _, views = S.render_batch(cams, prec, table, depth=depth, tri=tri, obj=obj)
    torch.cuda.synchronize()
    views = [v.clone() for v in views]
    off, hits = 0, 0
    for c, v in zip(cams, views):
        k = c.width * c.height
        rgba, d, t, o = _scene_alone(S, c, prec, table)
        assert torch.equal(v, rgba)
        assert torch.equal(depth[off:off + k], d) and torch.equal(tri[off:off + k], t)
        assert torch.equal(obj[off:off + k], o)
        hits += int((o >= 0).sum())
        off += k
    assert hits > 500 and len(torch.unique(obj[obj >= 0])) == 3


def test_scene_batch_limits(scene):
    sc, S = scene
    import ctypes
    import paper_2303_04086_amd as P
    from paper_2303_04086_amd import _lib as L
    assert P.lib().inrf_scene_batch_workspace_size(3, 17, 100) == -1
    assert P.lib().inrf_scene_batch_workspace_size(3, 0, 100) == -1
    assert P.lib().inrf_scene_batch_workspace_size(L.MAX_OBJECTS + 1, 1, 100) == -1
    one = S.batch_workspace_bytes(1, 64 * 64)
    assert S.batch_workspace_bytes(16, 64 * 64) > one > 0 and S.batch_workspace_bytes(4, 64 * 64) >= one
    arr = (L.CameraDesc * 1)()
    inst = S.instances("f32")
    assert P.lib().inrf_render_scene_batch(inst, 3, 0, arr, 17, None, None, None, None, None, 0, None) == -1
    cams = _scene_cams(sc, [(64, 64)])
    ws = torch.empty(one - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        S.render_batch(cams, ws=ws)


@pytest.mark.parametrize("prec,table", [("fp32", "f32"), ("fp16", "f16")])
def test_scene_server_frames_equal_alone(scene, prec, table):
    """The resident scene served to clients whose requests draw their
    resolution uniformly per request: every request is served, batches mix
    requests of several sizes, and every frame equals the same camera
    rendered alone, bit for bit."""
    from paper_2303_04086_amd.serve import Request, Server
    sc, S = scene
    sizes = ((64, 36), (96, 54), (128, 72), (192, 108))  # the 16:9 mix, scaled down
    reqs = [Request(k, t, c) for k, t, c in
            synth.orbit_requests(8, 0.05, 200.0, 21, distance=4.5, resolutions=sizes, center=(1.25, 1.25, 1.25),
                                 per_request=True)]
    assert len(reqs) > 40 and len({r.pixels for r in reqs}) == 4
    budget = _budget(S, 6, 3 * 192 * 108)
    server = Server(S, prec, table, hbm_budget=budget, max_batch=6, in_flight=2, max_request_pixels=192 * 108)
    seen, mixed = [], [0]

    def check(batch, views):
        if len({r.pixels for r in batch}) > 1:
            mixed[0] += 1
        for r, v in zip(batch, views):
            assert torch.equal(v, _scene_alone(S, r.camera, prec, table)[0])
        seen.extend(batch)

    out = server.run(reqs, on_batch=check, time_scale=0.0)
    print("scene serve:", out)
    assert out["requests"] == len(reqs) == len(seen) and out["max_batch_bytes"] <= budget
    assert mixed[0] > 0 and out["mean_batch"] > 1
