"""inrf_render and the stage-event entry point inrf_render_profiled must
give the same pixels, depth, triangle ids and hit count bit for bit, at
ragged sizes whose tile strips end part way, and frames of different sizes
issued back to back on one stream must each equal a lone render."""
import numpy as np
import pytest

import synth
from gpu_helpers import make_renderer

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R(tiny):
    return make_renderer(tiny, tables=("f32", "f16"), kind="uniform", sigma=0.5)


def _frame(R, cam, prec, table, profiled):
    n = cam.width * cam.height
    depth = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if profiled else None
    if ev:
        for e in ev:
            e.record()
    rgba = R.render(cam, prec, table, depth=depth, tri=tri, events=ev)
    torch.cuda.synchronize()
    return rgba.clone(), depth, tri, R.hit_count()


@pytest.mark.parametrize("wh", [(160, 300), (64, 520), (257, 450), (100, 1100)])
@pytest.mark.parametrize("prec,table", [("fp32", "f32"), ("fp16", "f16")])
def test_render_equals_profiled(R, wh, prec, table):
    cam = synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 1.6 * np.array([0.3, -0.8, 0.52]), (0.5, 0.5, 0.5),
                               40.0, *wh)
    a = _frame(R, cam, prec, table, profiled=False)
    b = _frame(R, cam, prec, table, profiled=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    assert a[3] == b[3] == int((b[2] >= 0).sum().item()) > 0


def test_frames_back_to_back_on_one_stream(R):
    """Frames of different sizes in a row without synchronisation in
    between: each equals its lone render."""
    cams = [synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 2.0 * d, (0.5, 0.5, 0.5), 40.0, w, h)
            for d, (w, h) in zip(synth.camera.fibonacci_directions(4), [(200, 300), (64, 32), (130, 520), (96, 96)])]
    outs = [R.render(c, "fp16", "f16") for c in cams]
    torch.cuda.synchronize()
    for c, o in zip(cams, outs):
        ref = _frame(R, c, "fp16", "f16", profiled=True)[0]
        assert torch.equal(o, ref)
