"""A render captured as a HIP graph (CapturedFrame) and replayed several
times, with the program's own eager renders and synchronisations between
the replays: every replay must equal the eager render bit for bit."""
import numpy as np
import pytest

import synth
from gpu_helpers import make_renderer

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R(tiny):
    return make_renderer(tiny, tables=("f32", "f16"), kind="uniform", sigma=0.5)


@pytest.mark.parametrize("prec,table,wh", [("fp16", "f16", (160, 300)), ("fp32", "f32", (37, 23))])
def test_captured_frame_replays_equal_eager(R, prec, table, wh):
    import paper_2303_04086_amd as P
    cam = synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 1.7 * np.array([0.6, 0.48, -0.64]), (0.5, 0.5, 0.5),
                               40.0, *wh)
    other = synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 2.0 * np.array([-0.3, 0.9, 0.3]), (0.5, 0.5, 0.5),
                                 40.0, 64, 48)
    n = wh[0] * wh[1]
    d_ref = torch.empty(n, device="cuda")
    t_ref = torch.empty(n, dtype=torch.int32, device="cuda")
    ref = R.render(cam, prec, table, depth=d_ref, tri=t_ref).clone()
    torch.cuda.synchronize()
    g = P.CapturedFrame(R, cam, prec, table, depth=True, tri=True)
    for i in range(4):
        R.render(other, prec, table)               # eager work between replays
        torch.cuda.synchronize()
        g.rgba.zero_()
        g.depth.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(g.rgba, ref), i
        assert torch.equal(g.depth, d_ref) and torch.equal(g.tri, t_ref), i
