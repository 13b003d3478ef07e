"""The allocation-free render (inrf_render_static: scratch in a static device
array of the library instead of a caller workspace) against inrf_render,
through the C ABI: two frames in a row, the second smaller than the first,
each equal to inrf_render's pixels bit for bit (colour, depth, triangle) in
FP32 and FP16; a frame beyond the static limit is refused with nothing
written."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_helpers import make_renderer

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    return make_renderer(synth.workload_tiny(), tables=("f32", "f16"))


def _cam(W, H):
    v = np.array([0.3, -0.8, 0.52])
    return synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 1.6 * v / np.linalg.norm(v), (0.5, 0.5, 0.5), 40.0, W, H)


def _static(R, cam, prec, table):
    from paper_2303_04086_amd import _lib as L
    from paper_2303_04086_amd.model import PRECISIONS, _camera_desc
    n = cam.width * cam.height
    rgba = torch.full((n, 4), -7.0, device="cuda")
    depth = torch.full((n,), -7.0, device="cuda")
    tri = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    st = L.lib().inrf_render_static(ctypes.byref(R.desc(table)), PRECISIONS[prec], ctypes.byref(_camera_desc(cam)),
                                    L.ptr(rgba), L.ptr(depth), L.ptr(tri),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, rgba, depth, tri


def _reference(R, cam, prec, table):
    n = cam.width * cam.height
    depth = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    rgba = R.render(cam, prec, table, depth=depth, tri=tri).reshape(-1, 4)
    return rgba, depth, tri


def test_static_render_equals_render(R):
    from paper_2303_04086_amd import _lib as L
    big = _cam(1024, 1000)            # 1,024,000 pixels: near the static limit of 1,048,576
    small = _cam(320, 203)
    for cam in (big, small):
        print(f"static render {cam.width}x{cam.height}", flush=True)
        for prec, table in (("fp32", "f32"), ("fp16", "f16")):
            st, rgba, depth, tri = _static(R, cam, prec, table)
            assert st == L.INRF_OK, L.lib().inrf_last_error()
            ref = _reference(R, cam, prec, table)
            torch.cuda.synchronize()
            assert (tri >= 0).sum().item() > 0.1 * cam.width * cam.height
            for got, want, name in zip((rgba, depth, tri), ref, ("rgba", "depth", "tri")):
                assert torch.equal(got, want), (cam.width, prec, name)


def test_static_render_refuses_large_frames(R):
    from paper_2303_04086_amd import _lib as L
    cam = _cam(1025, 1024)            # one row of pixels beyond the limit
    st, rgba, depth, tri = _static(R, cam, "fp32", "f32")
    torch.cuda.synchronize()
    assert st == L.INRF_E_SIZE and b"at most" in L.lib().inrf_last_error()
    assert bool((rgba == -7.0).all()) and bool((depth == -7.0).all()) and bool((tri == -7).all())
