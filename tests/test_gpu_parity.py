"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP32 path, features N(0, 0.01)): the network output differs from
FP64 by FP32 rounding of the gather, the hit point (FP32 x carries ~2^-24
relative error, amplified by N <= 2048 in the cell weights) and the matrix-core
accumulation; 1e-5 max abs bounds all three.  Reduced precision: 2e-3 max abs
and PSNR >= 50 dB against FP64.  Triangle ids and hash slots are compared bit
for bit; rays within rounding of an edge or the silhouette (the oracle's
`ambiguous` flag) may take either answer."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_hits, feature_fn, make_renderer, psnr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def R(tiny):
    return make_renderer(tiny)


@pytest.fixture(scope="module")
def tiny_psh(tiny, tiny_keys):
    return [oracle.build_psh_level(k, N, seed=tiny.psh_seed) for N, k in zip(tiny.res, tiny_keys)]


def test_trace_matches_brute_force(tiny, R):
    o, d = synth.random_rays(6000, 21)
    tri, t = R.trace(_dev(o), _dev(d))
    torch.cuda.synchronize()
    ora = oracle.closest_hit(o.astype(np.float64), d.astype(np.float64), tiny.verts, tiny.tris)
    tri = tri.cpu().numpy()
    t = t.cpu().numpy()
    agree = compare_hits(tri, {"tri": ora.tri, "ambiguous": ora.ambiguous})
    both = agree & (tri >= 0)
    assert both.sum() > 1000
    rel = np.abs(t[both] - ora.t[both]) / ora.t[both]
    print(f"trace: max rel t error {rel.max():.2e} over {both.sum()} hits")
    assert rel.max() <= 1e-5
    assert np.all(np.isinf(t[tri < 0]))


def test_trace_edge_cases(R):
    o = np.array([[0.5, 0.5, 3.0], [np.nan, 0, 0], [0.5, 0.5, 3.0], [0.5, 0.5, 0.5], [0.5, 0.5, 3.0]], np.float32)
    d = np.array([[0, 0, -1], [0, 0, 1], [0, 0, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    tri, t = R.trace(_dev(o), _dev(d))
    tri, t = tri.cpu().numpy(), t.cpu().numpy()
    assert tri[0] >= 0 and abs(t[0] - 2.0) < 1e-6        # top of the sphere at z = 1
    assert tri[1] == -1 and tri[2] == -1 and tri[4] == -1  # non-finite, zero direction, pointing away
    assert tri[3] >= 0 and 0.45 < t[3] <= 0.5             # from the centre: back faces count (two-sided)


def test_encode_matches_dictionary_lookup(tiny, R, tiny_oracle, tiny_psh):
    x = synth.surface_points(tiny.verts, tiny.tris, 3000, 5)
    # cell boundaries, the x = 1 face and points a hair inside it
    x = np.concatenate([x, np.array([[0.5, 0.5, 1.0], [1.0, 0.5, 0.5], [0.5, 0.0, 0.5],
                                     [0.5, 0.5, np.float32(1) - np.float32(2 ** -24)]], np.float32)])
    enc, sl = R.encode(_dev(x), slots=True)
    enc, sl = enc.cpu().numpy(), sl.cpu().numpy()
    want = oracle.encode_points(tiny_oracle, x)
    assert np.abs(enc - want).max() <= 1e-6
    for l, (N, L) in enumerate(zip(tiny.res, tiny_psh)):
        cv = oracle.encode.corner_vertices(x, N).reshape(-1, 3)
        assert np.array_equal(sl[:, l, :].reshape(-1).astype(np.int64), oracle.psh_slots(L, cv))


def test_encode_half_table(tiny, R, tiny_oracle):
    x = synth.surface_points(tiny.verts, tiny.tris, 2000, 6)
    enc = R.encode(_dev(x), table="f16").cpu().numpy()
    want = oracle.encode_points(tiny_oracle, x)
    assert np.abs(enc - want).max() <= 2e-5          # FP16 rounding of 0.01-scale features


@pytest.fixture(scope="module")
def R16(tiny):
    """Sixteen levels on the tiny proxy: the object workload's 48-wide input."""
    w = synth.workload_tiny()
    w.res = [4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19]
    w.weights = synth.xavier_mlp(3, w.d_in)
    return make_renderer(w, tables=("f32",)), w


@pytest.mark.parametrize("levels", [4, 16])
@pytest.mark.parametrize("n", [1, 15, 64, 1000, 4099])
def test_mlp_precisions(tiny, R, R16, n, levels):
    rng = np.random.default_rng(n)
    if levels == 16:
        R, tiny = R16
    d_in = tiny.d_in
    inp = np.concatenate([rng.normal(0, 0.02, (n, d_in - 16)), oracle.sh_real(rng.normal(size=(n, 3)))], 1)
    want = oracle.mlp_forward(inp, tiny.weights)
    x = _dev(inp.astype(np.float32))
    got = R.mlp(x, "fp32").cpu().numpy()
    got16 = R.mlp(x, "fp16").cpu().numpy()
    gotbf = R.mlp(x, "bf16").cpu().numpy()
    e32, e16, ebf = (np.abs(g - want).max() for g in (got, got16, gotbf))
    print(f"mlp L={levels} n={n}: fp32 {e32:.2e} fp16 {e16:.2e} bf16 {ebf:.2e}")
    assert e32 <= 1e-5
    assert e16 <= 2e-3
    assert ebf <= 2e-2        # BF16 is reported, not held to 2e-3
    loud = rng.uniform(-1, 1, (n, d_in))
    got = R.mlp(_dev(loud.astype(np.float32)), "fp32").cpu().numpy()
    assert np.abs(got - oracle.mlp_forward(loud, tiny.weights)).max() <= 1e-5


@pytest.mark.parametrize("levels", [4, 5, 16])
@pytest.mark.parametrize("n", [1, 15, 4099])
def test_mlp_encoded_inputs(levels, n):
    """The network on 16-bit encodings and view directions
    (inrf_mlp_encoded) against the FP64 network on the same 16-bit encoding
    values and the SH16 of the unit direction: FP16 to 2e-3, BF16 reported
    (2e-2).  Five levels give rows that are not 16-byte aligned."""
    w = synth.workload_tiny()
    w.res = [4 + 3 * k for k in range(levels)]
    w.weights = synth.xavier_mlp(11 + levels, w.d_in)
    Rl = make_renderer(w, tables=("f32",))
    rng = np.random.default_rng(100 * levels + n)
    enc = rng.normal(0, 0.3, (n, 2 * levels))
    dirs = rng.normal(size=(n, 3)) * rng.uniform(0.5, 2.0, (n, 1))     # not unit
    for prec, dt, tol in (("fp16", torch.float16, 2e-3), ("bf16", torch.bfloat16, 2e-2)):
        e16 = torch.from_numpy(enc).to(dt)
        want = oracle.mlp_forward(np.concatenate([e16.to(torch.float64).numpy(), oracle.sh_real(dirs)], 1), w.weights)
        got = Rl.mlp_encoded(e16.cuda(), _dev(dirs.astype(np.float32)), prec).cpu().numpy()
        err = np.abs(got - want).max()
        print(f"mlp_encoded L={levels} n={n} {prec}: {err:.2e}")
        assert err <= tol
    import paper_2303_04086_amd as P
    with pytest.raises(P.InrfError):
        Rl.mlp_encoded(e16.cuda(), _dev(dirs.astype(np.float32)), "fp32")


@pytest.mark.parametrize("n_levels", [5, 13])
def test_mlp_odd_levels_and_unaligned_inputs(n_levels):
    """Rows that are not 16-byte aligned (odd level count, or an input array
    starting 4 bytes into an allocation) take the element-wise load path."""
    w = synth.workload_tiny()
    w.res = list(range(4, 4 + n_levels))
    w.weights = synth.xavier_mlp(5, w.d_in)
    R5 = make_renderer(w, tables=("f32",))
    rng = np.random.default_rng(n_levels)
    n = 999
    inp = np.concatenate([rng.uniform(-1, 1, (n, w.d_in - 16)), oracle.sh_real(rng.normal(size=(n, 3)))], 1)
    want = oracle.mlp_forward(inp, w.weights)
    flat = torch.zeros(n * w.d_in + 1, device="cuda")
    flat[1:] = _dev(inp.astype(np.float32).reshape(-1))
    for x in (_dev(inp.astype(np.float32)), flat[1:].view(n, w.d_in)):
        for prec, tol in (("fp32", 1e-5), ("fp16", 2e-3)):
            got = R5.mlp(x, prec).cpu().numpy()
            assert np.abs(got - want).max() <= tol, (prec, x.data_ptr() % 16)


@pytest.mark.parametrize("N", [64, 40])
def test_single_resolution_model(N):
    """One level (the paper's single-resolution PSH): the LPG = 1 kernels."""
    w = synth.workload_tiny()
    w.res = [N]
    w.weights = synth.xavier_mlp(9, w.d_in)
    R1 = make_renderer(w, tables=("f32", "f16"), kind="uniform", sigma=0.5)
    cam = w.cameras[0]
    tri = torch.empty(cam.height * cam.width, dtype=torch.int32, device="cuda")
    got = R1.render(cam, "fp32", "f32", tri=tri).cpu().numpy().reshape(-1, 4)
    got16 = R1.render(cam, "fp16", "f16").cpu().numpy().reshape(-1, 4)
    ora = oracle.render_camera(oracle.Model.from_workload(w, kind="uniform", sigma=0.5), cam)
    agree = compare_hits(tri.cpu().numpy(), ora)
    assert np.abs(got[agree] - ora["rgba"][agree]).max() <= 1e-4   # loud features, N <= 64
    assert np.abs(got16[agree] - ora["rgba"][agree]).max() <= 2e-3


def test_render_full_frame_fp32(tiny, R, tiny_oracle):
    cam = tiny.cameras[0]
    depth = torch.empty(cam.height * cam.width, device="cuda")
    tri = torch.empty(cam.height * cam.width, dtype=torch.int32, device="cuda")
    rgba = R.render(cam, "fp32", "f32", depth=depth, tri=tri)
    torch.cuda.synchronize()
    ora = oracle.render_camera(tiny_oracle, cam)
    tri = tri.cpu().numpy()
    agree = compare_hits(tri, ora)
    rgba = rgba.cpu().numpy().reshape(-1, 4)
    assert np.abs(rgba[agree] - ora["rgba"][agree]).max() <= 1e-5
    assert np.all(rgba[tri < 0] == 0)
    dep = depth.cpu().numpy()
    hit = (tri >= 0) & agree
    assert np.allclose(dep[hit], ora["t"][hit], rtol=1e-5) and np.all(np.isinf(dep[tri < 0]))


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_render_full_frame_reduced_precision(tiny, R, tiny_oracle, prec):
    cam = tiny.cameras[0]
    tri = torch.empty(cam.height * cam.width, dtype=torch.int32, device="cuda")
    rgba = R.render(cam, prec, "f16", tri=tri).cpu().numpy().reshape(-1, 4)
    ora = oracle.render_camera(tiny_oracle, cam)
    tri = tri.cpu().numpy()
    agree = compare_hits(tri, ora)                      # ids bit-exact where unambiguous
    assert np.all(agree | ora["ambiguous"])             # every hit/miss disagreement is flagged
    assert np.all(rgba[tri < 0] == 0)
    hit = agree & (tri >= 0)
    err = np.abs(rgba[agree] - ora["rgba"][agree]).max()
    p = psnr(rgba[hit], ora["rgba"][hit])
    print(f"{prec}: max abs {err:.3e}, PSNR {p:.1f} dB over {hit.sum()} hits")
    if prec == "fp16":
        assert err <= 2e-3 and p >= 50.0
    else:
        assert err <= 2e-2


def _cam(W, H, direction=(0.3, -0.8, 0.52)):
    v = np.asarray(direction, np.float64)
    return synth.look_at_camera(np.array([0.5, 0.5, 0.5]) + 2.0 * v / np.linalg.norm(v), (0.5, 0.5, 0.5), 40.0, W, H)


@pytest.mark.parametrize("wh", [(64, 64), (37, 23), (200, 150)])
def test_render_is_deterministic_and_equals_forward(tiny, R, wh):
    """Two renders of a frame are identical, and equal inrf_forward on the
    camera's own rays (inrf_camera_rays) bit for bit: colour, depth and
    triangle, in every precision."""
    import paper_2303_04086_amd as P
    cam = tiny.cameras[0] if wh == (64, 64) else _cam(*wh)
    n = cam.width * cam.height
    o, d = P.camera_rays(cam)
    for prec, table in (("fp32", "f32"), ("fp16", "f16"), ("bf16", "f16"), ("fp32", "f16")):
        outs = []
        for k in range(2):
            dep = torch.empty(n, device="cuda")
            tri = torch.empty(n, dtype=torch.int32, device="cuda")
            rgba = R.render(cam, prec, table, depth=dep, tri=tri).reshape(-1, 4).clone()
            outs.append((rgba, dep, tri))
        assert all(torch.equal(x, y) for x, y in zip(*outs)), prec
        dep = torch.empty(n, device="cuda")
        tri = torch.empty(n, dtype=torch.int32, device="cuda")
        rgba = R.forward(o, d, prec, table, depth=dep, tri=tri)
        for x, y, name in zip(outs[0], (rgba, dep, tri), ("rgba", "depth", "tri")):
            assert torch.equal(x, y), (prec, table, name)


def test_camera_rays_match_the_camera_definition(tiny):
    """inrf_camera_rays against the FP64 camera convention (oracle.camera_rays):
    same origins, unit directions within FP32 rounding."""
    import paper_2303_04086_amd as P
    for cam in (tiny.cameras[0], _cam(37, 23), _cam(5, 200, (0.0, 0.0, 1.0))):
        o, d = P.camera_rays(cam)
        oo, od = oracle.camera_rays(cam)
        assert np.array_equal(o.cpu().numpy(), np.broadcast_to(oo, o.shape).astype(np.float32))
        assert np.abs(d.cpu().numpy() - od).max() <= 1e-6


def test_forward_matches_oracle(tiny, R, tiny_oracle):
    o, d = synth.random_rays(3000, 8)
    rgba = R.forward(_dev(o), _dev(d), "fp32").cpu().numpy()
    ora = oracle.render_rays(tiny_oracle, o.astype(np.float64), d.astype(np.float64))
    gtri = R.trace(_dev(o), _dev(d))[0].cpu().numpy()
    agree = compare_hits(gtri, ora)
    assert np.abs(rgba[agree] - ora["rgba"][agree]).max() <= 1e-5
    # a batch is independent of its composition: a sub-batch gives the same colours
    sub = R.forward(_dev(o[100:357]), _dev(d[100:357]), "fp32").cpu().numpy()
    assert np.array_equal(sub, rgba[100:357])


@pytest.mark.parametrize("wh", [(37, 23), (1, 1), (16, 16), (17, 33)])
def test_render_ragged_sizes(tiny, R, tiny_oracle, wh):
    cam = _cam(*wh)
    tri = torch.empty(wh[0] * wh[1], dtype=torch.int32, device="cuda")
    rgba = R.render(cam, "fp32", tri=tri).cpu().numpy().reshape(-1, 4)
    ora = oracle.render_camera(tiny_oracle, cam)
    tri = tri.cpu().numpy()
    clear = ~ora["ambiguous"]
    assert np.array_equal(tri[clear], ora["tri"][clear])
    agree = (tri >= 0) == (ora["tri"] >= 0)
    assert np.all(agree | ora["ambiguous"])
    assert np.abs(rgba[agree] - ora["rgba"][agree]).max() <= 1e-5


def test_empty_proxy_renders_zero(tiny):
    import paper_2303_04086_amd as P
    w = synth.workload_tiny()
    R0 = P.Renderer(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), w.res, w.weights,
                    lambda l, lv: np.zeros((len(lv.keys), 2), np.float32), tables=("f32",))
    rgba = R0.render(w.cameras[0], "fp32")
    assert torch.count_nonzero(rgba).item() == 0


def test_empty_batch_and_errors(R):
    z = torch.empty((0, 3), device="cuda")
    assert R.forward(z, z).shape == (0, 4)
    import paper_2303_04086_amd as P
    with pytest.raises(P.InrfError):
        R.render(synth.look_at_camera((0.5, -1.5, 0.5), width=0, height=4))


def test_loud_features_error_reported(tiny):
    """With U(-1, 1) features the colour depends strongly on the encoding; the
    FP32 path still matches FP64 to a bound set by the hit-point rounding."""
    R2 = make_renderer(tiny, tables=("f32",), kind="uniform", sigma=1.0)
    M = oracle.Model.from_workload(tiny, kind="uniform", sigma=1.0)
    o, d = synth.random_rays(2000, 9)
    rgba = R2.forward(_dev(o), _dev(d), "fp32").cpu().numpy()
    ora = oracle.render_rays(M, o.astype(np.float64), d.astype(np.float64))
    agree = compare_hits(R2.trace(_dev(o), _dev(d))[0].cpu().numpy(), ora)
    err = np.abs(rgba[agree] - ora["rgba"][agree]).max()
    print(f"loud features: max abs {err:.3e}")
    assert err <= 1e-4
