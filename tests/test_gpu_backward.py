"""GPU parity of the gradient (inrf_backward) and of the optimiser step
(inrf_adam) against the FP64 oracle, through the C ABI.

The oracle's gradient is itself pinned by FP64 finite differences
(test_oracle_backward.py).  Tolerance: 1e-4 of the largest gradient entry of
each array, for FP32 arithmetic on both the recomputed forward pass and the
adjoint (the gradient sums over up to a few thousand rays).  Rays whose hit
is ambiguous, or whose hidden pre-activations come within 1e-5 of a ReLU
kink (where FP32 may take the other side), get a zero upstream gradient on
both sides."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import compare_hits, make_renderer
from paper_2303_04086_amd.model import table_index

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KIND, SIGMA = "uniform", 0.5  # features large enough to move the network


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def R(tiny):
    return make_renderer(tiny, tables=("f32", "f16"), kind=KIND, sigma=SIGMA)


@pytest.fixture(scope="module")
def omodel(tiny):
    return oracle.Model.from_workload(tiny, kind=KIND, sigma=SIGMA)


@pytest.fixture(scope="module")
def opsh(tiny, tiny_keys):
    return [oracle.build_psh_level(k, N, seed=tiny.psh_seed) for N, k in zip(tiny.res, tiny_keys)]


def _kink_margin(model, o, d, hit):
    """Smallest |pre-activation| of either hidden layer per ray (inf for misses)."""
    out = np.full(len(o), np.inf)
    idx = np.nonzero(hit.hit)[0]
    if len(idx) == 0:
        return out
    x = np.clip(o[idx] + hit.t[idx, None] * d[idx], 0.0, 1.0)
    inp = np.concatenate([oracle.encode_points(model, x), oracle.sh_real(d[idx], model.sh_degree)], axis=1)
    W = [np.asarray(w, np.float64) for w in model.weights]
    z1 = inp @ W[0].T
    z2 = np.maximum(z1, 0.0) @ W[1].T
    out[idx] = np.minimum(np.abs(z1).min(axis=1), np.abs(z2).min(axis=1))
    return out


def _case(R, model, n, seed, table="f32"):
    o, d = synth.random_rays(n, seed, spread=0.3)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    g = np.random.default_rng(seed + 100).normal(size=(n, 4)).astype(np.float32)
    hit = oracle.closest_hit(o64, d64, model.verts, model.tris)
    gtri = R.trace(_dev(o), _dev(d))[0].cpu().numpy()
    agree = compare_hits(gtri, {"tri": hit.tri, "ambiguous": hit.ambiguous})
    keep = agree & ~hit.ambiguous & (_kink_margin(model, o64, d64, hit) > 1e-5)
    g[~keep] = 0.0
    dt = torch.zeros_like(R.tables["f32"])
    dw = torch.zeros_like(R.weights)
    rgba = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    R.backward(_dev(o), _dev(d), _dev(g), table=table, d_table=dt, d_weights=dw, rgba=rgba)
    torch.cuda.synchronize()
    ref = oracle.backward_rays(model, o64, d64, g.astype(np.float64))
    return o, d, g, keep, dt.cpu().numpy(), dw.cpu().numpy(), rgba.cpu().numpy(), ref


def _check_weights(R, dw, ref, what):
    sizes = [w.size for w in ref["weights"]]
    parts = np.split(dw, np.cumsum(sizes)[:-1])
    for i, (gw, rw) in enumerate(zip(parts, ref["weights"])):
        scale = np.abs(rw).max()
        err = np.abs(gw.reshape(rw.shape) - rw).max()
        print(f"{what} dW{i + 1}: max |grad| {scale:.3e}, max abs err {err:.2e} ({err / scale:.1e} rel)")
        assert scale > 0
        assert err <= 1e-4 * scale


def _check_table(R, dt, ref, opsh, what):
    scale = max(np.abs(np.array(list(f.values()))).max() for f in ref["features"] if f)
    touched = np.zeros(len(dt), bool)
    worst = 0.0
    for l, lv in enumerate(opsh):
        if not ref["features"][l]:
            continue
        verts = np.array(list(ref["features"][l].keys()), np.int64)
        want = np.array(list(ref["features"][l].values()))
        slots = table_index(R, l, oracle.psh_slots(lv, verts).astype(np.int64))
        touched[slots] = True
        worst = max(worst, np.abs(dt[slots] - want).max())
    print(f"{what} dTable: max |grad| {scale:.3e}, max abs err {worst:.2e} ({worst / scale:.1e} rel), "
          f"{touched.sum()} slots")
    assert worst <= 1e-4 * scale
    assert not np.any(dt[~touched])  # no other slot receives anything


def test_backward_matches_oracle(tiny, R, omodel, opsh):
    n = 4099  # several 64-hit wave steps and a ragged tail
    o, d, g, keep, dt, dw, rgba, ref = _case(R, omodel, n, 41)
    assert keep.sum() > 1000
    _check_weights(R, dw, ref, "fp32 table")
    _check_table(R, dt, ref, opsh, "fp32 table")
    # the forward output it reports is the FP32 path's, and the oracle's
    fwd = R.forward(_dev(o), _dev(d), "fp32").cpu().numpy()
    assert np.abs(rgba - fwd).max() <= 1e-6
    assert np.abs(rgba[keep] - ref["rgba"][keep]).max() <= 1e-5


@pytest.mark.parametrize("levels", [6, 10, 16])
def test_backward_more_levels(levels):
    """The gradient kernel's wider instantiations (5-8, 9-12 and 13-16
    levels; sixteen is the training configuration's input width of 48, with
    the whole weight gradient in accumulator registers) against the oracle:
    levels geometric from 8 to 96 on the tiny proxy, 2,400 rays."""
    w = synth.workload_tiny()
    w.res = [int(round(8 * 12.0 ** (l / (levels - 1)))) for l in range(levels)]
    w.weights = synth.xavier_mlp(3 + levels, w.d_in)
    Rl = make_renderer(w, tables=("f32",), kind=KIND, sigma=SIGMA)
    model = oracle.Model.from_workload(w, kind=KIND, sigma=SIGMA)
    opsh = [oracle.PSHLevel(lv.res, lv.mbar, lv.rbar, lv.phi, None) for lv in Rl.levels]
    _, _, _, keep, dt, dw, rgba, ref = _case(Rl, model, 2400, 50 + levels)
    assert keep.sum() > 1000
    _check_weights(Rl, dw, ref, f"{levels} levels")
    _check_table(Rl, dt, ref, opsh, f"{levels} levels")
    assert np.abs(rgba[keep] - ref["rgba"][keep]).max() <= 1e-5


def test_backward_half_table(tiny, R, opsh):
    """FP16 table: the oracle reads the same features rounded to FP16."""
    grids = []
    for l, N in enumerate(tiny.res):
        keys = oracle.shell_keys(tiny.verts, tiny.tris, N, tiny.dilate)
        f = synth.table_features(tiny.feature_seed, l, keys, N, F=tiny.F, kind=KIND, sigma=SIGMA)
        grids.append(oracle.FeatureGrid(N, keys, np.asarray(f, np.float32).astype(np.float16).astype(np.float64)))
    m16 = oracle.Model(np.asarray(tiny.verts), np.asarray(tiny.tris), grids, [np.asarray(w) for w in tiny.weights])
    _, _, _, keep, dt, dw, _, ref = _case(R, m16, 2000, 43, table="f16")
    assert keep.sum() > 500
    _check_weights(R, dw, ref, "fp16 table")
    _check_table(R, dt, ref, opsh, "fp16 table")


def test_backward_accumulates_and_weights_are_deterministic(tiny, R):
    o, d = synth.random_rays(3000, 45)
    g = _dev(np.random.default_rng(1).normal(size=(3000, 4)).astype(np.float32))
    o, d = _dev(o), _dev(d)
    dw1 = torch.zeros_like(R.weights)
    dw2 = torch.zeros_like(R.weights)
    dt = torch.zeros_like(R.tables["f32"])
    R.backward(o, d, g, d_weights=dw1, d_table=dt)
    R.backward(o, d, g, d_weights=dw2)
    torch.cuda.synchronize()
    assert torch.equal(dw1, dw2)
    R.backward(o, d, g, d_weights=dw2)  # adds
    torch.cuda.synchronize()
    assert torch.allclose(dw2, 2 * dw1, rtol=1e-6, atol=0)
    dt2 = torch.zeros_like(dt)
    R.backward(o, d, g, d_table=dt2)
    torch.cuda.synchronize()
    # table gradients are FP32 atomic sums: equal up to the order of addition
    scale = dt.abs().max().item()
    assert scale > 0
    assert torch.allclose(dt, dt2, rtol=1e-4, atol=1e-6 * scale)


def test_backward_edge_cases(tiny, R):
    import paper_2303_04086_amd as P
    z = torch.empty((0, 3), device="cuda")
    dw = torch.zeros_like(R.weights)
    R.backward(z, z, torch.empty((0, 4), device="cuda"), d_weights=dw)  # empty batch: nothing
    # rays that all miss contribute nothing
    o = _dev(np.tile(np.array([[0.5, 0.5, 3.0]], np.float32), (100, 1)))
    d = _dev(np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (100, 1)))
    dt = torch.zeros_like(R.tables["f32"])
    rgba = torch.full((100, 4), 7.0, device="cuda")
    R.backward(o, d, torch.ones((100, 4), device="cuda"), d_table=dt, d_weights=dw, rgba=rgba)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dw).item() == 0 and torch.count_nonzero(dt).item() == 0
    assert torch.count_nonzero(rgba).item() == 0
    # workspace too small is an error, nothing enqueued
    import ctypes
    from paper_2303_04086_amd import _lib as L
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    st = L.lib().inrf_backward(ctypes.byref(R.desc("f32")), L.ptr(o), L.ptr(d), 100,
                               L.ptr(torch.ones((100, 4), device="cuda")), L.ptr(dt), L.ptr(dw), 0,
                               L.ptr(ws), ws.numel(), None)
    assert st == -2
    # misaligned upstream gradient: invalid argument, nothing enqueued
    big = R.backward_workspace(100)
    g4 = torch.ones(401, device="cuda")
    st = L.lib().inrf_backward(ctypes.byref(R.desc("f32")), L.ptr(o), L.ptr(d), 100, L.ptr(g4) + 4, L.ptr(dt),
                               L.ptr(dw), 0, L.ptr(big), big.numel(), None)
    assert st == -1
    with pytest.raises(ValueError):
        R.backward(o, d, torch.ones((100, 4), device="cuda"), d_weights=dw, d_table=dt[:-1])
    assert P.lib().inrf_backward_workspace_size(ctypes.byref(R.desc("f32")), -1) == -1


@pytest.mark.parametrize("n", [1, 7, 4096, 100003])
def test_adam_matches_oracle(n):
    import paper_2303_04086_amd as P
    from paper_2303_04086_amd.model import adam_step
    rng = np.random.default_rng(n)
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    tp, tm, tv = _dev(p), _dev(m), _dev(v)
    half = torch.empty(n, dtype=torch.float16, device="cuda")
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        g[::5] = 0.0
        tg = _dev(g)
        adam_step(tp, tg, tm, tv, t, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, param_f16=half)
        rp, rm, rv = oracle.adam_step(rp, g, rm, rv, t, 1e-2, 0.9, 0.99, 1e-15)
        torch.cuda.synchronize()
        assert torch.count_nonzero(tg).item() == 0  # cleared
        assert np.abs(tp.cpu().numpy() - rp).max() <= 1e-6
        assert np.abs(tm.cpu().numpy() - rm).max() <= 1e-6 and np.abs(tv.cpu().numpy() - rv).max() <= 1e-6
        assert torch.equal(half, tp.to(torch.float16))
    with pytest.raises(P.InrfError):
        adam_step(tp, tg, tm, tv, 0)


@pytest.mark.parametrize("n", [4099, 1 << 16])
def test_adam_lazy_matches_oracle(n):
    """Lazy Adam: entries with a zero gradient keep value, moments and FP16
    copy; the others match the FP64 lazy step."""
    from paper_2303_04086_amd.model import adam_step
    rng = np.random.default_rng(n + 1)
    p = rng.normal(size=n).astype(np.float32)
    m = (0.1 * rng.normal(size=n)).astype(np.float32)
    v = np.abs(0.1 * rng.normal(size=n)).astype(np.float32)
    tp, tm, tv = _dev(p), _dev(m), _dev(v)
    half = tp.to(torch.float16)
    rp, rm, rv = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        g[rng.random(n) < 0.6] = 0.0
        g[:8] = 0.0  # a whole 4-group of zeros (skipped), and a ragged tail below
        g[-3:] = [0.0, 1.5, 0.0]
        tg = _dev(g)
        adam_step(tp, tg, tm, tv, t, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, param_f16=half, lazy=True)
        rp, rm, rv = oracle.adam_step(rp, g, rm, rv, t, 1e-2, 0.9, 0.99, 1e-15, lazy=True)
        torch.cuda.synchronize()
        assert torch.count_nonzero(tg).item() == 0
        assert np.abs(tp.cpu().numpy() - rp).max() <= 1e-6
        assert np.abs(tm.cpu().numpy() - rm).max() <= 1e-6 and np.abs(tv.cpu().numpy() - rv).max() <= 1e-6
        assert torch.equal(half, tp.to(torch.float16))
    assert np.array_equal(tp.cpu().numpy()[:8], p[:8]) and np.array_equal(tm.cpu().numpy()[:8], m[:8])


def test_backward_rejects_more_than_16_levels():
    import paper_2303_04086_amd as P
    w = synth.workload_tiny()
    w.res = list(range(4, 21))                 # 17 levels
    w.weights = synth.xavier_mlp(3, w.d_in)
    R17 = make_renderer(w, tables=("f32",))
    o, d = synth.random_rays(64, 2)
    with pytest.raises(P.InrfError):
        R17.backward(_dev(o), _dev(d), torch.ones((64, 4), device="cuda"), d_weights=torch.zeros_like(R17.weights))
