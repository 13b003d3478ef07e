"""Training on the GPU (Sec. 4.2, loss of Eq. 8, Adam): the autograd binding
agrees with the library's gradient, and fitting a second seeded i-NOLF of
the same proxy (targets rendered by the FP64 oracle) lowers the loss."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import make_renderer

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _target_model(tiny):
    grids = []
    for l, N in enumerate(tiny.res):
        keys = oracle.shell_keys(tiny.verts, tiny.tris, N, tiny.dilate)
        f = synth.table_features(tiny.feature_seed + 1000, l, keys, N, F=tiny.F, kind="uniform", sigma=0.5)
        grids.append(oracle.FeatureGrid(N, keys, f))
    w = synth.xavier_mlp(99, 2 * len(tiny.res) + 16)
    return oracle.Model(np.asarray(tiny.verts), np.asarray(tiny.tris), grids, [np.asarray(x) for x in w])


def test_autograd_matches_backward(tiny):
    from paper_2303_04086_amd.train import render_rays
    R = make_renderer(tiny, tables=("f32",), kind="uniform", sigma=0.5)
    o, d = synth.random_rays(2048, 61)
    o, d = _dev(o), _dev(d)
    table = R.tables["f32"].detach().requires_grad_(True)
    weights = R.weights.detach().requires_grad_(True)
    target = torch.rand((2048, 4), device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    rgba = render_rays(R, o, d, table, weights)
    loss = ((rgba - target) ** 2).sum() / 2048
    loss.backward()
    dt = torch.zeros_like(R.tables["f32"])
    dw = torch.zeros_like(R.weights)
    R.backward(o, d, (2.0 / 2048) * (rgba.detach() - target), d_table=dt, d_weights=dw)
    torch.cuda.synchronize()
    assert torch.equal(weights.grad, dw)
    assert torch.allclose(table.grad, dt, rtol=1e-5, atol=1e-10)
    assert torch.count_nonzero(dw).item() > 0


def test_training_lowers_the_loss(tiny):
    from paper_2303_04086_amd.train import Trainer
    target_model = _target_model(tiny)
    cams = synth.fibonacci_cameras(4, 2.0, 48, 48)
    rays, targets = [], []
    for cam in cams:
        o, d = oracle.camera_rays(cam)
        ref = oracle.render_rays(target_model, o, d)
        rays.append((o.astype(np.float32), d.astype(np.float32)))
        targets.append(ref["rgba"].astype(np.float32))
    o_all = np.concatenate([r[0] for r in rays])
    d_all = np.concatenate([r[1] for r in rays])
    t_all = np.concatenate(targets)
    R = make_renderer(tiny, tables=("f32", "f16"), kind="normal", sigma=1e-2)
    tr = Trainer(R, lr=1e-2)
    O, D, T = _dev(o_all), _dev(d_all), _dev(t_all)
    gen = torch.Generator("cuda").manual_seed(1)
    n = len(o_all)

    def full_loss():
        rgba = R.forward(O, D, "fp32", "f32")
        return float(((rgba - T) ** 2).sum() / n)

    l0 = full_loss()
    for _ in range(150):
        idx = torch.randint(0, n, (2048,), device="cuda", generator=gen)
        tr.step(O[idx], D[idx], T[idx])
    torch.cuda.synchronize()
    l1 = full_loss()
    print(f"training: loss {l0:.4e} -> {l1:.4e}")
    assert l1 < 0.3 * l0
    # the FP16 table follows the master table
    assert torch.equal(R.tables["f16"], R.tables["f32"].to(torch.float16))
