"""Python binding of libinrf: host builders, a device-resident model, and the
render / forward / trace / encode / mlp calls.

PyTorch provides device memory and the stream; every step of the path runs in
the library's kernels.  There is no fallback: a missing library or a missing
GPU raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Callable, Optional, Sequence

import numpy as np

from . import _lib as L


@dataclass
class PshLevel:
    res: int
    mbar: int
    rbar: int
    restarts: int
    keys: np.ndarray   # int64 [n] linear keys (z*(N+1)+y)*(N+1)+x, ascending
    phi: np.ndarray    # uint32 [rbar^3] packed offsets
    slots: np.ndarray  # int32 [n] slot of each key

    def vertices(self) -> np.ndarray:
        M = self.res + 1
        k = self.keys
        return np.stack([k % M, (k // M) % M, k // (M * M)], axis=1)


def brick_entries(side: int) -> int:
    """Entries one level's cube of the given side occupies on the device."""
    n = int(L.lib().inrf_brick_entries(int(side)))
    if n < 0:
        raise ValueError(f"side {side} not in [1, 1024]")
    return n


def brick_index(side: int, linear) -> np.ndarray:
    """Device storage index of linear cell indices (z*side + y)*side + x."""
    lin = np.ascontiguousarray(linear, np.int64)
    out = np.empty_like(lin)
    L.check(L.lib().inrf_brick_index(int(side), L.ptr(lin), lin.size, L.ptr(out)))
    return out


def table_index(R, level: int, slots) -> np.ndarray:
    """Row of the device table holding linear slot(s) `slots` of `level`."""
    _, mbar, _, _, so = R.level_desc[level]
    return so + brick_index(mbar, slots)


def psh_params(**kw) -> L.PshParams:
    p = L.PshParams()
    L.lib().inrf_psh_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _levels_out(h) -> list:
    lib = L.lib()
    out = []
    try:
        for l in range(lib.inrf_psh_levels(h)):
            info = L.PshLevelInfo()
            L.check(lib.inrf_psh_level(h, l, ctypes.byref(info), None, None, None))
            keys = np.empty(info.n_keys, np.int64)
            phi = np.empty(info.n_phi, np.uint32)
            slots = np.empty(info.n_keys, np.int32)
            L.check(lib.inrf_psh_level(h, l, ctypes.byref(info), L.ptr(keys), L.ptr(phi), L.ptr(slots)))
            out.append(PshLevel(info.res, info.mbar, info.rbar, info.restarts, keys, phi, slots))
    finally:
        lib.inrf_psh_free(h)
    return out


def _mesh_args(verts, tris):
    v = np.ascontiguousarray(verts, np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(tris, np.int32).reshape(-1, 3)
    return v, t


def build_psh(verts, tris, res: Sequence[int], **params) -> list:
    """Voxelise the proxy at each resolution and build each level's PSH."""
    v, t = _mesh_args(verts, tris)
    r = np.ascontiguousarray(res, np.int32)
    p = psh_params(**params)
    h = ctypes.c_void_p()
    L.check(L.lib().inrf_build_psh(L.ptr(v), len(v), L.ptr(t), len(t), len(r), L.ptr(r), ctypes.byref(p),
                                   ctypes.byref(h)))
    return _levels_out(h)


def build_psh_keys(res: int, keys, **params) -> PshLevel:
    """Build one level's PSH from a caller-supplied ascending key list."""
    k = np.ascontiguousarray(keys, np.int64)
    p = psh_params(**params)
    h = ctypes.c_void_p()
    L.check(L.lib().inrf_build_psh_keys(int(res), L.ptr(k), len(k), ctypes.byref(p), ctypes.byref(h)))
    return _levels_out(h)[0]


@dataclass
class BvhImage:
    nodes: np.ndarray  # uint8
    tris: np.ndarray   # uint8
    n_nodes: int
    depth: int
    stack: int


def build_bvh(verts, tris) -> BvhImage:
    v, t = _mesh_args(verts, tris)
    lib = L.lib()
    h = ctypes.c_void_p()
    L.check(lib.inrf_build_bvh(L.ptr(v), len(v), L.ptr(t), len(t), ctypes.byref(h)))
    try:
        info = L.BvhInfo()
        L.check(lib.inrf_bvh_get_info(h, ctypes.byref(info)))
        nodes = np.zeros(max(info.node_bytes, 128), np.uint8)
        tri = np.zeros(max(info.tri_bytes, 48), np.uint8)
        L.check(lib.inrf_bvh_copy(h, L.ptr(nodes), L.ptr(tri)))
        return BvhImage(nodes, tri, info.n_nodes, info.depth, info.stack)
    finally:
        lib.inrf_bvh_free(h)


PRECISIONS = {"fp32": L.PREC_FP32, "fp16": L.PREC_FP16, "bf16": L.PREC_BF16}
TABLES = {"f32": L.INRF_F32, "f16": L.INRF_F16}


def _camera_desc(cam) -> L.CameraDesc:
    c = L.CameraDesc()
    for name in ("origin", "right", "up", "forward"):
        getattr(c, name)[:] = [float(x) for x in np.asarray(getattr(cam, name), np.float32)]
    c.tan_half_fov_y = float(np.float32(cam.tan_half_fov_y))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def camera_rays(cam, device="cuda", stream=None):
    """The camera's primary rays as the render kernels generate them
    (inrf_camera_rays): origins and unit directions, float32 [H*W, 3] each."""
    import torch
    n = int(cam.width) * int(cam.height)
    o = torch.empty((n, 3), dtype=torch.float32, device=device)
    d = torch.empty((n, 3), dtype=torch.float32, device=device)
    s = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
    L.check(L.lib().inrf_camera_rays(ctypes.byref(_camera_desc(cam)), L.ptr(o), L.ptr(d), ctypes.c_void_p(s.cuda_stream)))
    return o, d


class Renderer:
    """A device-resident i-NOLF object: PSH offset tables and feature tables
    (FP32 and/or FP16), FP32 network weights, and the proxy BVH."""

    def __init__(self, verts, tris, res: Sequence[int], weights: Sequence[np.ndarray],
                 features: Callable[[int, PshLevel], np.ndarray], tables=("f32",), device="cuda",
                 psh_levels: Optional[list] = None, **psh_kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the render path runs only on the device")
        self.torch = torch
        self.device = torch.device(device)
        self.res = [int(r) for r in res]
        self.n_levels = len(self.res)
        self.levels = psh_levels if psh_levels is not None else build_psh(verts, tris, self.res, **psh_kw)
        d_in = 2 * self.n_levels + L.SH_DIM
        w = [np.asarray(x, np.float32) for x in weights]
        if [x.shape for x in w] != [(L.HIDDEN, d_in), (L.HIDDEN, L.HIDDEN), (L.OUT, L.HIDDEN)]:
            raise ValueError(f"weights must be shaped [64,{d_in}], [64,64], [4,64]")
        self.weights = torch.from_numpy(np.concatenate([x.reshape(-1) for x in w])).to(self.device)
        phi_off, slot_off = 0, 0
        self.level_desc = []
        for lv in self.levels:
            self.level_desc.append((lv.res, lv.mbar, lv.rbar, phi_off, slot_off))
            phi_off += brick_entries(lv.rbar)
            slot_off += brick_entries(lv.mbar)
        self.n_slots = slot_off
        phi = np.zeros(phi_off, np.uint32)
        host = np.zeros((slot_off, L.FEATURES), np.float32)
        for l, lv in enumerate(self.levels):
            po, so = self.level_desc[l][3], self.level_desc[l][4]
            phi[po + brick_index(lv.rbar, np.arange(len(lv.phi), dtype=np.int64))] = lv.phi
            f = np.asarray(features(l, lv), np.float32)
            host[so + brick_index(lv.mbar, lv.slots.astype(np.int64))] = f
        self.phi = torch.from_numpy(phi.view(np.int32)).to(self.device)
        del phi
        self.tables = {}
        t32 = torch.from_numpy(host)
        for name in tables:
            if name == "f32":
                self.tables[name] = t32.to(self.device)
            elif name == "f16":
                self.tables[name] = t32.to(torch.float16).to(self.device)
            else:
                raise ValueError(name)
        del host, t32
        self.bvh = build_bvh(verts, tris)
        self.n_tris = int(np.asarray(tris).reshape(-1, 3).shape[0])
        self.bvh_nodes = torch.from_numpy(self.bvh.nodes).to(self.device)
        self.bvh_tris = torch.from_numpy(self.bvh.tris).to(self.device)
        self._ws = None
        self._descs = {}

    # -- descriptors -------------------------------------------------------
    def desc(self, table: str = "f32") -> L.ModelDesc:
        if table not in self._descs:
            if table not in self.tables:
                raise KeyError(f"table {table!r} not resident (have {list(self.tables)})")
            m = L.ModelDesc()
            m.n_levels = self.n_levels
            m.table_dtype = TABLES[table]
            for l, (res, mbar, rbar, po, so) in enumerate(self.level_desc):
                m.levels[l].res, m.levels[l].mbar, m.levels[l].rbar = res, mbar, rbar
                m.levels[l].phi_offset, m.levels[l].slot_offset = po, so
            m.phi = self.phi.data_ptr()
            m.table = self.tables[table].data_ptr()
            m.weights = self.weights.data_ptr()
            m.bvh_nodes = self.bvh_nodes.data_ptr()
            m.bvh_tris = self.bvh_tris.data_ptr()
            m.n_tris = self.n_tris
            m.bvh_stack = self.bvh.stack
            m.bvh_n_nodes = self.bvh.n_nodes
            self._descs[table] = m
        return self._descs[table]

    def workspace(self, n_rays: int):
        need = int(L.lib().inrf_workspace_size(n_rays))
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self._ws

    def _stream(self, stream):
        s = stream if stream is not None else self.torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    # -- calls -------------------------------------------------------------
    def render(self, cam, precision="fp32", table="f32", rgba=None, depth=None, tri=None, stream=None,
               events=None, ws=None):
        """Render one camera.  `events`: optional three recorded
        torch.cuda.Event objects marking trace start, shading start and end
        (inrf_render_profiled).  `ws`: optional uint8 workspace of the
        caller (frames in flight on different streams need one each); else
        the renderer's own."""
        torch = self.torch
        n = int(cam.width) * int(cam.height)
        if rgba is None:
            rgba = torch.empty((int(cam.height), int(cam.width), 4), dtype=torch.float32, device=self.device)
        ws = self.workspace(n) if ws is None else ws
        c = _camera_desc(cam)
        args = (ctypes.byref(self.desc(table)), PRECISIONS[precision], ctypes.byref(c), L.ptr(rgba), L.ptr(depth),
                L.ptr(tri), L.ptr(ws), ws.numel(), self._stream(stream))
        if events is None:
            L.check(L.lib().inrf_render(*args))
        else:
            arr = (ctypes.c_void_p * 3)(*[e.cuda_event if e is not None else 0 for e in events])
            L.check(L.lib().inrf_render_profiled(*args, arr))
        return rgba

    def batch_workspace_bytes(self, n_cameras: int, n_pixels: int) -> int:
        """Workspace bytes of a batch of n_cameras cameras with n_pixels in all."""
        need = int(L.lib().inrf_batch_workspace_size(int(n_cameras), int(n_pixels)))
        if need < 0:
            raise ValueError("invalid batch")
        return need

    def render_batch(self, cams, precision="fp32", table="f32", rgba=None, depth=None, tri=None, stream=None,
                     ws=None):
        """Render several cameras in one pass (inrf_render_batch).  Returns
        the flat [sum(W*H), 4] RGBA buffer and the list of per-camera
        [H, W, 4] views into it.  `ws` as for render()."""
        torch = self.torch
        cams = list(cams)
        if not 1 <= len(cams) <= L.MAX_CAMERAS:
            raise ValueError(f"1..{L.MAX_CAMERAS} cameras per batch")
        sizes = [int(c.width) * int(c.height) for c in cams]
        n = sum(sizes)
        if rgba is None:
            rgba = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        need = int(L.lib().inrf_batch_workspace_size(len(cams), n))
        if need < 0:
            raise ValueError("invalid batch")
        if ws is None:
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            ws = self._ws
        arr = (L.CameraDesc * len(cams))(*[_camera_desc(c) for c in cams])
        L.check(L.lib().inrf_render_batch(ctypes.byref(self.desc(table)), PRECISIONS[precision], arr, len(cams),
                                          L.ptr(rgba), L.ptr(depth), L.ptr(tri), L.ptr(ws), ws.numel(),
                                          self._stream(stream)))
        views, off = [], 0
        for c, k in zip(cams, sizes):
            views.append(rgba[off:off + k].view(int(c.height), int(c.width), 4))
            off += k
        return rgba, views

    def hit_count(self) -> int:
        """Hit rays of the last render/forward (reads the workspace header:
        the frame's hit count, then a counter kept at zero)."""
        return int(self._ws[:8].view(self.torch.int32).sum().item())

    def forward(self, o, d, precision="fp32", table="f32", depth=None, tri=None, rgba=None, stream=None):
        torch = self.torch
        o = o.contiguous()
        d = d.contiguous()
        n = o.shape[0]
        if rgba is None:
            rgba = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        ws = self.workspace(n)
        L.check(L.lib().inrf_forward(ctypes.byref(self.desc(table)), PRECISIONS[precision], L.ptr(o), L.ptr(d), n,
                                     L.ptr(rgba), L.ptr(depth), L.ptr(tri), L.ptr(ws), ws.numel(),
                                     self._stream(stream)))
        return rgba

    def trace(self, o, d, stream=None):
        torch = self.torch
        o = o.contiguous()
        d = d.contiguous()
        n = o.shape[0]
        tri = torch.empty(n, dtype=torch.int32, device=self.device)
        t = torch.empty(n, dtype=torch.float32, device=self.device)
        L.check(L.lib().inrf_trace(ctypes.byref(self.desc(next(iter(self.tables)))), L.ptr(o), L.ptr(d), n,
                                   L.ptr(tri), L.ptr(t), self._stream(stream)))
        return tri, t

    def encode(self, x, table="f32", slots=False, stream=None):
        torch = self.torch
        x = x.contiguous()
        n = x.shape[0]
        enc = torch.empty((n, 2 * self.n_levels), dtype=torch.float32, device=self.device)
        sl = torch.empty((n, self.n_levels, 8), dtype=torch.int32, device=self.device) if slots else None
        L.check(L.lib().inrf_encode(ctypes.byref(self.desc(table)), L.ptr(x), n, L.ptr(enc), L.ptr(sl),
                                    self._stream(stream)))
        return (enc, sl) if slots else enc

    def mlp(self, inputs, precision="fp32", out=None, stream=None):
        torch = self.torch
        inputs = inputs.contiguous()
        n = inputs.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        L.check(L.lib().inrf_mlp(ctypes.byref(self.desc(next(iter(self.tables)))), PRECISIONS[precision],
                                 L.ptr(inputs), n, L.ptr(out), self._stream(stream)))
        return out

    def mlp_encoded(self, enc, dirs, precision="fp16", out=None, stream=None):
        """The network on 16-bit encodings enc [n, 2L] (float16 for "fp16",
        bfloat16 for "bf16") and view directions dirs [n, 3] (inrf_mlp_encoded)."""
        torch = self.torch
        enc, dirs = enc.contiguous(), dirs.contiguous()
        n = enc.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        L.check(L.lib().inrf_mlp_encoded(ctypes.byref(self.desc(next(iter(self.tables)))), PRECISIONS[precision],
                                         L.ptr(enc), L.ptr(dirs), n, L.ptr(out), self._stream(stream)))
        return out

    # -- gradient ------------------------------------------------------------
    def backward_workspace(self, n_rays: int, table: str = "f32"):
        need = int(L.lib().inrf_backward_workspace_size(ctypes.byref(self.desc(table)), n_rays))
        if need < 0:
            L.check(-1)
        if getattr(self, "_bws", None) is None or self._bws.numel() < need:
            self._bws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self._bws

    def backward(self, o, d, d_rgba, table="f32", d_table=None, d_weights=None, rgba=None, stream=None):
        """Adds dL/d(table) to d_table (float32, shaped like the table) and
        dL/d(weights) to d_weights (float32, shaped like the flat weights),
        given d_rgba = dL/d(rgba) for the rays o, d; either may be None.
        `rgba`, if given, receives the forward output (FP32 network)."""
        o = o.contiguous()
        d = d.contiguous()
        d_rgba = d_rgba.contiguous()
        n = o.shape[0]
        for name, t, shape in (("d_table", d_table, (self.n_slots, L.FEATURES)),
                               ("d_weights", d_weights, tuple(self.weights.shape)),
                               ("rgba", rgba, (n, 4)), ("d_rgba", d_rgba, (n, 4))):
            if t is not None and (tuple(t.shape) != shape or t.dtype != self.torch.float32 or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float32 tensor of shape {shape}")
        ws = self.backward_workspace(n, table)
        L.check(L.lib().inrf_backward(ctypes.byref(self.desc(table)), L.ptr(o), L.ptr(d), n, L.ptr(d_rgba),
                                      L.ptr(d_table), L.ptr(d_weights), L.ptr(rgba), L.ptr(ws), ws.numel(),
                                      self._stream(stream)))


class NolfRenderer:
    """A device-resident object in the paper's own i-NOLF form (Sec. 4.2):
    density and diffuse texture cubes (FP16) over one base-cell index, PSH
    level tables built from the given key sets, and FP32 network weights
    whose first layer also takes the coarse opacity (d_in = 2L + 17)."""

    def __init__(self, base_res: int, cube_res: int, index, density, diffuse, res: Sequence[int], level_keys,
                 weights: Sequence[np.ndarray], features: Callable[[int, PshLevel], np.ndarray], step: float,
                 t_stop: float = 1e-4, w_min: float = 1e-4, tables=("f32",), device="cuda", psh_seed: int = 1):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the render path runs only on the device")
        self.torch = torch
        self.device = torch.device(device)
        self.res = [int(r) for r in res]
        self.n_levels = len(self.res)
        levels = [build_psh_keys(N, level_keys(l), seed=psh_seed) for l, N in enumerate(self.res)]
        d_in = 2 * self.n_levels + L.SH_DIM + 1
        w = [np.asarray(x, np.float32) for x in weights]
        if [x.shape for x in w] != [(L.HIDDEN, d_in), (L.HIDDEN, L.HIDDEN), (L.OUT, L.HIDDEN)]:
            raise ValueError(f"weights must be shaped [64,{d_in}], [64,64], [4,64]")
        self.weights = torch.from_numpy(np.concatenate([x.reshape(-1) for x in w])).to(self.device)
        phi_off, slot_off = 0, 0
        self.level_desc = []
        for lv in levels:
            self.level_desc.append((lv.res, lv.mbar, lv.rbar, phi_off, slot_off))
            phi_off += brick_entries(lv.rbar)
            slot_off += brick_entries(lv.mbar)
        phi = np.zeros(phi_off, np.uint32)
        host = np.zeros((slot_off, L.FEATURES), np.float32)
        for l, lv in enumerate(levels):
            po, so = self.level_desc[l][3], self.level_desc[l][4]
            phi[po + brick_index(lv.rbar, np.arange(len(lv.phi), dtype=np.int64))] = lv.phi
            host[so + brick_index(lv.mbar, lv.slots.astype(np.int64))] = np.asarray(features(l, lv), np.float32)
        self.n_keys = sum(len(lv.keys) for lv in levels)
        del levels
        self.phi = torch.from_numpy(phi.view(np.int32)).to(self.device)
        t32 = torch.from_numpy(host)
        self.tables = {}
        for name in tables:
            self.tables[name] = t32.to(self.device) if name == "f32" else t32.to(torch.float16).to(self.device)
        del host, t32
        r1 = int(cube_res) + 1
        dens = np.asarray(density, np.float32).reshape(-1, r1 ** 3)
        diff = np.asarray(diffuse, np.float32).reshape(-1, r1 ** 3, 4)
        if len(dens) != len(diff) or len(dens) < 1:
            raise ValueError("density and diffuse cubes must have the same, non-zero count")
        self.index = torch.from_numpy(np.ascontiguousarray(np.asarray(index, np.int32))).to(self.device)
        self.density = torch.from_numpy(dens).to(torch.float16).to(self.device)
        self.diffuse = torch.from_numpy(diff).to(torch.float16).to(self.device)
        self.cubes = L.CubesDesc(int(base_res), int(cube_res), self.index.data_ptr(), self.density.data_ptr(),
                                 self.diffuse.data_ptr(), len(dens), float(step), float(t_stop), float(w_min), 0)
        self._ws = None
        self._descs = {}

    @classmethod
    def from_workload(cls, w, tables=("f32", "f16"), kind: str = "normal", sigma: float = 1e-2):
        import synth
        feats = lambda l, lv: synth.feature_values(w.feature_seed, l, lv.keys, F=w.F, kind=kind, sigma=sigma)
        return cls(w.b, w.r, w.index, w.density, w.diffuse, w.res, w.level_keys, w.weights, feats, w.step,
                   tables=tables, psh_seed=w.psh_seed)

    def desc(self, table: str = "f32") -> L.ModelDesc:
        if table not in self._descs:
            m = L.ModelDesc()
            m.n_levels = self.n_levels
            m.table_dtype = TABLES[table]
            for l, (res, mbar, rbar, po, so) in enumerate(self.level_desc):
                m.levels[l].res, m.levels[l].mbar, m.levels[l].rbar = res, mbar, rbar
                m.levels[l].phi_offset, m.levels[l].slot_offset = po, so
            m.phi = self.phi.data_ptr()
            m.table = self.tables[table].data_ptr()
            m.weights = self.weights.data_ptr()
            self._descs[table] = m
        return self._descs[table]

    def workspace(self, n_rays: int):
        need = int(L.lib().inrf_workspace_size(n_rays))
        if self._ws is None or self._ws.numel() < need:
            self._ws = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        return self._ws

    def hit_count(self) -> int:
        return int(self._ws[:8].view(self.torch.int32).sum().item())

    def render(self, cam, precision="fp32", table="f32", rgba=None, depth=None, alpha_c=None, stream=None):
        torch = self.torch
        n = int(cam.width) * int(cam.height)
        if rgba is None:
            rgba = torch.empty((int(cam.height), int(cam.width), 4), dtype=torch.float32, device=self.device)
        ws = self.workspace(n)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        c = _camera_desc(cam)
        L.check(L.lib().inrf_render_nolf(ctypes.byref(self.desc(table)), ctypes.byref(self.cubes), PRECISIONS[precision],
                                         ctypes.byref(c), L.ptr(rgba), L.ptr(depth), L.ptr(alpha_c), L.ptr(ws),
                                         ws.numel(), ctypes.c_void_p(s.cuda_stream)))
        return rgba


    def shade(self, x, d, alpha_c, precision="fp32", table="f32", rgba=None, stream=None):
        """The shading stage alone (inrf_shade_nolf) on hit points x [n, 3],
        directions d [n, 3] and coarse opacities alpha_c [n]."""
        torch = self.torch
        x, d, alpha_c = x.contiguous(), d.contiguous(), alpha_c.contiguous()
        n = x.shape[0]
        if rgba is None:
            rgba = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        ws = self.workspace(n)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        L.check(L.lib().inrf_shade_nolf(ctypes.byref(self.desc(table)), ctypes.byref(self.cubes), PRECISIONS[precision],
                                        L.ptr(x), L.ptr(d), L.ptr(alpha_c), n, L.ptr(rgba), L.ptr(ws), ws.numel(),
                                        ctypes.c_void_p(s.cuda_stream)))
        return rgba


class CapturedFrame:
    """One camera frame captured as a HIP graph (torch.cuda.CUDAGraph) and
    replayed: the launches of a render of a fixed camera into
    fixed buffers with a workspace of its own, enqueued with one call.  The
    path records no memset (counters are written by kernels), so a replay
    recomputes the frame exactly as the eager render does."""

    def __init__(self, renderer, cam, precision="fp16", table="f16", depth: bool = False, tri: bool = False):
        torch = renderer.torch
        self.R, self.torch = renderer, torch
        n = int(cam.width) * int(cam.height)
        dev = renderer.device
        self.rgba = torch.empty((int(cam.height), int(cam.width), 4), dtype=torch.float32, device=dev)
        self.depth = torch.empty(n, dtype=torch.float32, device=dev) if depth else None
        self.tri = torch.empty(n, dtype=torch.int32, device=dev) if tri else None
        self.ws = torch.empty(int(L.lib().inrf_workspace_size(n)), dtype=torch.uint8, device=dev)
        args = (cam, precision, table)
        kw = dict(rgba=self.rgba, depth=self.depth, tri=self.tri, ws=self.ws)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):   # warm-up: kernel attributes and occupancy queries happen here
            renderer.render(*args, stream=side, **kw)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, capture_error_mode="relaxed"):
            renderer.render(*args, stream=torch.cuda.current_stream(dev), **kw)

    def replay(self):
        self.graph.replay()
        return self.rgba


class FramePipeline:
    """Frames in flight on `depth` streams of default priority, each with a
    workspace of its own.  A frame's trace (ALU-bound) then overlaps the
    shading of the frame before it (bound by gathers from HBM), which
    raises throughput; every frame's pixels are those of a lone render.
    submit() returns the frame's RGBA buffer (the event recorded after the
    frame is in `events`); wait() makes the caller's current stream wait
    for every submitted frame."""

    def __init__(self, renderer, depth: int = 2):
        torch = renderer.torch
        self.R, self.torch = renderer, torch
        self.streams = [torch.cuda.Stream(device=renderer.device) for _ in range(int(depth))]
        self.ws = [None] * int(depth)
        self.events = [None] * int(depth)
        self.k = 0

    def _workspace(self, slot: int, need: int):
        if self.ws[slot] is None or self.ws[slot].numel() < need:
            # the slot's stream may still use the old buffer: let it drain first
            self.streams[slot].synchronize()
            self.ws[slot] = self.torch.empty(need, dtype=self.torch.uint8, device=self.R.device)
        return self.ws[slot]

    def submit(self, cam, precision="fp16", table="f16", rgba=None, depth=None, tri=None):
        torch = self.torch
        slot = self.k % len(self.streams)
        self.k += 1
        s = self.streams[slot]
        n = int(cam.width) * int(cam.height)
        ws = self._workspace(slot, int(L.lib().inrf_workspace_size(n)))
        if rgba is None:
            rgba = torch.empty((int(cam.height), int(cam.width), 4), dtype=torch.float32, device=self.R.device)
        s.wait_stream(torch.cuda.current_stream(self.R.device))  # outputs allocated / reused by the caller
        for t in (rgba, depth, tri):
            if t is not None:
                t.record_stream(s)
        self.R.render(cam, precision, table, rgba=rgba, depth=depth, tri=tri, stream=s, ws=ws)
        ev = torch.cuda.Event()
        ev.record(s)
        self.events[slot] = ev
        return rgba

    def wait(self):
        cur = self.torch.cuda.current_stream(self.R.device)
        for s in self.streams:
            cur.wait_stream(s)


def adam_step(param, grad, m, v, step: int, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.99,
              eps: float = 1e-15, zero_grad: bool = True, param_f16=None, stream=None, lazy: bool = False):
    """One Adam step in place on contiguous float32 device tensors of equal
    size (the library's k_adam); param_f16, if given, receives the updated
    parameters in FP16.  lazy: step only parameters with a nonzero gradient."""
    import torch
    n = param.numel()
    for t in (grad, m, v):
        if t.numel() != n or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("grad, m, v must be contiguous float32 tensors of param's size")
    if param_f16 is not None and (param_f16.numel() != n or param_f16.dtype != torch.float16):
        raise ValueError("param_f16 must be a float16 tensor of param's size")
    p = L.AdamParams()
    p.lr, p.beta1, p.beta2, p.eps, p.step, p.zero_grad = lr, beta1, beta2, eps, int(step), int(bool(zero_grad))
    p.lazy = int(bool(lazy))
    s = stream if stream is not None else torch.cuda.current_stream(param.device)
    L.check(L.lib().inrf_adam(L.ptr(param), L.ptr(grad), L.ptr(m), L.ptr(v), n, ctypes.byref(p), L.ptr(param_f16),
                              ctypes.c_void_p(s.cuda_stream)))


class Scene:
    """Several device-resident objects (Renderers) placed in the world by
    similarity transforms x_world = scale * R @ x_object + t, rendered with
    inrf_render_scene (nearest hit over the objects, per-object shading)."""

    def __init__(self, renderers, placements):
        """placements: one (scale, rotation [3, 3], translation [3]) per renderer."""
        if len(renderers) != len(placements):
            raise ValueError("one placement per renderer")
        if len(renderers) > L.MAX_OBJECTS:
            raise ValueError(f"at most {L.MAX_OBJECTS} objects")
        self.objects = list(renderers)
        self.placements = [(float(s), np.asarray(R, np.float32).reshape(3, 3), np.asarray(t, np.float32).reshape(3))
                           for s, R, t in placements]
        self._ws = None
        self.torch = renderers[0].torch if renderers else None
        self.device = renderers[0].device if renderers else "cuda"

    def instances(self, table: str):
        arr = (L.InstanceDesc * max(1, len(self.objects)))()
        for k, (R, (s, rot, t)) in enumerate(zip(self.objects, self.placements)):
            arr[k].model = ctypes.addressof(R.desc(table))
            arr[k].scale = s
            arr[k].rotation[:] = [float(v) for v in rot.reshape(-1)]
            arr[k].translation[:] = [float(v) for v in t]
        return arr

    def workspace(self, n_rays: int):
        import torch
        need = int(L.lib().inrf_scene_workspace_size(len(self.objects), n_rays))
        if need < 0:
            raise ValueError("invalid scene size")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def batch_workspace_bytes(self, n_cameras: int, n_pixels: int) -> int:
        """Workspace bytes of a batch of n_cameras cameras with n_pixels in all."""
        need = int(L.lib().inrf_scene_batch_workspace_size(len(self.objects), int(n_cameras), int(n_pixels)))
        if need < 0:
            raise ValueError("invalid scene batch")
        return need

    def render_batch(self, cams, precision="fp32", table="f32", rgba=None, depth=None, tri=None, obj=None,
                     stream=None, ws=None):
        """Several cameras over the scene in one pass (inrf_render_scene_batch).
        Returns the flat [sum(W*H), 4] RGBA buffer and the per-camera
        [H, W, 4] views into it; `ws` an optional caller workspace."""
        import torch
        cams = list(cams)
        if not 1 <= len(cams) <= L.MAX_CAMERAS:
            raise ValueError(f"1..{L.MAX_CAMERAS} cameras per batch")
        sizes = [int(c.width) * int(c.height) for c in cams]
        n = sum(sizes)
        if rgba is None:
            rgba = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        if ws is None:
            ws = self.workspace_bytes(self.batch_workspace_bytes(len(cams), n))
        inst = self.instances(table)
        arr = (L.CameraDesc * len(cams))(*[_camera_desc(c) for c in cams])
        s = stream if stream is not None else torch.cuda.current_stream()
        L.check(L.lib().inrf_render_scene_batch(inst, len(self.objects), PRECISIONS[precision], arr, len(cams),
                                                L.ptr(rgba), L.ptr(depth), L.ptr(tri), L.ptr(obj), L.ptr(ws),
                                                ws.numel(), ctypes.c_void_p(s.cuda_stream)))
        views, off = [], 0
        for c, k in zip(cams, sizes):
            views.append(rgba[off:off + k].view(int(c.height), int(c.width), 4))
            off += k
        return rgba, views

    def workspace_bytes(self, need: int):
        import torch
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def render(self, cam, precision="fp32", table="f32", rgba=None, depth=None, tri=None, obj=None, stream=None):
        import torch
        H, W = int(cam.height), int(cam.width)
        if rgba is None:
            rgba = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        ws = self.workspace(H * W)
        inst = self.instances(table)
        c = _camera_desc(cam)
        s = stream if stream is not None else torch.cuda.current_stream()
        L.check(L.lib().inrf_render_scene(inst, len(self.objects), PRECISIONS[precision], ctypes.byref(c),
                                          L.ptr(rgba), L.ptr(depth), L.ptr(tri), L.ptr(obj), L.ptr(ws), ws.numel(),
                                          ctypes.c_void_p(s.cuda_stream)))
        return rgba
