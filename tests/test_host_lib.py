"""Host side of libinrf (no GPU): exports, PSH / occupancy bit-identity with
the oracle, BVH invariants, argument errors."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

P = pytest.importorskip("paper_2303_04086_amd")
from paper_2303_04086_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "inrf.h")).read()
    declared = set(re.findall(r"\b(inrf_[a-z_]+)\s*\(", hdr))
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTED)
    assert lib.inrf_version() >= 100


def test_peaks_library_exports_every_declared_symbol():
    """The benchmark's measurement kernels (include/inrf_peaks.h) load and
    refuse bad arguments on the host, before touching a device."""
    from paper_2303_04086_amd import peaks
    hdr = open(os.path.join(ROOT, "include", "inrf_peaks.h")).read()
    declared = set(re.findall(r"\b(inrf_[a-z_]+)\s*\(", hdr))
    lib = peaks.lib()
    assert declared == set(peaks.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.inrf_peak_read_sink_size() >= 256
    assert lib.inrf_peak_hbm_read(None, 16, 1, None, None) == -1
    assert lib.inrf_peak_mfma(7, 2, 10, 256, None) == -1 and b"precision" in lib.inrf_peaks_last_error()


# Entry points that carry out a step of the paper's method: each one's
# comment block in the header cites the passage that defines it.
CITED = ["inrf_build_psh", "inrf_build_bvh", "inrf_render", "inrf_camera_rays", "inrf_forward", "inrf_render_batch",
         "inrf_encode", "inrf_mlp", "inrf_render_scene", "inrf_render_nolf", "inrf_shade_nolf", "inrf_backward",
         "inrf_adam"]


def _comment_before(hdr: str, name: str) -> str:
    """All comment text between the end of the previous top-level
    declaration (a ';' outside comments and braces) and the declaration of
    `name`, so a block describing a group, or a parameter struct, counts."""
    code = re.sub(r"/\*.*?\*/", lambda m: " " * len(m.group(0)), hdr, flags=re.S)
    at = re.search(r"\b" + name + r"\s*\(", code).start()
    depth, prev = 0, 0
    for i, ch in enumerate(code[:at]):
        depth += ch == "{"
        depth -= ch == "}"
        if ch == ";" and depth == 0:
            prev = i
    return " ".join(re.findall(r"/\*(.*?)\*/", hdr[prev:at], re.S))


def test_header_cites_the_paper_for_every_path_call():
    hdr = open(os.path.join(ROOT, "include", "inrf.h")).read()
    for name in CITED:
        text = _comment_before(hdr, name)
        assert re.search(r"Sec\. \d|Eqs?\. \d|Kingma", text), f"{name}: no citation in {text[:200]!r}"
    # the render call cites where poses come from (clients send them per frame)
    assert "Sec. 5" in _comment_before(hdr, "inrf_render")


def test_psh_identical_to_oracle_on_tiny_workload(tiny, tiny_keys):
    levels = P.build_psh(tiny.verts, tiny.tris, tiny.res)
    for N, k, lv in zip(tiny.res, tiny_keys, levels):
        M = N + 1
        assert np.array_equal((k[:, 2] * M + k[:, 1]) * M + k[:, 0], lv.keys)
        O = oracle.build_psh_level(k, N, seed=1)
        assert (lv.mbar, lv.rbar) == (O.mbar, O.rbar)
        assert np.array_equal(lv.phi, O.phi)
        assert np.array_equal(lv.slots.astype(np.int64), O.slots)


def test_psh_identical_to_oracle_other_parameters(tiny_keys, tiny):
    k = tiny_keys[1]
    N = tiny.res[1]
    M = N + 1
    lin = (k[:, 2] * M + k[:, 1]) * M + k[:, 0]
    for kw in ({"seed": 7, "load_pct": 95, "bucket_keys": 6}, {"seed": 3, "load_pct": 60, "bucket_keys": 1},
               {"seed": 1, "load_pct": 100, "bucket_keys": 6, "n_random": 0}):
        lv = P.build_psh_keys(N, lin, **kw)
        O = oracle.build_psh_level(k, N, **kw)
        assert (lv.mbar, lv.rbar, lv.restarts >= 0) == (O.mbar, O.rbar, True)
        assert np.array_equal(lv.phi, O.phi), kw
        assert np.array_equal(lv.slots.astype(np.int64), O.slots), kw


def test_occupancy_identical_to_oracle_on_random_soup():
    rng = np.random.default_rng(5)
    v = synth.quantize_vertices(rng.uniform(0.05, 0.95, (60, 3)))
    t = rng.integers(0, 60, (20, 3)).astype(np.int32)
    for N, dil in ((7, 0), (13, 1), (20, 2)):
        lv = P.build_psh(v, t, [N], dilate=dil)[0]
        k = oracle.shell_keys(v, t, N, dil)
        M = N + 1
        assert np.array_equal((k[:, 2] * M + k[:, 1]) * M + k[:, 0], lv.keys), (N, dil)


def test_bvh_invariants(tiny):
    v, t = synth.displaced_sphere(12)
    b = P.build_bvh(v, t)
    f = b.nodes.view(np.float32).reshape(-1, 32)
    refs = b.nodes.view(np.int32).reshape(-1, 32)[:, 24:28]
    tri_img = b.tris.view(np.float32).reshape(-1, 12)
    idx = b.tris.view(np.int32).reshape(-1, 12)[:, 3]
    assert sorted(idx.tolist()) == list(range(len(t)))          # every triangle exactly once
    V = v.astype(np.float32)
    assert np.array_equal(tri_img[:, 0:3], V[t[idx, 0]]) and np.array_equal(tri_img[:, 8:11], V[t[idx, 2]])
    seen = []

    def walk(node, lo, hi, depth):
        """Returns (deepest leaf level, traversal stack need) of the subtree."""
        n = f[node]
        deepest, need, interior = depth, 0, 0
        for c in range(4):
            ref = refs[node][c]
            if ref == -1:
                continue
            a = np.array([n[c], n[4 + c], n[8 + c]])
            z = np.array([n[12 + c], n[16 + c], n[20 + c]])
            if lo is not None:
                assert np.all(a >= lo) and np.all(z <= hi)           # children inside the parent
            if ref < 0:
                code = ~ref
                first, count = code >> 3, code & 7
                assert 1 <= count <= 4
                for i in range(first, first + count):
                    p = tri_img[i].reshape(3, 4)[:, :3]
                    assert np.all(p >= a) and np.all(p <= z)        # triangles inside the leaf box
                    seen.append(i)
                deepest = max(deepest, depth + 1)
            else:
                interior += 1
                d, s = walk(ref, a, z, depth + 1)
                deepest, need = max(deepest, d), max(need, s)
        return deepest, max(0, interior - 1) + need

    depth, need = walk(0, None, None, 1)
    assert sorted(seen) == list(range(len(t)))
    assert depth == b.depth and max(1, need) == b.stack and b.stack <= 64
    assert b.n_nodes < len(t) / 2                                   # four-wide: far fewer nodes than leaves


def test_argument_errors():
    lib = L.lib()
    h = ctypes.c_void_p()
    p = P.psh_params()
    bad_v = np.array([[0.1, 0.2, 0.3]], np.float32)          # 0.1 is off the 2^-16 lattice
    t = np.array([[0, 0, 0]], np.int32)
    r = np.array([8], np.int32)
    assert lib.inrf_build_psh(L.ptr(bad_v), 1, L.ptr(t), 1, 1, L.ptr(r), ctypes.byref(p), ctypes.byref(h)) == L.INRF_E_INVALID
    assert b"2^-16" in lib.inrf_last_error()
    good_v = synth.quantize_vertices(bad_v)
    t_bad = np.array([[0, 0, 5]], np.int32)
    assert lib.inrf_build_psh(L.ptr(good_v), 1, L.ptr(t_bad), 1, 1, L.ptr(r), ctypes.byref(p), ctypes.byref(h)) == L.INRF_E_INVALID
    r0 = np.array([0], np.int32)
    assert lib.inrf_build_psh(L.ptr(good_v), 1, L.ptr(t), 1, 1, L.ptr(r0), ctypes.byref(p), ctypes.byref(h)) == L.INRF_E_INVALID
    p.load_pct = 0
    assert lib.inrf_build_psh(L.ptr(good_v), 1, L.ptr(t), 1, 1, L.ptr(r), ctypes.byref(p), ctypes.byref(h)) == L.INRF_E_INVALID
    keys = np.array([5, 3], np.int64)
    assert lib.inrf_build_psh_keys(4, L.ptr(keys), 2, ctypes.byref(P.psh_params()), ctypes.byref(h)) == L.INRF_E_INVALID
    # device calls validate before touching the device
    m = L.ModelDesc()
    m.n_levels = 0
    assert lib.inrf_encode(ctypes.byref(m), None, 0, None, None, None) == L.INRF_E_INVALID
    m.n_levels = 1
    m.table_dtype = 7
    assert lib.inrf_encode(ctypes.byref(m), None, 0, None, None, None) == L.INRF_E_INVALID
    assert lib.inrf_workspace_size(-1) == -1
    assert lib.inrf_workspace_size(1000) > 1000 * 16


def test_nolf_rejects_nonpositive_w_min():
    """A largest sample weight of 0 must not count as a hit: w_min <= 0 is an
    invalid argument, refused on the host before anything touches a device
    (the pointers below are never dereferenced)."""
    lib = L.lib()
    m = L.ModelDesc()
    m.n_levels, m.table_dtype = 1, L.INRF_F32
    m.levels[0].res, m.levels[0].mbar, m.levels[0].rbar = 16, 17, 5
    m.phi = m.table = m.weights = 256
    cam = L.CameraDesc()
    cam.forward[:] = [0.0, 0.0, 1.0]
    cam.right[:] = [1.0, 0.0, 0.0]
    cam.up[:] = [0.0, 1.0, 0.0]
    cam.tan_half_fov_y, cam.width, cam.height = 0.36, 4, 4
    for w_min, ok in ((0.0, False), (-1e-4, False), (float("nan"), False), (1e-4, True)):
        cubes = L.CubesDesc(16, 4, 256, 256, 256, 1, 0.01, 1e-4, w_min, 0)
        # a valid w_min passes validation and then stops at the undersized workspace
        st = lib.inrf_render_nolf(ctypes.byref(m), ctypes.byref(cubes), 0, ctypes.byref(cam), 256, None, None, 256,
                                  16, None)
        if ok:
            assert st == L.INRF_E_SIZE, lib.inrf_last_error()
        else:
            assert st == L.INRF_E_INVALID and b"w_min" in lib.inrf_last_error()


def test_empty_mesh_builds():
    v = np.zeros((0, 3), np.float32)
    t = np.zeros((0, 3), np.int32)
    lv = P.build_psh(v, t, [4])[0]
    assert len(lv.keys) == 0 and lv.mbar == 2  # smallest with 80*m^3 >= 100*max(n, 1)
    # few keys at a large resolution: library and oracle agree on the raised sizes
    lv = P.build_psh_keys(4000, [((17 * 4001) + 0) * 4001 + 3999])
    O = oracle.build_psh_level(np.array([[3999, 0, 17]]), 4000, seed=1)
    assert (lv.mbar, lv.rbar) == (O.mbar, O.rbar) and np.array_equal(lv.phi, O.phi)
    b = P.build_bvh(v, t)
    assert b.n_nodes == 1 and b.stack == 1


def test_brick_layout():
    """Storage order of the device cubes: a bijection into the padded cube,
    bricks of 8 x 4 x 1 cells on one 128-byte line, hand-checked entries."""
    from paper_2303_04086_amd.model import brick_entries, brick_index
    for side in (1, 2, 3, 5, 8, 13, 64):
        n = side ** 3
        idx = brick_index(side, np.arange(n))
        assert len(np.unique(idx)) == n and idx.min() >= 0 and idx.max() < brick_entries(side)
        v = np.arange(n)
        x, y, z = v % side, (v // side) % side, v // (side * side)
        key = (z * 1000 + y // 4) * 1000 + x // 8
        for k in np.unique(key)[:50]:
            assert len(np.unique(idx[key == k] // 32)) == 1   # one brick = one line
        assert np.array_equal(idx % 32, (y % 4) * 8 + x % 8)
        bx = -(-side // 8)
        assert brick_entries(side) == 32 * bx * (-(-side // 4)) * side
    lin = lambda x, y, z, s: (z * s + y) * s + x
    got = brick_index(5, [lin(4, 0, 0, 5), lin(0, 4, 0, 5), lin(0, 0, 2, 5), lin(1, 1, 1, 5)])
    assert list(got) == [4, 32, 128, 73]
    got = brick_index(20, [lin(8, 0, 0, 20), lin(0, 4, 0, 20), lin(9, 5, 1, 20)])
    # row = 32 * 3 bricks = 96 entries, plane = 96 * 5 = 480
    assert list(got) == [32, 96, 480 + 96 + 32 + 1 * 8 + 1]
    import paper_2303_04086_amd as P
    assert P.lib().inrf_brick_entries(0) == -1 and P.lib().inrf_brick_entries(1025) == -1
    with pytest.raises(P.InrfError):
        brick_index(5, [0, 125])
