"""The perfect spatial hash of the benchmark object at full size, on the CPU:
all 16 levels (16..2048, about 137.6M occupied vertices) built by the
library, checked level by level against what Sec. 4.1 requires of it.

  * Eq. 1 reproduced: the oracle's own arithmetic, slot(v) = (v mod mbar +
    Phi[v mod rbar]) mod mbar per axis, applied to the library's offset
    table gives the library's slot for every key;
  * injective: no two keys share a slot, and every slot lies in the table;
  * corner coverage (the occupancy reading of Sec. 4.2: features stored
    around every possible hit point): the eight corners of the cell of
    every one of 400,000 seeded points on the proxy surface are keys at
    every level.
The offset tables of the tiny workload are also compared bit for bit with
the oracle's own construction (test_host_lib.py)."""
import numpy as np
import pytest

import oracle
import synth
import paper_2303_04086_amd as P

CHUNK = 1 << 23


@pytest.fixture(scope="module")
def levels():
    w = synth.workload_object(64, 64)
    return w, P.build_psh(w.verts, w.tris, w.res, dilate=w.dilate, seed=w.psh_seed)


def test_full_scale_key_count(levels):
    w, lv = levels
    total = sum(len(l.keys) for l in lv)
    print(f"{total} keys over {len(lv)} levels; finest level {len(lv[-1].keys)}")
    assert [l.res for l in lv] == list(w.res)
    assert 1.2e8 < total < 1.6e8


@pytest.mark.parametrize("level", range(16))
def test_full_scale_level(levels, level):
    w, lv = levels
    L = lv[level]
    n = len(L.keys)
    assert n > 0 and np.all(np.diff(L.keys) > 0)          # canonical ascending order
    # Eq. 1 by the oracle's arithmetic on the library's offsets, chunk by chunk
    ol = oracle.PSHLevel(L.res, L.mbar, L.rbar, L.phi, None)
    M = L.res + 1
    for a in range(0, n, CHUNK):
        k = L.keys[a:a + CHUNK]
        v = np.stack([k % M, (k // M) % M, k // (M * M)], axis=1)
        assert np.array_equal(oracle.psh_slots(ol, v), L.slots[a:a + CHUNK].astype(np.int64))
    # injective into the table
    s = np.sort(L.slots.astype(np.int64))
    assert s[0] >= 0 and s[-1] < L.mbar ** 3
    assert np.all(np.diff(s) > 0)
    del s
    # corner coverage on points of the proxy surface
    x = synth.surface_points(w.verts, w.tris, 400_000, 900 + level)
    corners = oracle.encode.corner_vertices(x, L.res).reshape(-1, 3)
    lin = (corners[:, 2] * M + corners[:, 1]) * M + corners[:, 0]
    pos = np.searchsorted(L.keys, lin)
    found = (pos < n) & (L.keys[np.minimum(pos, n - 1)] == lin)
    assert found.all(), f"{int((~found).sum())} corners of surface cells are not keys at N={L.res}"
    print(f"N={L.res}: {n} keys, mbar {L.mbar}, rbar {L.rbar}, load {n / L.mbar ** 3:.3f}")
