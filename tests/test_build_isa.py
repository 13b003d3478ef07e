"""Static checks of the gfx950 code the build produces (no GPU needed)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


_CACHE = {}


def _assembly(tmp_path):
    if "asm" in _CACHE:
        return _CACHE["asm"]
    from paper_2303_04086_amd import build as b
    out = tmp_path / "render.s"
    cmd = [b._hipcc(), *b.HIP_FLAGS, *b.COMMON, "--cuda-device-only", "-S",
           os.path.join(b.CSRC, "render.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"hipcc unavailable: {r.stderr[:200]}")
    _CACHE["asm"] = out.read_text()
    return _CACHE["asm"]


def test_no_partially_overlapping_matrix_accumulators(tmp_path):
    """An MFMA whose destination partially overlaps its own accumulator input
    produced wrong sums on the device; the build must emit none."""
    asm = _assembly(tmp_path)
    pat = re.compile(r"v_mfma_\S+\s+([av])\[(\d+):(\d+)\],\s*\S+,\s*\S+,\s*([av])\[(\d+):(\d+)\]")
    n_mfma, bad = 0, []
    for line in asm.splitlines():
        m = pat.search(line)
        if not m:
            continue
        n_mfma += 1
        r1, d0, d1, r2, c0, c1 = m.groups()
        d0, d1, c0, c1 = int(d0), int(d1), int(c0), int(c1)
        if r1 == r2 and (d0, d1) != (c0, c1) and not (d1 < c0 or c1 < d0):
            bad.append(line.strip())
    assert n_mfma > 100
    assert not bad, bad[:5]


def test_no_packed_fp32_and_no_scratch(tmp_path):
    asm = _assembly(tmp_path)
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", asm)
    sizes = [int(x) for x in re.findall(r"\.private_segment_fixed_size:\s*(\d+)", asm)]
    assert sizes and max(sizes) == 0, "a kernel spills to scratch"
