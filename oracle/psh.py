"""Perfect spatial hash of one level, built and queried in plain Python (test
infrastructure only).

Hash form (Sec. 4.1, Eq. 1): h(p) = h0(p) + Phi(h1(p)), with the readings
  h0(p) = p mod mbar,  h1(p) = p mod rbar  (component-wise),
  slot(p) = (p + Phi[p mod rbar]) mod mbar  (component-wise),
  linear slot = (s_z * mbar + s_y) * mbar + s_x,
so a table of mbar**3 slots holds one feature vector per key with no
collision.  The paper builds Phi with a heuristic that favours mapping
neighbouring points to neighbouring slots (Sec. 4.1 and the PSH figure) but
does not spell it out; the deterministic greedy adopted here is:

  sizes   mbar = smallest integer with load_pct * mbar**3 >= 100 * n (the
          table is at most load_pct % full; default 80) and 1024 * mbar >= N + 1
          (which keeps rbar <= 1024);
          rbar = smallest integer >= 2 with bucket_keys * rbar**3 >= n (about
          bucket_keys keys per offset entry; default 2), then increased until
          gcd(mbar, rbar) = 1 and mbar * rbar >= N + 1.  Keys sharing a bucket
          then differ modulo mbar (Chinese remainder theorem), so any offset
          keeps a bucket's own keys apart.  A table with slack and small
          buckets lets more buckets take a neighbour's offset, which is what
          makes neighbouring keys share cache lines.
  order   buckets B_q = {p : p mod rbar = q}, largest first, ties by linear q
          = (q_z * rbar + q_y) * rbar + q_x ascending.
  offsets for each bucket, try in turn
          (i)   the offsets already given to its six face neighbours in
                offset space (-x, +x, -y, +y, -z, +z, wrapping), duplicates
                skipped -- equal neighbouring offsets put neighbouring keys in
                neighbouring slots;
          (ii)  n_random (default 32) pseudo-random offsets: r_k = splitmix64(splitmix64(seed) +
                q * 256 + k), offset = (r mod mbar, (r >> 21) mod mbar,
                (r >> 42) mod mbar);
          (iii) every offset that puts the bucket's first key on a free slot,
                free slots in ascending linear order (exhaustive);
          and keep the first offset under which every key of the bucket lands
          on a free slot.  If a bucket admits none, rbar is raised (keeping
          the conditions above) and the build restarts; after max_restarts
          (default 4) restarts mbar is raised by one.  Empty buckets get offset 0.
  storage Phi entries are packed as x | y << 10 | z << 20 (mbar <= 1024).

Pins: injectivity by brute force; PSH lookup equals a dictionary lookup on
every key; the bucket CRT property; reproducibility from the seed.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import gcd

import numpy as np

M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (Steele, Lea & Flood, 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _icbrt_ceil(n: int, mult: int = 1) -> int:
    """Smallest r >= 1 with mult * r**3 >= n (exact integer arithmetic)."""
    r = max(1, int(round((n / mult) ** (1.0 / 3.0))) - 2)
    while mult * r ** 3 < n:
        r += 1
    while r > 1 and mult * (r - 1) ** 3 >= n:
        r -= 1
    return r


def _fix_rbar(r: int, mbar: int, N: int) -> int:
    while gcd(mbar, r) != 1 or mbar * r < N + 1:
        r += 1
    return r


@dataclass
class PSHLevel:
    res: int
    mbar: int
    rbar: int
    phi: np.ndarray    # uint32 [rbar**3], packed
    slots: np.ndarray  # int64 [n], linear slot of each key (canonical order)


def _try_build(keys, N, mbar, rbar, seed, n_random=32):
    n = len(keys)
    R3 = rbar ** 3
    q3 = [(int(x) % rbar, int(y) % rbar, int(z) % rbar) for x, y, z in keys]
    qlin = [(qz * rbar + qy) * rbar + qx for qx, qy, qz in q3]
    h0 = [(int(x) % mbar, int(y) % mbar, int(z) % mbar) for x, y, z in keys]
    buckets: dict = {}
    for i, q in enumerate(qlin):
        buckets.setdefault(q, []).append(i)
    order = sorted(buckets, key=lambda q: (-len(buckets[q]), q))
    used = bytearray(mbar ** 3)
    phi: dict = {}
    s0 = splitmix64(seed)

    def lin(s):
        return (s[2] * mbar + s[1]) * mbar + s[0]

    def fits(members, off):
        out = []
        for i in members:
            s = lin(((h0[i][0] + off[0]) % mbar, (h0[i][1] + off[1]) % mbar, (h0[i][2] + off[2]) % mbar))
            if used[s]:
                return None
            out.append(s)
        return out

    for q in order:
        members = buckets[q]
        qz, rem = divmod(q, rbar * rbar)
        qy, qx = divmod(rem, rbar)
        cands = []
        for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            nq = (((qz + dz) % rbar) * rbar + (qy + dy) % rbar) * rbar + (qx + dx) % rbar
            if nq in phi and phi[nq] not in cands:
                cands.append(phi[nq])
        chosen = None
        for off in cands:
            chosen = fits(members, off)
            if chosen is not None:
                phi[q] = off
                break
        if chosen is None:
            for k in range(n_random):
                r = splitmix64((s0 + q * 256 + k) & M64)
                off = (r % mbar, (r >> 21) % mbar, (r >> 42) % mbar)
                chosen = fits(members, off)
                if chosen is not None:
                    phi[q] = off
                    break
        if chosen is None:
            p0 = h0[members[0]]
            s = used.find(0)
            while s >= 0:
                sz, rem = divmod(s, mbar * mbar)
                sy, sx = divmod(rem, mbar)
                off = ((sx - p0[0]) % mbar, (sy - p0[1]) % mbar, (sz - p0[2]) % mbar)
                chosen = fits(members, off)
                if chosen is not None:
                    phi[q] = off
                    break
                s = used.find(0, s + 1)
        if chosen is None:
            return None
        for s in chosen:
            used[s] = 1
    packed = np.zeros(R3, np.uint32)
    for q, (ox, oy, oz) in phi.items():
        packed[q] = ox | (oy << 10) | (oz << 20)
    slots = np.array([lin(((h0[i][0] + phi[qlin[i]][0]) % mbar, (h0[i][1] + phi[qlin[i]][1]) % mbar,
                           (h0[i][2] + phi[qlin[i]][2]) % mbar)) for i in range(n)], np.int64)
    return packed, slots


def build_psh_level(keys, N: int, seed: int = 1, load_pct: int = 80, bucket_keys: int = 2,
                    n_random: int = 32, max_restarts: int = 4) -> PSHLevel:
    """Build Phi and the slot of each key; keys int [n, 3] in canonical order."""
    keys = np.asarray(keys, np.int64).reshape(-1, 3)
    n = len(keys)
    mbar = max(_icbrt_ceil(100 * max(n, 1), load_pct), -(-(N + 1) // 1024))
    rbar = _fix_rbar(max(2, _icbrt_ceil(max(n, 1), bucket_keys)), mbar, N)
    while True:
        for _ in range(max_restarts + 1):
            if mbar > 1024:
                raise RuntimeError("offset components exceed 10 bits")
            got = _try_build(keys, N, mbar, rbar, seed, n_random)
            if got is not None:
                return PSHLevel(N, mbar, rbar, got[0], got[1])
            rbar = _fix_rbar(rbar + 1, mbar, N)
        mbar += 1
        rbar = _fix_rbar(rbar, mbar, N)


def psh_slots(level: PSHLevel, vertices) -> np.ndarray:
    """Linear slots of integer vertices [k, 3] under the level's hash (Eq. 1)."""
    v = np.asarray(vertices, np.int64).reshape(-1, 3)
    r, m = level.rbar, level.mbar
    q = v % r
    ql = (q[:, 2] * r + q[:, 1]) * r + q[:, 0]
    ph = level.phi[ql].astype(np.int64)
    off = np.stack([ph & 1023, (ph >> 10) & 1023, (ph >> 20) & 1023], axis=1)
    s = (v % m + off) % m
    return (s[:, 2] * m + s[:, 1]) * m + s[:, 0]
