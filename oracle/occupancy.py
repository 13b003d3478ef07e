"""Occupied grid vertices ("keys") of one level, in exact arithmetic (test
infrastructure only).

The paper stores features only for voxels around the possible hit points
(Sec. 4.2, "Implementation with PSH encoding") and computes the PSH offset
table from an occupancy field (Sec. 4.1, "Implementation for i-NGP").  Reading
adopted for a triangle-mesh proxy at grid resolution N (cells 0..N-1 per axis,
vertices 0..N):
  * surface cell: a cell whose closed box [p/N, (p+1)/N] meets a triangle;
  * occupied cell: a cell within Chebyshev distance `dilate` of a surface
    cell, clipped to the grid;
  * keys: every corner of every occupied cell, as integer vertex coordinates,
    in canonical order (linear key (z*(N+1)+y)*(N+1)+x ascending).

Triangle/box overlap is the separating-axis test (13 axes: 3 box normals,
the triangle normal, 9 edge cross products).  Vertex coordinates are
multiples of 2**-16, so N * 2**17 * v is an integer and the test is carried
out on integers: exactly.  The 12 axes whose projections fit int64 are
evaluated in numpy int64; the triangle-normal axis is evaluated in FP64 with
a rounding bound and, when the bound does not decide it, again in Python's
arbitrary-precision integers.

Pins: against an independent exact test (clipping the triangle to the box
with rational arithmetic) on small grids; every corner of the cell holding a
surface point is a key; the key count of a sphere follows its area.
"""
from __future__ import annotations

import numpy as np

FRAC_BITS = 16


def _integer_vertices(verts, N):
    """2 * N * v * 2**16 as int64 (exact); asserts the 2**-16 lattice."""
    v = np.asarray(verts, np.float64)
    s = v * float(1 << FRAC_BITS)
    q = np.rint(s)
    if not np.array_equal(q, s):
        raise ValueError("vertex coordinates must be multiples of 2**-16")
    return q.astype(np.int64) * (2 * int(N))


def _sat_overlap(X, C, h):
    """Closed-box / triangle overlap by the 13-axis separating-axis test.

    X: triangle corners int64 [3, 3]; C: box centres int64 [k, 3]; h: box
    half-extents int64 [k, 3] or [3].  All in the doubled integer units of
    _integer_vertices.  Returns bool [k]."""
    h = np.broadcast_to(np.asarray(h, np.int64), C.shape)
    w = X[None, :, :] - C[:, None, :]                  # [k, 3 vertices, 3]
    keep = np.ones(len(C), bool)
    # box normals
    keep &= ~np.any((w.min(axis=1) > h) | (w.max(axis=1) < -h), axis=1)
    # nine edge cross-product axes e_ax x f_j
    for fj in (X[1] - X[0], X[2] - X[1], X[0] - X[2]):
        for ax in range(3):
            b1, b2 = (ax + 1) % 3, (ax + 2) % 3
            a1, a2 = -int(fj[b2]), int(fj[b1])
            p = w[:, :, b1] * a1 + w[:, :, b2] * a2
            r = h[:, b1] * abs(a1) + h[:, b2] * abs(a2)
            keep &= ~((p.min(axis=1) > r) | (p.max(axis=1) < -r))
    # triangle normal axis, FP64 with exact fallback
    nrm = [int(x) for x in np.cross(X[1] - X[0], X[2] - X[0])]   # fits int64
    idx = np.nonzero(keep)[0]
    if len(idx):
        w0 = w[idx, 0, :].astype(np.float64)
        nf = np.array(nrm, np.float64)
        hf = h[idx].astype(np.float64)
        dist = w0 @ nf
        rad = hf @ np.abs(nf)
        bound = 2.0 ** -50 * ((np.abs(w0) @ np.abs(nf)) + rad)
        sep = np.abs(dist) - rad
        decided_sep = sep > bound
        decided_ok = sep < -bound
        res = ~decided_sep
        for k in np.nonzero(~(decided_sep | decided_ok))[0]:
            wk = [int(x) for x in w[idx[k], 0, :]]
            hk = [int(x) for x in h[idx[k]]]
            dd = sum(wk[c] * nrm[c] for c in range(3))
            res[k] = abs(dd) <= sum(hk[c] * abs(nrm[c]) for c in range(3))
        keep[idx] = res
    return keep


def _cells_of_triangle(X, N):
    """Surface cells (int64 [k, 3]) of one triangle with integer corners X
    [3, 3], in units where a cell spans 2**17."""
    S = 1 << (FRAC_BITS + 1)
    h = 1 << FRAC_BITS
    lo = np.maximum(-(-X.min(axis=0) // S) - 1, 0)   # ceil(min/S) - 1
    hi = np.minimum(X.max(axis=0) // S, N - 1)
    if np.any(lo > hi):
        return np.zeros((0, 3), np.int64)
    g = np.stack(np.meshgrid(*[np.arange(lo[k], hi[k] + 1, dtype=np.int64) for k in range(3)],
                             indexing="ij"), axis=-1).reshape(-1, 3)
    return g[_sat_overlap(X, (2 * g + 1) * h, np.array([h, h, h], np.int64))]


def is_key(verts, tris, N: int, vertices, dilate: int = 1) -> np.ndarray:
    """Whether each integer vertex [k, 3] is a key of the level, decided
    locally: v is a corner of an occupied cell iff some triangle meets the
    closed union of the cells v-1-dilate .. v+dilate (clipped to the grid)."""
    X = _integer_vertices(verts, N)
    v = np.asarray(vertices, np.int64).reshape(-1, 3)
    lo = np.maximum(v - 1 - dilate, 0)
    hi = np.minimum(v + dilate, N - 1) + 1             # exclusive cell bound = box max
    S = 1 << (FRAC_BITS + 1)
    C = (lo + hi) * (S // 2)                           # box centre, doubled units
    H = (hi - lo) * (S // 2)
    ok = (lo < hi).all(axis=1)
    out = np.zeros(len(v), bool)
    if len(v) == 0:
        return out
    # only triangles whose bounding box meets the bounding box of all query
    # boxes can meet one of them; the others are skipped unexamined
    T = np.asarray(tris, np.int64).reshape(-1, 3)
    bmin, bmax = (C - H).min(axis=0), (C + H).max(axis=0)
    tmin, tmax = X[T].min(axis=1), X[T].max(axis=1)
    near = np.all((tmin <= bmax) & (tmax >= bmin), axis=1)
    for t in T[near]:
        out |= _sat_overlap(X[t], C, H) & ok
    return out


def surface_cells(verts, tris, N: int) -> np.ndarray:
    """Sorted unique linear cell indices (z*N+y)*N+x of surface cells."""
    X = _integer_vertices(verts, N)
    tris = np.asarray(tris, np.int64).reshape(-1, 3)
    out = [_cells_of_triangle(X[t], N) for t in tris]
    if not out:
        return np.zeros(0, np.int64)
    c = np.concatenate(out)
    return np.unique((c[:, 2] * N + c[:, 1]) * N + c[:, 0])


def shell_keys(verts, tris, N: int, dilate: int = 1) -> np.ndarray:
    """Keys of one level: integer vertex coordinates [n, 3] (x, y, z) in
    canonical order."""
    cells = surface_cells(verts, tris, N)
    if len(cells) == 0:
        return np.zeros((0, 3), np.int64)
    cz, rem = np.divmod(cells, N * N)
    cy, cx = np.divmod(rem, N)
    base = np.stack([cx, cy, cz], axis=1)
    rng = np.arange(-dilate, dilate + 1)
    offs = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), axis=-1).reshape(-1, 3)
    occ = (base[:, None, :] + offs[None, :, :]).reshape(-1, 3)
    occ = occ[np.all((occ >= 0) & (occ < N), axis=1)]
    occ = np.unique((occ[:, 2] * N + occ[:, 1]) * N + occ[:, 0])
    oz, rem = np.divmod(occ, N * N)
    oy, ox = np.divmod(rem, N)
    occ3 = np.stack([ox, oy, oz], axis=1)
    corners = np.array([[cx_, cy_, cz_] for cz_ in (0, 1) for cy_ in (0, 1) for cx_ in (0, 1)], np.int64)
    v = (occ3[:, None, :] + corners[None]).reshape(-1, 3)
    M = N + 1
    lin = np.unique((v[:, 2] * M + v[:, 1]) * M + v[:, 0])
    vz, rem = np.divmod(lin, M * M)
    vy, vx = np.divmod(rem, M)
    return np.stack([vx, vy, vz], axis=1)
