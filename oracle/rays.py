"""Primary rays of a pinhole camera, FP64 (test infrastructure only).

The paper receives camera pose and intrinsics from clients (Sec. 5, data
streaming) and renders one query per ray (Sec. 4.2).  Reading adopted here:
the vertical field of view is given by tan(fov_y/2); pixel (i from the top,
j from the left) looks through its centre,
    s_x = (2 (j + 1/2) / W - 1) * tan(fov_y/2) * W / H
    s_y = (1 - 2 (i + 1/2) / H) * tan(fov_y/2)
    d   = normalize(forward + s_x * right + s_y * up),  o = camera origin,
and ray index = i * W + j.

Pins: the centre of an odd-sized image looks along `forward`; the rays
through the image's top and bottom edge span the field of view; mirror
pixels give mirror rays.
"""
from __future__ import annotations

import numpy as np


def camera_rays(cam, rows=None, cols=None):
    """Return (o, d) float64 arrays [n, 3]; all pixels in row-major order, or
    the pixels (rows[k], cols[k]) when given."""
    W, H = int(cam.width), int(cam.height)
    if rows is None:
        i, j = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
        i, j = i.reshape(-1), j.reshape(-1)
    else:
        i, j = np.asarray(rows, np.float64), np.asarray(cols, np.float64)
    t = float(cam.tan_half_fov_y)
    sx = (2.0 * (j + 0.5) / W - 1.0) * t * W / H
    sy = (1.0 - 2.0 * (i + 0.5) / H) * t
    f, r, u = (np.asarray(a, np.float64) for a in (cam.forward, cam.right, cam.up))
    d = f[None, :] + sx[:, None] * r[None, :] + sy[:, None] * u[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(np.asarray(cam.origin, np.float64), d.shape).copy()
    return o, d
