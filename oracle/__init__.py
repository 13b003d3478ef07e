"""FP64 CPU oracle for the i-NOLF one-query-per-ray render path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library; the two
meet only through the seeded inputs of the ``synth`` package.

Every function is written from the paper's definitions (arXiv 2303.04086,
Sec. 4.1 "Perfect Spatial Hashing Encoding" with Eq. 1, Sec. 4.2 "Instant
Neural Opacity Light Fields" with Eqs. 2-3) and computes the plain definition
of what the fast path reaches:
  * the proxy hit is a brute-force closest hit over all triangles
    (the fast path uses a BVH);
  * the per-level feature lookup is a dictionary keyed by grid vertex
    (the fast path uses a perfect spatial hash); a separate PSH construction
    (psh.py) exists only to check the library's offset tables;
  * the network is evaluated with numpy FP64 matrix products.

Parity status of each function (what pins it) is listed in its module
header; functions that no independent pin covers say "parity unpinned".
"""
from .rays import camera_rays
from .hit import closest_hit, HitResult
from .occupancy import surface_cells, shell_keys
from . import psh
from .psh import build_psh_level, psh_slots, PSHLevel
from .encode import grid_cell, trilinear_encode, FeatureGrid
from .sh import sh_real
from .mlp import mlp_forward
from .render import Model, render_rays, render_camera, encode_points
from .backward import backward_rays, mse_loss, mse_grad
from .optim import adam_step
from .scene import Instance, render_scene_rays

__all__ = [
    "camera_rays", "closest_hit", "HitResult", "surface_cells", "shell_keys",
    "build_psh_level", "psh_slots", "PSHLevel", "grid_cell", "trilinear_encode",
    "FeatureGrid", "sh_real", "mlp_forward", "Model", "render_rays",
    "render_camera", "encode_points", "backward_rays", "mse_loss", "mse_grad", "adam_step", "Instance", "render_scene_rays",
]
