"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module holds data only: proxy meshes, camera poses, MLP parameters,
feature values and ray/point batches.  It contains none of the rendering
method's arithmetic (no ray generation, intersection, hashing, encoding or
network evaluation); every consumer receives the same arrays.

The paper's workloads are trained objects from public datasets that are not
available here; these procedural objects stand in for "one object inside the
unit cube" with seeded random parameters.
"""
from .mesh import icosphere, displaced_sphere, quantize_vertices, VERTEX_FRAC_BITS
from .camera import (Camera, look_at_camera, fibonacci_cameras, random_cameras, orbit_requests,
                     SERVING_RESOLUTIONS)
from .params import xavier_mlp, level_resolutions, feature_values, table_features
from .batches import random_rays, surface_points, view_rays
from .workloads import (Workload, workload_tiny, workload_object, SceneObject, SceneWorkload, random_rotation,
                        scene_tiny, scene_objects)
from .nolf import NolfWorkload, make_nolf, nolf_tiny, nolf_object

__all__ = [
    "icosphere", "displaced_sphere", "quantize_vertices", "VERTEX_FRAC_BITS",
    "Camera", "look_at_camera", "fibonacci_cameras", "random_cameras", "orbit_requests", "SERVING_RESOLUTIONS",
    "xavier_mlp", "level_resolutions", "feature_values", "table_features",
    "random_rays", "surface_points", "view_rays",
    "Workload", "workload_tiny", "workload_object", "SceneObject", "SceneWorkload", "random_rotation",
    "scene_tiny", "scene_objects", "NolfWorkload", "make_nolf", "nolf_tiny", "nolf_object",
]
