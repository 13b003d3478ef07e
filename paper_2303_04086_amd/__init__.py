"""MI355X-native i-NOLF one-query-per-ray render path (arXiv 2303.04086).

The product is libinrf.so (C ABI in include/inrf.h): host builders for the
perfect spatial hash and the proxy BVH, and HIP kernels for gfx950.  This
package is its binding."""
from ._lib import InrfError, lib, EXPORTED, PREC_FP32, PREC_FP16, PREC_BF16
from .model import (PshLevel, BvhImage, CapturedFrame, FramePipeline, NolfRenderer, Renderer, Scene, build_bvh, build_psh, build_psh_keys,
                    camera_rays, psh_params)

__all__ = ["InrfError", "lib", "EXPORTED", "PREC_FP32", "PREC_FP16", "PREC_BF16", "PshLevel", "BvhImage",
           "CapturedFrame", "FramePipeline", "NolfRenderer", "Renderer", "Scene", "build_bvh", "build_psh", "build_psh_keys", "camera_rays",
           "psh_params"]
