"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws random numbers and lays out arrays: Gaussian parameter
sets shaped like the pruned / unpruned scenes the paper renders (Sec. 5,
Tab. 3 model sizes), pinhole cameras (stereo head, rings, yaw arcs), fovea
descriptions and the renderer's scalar knobs.  It contains none of the
rendering arithmetic: no projection, no colour evaluation, no blending.

Every float that crosses the library boundary as ``float`` in C is produced
here already rounded to float32, so that the FP64 oracle and the FP32 GPU path
start from the very same input bits.
"""
from .scenes import (  # noqa: F401
    Params, Camera, Fovea, Scene,
    default_params, make_scene, uniform_scene, cluster_scene,
    camera_lookat, camera_translate, stereo_head, ring_cameras,
    fovea_off, fovea_at_center, fovea_rect, lens_mask, LENS_AXES,
    config_tiny, config_stereo, config_unpruned, config_batch, config_diff,
    subset_scene, permute_scene,
)
