"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Holds scene rendering and workload parameters only; no matching arithmetic.
"""
from .scenes import Scene, SceneSpec, make_scene, smoothed_noise  # noqa: F401
from .configs import (params_dict, tiny_spec, tiny_params, kitti_spec,  # noqa: F401
                      kitti_params, kitti_batch_specs, small_spec, sintel_spec,
                      sintel_params, sintel_sequence_specs)
