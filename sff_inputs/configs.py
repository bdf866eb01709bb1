"""Named workloads: scene specifications plus matcher parameters.

* ``tiny``   -- 160x96 grey pairs, one pyramid level, 4 iterations.
* ``kitti``  -- 1242x375 RGB pairs shaped like KITTI scene-flow frames (large
  stereo and flow displacements, an occluder, salt noise), 3 levels x 6
  iterations.  Synthetic stand-in for KITTI 2015 (Section 5 evaluates there;
  the dataset is not available here).
* ``kitti_batch`` -- 16 such pairs with per-pair seeds and mixed motion
  magnitudes (flow <= 64 for pairs 0..7, <= 256 for pairs 8..15).

Matcher parameters are plain dicts with the fields of ``sff_params``.
"""
from __future__ import annotations

from .scenes import SceneSpec, make_scene


def params_dict(H, W, C, levels, iters, rs_r0=32, rs_samples=6, fmax=32, dmax=32,
                tau=1):
    return dict(H=H, W=W, C=C, levels=levels, iters=iters, rs_r0=rs_r0,
                rs_samples=rs_samples, fmax=fmax, dmax=dmax, tau=tau)


def tiny_spec(seed: int = 1) -> SceneSpec:
    return SceneSpec(H=96, W=160, C=1, seed=seed, n_segments=(3, 3), d_range=(5, 30),
                     flow_max=20, delta_max=0, occluder=False, salt=0.0)


def tiny_params() -> dict:
    return params_dict(96, 160, 1, levels=1, iters=4, fmax=32, dmax=32, tau=1)


def kitti_spec(seed: int = 2, flow_max: int = 256) -> SceneSpec:
    return SceneSpec(H=375, W=1242, C=3, seed=seed, n_segments=(8, 20), d_range=(0, 192),
                     flow_max=flow_max, delta_max=4, occluder=True, salt=0.05)


def kitti_params() -> dict:
    return params_dict(375, 1242, 3, levels=3, iters=6, fmax=256, dmax=192, tau=1)


def kitti_batch_specs(n: int = 16, first_seed: int = 100):
    """Per-pair specs: the first half with flow <= 64, the rest <= 256."""
    return [kitti_spec(seed=first_seed + i, flow_max=64 if i < n // 2 else 256)
            for i in range(n)]


def sintel_spec(seed: int) -> SceneSpec:
    """1024x436 RGB pair shaped like MPI Sintel frames (Section 5 evaluates on
    Sintel; not available here): motions up to |u| <= 400, |v| <= 100 px with
    a heavy tail (|u| = 400 r^3), disparities up to 128 px and an occluder."""
    return SceneSpec(H=436, W=1024, C=3, seed=seed, n_segments=(8, 16), d_range=(0, 128),
                     flow_max=400, flow_max_v=100, flow_power=3.0, delta_max=4, occluder=True,
                     occluder_scale=0.8, salt=0.0)


def sintel_params() -> dict:
    return params_dict(436, 1024, 3, levels=3, iters=6, fmax=400, dmax=128, tau=1)


def sintel_sequence_specs(n_pairs: int = 49, first_seed: int = 600):
    """The 49 frame pairs of a 50-frame sequence, one seed each."""
    return [sintel_spec(first_seed + i) for i in range(n_pairs)]


def small_spec(H: int, W: int, C: int, seed: int, flow_max: int = 8,
               d_range=(0, 12), **kw) -> SceneSpec:
    """A small scene for tests whose oracle runs must finish in seconds."""
    return SceneSpec(H=H, W=W, C=C, seed=seed, n_segments=(2, 4), d_range=d_range,
                     flow_max=flow_max, **kw)


__all__ = ["SceneSpec", "make_scene", "params_dict", "tiny_spec", "tiny_params",
           "kitti_spec", "kitti_params", "kitti_batch_specs", "small_spec", "sintel_spec",
           "sintel_params", "sintel_sequence_specs"]
