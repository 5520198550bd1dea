"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the oracle.

This package only draws random numbers and places cameras. It contains none of
the rendering arithmetic (no projection, colour, sorting or blending), so that
the two implementations it feeds stay independent of each other.
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    ball_scene,
    cluster_scene,
    crop_camera,
    look_at,
    orbit_cameras,
    sampled_orbit_poses,
    perturbed_scene,
    sphere_cameras,
    hp_membership,
    reorder_segments,
    HPLayout,
)
from .configs import config  # noqa: F401
