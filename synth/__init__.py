"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package draws random numbers and lays them out; it holds none of the
renderer's arithmetic (no projection, no compositing, no sorting).
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    camera_look_at,
    camera_front,
    random_cameras,
    scene_uniform_cube,
    scene_clusters,
    request_stream,
    CONFIGS,
)
