"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark."""
from .scenes import (CONFIGS, Camera, SceneConfig, make_cameras, make_scene,  # noqa: F401
                     make_targets, make_workload, look_at_camera, custom_scene,
                     subset_scene, cmlp_param_count, XI_DIM)
