"""Seeded synthetic bundle-adjustment scenes.

This package only *makes inputs*: camera rigs, scene points, visibility,
noisy pixel observations and perturbed initial estimates.  It holds none of
the solver's arithmetic; both the FP64 oracle (``oracle/``) and the GPU path
(``paper_1708_07954_amd``) consume what it produces and nothing else is shared
between them.
"""
from .generate import (  # noqa: F401
    Scene,
    make_config0,
    make_config1,
    make_config2,
    make_config3,
    make_ring_scene,
    make_sphere_scene,
    make_trajectory_scene,
    make_tiny_paper_scene,
    point_shard,
)
