"""Seeded synthetic inputs for the distributed radar imaging problem.

This package builds the *inputs* of the solver: sensor geometry, the
measurement operator A_q of the signal model (Sec. II, eq. (1)), target
scenes and noisy measurements y_q.  It holds none of the solver's
arithmetic (no ADMM step, no threshold, no factorisation, no pruning) and is
the only code shared by the FP64 oracle and the GPU engine's tests/bench.

Random numbers come from numpy's PCG64 (`numpy.random.default_rng(seed)`).
"""

from .geometry import Geometry, make_geometry, steering, SPEED_OF_LIGHT
from .scene import Scene, make_scene
from .configs import CONFIGS, config_geometry, config_scene

__all__ = [
    "Geometry", "make_geometry", "steering", "SPEED_OF_LIGHT",
    "Scene", "make_scene", "CONFIGS", "config_geometry", "config_scene",
]
