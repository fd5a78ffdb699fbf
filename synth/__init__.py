"""Seeded synthetic inputs for the splatting path (driving scenes, rigs, trajectories).

This package only draws numbers: it holds none of the rendering, projection or
pose arithmetic. Both the CPU oracle tests and the GPU path are fed from it.
"""
from .scenes import *  # noqa: F401,F403
