"""Seeded synthetic inputs for fractured-media pressure systems.

This package only draws and describes raw problem data (grid size, host
permeability field, fracture geometry and properties, boundary values,
source fields, random vectors).  It holds none of the discretisation or
solver arithmetic: both the plain CPU oracle and the GPU library build their
own matrices from what is returned here.
"""

from .scenarios import (  # noqa: F401
    Fracture,
    Scenario,
    grid_2d_four_lines,
    regular_3d,
    random_2d,
    random_3d,
    host_sources,
    random_vector,
    tiny_2d,
    tiny_3d,
)
