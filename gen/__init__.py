"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package holds curve generators only: vertex coordinates and edge lists.
It contains none of the method's arithmetic (no energy, no operator, no
constraint), so that the oracle and the HIP path can both draw their inputs
from it without sharing any computation.
"""

from .curves import (  # noqa: F401
    trefoil,
    fourier_knot,
    regular_ngon,
    packing_instance,
    packing_batch,
    round_to_f32,
    loop_edges,
    theta_graph,
    tennis_ball,
    torus_knot,
    icosphere,
    torus_mesh,
    star_graph,
)
