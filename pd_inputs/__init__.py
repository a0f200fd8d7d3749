"""Seeded synthetic inputs for the linearized OSB-PD explicit solver.

This package builds node lattices, boundary-condition flags, nodal external
forces, notch descriptions and material tables for the five workloads the
solver is exercised on (a 3D cantilever, a 2D edge-notched plate, a 3D
double-notched plate under edge impact, a 3D notched cylinder under torsion,
and a batch of 256 random 2D plates).

It holds none of the peridynamic arithmetic: no horizon search, no bond
geometry, no critical stretch, no force.  Quantities that do depend on that
arithmetic (the stable time step of each specimen and the end-twist rate of
the cylinder, which is scaled by the critical stretch) are plain input
parameters read from ``params.json``; that file is written by a script that
calls only the CPU reference implementation.

Both the GPU library's tests and the CPU reference take their inputs from
here, so the two sides see bit-identical inputs.
"""

from .workloads import (  # noqa: F401
    Material,
    Cut,
    Workload,
    cantilever3d,
    plate2d,
    impact3d,
    cylinder3d,
    batch2d,
    workload,
    WORKLOAD_NAMES,
    load_params,
)
