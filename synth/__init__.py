"""Seeded synthetic inputs for the SIPG Helmholtz operator.

This package only builds inputs: mesh vertex coordinates, element-to-vertex
connectivity, per-element polynomial orders, Helmholtz coefficients and random
coefficient vectors.  It holds none of the method's arithmetic (no bases, no
quadrature, no geometric factors) and is the one module that both the oracle
tests and the HIP path's tests and benchmark draw their inputs from.
"""

from .meshes import (
    Mesh,
    structured_mesh,
    rotate_elements,
    cube_rotations,
    num_dofs,
    random_coefficients,
    affine_mesh,
)
from .configs import (
    WORKLOADS,
    workload,
    small_mesh,
)

__all__ = [
    "Mesh",
    "structured_mesh",
    "rotate_elements",
    "cube_rotations",
    "num_dofs",
    "random_coefficients",
    "affine_mesh",
    "WORKLOADS",
    "workload",
    "small_mesh",
]
