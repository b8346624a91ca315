"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only *describes* inputs: which octree leaves exist (as treeIDs),
which finest-level cells are solid, the domain box with its face boundary
kinds, and analytic initial fields evaluated at caller-supplied positions.
It holds none of the method's arithmetic (no lattice, no equilibrium, no
interpolation, no neighbour search); both sides decode the treeIDs and build
everything else themselves.

treeID format (paper, Sec. 3.1 and the quadtree example figure): the root
element has id 0 at level 0; the first id at level L is
sum_{k<L} 2^(d*k); inside a level, ids follow the Morton (Z) order with the
x bit least significant, then y, then z.  Encoding lives here only to
produce inputs; each consumer has its own decoder.
"""
from .meshes import (MeshSpec, partition_example, refined_box_mesh,
                     half_refined_2d, sphere_channel_mesh, uniform_box_mesh,
                     plane_channel_mesh, plane_wall_links, sphere_wall_links,
                     two_level_channel_mesh)
from .fields import (tgv_fields, tgv_perturbed_fields, fourier_perturbation,
                     uniform_fields, shear_wave_fields)

__all__ = [
    "MeshSpec", "partition_example", "refined_box_mesh", "half_refined_2d",
    "sphere_channel_mesh", "uniform_box_mesh", "tgv_fields",
    "tgv_perturbed_fields", "fourier_perturbation", "uniform_fields",
    "plane_channel_mesh", "plane_wall_links", "sphere_wall_links",
    "shear_wave_fields", "two_level_channel_mesh",
]
