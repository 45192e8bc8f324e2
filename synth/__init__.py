"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This package holds no arithmetic of the method itself: it builds problem
descriptions (box, boundary kinds, sphere lists, parameters), initial density
fields and random numbers.  The lattice Boltzmann update, the voxelization of
spheres into solid nodes, the reductions and the drainage ramp live in the two
independent implementations (the FP64 CPU oracle and the HIP library).
"""
from .spec import Problem, BC_PERIODIC, BC_WALLS, BC_RESERVOIR
from .rng import splitmix64, uniform_pm
from .fields import layered_density, flat_interface_density, droplet_density
from .throats import (tetra_throat, c1_problem, c2_problem, throat_incircle, pc_ramp, GAMMA_LAPLACE,
                      small_throat_problem, three_sphere_throat, constriction_problem)
from .packing import (dense_packing, regular_triangulation, interior_facets, packing_throats,
                      packed_sample)
from .network import pore_network, pore_void_volume
from .membrane import membrane_sample

__all__ = [
    "Problem", "BC_PERIODIC", "BC_WALLS", "BC_RESERVOIR", "splitmix64", "uniform_pm",
    "layered_density", "flat_interface_density", "droplet_density", "tetra_throat",
    "c1_problem", "c2_problem", "small_throat_problem", "three_sphere_throat", "constriction_problem", "throat_incircle", "pc_ramp", "GAMMA_LAPLACE",
    "dense_packing", "regular_triangulation", "interior_facets", "packing_throats",
    "packed_sample", "pore_network", "pore_void_volume", "membrane_sample",
]
