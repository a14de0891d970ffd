"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only *describes workloads*: lattice geometry (node tags, wall
links with their wall-crossing fraction q), inlet/outlet data, initial
macroscopic fields and triangulated capsule meshes with their material
parameters.  It contains none of the lattice-Boltzmann or immersed-boundary
arithmetic: every collision, boundary rule, interpolation or force is
implemented separately by the oracle and by the HIP library.

Every random draw uses ``numpy.random.default_rng(seed)`` (PCG64) in the
order documented by each generator.
"""
from .geometry import (FLUID, SOLID, INLET, OUTLET, D3Q19_DIRS, Domain,
                       periodic_box, pipe, bifurcation)
from .mesh import icosphere, Body
from .configs import (Workload, pipe_sphere, bifurcation_capsule,
                      precision_form, periodic_r0, pipe_r1, tiny_pipe,
                      tiny_bifurcation, facing_pair, batch_instance, batch_instances, get,
                      capsule_train, tiny_train, TRAIN_KINDS, outlet_flux_weights, terminal_weights)

__all__ = [
    "FLUID", "SOLID", "INLET", "OUTLET", "D3Q19_DIRS", "Domain",
    "periodic_box", "pipe", "bifurcation", "icosphere", "Body", "Workload", "facing_pair", "batch_instance",
    "pipe_sphere", "bifurcation_capsule", "precision_form", "periodic_r0",
    "pipe_r1", "tiny_pipe", "tiny_bifurcation", "batch_instances", "get", "capsule_train", "tiny_train",
    "TRAIN_KINDS", "outlet_flux_weights", "terminal_weights",
]
