"""Seeded synthetic inputs shared by the library caller and the test oracle.

This subpackage holds no arithmetic of the method itself: it builds meshes
(vertex coordinates and connectivity), reads stored cubature rules, evaluates
initial-condition functions at coordinates that the caller supplies, and
defines the workload recipes (mesh size, order, absorbing-layer profile,
source and probe parameters).  Everything the DG/PML method computes from these
inputs lives either in the HIP library or, independently, in the oracle.
"""
from .configs import (CONFIGS, column_for, config, gaussian_fields, load_rule, mesh_for, plane_pulse_fields,  # noqa: F401
                      product_rule)
from .mesh import kuhn_box, kuhn_grid, orient_positive  # noqa: F401
from .batch import batch_meshes, batch_recipe, concat_meshes  # noqa: F401
