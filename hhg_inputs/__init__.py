"""Seeded synthetic inputs shared by the product's tests/benchmarks and the oracle.

This package holds no arithmetic of the method: macro meshes (vertex
coordinates and tetrahedra), coefficient fields evaluated at given points, and
seeded random vectors.  Both the oracle and the GPU path consume what it
produces; neither side's code lives here.
"""
from .meshes import (unit_tet, regular_tet, flat_tet, kuhn_cube, kuhn_cube_2x2x2, cube12, MESHES,
                     kuhn_box, cylinder_reference_box, CYLINDER_BOX,
                     obtuse_triangle, square_right4, square_nondelaunay8, MESHES2D)
from .fields import (smooth_k, cosine_k, lognormal_params, lognormal_k, lognormal_k_torch, sigmoid_k,
                     TENSOR_DIRS, tensor_K, tensor_fields, tensor_fields_torch,
                     polynomial_tensor_K, polynomial_tensor_fields_torch, affine_k, uniform_vector, manufactured_u, manufactured_f,
                     kuhn_cube_mass_rhs, kuhn_box_mass_rhs, cylinder_warp, cylinder_mapping_K,
                     cylinder_phi, cylinder_phi_inverse, cylinder_tensor, cylinder_tensor_fields_torch,
                     cylinder_u, cylinder_f)

__all__ = ["unit_tet", "regular_tet", "flat_tet", "kuhn_cube", "kuhn_cube_2x2x2", "cube12", "MESHES",
           "obtuse_triangle", "square_right4", "square_nondelaunay8", "MESHES2D",
           "smooth_k", "cosine_k", "lognormal_params", "lognormal_k", "lognormal_k_torch", "sigmoid_k",
           "TENSOR_DIRS", "tensor_K", "tensor_fields", "tensor_fields_torch", "polynomial_tensor_K",
           "polynomial_tensor_fields_torch", "affine_k",
           "uniform_vector", "manufactured_u", "manufactured_f", "kuhn_cube_mass_rhs",
           "kuhn_box", "cylinder_reference_box", "CYLINDER_BOX", "kuhn_box_mass_rhs", "cylinder_warp",
           "cylinder_mapping_K", "cylinder_phi", "cylinder_phi_inverse", "cylinder_tensor",
           "cylinder_tensor_fields_torch", "cylinder_u", "cylinder_f"]
