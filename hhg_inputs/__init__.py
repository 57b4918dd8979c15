"""Seeded synthetic inputs shared by the product's tests/benchmarks and the oracle.

This package holds no arithmetic of the method: macro meshes (vertex
coordinates and tetrahedra), coefficient fields evaluated at given points, and
seeded random vectors.  Both the oracle and the GPU path consume what it
produces; neither side's code lives here.
"""
from .meshes import (unit_tet, regular_tet, flat_tet, kuhn_cube, kuhn_cube_2x2x2, cube12, MESHES,
                     obtuse_triangle, square_right4, square_nondelaunay8, MESHES2D)
from .fields import (smooth_k, cosine_k, lognormal_params, lognormal_k, lognormal_k_torch, sigmoid_k,
                     TENSOR_DIRS, tensor_K, tensor_fields, tensor_fields_torch,
                     polynomial_tensor_K, polynomial_tensor_fields_torch, affine_k, uniform_vector, manufactured_u, manufactured_f,
                     kuhn_cube_mass_rhs)

__all__ = ["unit_tet", "regular_tet", "flat_tet", "kuhn_cube", "kuhn_cube_2x2x2", "cube12", "MESHES",
           "obtuse_triangle", "square_right4", "square_nondelaunay8", "MESHES2D",
           "smooth_k", "cosine_k", "lognormal_params", "lognormal_k", "lognormal_k_torch", "sigmoid_k",
           "TENSOR_DIRS", "tensor_K", "tensor_fields", "tensor_fields_torch", "polynomial_tensor_K",
           "polynomial_tensor_fields_torch", "affine_k",
           "uniform_vector", "manufactured_u", "manufactured_f", "kuhn_cube_mass_rhs"]
