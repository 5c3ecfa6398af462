"""Seeded synthetic inputs (surfaces, point clouds, linear systems).

This package produces the *inputs* of the multigrid pipeline only: point
positions, an edge array, the system matrix A and the right-hand side.  It
holds none of the multigrid method's arithmetic and is imported by both the
CPU oracle's tests and the GPU path's tests and benchmark, so that both sides
see exactly the same arrays.
"""
from .rng import mix64, uniform, normal
from .meshes import icosphere, torus_grid, flat_grid, bumpy_sphere_points, edges_from_faces, knn_edges
from .operators import cotan_laplacian, lumped_mass, gaussian_knn_laplacian, Problem
from .configs import (config_icosphere, config_torus, config_bumpy_sphere, config_adjoint, config_poisson, config_batched,
                      small_icosphere,
                      small_torus, small_flat_grid, small_pointcloud, small_hubs, CONFIGS)

__all__ = [
    "mix64", "uniform", "normal", "icosphere", "torus_grid", "flat_grid", "bumpy_sphere_points",
    "edges_from_faces", "knn_edges", "cotan_laplacian", "lumped_mass", "gaussian_knn_laplacian",
    "Problem", "config_icosphere", "config_torus", "config_bumpy_sphere", "config_adjoint", "config_poisson", "config_batched",
    "small_icosphere",
    "small_torus", "small_flat_grid", "small_pointcloud", "small_hubs", "CONFIGS",
]
