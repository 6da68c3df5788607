"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds only input generation: media, right-hand sides, random
vectors and receiver masks.  It contains none of the solver's arithmetic
(no stencil, transfer, smoother or Krylov code), so both sides of every
parity test can draw identical inputs from it without sharing method code.
"""
from .media import (make_media, constant_media, linear_media, omega_for_ppw,
                    velocities_to_lame)
from .vectors import (random_field, point_source, lattice_sources,
                      receiver_plane_mask, zero_boundary_faces, plane_wave_field)

__all__ = ["make_media", "constant_media", "linear_media", "omega_for_ppw",
           "velocities_to_lame", "random_field", "point_source",
           "lattice_sources", "receiver_plane_mask", "zero_boundary_faces",
           "plane_wave_field"]
