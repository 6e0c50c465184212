"""Seeded synthetic inputs shared by the oracle and the GPU library's tests.

This package only produces geometry (triangle meshes), plane-wave angle sets and
the named workload definitions.  It contains none of the solver's arithmetic:
no basis functions, no integrals, no matrices.  Both the CPU oracle and the
HIP library receive its arrays as plain inputs.
"""

from .meshes import icosphere, geodesic_sphere, ellipsoid_mesh, flat_plate  # noqa: F401
from .configs import (WORKLOADS, BATCH_WORKLOADS, workload, batch_workload,  # noqa: F401
                      monostatic_angles, plane_wave_dirs)
