"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark: triangle meshes of closed star-shaped surfaces, plane-wave
directions and request streams.  This package holds no boundary-element
arithmetic: it only produces geometry and parameters."""
from .meshes import (icosphere, fibonacci_sphere, random_rotation, jitter_on_sphere,
                     scale_to_ellipsoid, mesh_check, mean_edge_length, orient_outward,
                     planar_square)
from .configs import (CONFIGS, make_config, make_pair, plane_wave_directions, serving_stream,  # noqa: F401
                      request_meshes, request_directions)
