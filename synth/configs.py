"""The five benchmark workloads (C1..C5) as seeded recipes.

C1  tiny, FP64:   unit sphere; ext = icosphere L2 (320 tri, 162 nodes);
                  int = icosphere L2 rotated by a seeded rotation, jitter 1 %;
                  k_ext = 2, k_int = 4, rho_int/rho_ext = 1; d = +z; tol 1e-8.
C2  FP64 on GPU:  unit sphere; ext = icosphere L4 (5120 tri, 2562 nodes);
                  int = Fibonacci hull, 2002 nodes (4000 tri), rotated, jitter 2 %;
                  k_ext = 5, k_int = 8, rho ratio 1.5; one plane wave; tol 1e-6.
C3  precision:    ellipsoid (1.0, 0.8, 0.6); ext = icosphere L5 (20480 tri);
                  int = Fibonacci 8002 nodes (16000 tri), jitter 1 %;
                  k_ext = 10, k_int = 20, rho ratio 2.
C4  batching:     same ellipsoid; ext 10242 nodes; int Fibonacci 8000 nodes;
                  k_ext = 8, k_int = 12, rho ratio 2; 64 seeded directions.
C5  serving:      Poisson stream (mean 20 req/s) of random ellipsoids, see
                  ``serving_stream``.
"""
import numpy as np

from .meshes import (icosphere, fibonacci_sphere, random_rotation, jitter_on_sphere,
                     scale_to_ellipsoid, orient_outward)

CONFIGS = {
    "C1": dict(seed=1, ext_level=2, int_kind="ico", int_level=2, jitter=0.01,
               axes=(1.0, 1.0, 1.0), k_ext=2.0, k_int=4.0, rho_ext=1.0, rho_int=1.0,
               nrhs=1, tol=1e-8, dtype="c128"),
    "C2": dict(seed=2, ext_level=4, int_kind="fib", int_n=2002, jitter=0.02,
               axes=(1.0, 1.0, 1.0), k_ext=5.0, k_int=8.0, rho_ext=1.0, rho_int=1.5,
               nrhs=1, tol=1e-6, dtype="c128"),
    "C3": dict(seed=3, ext_level=5, int_kind="fib", int_n=8002, jitter=0.01,
               axes=(1.0, 0.8, 0.6), k_ext=10.0, k_int=20.0, rho_ext=1.0, rho_int=2.0,
               nrhs=1, tol=1e-6, dtype="c64"),
    "C4": dict(seed=4, ext_level=5, int_kind="fib", int_n=8000, jitter=0.01,
               axes=(1.0, 0.8, 0.6), k_ext=8.0, k_int=12.0, rho_ext=1.0, rho_int=2.0,
               nrhs=64, tol=1e-6, dtype="c64"),
}


def plane_wave_directions(n, rng):
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def make_pair(seed, ext_level, int_kind, jitter, axes, int_level=None, int_n=None):
    """Exterior icosphere and an independent, rotated, jittered interior grid."""
    rng = np.random.default_rng(seed)
    xe, te = icosphere(ext_level)
    if int_kind == "ico":
        xi, ti = icosphere(int_level)
    elif int_kind == "fib":
        xi, ti = fibonacci_sphere(int_n)
    else:
        raise ValueError(int_kind)
    R = random_rotation(rng)
    xi = xi @ R.T
    xi = jitter_on_sphere(xi, ti, jitter, rng)
    xe = scale_to_ellipsoid(xe, axes)
    xi = scale_to_ellipsoid(xi, axes)
    te = orient_outward(xe, te)
    ti = orient_outward(xi, ti)
    return (xe, te), (xi, ti), rng


def make_config(name):
    """Return a dict with meshes, physical parameters and plane-wave directions."""
    c = dict(CONFIGS[name])
    (xe, te), (xi, ti), rng = make_pair(c["seed"], c["ext_level"], c["int_kind"], c["jitter"],
                                        c["axes"], c.get("int_level"), c.get("int_n"))
    if c["nrhs"] == 1 and name in ("C1", "C2", "C3"):
        dirs = np.array([[0.0, 0.0, 1.0]]) if name == "C1" else plane_wave_directions(1, rng)
    else:
        dirs = plane_wave_directions(c["nrhs"], rng)
    c.update(ext=(xe, te), int=(xi, ti), dirs=dirs, name=name)
    return c


def serving_stream(n_requests=500, rate=20.0, seed=5):
    """C5: Poisson arrivals of transmission solves on random ellipsoids."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n_requests))
    reqs = []
    for r in range(n_requests):
        axes = rng.uniform(0.5, 1.5, 3)
        level = int(rng.integers(3, 6))
        ne = 10 * 4 ** level + 2
        ni = int(round(rng.uniform(0.7, 1.3) * ne))
        ke = rng.uniform(1.0, 15.0)
        ki = ke * rng.uniform(1.2, 2.5)
        nrhs = int(rng.integers(1, 17))
        reqs.append(dict(t_arrival=float(t[r]), axes=tuple(axes), ext_level=level, int_n=ni,
                         k_ext=ke, k_int=ki, rho_ext=1.0, rho_int=1.5, nrhs=nrhs,
                         seed=int(rng.integers(1 << 31))))
    return reqs


def request_meshes(req):
    """Exterior icosphere and independent interior Fibonacci grid of one
    serving request (ellipsoid with the request's semi-axes, 1 % jitter)."""
    (xe, te), (xi, ti), _ = make_pair(req["seed"], req["ext_level"], "fib", 0.01, req["axes"],
                                      int_n=req["int_n"])
    return (xe, te), (xi, ti)


def request_directions(req):
    """The request's plane-wave directions (seeded by the request)."""
    return plane_wave_directions(req["nrhs"], np.random.default_rng(req["seed"] + 1))

