"""Pins of the field-evaluation oracle (representation formulas of Sec. 2):
closed-form solid angles, brute-force triangle integrals, the winding number
of closed meshes, and the Mie series for the full solve followed by field
evaluation (conforming and nonconforming grids)."""
import numpy as np
import pytest

import synth
from mie import mie_field
from oracle import field as F


def _tri(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((3, 3)) * scale
    if np.dot(np.cross(P[1] - P[0], P[2] - P[0]), P.mean(axis=0)) < 0:
        P = P[[0, 2, 1]]
    return P, np.array([[0, 1, 2]])


def _far_points(P, dist, m, seed=1):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((m, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    diam = max(np.linalg.norm(P[i] - P[j]) for i in range(3) for j in range(3))
    return P.mean(axis=0) + dist * diam * u


def _brute(P, k, phi, psi, x, n=40):
    """The same triangle integrals by a Duffy-mapped n x n Gauss-Legendre rule
    (y = p0 + u (p1 - p0) + u v (p2 - p1), dy = 2 A u du dv)."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1); w = 0.5 * w
    U, V = np.meshgrid(g, g, indexing="ij"); WU, WV = np.meshgrid(w, w, indexing="ij")
    U, V, W = U.ravel(), V.ravel(), (WU * WV).ravel()
    lam = np.stack([1 - U, U * (1 - V), U * V], axis=1)
    Y = lam @ P
    cr = np.cross(P[1] - P[0], P[2] - P[0]); A2 = np.linalg.norm(cr); nrm = cr / A2
    jac = A2 * U * W
    out = []
    for xx in x:
        dv = Y - xx; r = np.linalg.norm(dv, axis=1); e = np.exp(1j * k * r)
        G = e / (4 * np.pi * r)
        dG = e * (1j * k * r - 1) * (dv @ nrm) / (4 * np.pi * r ** 3)
        out.append(np.sum(jac * (G * (lam @ psi) - dG * (lam @ phi))))
    return np.array(out)


def test_dlp_of_one_is_solid_angle():
    """k = 0, phi = 1: -[DLP 1](x) is the solid angle over 4 pi (Gauss); the
    6-point sum approaches the closed form as the point recedes."""
    P, T = _tri(3)
    errs = []
    for dist in (5.0, 10.0, 20.0):
        x = _far_points(P, dist, 16)
        q = F.potentials(P, T, 0.0, np.ones(3), np.zeros(3), x)
        ex = np.array([F.solid_angles(P, T, xx)[0] for xx in x]) / (4 * np.pi)
        assert np.max(np.abs(q.imag)) < 1e-18
        errs.append(np.max(np.abs(q.real - ex) / np.abs(ex)))
    assert errs[0] < 1e-3 and errs[2] < 2e-6 and errs[2] < errs[0] / 100, errs


@pytest.mark.parametrize("k", [0.0, 3.0])
def test_potentials_match_brute_force(k):
    """P1 densities, SLP and DLP together, against a 40 x 40 Duffy rule, on a
    triangle the 6-point rule resolves (k diam about 0.7; the rule's error
    is then set by the distance for k = 0 and by the phase across the
    triangle for k = 3, a few 1e-6 either way)."""
    P, T = _tri(5, scale=0.1)
    rng = np.random.default_rng(2)
    phi = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    psi = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    for dist, tol in ((4.0, 1e-5), (12.0, 1e-5)):
        x = _far_points(P, dist, 8, seed=4)
        q = F.potentials(P, T, k, phi, psi, x)
        b = _brute(P, k, phi, psi, x)
        assert np.max(np.abs(q - b)) / np.max(np.abs(b)) < tol, (dist, np.max(np.abs(q - b)) / np.max(np.abs(b)))
    # each density enters on its own: SLP alone and DLP alone
    x = _far_points(P, 12.0, 4, seed=6)
    for ph, ps in ((np.zeros(3), psi), (phi, np.zeros(3))):
        q = F.potentials(P, T, k, ph, ps, x); b = _brute(P, k, ph, ps, x)
        assert np.max(np.abs(q - b)) / np.max(np.abs(b)) < 1e-5


def test_winding_of_closed_meshes():
    """Sum of solid angles over 4 pi: 1 inside, 0 outside, for both meshes of
    a nonconforming pair (any closed outward polyhedron)."""
    (xe, te), (xi, ti), _ = synth.configs.make_pair(3, 2, "fib", 0.02, (1.0, 0.8, 0.6), int_n=200)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((20, 3)); u /= np.linalg.norm(u, axis=1)[:, None]
    inner = 0.4 * u * np.array([1.0, 0.8, 0.6])
    outer = 1.6 * u
    for X, Tm in ((xe, te), (xi, ti)):
        assert np.max(np.abs(F.winding(X, Tm, inner) - 1)) < 1e-12
        assert np.max(np.abs(F.winding(X, Tm, outer))) < 1e-12
        assert abs(F.winding(X, Tm, [[0.0, 0.0, 0.0]])[0] - 1) < 1e-12


def test_constant_densities_on_a_closed_mesh():
    """k = 0 on the unit icosphere: -[DLP 1] = 1 inside and 0 outside (the
    6-point sums of all triangles, away from the surface), and the single
    layer of psi = 1 is 1 inside, 1/|x| outside, to the O(h^2) of the
    polyhedral surface."""
    (xe, te), _, _ = synth.configs.make_pair(1, 4, "ico", 0.0, (1, 1, 1), int_level=1)
    nv = len(xe)
    xin = np.array([[0.0, 0.0, 0.0], [0.2, -0.1, 0.3]])
    xout = np.array([[3.0, 0.0, 0.0], [0.0, -2.5, 1.0]])
    d_in = F.potentials(xe, te, 0.0, np.ones(nv), np.zeros(nv), xin)
    d_out = F.potentials(xe, te, 0.0, np.ones(nv), np.zeros(nv), xout)
    assert np.max(np.abs(d_in - 1)) < 1e-5 and np.max(np.abs(d_out)) < 1e-5
    s_in = F.potentials(xe, te, 0.0, np.zeros(nv), np.ones(nv), xin)
    s_out = F.potentials(xe, te, 0.0, np.zeros(nv), np.ones(nv), xout)
    assert np.max(np.abs(s_in - 1)) < 5e-3
    assert np.max(np.abs(s_out - 1 / np.linalg.norm(xout, axis=1))) < 5e-3


def test_field_converges_to_mie(orc):
    """Discrete MTF solve, then the field off the surface by the representation
    formulas: O(h^2) towards the penetrable-sphere series inside and outside,
    for independent interior and exterior grids.  A wrong sign on either
    potential or on the interior unknowns leaves an O(1) error."""
    ke, ki, re, ri = 2.0, 3.0, 1.0, 1.5
    d = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(3)
    u = rng.standard_normal((12, 3)); u /= np.linalg.norm(u, axis=1)[:, None]
    pts = np.concatenate([0.5 * u, 1.8 * u])
    region = np.array([1] * 12 + [0] * 12)
    ref = mie_field(pts, d, ke, ki, re, ri)
    errs = []
    for L in (1, 2, 3):
        (xe, te), (xi, ti), _ = synth.configs.make_pair(7, L, "ico", 0.01, (1, 1, 1), int_level=L)
        X, _ = orc.solve_mtf((xe, te), (xi, ti), ke, ki, re, ri, d)
        f = F.mtf_field((xe, te), (xi, ti), ke, ki, X[0], d, pts, region)
        errs.append([np.linalg.norm(f[:12] - ref[:12]) / np.linalg.norm(ref[:12]),
                     np.linalg.norm(f[12:] - ref[12:]) / np.linalg.norm(ref[12:])])
    errs = np.array(errs)
    assert np.all(errs[1] < errs[0] / 2.5) and np.all(errs[2] < errs[1] / 2.5), errs
    assert np.all(errs[2] < 0.01), errs


def test_field_of_transparent_body(orc):
    """k_int = k_ext, equal densities: the field is the incident wave inside
    and outside, to the discretisation error."""
    k = 1.5
    d = np.array([0.6, 0.0, 0.8])
    (xe, te), (xi, ti), _ = synth.configs.make_pair(8, 3, "fib", 0.02, (1, 1, 1), int_n=500)
    X, _ = orc.solve_mtf((xe, te), (xi, ti), k, k, 1.0, 1.0, d)
    pts = np.array([[0.1, 0.2, -0.3], [0.0, 0.0, 0.4], [2.0, 0.5, 0.0], [-1.0, 1.5, 1.0]])
    f = F.mtf_field((xe, te), (xi, ti), k, k, X[0], d, pts, np.array([1, 1, 0, 0]))
    inc = np.exp(1j * k * pts @ d)
    assert np.max(np.abs(f - inc)) < 0.02, np.abs(f - inc)


def test_absorbing_interior_field_converges_to_mie(orc):
    """Absorbing interior (k_int = 3 + 0.6 i, Sec. 5.7): the field off the
    surface converges at O(h^2) to the penetrable-sphere series evaluated with
    the complex wavenumber, inside (where the interior potentials carry
    exp(i k r) with the complex k) and outside."""
    ke, ki, re, ri = 2.0, 3.0 + 0.6j, 1.0, 1.5
    d = np.array([0.0, 0.0, 1.0])
    rng = np.random.default_rng(5)
    u = rng.standard_normal((12, 3)); u /= np.linalg.norm(u, axis=1)[:, None]
    pts = np.concatenate([0.5 * u, 1.8 * u])
    region = np.array([1] * 12 + [0] * 12)
    ref = mie_field(pts, d, ke, ki, re, ri)
    errs = []
    for L in (1, 2, 3):
        (xe, te), (xi, ti), _ = synth.configs.make_pair(7, L, "ico", 0.01, (1, 1, 1), int_level=L)
        X, _ = orc.solve_mtf((xe, te), (xi, ti), ke, ki, re, ri, d)
        f = F.mtf_field((xe, te), (xi, ti), ke, ki, X[0], d, pts, region)
        errs.append([np.linalg.norm(f[:12] - ref[:12]) / np.linalg.norm(ref[:12]),
                     np.linalg.norm(f[12:] - ref[12:]) / np.linalg.norm(ref[12:])])
    errs = np.array(errs)
    assert np.all(errs[1] < errs[0] / 2.5) and np.all(errs[2] < errs[1] / 2.5), errs
    assert np.all(errs[2] < 0.01), errs
