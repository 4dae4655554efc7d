"""ORACLE -- TEST INFRASTRUCTURE ONLY.

Plain FP64 evaluation of the acoustic field from the surface potentials of a
solve, by the representation formulas of Sec. 2 (Eq. "representation"):

  interior:  p(x)   = [SLP_int psi_int](x) - [DLP_int phi_int](x)
  exterior:  u_s(x) = [SLP_ext psi_ext](x) - [DLP_ext phi_ext](x),
             p(x)   = u_inc(x) + u_s(x)

with [SLP psi](x) = int G(x, y) psi(y) dy, [DLP phi](x) = int dG/dn(y) phi(y) dy,
G = exp(i k r) / (4 pi r), r = |x - y|, outward normals, so that
dG/dn(y) = exp(i k r) (i k r - 1) ((y - x).n_y) / (4 pi r^3).

The densities are the P1 functions of the solve's nodal values.  Each
triangle integral is the 6-point rule of the regular assembly (weights summing
to one, times the area) -- the same discrete sum the device evaluates, with
no near-surface refinement, so points close to a mesh see the rule's
nearly-singular error in both.

Surface potentials of the multiple-traces unknowns [v_e, w_e, v_i, w_i] as
the system is printed (Sec. 3.3): p = -v and dp/dn = -w on each mesh, so
phi_ext = v_e and psi_ext = w_e (phi_ext = -gamma_D p, psi_ext = -gamma_N p,
Eq. "potentials:traces"), while phi_int = gamma_D p = -v_i and
psi_int = gamma_N p = -w_i.

winding(xyz, tri, x) is the sum over triangles of the signed solid angle
(Van Oosterom and Strackee, 1983) over 4 pi: 1 inside a closed outward mesh,
0 outside.  It decides which formula applies to a point.

Only tests, the smoke check and the CPU-baseline leg of the benchmark import
this module.
"""
import numpy as np

from oracle import oracle as _O


def _rule():
    bary, w = _O.rule6()
    return bary, w


def potentials(xyz, tri, k, phi, psi, points, chunk=256):
    """[SLP psi - DLP phi](x) at points [m][3] for P1 nodal phi, psi."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    phi = np.asarray(phi, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    bary, w = _rule()
    P = xyz[tri]                                   # [T][3 corners][3]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2.0 * area)[:, None]
    Y = np.einsum("qa,tac->tqc", bary, P)          # quadrature points [T][6][3]
    ph = np.einsum("qa,ta->tq", bary, phi[tri])    # densities at the points
    ps = np.einsum("qa,ta->tq", bary, psi[tri])
    W = area[:, None] * w[None, :]                 # [T][6]
    out = np.zeros(points.shape[0], dtype=np.complex128)
    for c0 in range(0, points.shape[0], chunk):
        x = points[c0:c0 + chunk]                  # [m][3]
        d = Y[None] - x[:, None, None, :]          # y - x, [m][T][6][3]
        r = np.sqrt(np.sum(d * d, axis=-1))
        e = np.exp(1j * k * r)
        G = e / (4.0 * np.pi * r)
        dn = np.einsum("mtqc,tc->mtq", d, n)
        dG = e * (1j * k * r - 1.0) * dn / (4.0 * np.pi * r ** 3)
        out[c0:c0 + chunk] = np.sum(W[None] * (G * ps[None] - dG * ph[None]), axis=(1, 2))
    return out


def solid_angles(xyz, tri, x):
    """Signed solid angle of every triangle seen from x, [T]."""
    P = np.asarray(xyz, dtype=np.float64)[np.asarray(tri)] - np.asarray(x, dtype=np.float64)[None, None, :]
    a, b, c = P[:, 0], P[:, 1], P[:, 2]
    la, lb, lc = (np.linalg.norm(v, axis=1) for v in (a, b, c))
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = la * lb * lc + np.einsum("ij,ij->i", a, b) * lc + np.einsum("ij,ij->i", a, c) * lb \
        + np.einsum("ij,ij->i", b, c) * la
    return 2.0 * np.arctan2(num, den)


def winding(xyz, tri, points):
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    return np.array([np.sum(solid_angles(xyz, tri, x)) / (4.0 * np.pi) for x in points])


def incident(k, d, points, kind=0):
    """The plane wave exp(i k d.x) (kind 0) or the point source
    exp(i k |x - d|) / (4 pi |x - d|) (kind 1) at points [m][3]."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    if kind == 0:
        return np.exp(1j * k * (points @ np.asarray(d, dtype=np.float64)))
    r = np.linalg.norm(points - np.asarray(d, dtype=np.float64)[None, :], axis=1)
    return np.exp(1j * k * r) / (4.0 * np.pi * r)


def mtf_field(ext_mesh, int_mesh, k_ext, k_int, x, d, points, region, kind=0):
    """Total field at points from the unknowns x = [v_e, w_e, v_i, w_i] of one
    incident field (kind 0: plane wave exp(i k_ext d.x); kind 1: point source
    at d); region[m] = 1 for interior points (interior formula), 0 for
    exterior ones (incident plus scattered field)."""
    ne, ni = len(ext_mesh[0]), len(int_mesh[0])
    x = np.asarray(x, dtype=np.complex128)
    v_e, w_e = x[:ne], x[ne:2 * ne]
    v_i, w_i = x[2 * ne:2 * ne + ni], x[2 * ne + ni:]
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    region = np.asarray(region)
    out = np.zeros(points.shape[0], dtype=np.complex128)
    ext = region == 0
    if ext.any():
        xe = points[ext]
        out[ext] = incident(k_ext, d, xe, kind) + potentials(*ext_mesh, k_ext, v_e, w_e, xe)
    if (~ext).any():
        out[~ext] = potentials(*int_mesh, k_int, -v_i, -w_i, points[~ext])
    return out
