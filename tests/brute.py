"""Independent brute-force element integrals for the oracle pins.

    I_ab = int_tau int_sigma  phi_a(x) kern(x, y) phi_b(y)  dy dx

The inner integral over sigma is done in polar coordinates centred at the
orthogonal projection c of x onto the plane of sigma (signed sub-triangles
(c, v_m, v_m+1)), with the radial substitution rho = h sinh(u) when x is off
the plane (h > 0) so that 1/r and h/r^3 become smooth.  The outer integral
over tau is a composite collapsed-square Gauss rule on a uniform refinement.
Kernels: 'V' = G, 'K' = dG/dn_y, 'T' = dG/dn_x, and the double-layer is
checked through finite differences of G along the normals (no analytic
derivative is used).  Nothing here is shared with the oracle.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss


def _gl01(n):
    x, w = leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _subdivide(P, m):
    tris = [np.asarray(P, dtype=float)]
    for _ in range(m):
        nt = []
        for A, B, C in tris:
            ab, bc, ca = (A + B) / 2, (B + C) / 2, (C + A) / 2
            nt += [np.array([A, ab, ca]), np.array([ab, B, bc]), np.array([ca, bc, C]), np.array([ab, bc, ca])]
        tris = nt
    return tris


def _graded_edge(A, B, C, n, q):
    """Rule on triangle (A,B,C) graded towards edge AB: x = (1-w)(A + v(B-A)) + w C,
    w = z^q."""
    x, w = _gl01(n)
    V, Z = np.meshgrid(x, x, indexing="ij")
    WV, WZ = np.meshgrid(w, w, indexing="ij")
    v = V.ravel(); z = Z.ravel()
    ww = q * z ** (q - 1)
    wz = z ** q
    area2 = np.linalg.norm(np.cross(B - A, C - A))
    pts = (1 - wz)[:, None] * (A + v[:, None] * (B - A)) + wz[:, None] * C
    wts = (WV * WZ).ravel() * ww * (1 - wz) * area2
    return pts, wts


def _graded_vertex(A, B, C, n, q):
    """Rule on triangle (A,B,C) graded towards vertex A: x = A + w((1-v)B + vC - A), w = z^q."""
    x, w = _gl01(n)
    V, Z = np.meshgrid(x, x, indexing="ij")
    WV, WZ = np.meshgrid(w, w, indexing="ij")
    v = V.ravel(); z = Z.ravel()
    wz = z ** q
    area2 = np.linalg.norm(np.cross(B - A, C - A))
    pts = A + wz[:, None] * ((1 - v)[:, None] * B + v[:, None] * C - A)
    wts = (WV * WZ).ravel() * q * z ** (q - 1) * wz * area2
    return pts, wts


def outer_points(P, kind, n, q=3, shared=None):
    """Outer rule on P (3x3) graded towards the set where the inner integral is
    not smooth: 'coinc' -> all edges (centroid split), 'edge' -> the edge
    P[0]P[1], 'vertex' -> P[0], 'regular' -> plain collapsed Gauss."""
    P = np.asarray(P, dtype=float)
    if kind == "coinc":
        g = P.mean(axis=0)
        parts = [_graded_edge(P[m], P[(m + 1) % 3], g, n, q) for m in range(3)]
        return np.concatenate([p for p, _ in parts]), np.concatenate([w for _, w in parts])
    if kind == "edge":
        return _graded_edge(P[0], P[1], P[2], n, q)
    if kind == "vertex":
        return _graded_vertex(P[0], P[1], P[2], n, q)
    return _graded_edge(P[0], P[1], P[2], n, 1)


def barycentric(P, x):
    A, B, C = P
    n = np.cross(B - A, C - A)
    nn = n @ n
    l1 = np.cross(x - A, C - A) @ n / nn
    l2 = np.cross(B - A, x - A) @ n / nn
    return np.stack([1 - l1 - l2, l1, l2], axis=-1)


def inner_integral(x, S, k, nth=24, nr=24):
    """For each point x (M,3): int_S G(x,y) phi_b(y) dy and
    int_S dG/dn_y phi_b(y) dy, b = 0..2.  Returns (M,3) complex arrays.

    Polar coordinates around the projection c of x on the plane of S, one
    signed sub-triangle (c, v_m, v_m+1) per edge.  On each, the angle is
    parametrised by the edge coordinate t measured from the foot point of c,
    t = delta sinh(v) (delta = distance of c to the edge line), which makes
    thin sub-triangles harmless; the radius uses rho = h sinh(u) when x is
    off the plane (h > 0), which makes 1/r and h/r^3 smooth."""
    S = np.asarray(S, dtype=float)
    n = np.cross(S[1] - S[0], S[2] - S[0]); n /= np.linalg.norm(n)
    h = (x - S[0]) @ n
    c = x - h[:, None] * n
    ah = np.abs(h)
    tx, tw = _gl01(nth); rx, rw = _gl01(nr)
    JV = np.zeros((x.shape[0], 3), dtype=complex)
    JK = np.zeros_like(JV)
    for m in range(3):
        a, b = S[m], S[(m + 1) % 3]
        L = np.linalg.norm(b - a)
        eh = (b - a) / L
        ta = (a - c) @ eh                        # edge coordinate of a from the foot point
        tb = ta + L
        f = a - ta[:, None] * eh                 # foot point of c on the edge line
        dsg = np.cross(a - c, b - a) @ n / L     # signed distance (CCW positive)
        dl = np.abs(dsg)
        ok = dl > 1e-14 * L
        dls = np.where(ok, dl, 1.0)
        va, vb = np.arcsinh(ta / dls), np.arcsinh(tb / dls)
        sgn = np.sign(dsg)
        for ti, twi in zip(tx, tw):
            v = va + ti * (vb - va)
            t = dls * np.sinh(v)
            e = f + t[:, None] * eh
            R = dls * np.cosh(v)
            dirv = (e - c) / R[:, None]
            dth = sgn / np.cosh(v) * (vb - va) * twi       # d(theta)
            off = ah > 1e-13 * (1 + R)
            Umax = np.where(off, np.arcsinh(R / np.where(off, ah, 1)), 1.0)
            for ri, rwi in zip(rx, rw):
                uu = ri * Umax
                rho = np.where(off, ah * np.sinh(uu), R * ri)
                drho = np.where(off, ah * np.cosh(uu) * Umax, R) * rwi
                y = c + rho[:, None] * dirv
                r = np.sqrt(ah ** 2 + rho ** 2)
                G = np.exp(1j * k * r) / (4 * np.pi * r)
                dGn = G * (1j * k * r - 1) / r ** 2 * ((y - x) @ n)
                wgt = np.where(ok, rho * drho * dth, 0.0)
                ph = barycentric(S, y)
                JV += (wgt * G)[:, None] * ph
                JK += (wgt * dGn)[:, None] * ph
    return JV, JK


def element_blocks(Ptau, Psig, k, kind, n=24, q=3, nth=24, nr=24):
    """Brute-force V and K element blocks [a][b] (a on tau, b on sigma).  For
    kind 'edge' the shared edge must be Ptau[0]Ptau[1]; for 'vertex' the
    shared vertex must be Ptau[0]."""
    X, W = outer_points(Ptau, kind, n, q)
    JV, JK = inner_integral(X, Psig, k, nth, nr)
    ph = barycentric(np.asarray(Ptau, float), X)
    V = (ph * W[:, None]).T @ JV
    K = (ph * W[:, None]).T @ JK
    return V, K
