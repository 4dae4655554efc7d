"""Penetrable unit-sphere (Mie) solution of the transmission problem, used as
an independent pin of the full solve.  Time convention exp(-i omega t), so the
scattered field uses spherical Hankel functions of the first kind.

Exterior total field on r = a = 1 (cos t = x.d):
  p(t)     = sum_n (2n+1) i^n [j_n(x_e) + a_n h_n(x_e)] P_n(cos t)
  dp+/dr   = k_e sum_n (2n+1) i^n [j_n'(x_e) + a_n h_n'(x_e)] P_n(cos t)
  dp-/dr   = (rho_int / rho_ext) dp+/dr         (flux condition)
  a_n = [g j_n'(x_i) j_n(x_e) - j_n(x_i) j_n'(x_e)] / [j_n(x_i) h_n'(x_e) - g j_n'(x_i) h_n(x_e)]
with x_e = k_e, x_i = k_i, g = (k_i rho_e) / (k_e rho_i).  These follow from
continuity of p and of (1/rho) dp/dr at r = 1.
"""
import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def _h(n, x, d=False):
    return spherical_jn(n, x, d) + 1j * spherical_yn(n, x, d)


def mie_traces(points, d, k_e, k_i, rho_e, rho_i, nmax=None):
    """Surface values p, dp+/dr, dp-/dr at unit-sphere points (radial normal)."""
    xe, xi = k_e, k_i
    if nmax is None:
        nmax = int(abs(xe) + 4 * abs(xe) ** (1 / 3) + 10 + abs(xi))
    g = (k_i * rho_e) / (k_e * rho_i)
    ct = np.clip(points @ d / np.linalg.norm(points, axis=1), -1, 1)
    p = np.zeros(points.shape[0], dtype=complex)
    dp = np.zeros_like(p)
    for n in range(nmax + 1):
        jn_e, jnp_e = spherical_jn(n, xe), spherical_jn(n, xe, True)
        jn_i, jnp_i = spherical_jn(n, xi), spherical_jn(n, xi, True)
        hn_e, hnp_e = _h(n, xe), _h(n, xe, True)
        an = (g * jnp_i * jn_e - jn_i * jnp_e) / (jn_i * hnp_e - g * jnp_i * hn_e)
        Pn = eval_legendre(n, ct)
        c = (2 * n + 1) * (1j ** n)
        p += c * (jn_e + an * hn_e) * Pn
        dp += c * k_e * (jnp_e + an * hnp_e) * Pn
    return p, dp, (rho_i / rho_e) * dp


def mie_field(points, d, k_e, k_i, rho_e, rho_i, nmax=None):
    """Total field off the unit sphere: outside (r > 1)
    sum_n (2n+1) i^n [j_n(k_e r) + a_n h_n(k_e r)] P_n(cos t), inside (r < 1)
    sum_n (2n+1) i^n b_n j_n(k_i r) P_n(cos t) with b_n j_n(x_i) = j_n(x_e) + a_n h_n(x_e)
    (continuity of p at r = 1)."""
    xe, xi = k_e, k_i
    if nmax is None:
        nmax = int(abs(xe) + 4 * abs(xe) ** (1 / 3) + 10 + abs(xi))
    g = (k_i * rho_e) / (k_e * rho_i)
    points = np.asarray(points, dtype=float)
    r = np.linalg.norm(points, axis=1)
    ct = np.clip(points @ d / r, -1, 1)
    out = np.zeros(points.shape[0], dtype=complex)
    inside = r < 1
    for n in range(nmax + 1):
        jn_e, jnp_e = spherical_jn(n, xe), spherical_jn(n, xe, True)
        jn_i, jnp_i = spherical_jn(n, xi), spherical_jn(n, xi, True)
        hn_e, hnp_e = _h(n, xe), _h(n, xe, True)
        an = (g * jnp_i * jn_e - jn_i * jnp_e) / (jn_i * hnp_e - g * jnp_i * hn_e)
        bn = (jn_e + an * hn_e) / jn_i
        Pn = eval_legendre(n, ct)
        c = (2 * n + 1) * (1j ** n)
        rad = np.where(inside, bn * spherical_jn(n, k_i * r), spherical_jn(n, k_e * r) + an * _h(n, k_e * r))
        out += c * rad * Pn
    return out
