"""ORACLE -- TEST INFRASTRUCTURE ONLY.

Python side of the plain FP64 reference for the nonconforming multiple-traces
boundary element method (van 't Wout, "The Boundary Element Method for
Acoustic Transmission with Nonconforming Grids").  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark import this module; the
product library never does.  It shares no code with the GPU path.

Element integrals and the mortar matrix come from ``bem_oracle.c`` (plain C,
ordered-pair loops).  Everything else is written here with numpy/scipy
primitives and no blocking or reordering:

  mass(xyz, tri)          M[i][j] = <phi_i, phi_j>  (Sec. 3.1)
  plane_wave_rhs(...)     f_j = <u_inc, phi_j>, g_j = <d_n u_inc, phi_j>
                          with u_inc = exp(i k d.x)  (plane wave, Sec. 5.3)
  point_source_rhs(...)   the same for u_inc = exp(i k r) / (4 pi r),
                          r = |x - x0|  (point source, Sec. 5.7)
  mtf_system(...)         the discrete multiple-traces system as printed in
                          Sec. 3.3, with right-hand side [-f, -g, 0, 0]
  solve_mtf(...)          x = A^{-1} b by dense LU: GMRES on the mass-
                          preconditioned (strong) form M^{-1} A x = M^{-1} b
                          reaches exactly this solution (Sec. 3.3, 5.1)
  solve_mtf_inplace(...)  the same solution for systems of tens of thousands
                          of unknowns: the block matrix is filled in place,
                          operator rows a chunk at a time, and factorised in
                          place (no second copy of the matrix)
  pmchwt_system(...)      the exterior PMCHWT matrix as printed in Sec. 3.3,
                          interior operators scaled as in the single-trace
                          Calderon system of Sec. 2.2
  solve_pmchwt(...)       its exact discrete solution by dense LU
  high_contrast_neumann_system(...), solve_high_contrast_neumann(...)
                          the exterior high-contrast Neumann formulation
                          (indirect single-layer representation outside)
  projection_error(...)   E_int, E_ext of Sec. 5.2
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the C part of the oracle (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        p, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.orc_assemble_rows.argtypes = [i64, p, i64, p, d, d, i32, i32, i64, p, p, p, p, p]
        L.orc_assemble_rows.restype = i32
        L.orc_mortar_rows.argtypes = [i64, p, i64, p, i64, p, i64, p, i32, p, i64, p, p]
        L.orc_mortar_rows.restype = i32
        L.orc_plane_wave_rhs.argtypes = [i64, p, i64, p, d, d, p, p, p]
        L.orc_plane_wave_rhs.restype = i32
        L.orc_pair_blocks.argtypes = [p, p, i64, i64, d, d, i32, p]
        L.orc_rule6.argtypes = [p, p]
        L.orc_gauss01.argtypes = [i32, p, p]
        L.orc_ss_poly.argtypes = [i32, i32, i32, i32, i32, i32]
        L.orc_ss_poly.restype = d
        L.orc_set_threads.argtypes = [i32]
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP threads of the C loops (for timing at one thread and at all)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _mesh(xyz, tri):
    return (np.ascontiguousarray(xyz, dtype=np.float64),
            np.ascontiguousarray(tri, dtype=np.int32))


def rule6():
    b = np.zeros((6, 3)); w = np.zeros(6)
    lib().orc_rule6(_ptr(b), _ptr(w))
    return b, w


def gauss01(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().orc_gauss01(n, _ptr(x), _ptr(w))
    return x, w


def ss_poly(kind, ng, a, b, c, d):
    """Integral of x1^a x2^b y1^c y2^d over {0<=x2<=x1<=1}^2 via the singular
    rule's regions; kind = number of shared vertices."""
    return lib().orc_ss_poly(int(kind), int(ng), a, b, c, d)


def pair_blocks(xyz, tri, t, s, k, ng=4):
    """Element blocks [op][a][b] (op = V, K, T, D) of the ordered pair (t, s)."""
    xyz, tri = _mesh(xyz, tri)
    out = np.zeros((4, 3, 3), dtype=np.complex128)
    lib().orc_pair_blocks(_ptr(xyz), _ptr(tri), int(t), int(s), float(np.real(k)),
                          float(np.imag(k)), int(ng), _ptr(out))
    return out


def assemble(xyz, tri, k, ng=4, which=3, rows=None, ops="VKTD"):
    """Dense Galerkin matrices V, K, T, D (rows = test vertices).  Returns a
    dict op -> complex128 [len(rows), nv].  which: 1 regular pairs only,
    2 singular pairs only, 3 all."""
    xyz, tri = _mesh(xyz, tri)
    nv = xyz.shape[0]
    rows = np.arange(nv, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    out = {o: np.zeros((rows.size, nv), dtype=np.complex128) for o in ops}
    ptrs = [(_ptr(out[o]) if o in out else None) for o in "VKTD"]
    rc = lib().orc_assemble_rows(nv, _ptr(xyz), tri.shape[0], _ptr(tri), float(np.real(k)),
                                 float(np.imag(k)), int(ng), int(which), rows.size, _ptr(rows), *ptrs)
    if rc != 0:
        raise ValueError("orc_assemble_rows failed")
    return out


def mortar(int_mesh, ext_mesh, mode=0, centre=(0.0, 0.0, 0.0), rows=None):
    """Dense mortar matrix P_int,ext [N_int, N_ext] (or selected rows)."""
    xi, ti = _mesh(*int_mesh)
    xe, te = _mesh(*ext_mesh)
    rows = (np.arange(xi.shape[0], dtype=np.int64) if rows is None
            else np.ascontiguousarray(rows, dtype=np.int64))
    P = np.zeros((rows.size, xe.shape[0]))
    c = np.ascontiguousarray(centre, dtype=np.float64)
    rc = lib().orc_mortar_rows(xi.shape[0], _ptr(xi), ti.shape[0], _ptr(ti), xe.shape[0], _ptr(xe),
                               te.shape[0], _ptr(te), int(mode), _ptr(c), rows.size, _ptr(rows), _ptr(P))
    if rc != 0:
        raise ValueError("orc_mortar_rows failed")
    return P


def mass(xyz, tri):
    """Dense P1 mass matrix: element matrix (A/12) [[2,1,1],[1,2,1],[1,1,2]]."""
    xyz, tri = _mesh(xyz, tri)
    nv = xyz.shape[0]
    M = np.zeros((nv, nv))
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(p1 - p0, p2 - p0), axis=1)
    for t in range(tri.shape[0]):
        for a in range(3):
            for b in range(3):
                M[tri[t, a], tri[t, b]] += area[t] / 12.0 * (2.0 if a == b else 1.0)
    return M


def plane_wave_rhs(xyz, tri, k, d):
    xyz, tri = _mesh(xyz, tri)
    d = np.ascontiguousarray(d, dtype=np.float64)
    f = np.zeros(xyz.shape[0], dtype=np.complex128)
    g = np.zeros(xyz.shape[0], dtype=np.complex128)
    lib().orc_plane_wave_rhs(xyz.shape[0], _ptr(xyz), tri.shape[0], _ptr(tri), float(np.real(k)),
                             float(np.imag(k)), _ptr(d), _ptr(f), _ptr(g))
    return f, g


def point_source_rhs(xyz, tri, k, x0):
    """f_j = <u_inc, phi_j>, g_j = <d_n u_inc, phi_j> for the point source
    u_inc(x) = exp(i k |x - x0|) / (4 pi |x - x0|) (Sec. 5.7), with
    d_n u_inc = exp(i k r)(i k r - 1)((x - x0).n) / (4 pi r^3); every
    triangle by the 6-point rule (area times the weights)."""
    xyz, tri = _mesh(xyz, tri)
    bary, w = rule6()
    P = xyz[tri]
    cr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2.0 * area)[:, None]
    Y = np.einsum("qa,tac->tqc", bary, P)
    R = Y - np.asarray(x0, dtype=np.float64)[None, None, :]
    r = np.linalg.norm(R, axis=2)
    e = np.exp(1j * k * r) / (4.0 * np.pi * r)
    du = e * (1j * k * r - 1.0) * np.einsum("tqc,tc->tq", R, n) / r ** 2
    f = np.zeros(xyz.shape[0], dtype=np.complex128)
    g = np.zeros(xyz.shape[0], dtype=np.complex128)
    for a in range(3):
        wa = area[:, None] * w[None, :] * bary[None, :, a]
        np.add.at(f, tri[:, a], np.sum(wa * e, axis=1))
        np.add.at(g, tri[:, a], np.sum(wa * du, axis=1))
    return f, g


def operators(ext_mesh, int_mesh, k_ext, k_int, ng=4):
    """All dense operators and sparse couplings of the multiple-traces system."""
    Oe = assemble(*ext_mesh, k_ext, ng=ng)
    Oi = assemble(*int_mesh, k_int, ng=ng)
    P_ie = mortar(int_mesh, ext_mesh)
    return dict(ext=Oe, int=Oi, P_ie=P_ie, M_e=mass(*ext_mesh), M_i=mass(*int_mesh))


def mtf_system(ops, rho_ext, rho_int):
    """The weak-form multiple-traces block matrix, signs as printed:
        [ -K_e   V_e    1/2 P_ei              0                 ]
        [  D_e   T_e    0                    1/2 (re/ri) P_ei   ]
        [ -1/2 P_ie     0      -K_i          V_i                ]
        [  0  -1/2 (ri/re) P_ie  D_i         T_i                ]
    with P_ei = P_ie^T; unknowns [v_ext, w_ext, v_int, w_int]."""
    Oe, Oi, P_ie = ops["ext"], ops["int"], ops["P_ie"]
    ne, ni = Oe["V"].shape[0], Oi["V"].shape[0]
    P_ei = P_ie.T
    Z = np.zeros
    A = np.block([
        [-Oe["K"], Oe["V"], 0.5 * P_ei, Z((ne, ni))],
        [Oe["D"], Oe["T"], Z((ne, ni)), 0.5 * (rho_ext / rho_int) * P_ei],
        [-0.5 * P_ie, Z((ni, ne)), -Oi["K"], Oi["V"]],
        [Z((ni, ne)), -0.5 * (rho_int / rho_ext) * P_ie, Oi["D"], Oi["T"]],
    ])
    return A


def mtf_rhs(ext_mesh, k_ext, d, n_int, incident=0):
    """[-f, -g, 0, 0] for the plane wave of direction d (incident 0) or the
    point source at d (incident 1)."""
    f, g = plane_wave_rhs(*ext_mesh, k_ext, d) if incident == 0 else point_source_rhs(*ext_mesh, k_ext, d)
    return np.concatenate([-f, -g, np.zeros(2 * n_int, dtype=np.complex128)])


def block_mass(ops):
    Me, Mi = ops["M_e"], ops["M_i"]
    ne, ni = Me.shape[0], Mi.shape[0]
    M = np.zeros((2 * ne + 2 * ni,) * 2)
    M[:ne, :ne] = Me
    M[ne:2 * ne, ne:2 * ne] = Me
    M[2 * ne:2 * ne + ni, 2 * ne:2 * ne + ni] = Mi
    M[2 * ne + ni:, 2 * ne + ni:] = Mi
    return M


def strong_matvec(A, M, x):
    """z = M^{-1} A x (mass-matrix preconditioned form, Sec. 3.3)."""
    return np.linalg.solve(M, A @ x)


def solve_mtf(ext_mesh, int_mesh, k_ext, k_int, rho_ext, rho_int, dirs, ng=4, ops=None, incident=0):
    """Exact discrete MTF solution(s) by dense LU; returns (x [nrhs, n], ops).
    dirs: plane-wave directions (incident 0) or point-source positions (1)."""
    if ops is None:
        ops = operators(ext_mesh, int_mesh, k_ext, k_int, ng=ng)
    A = mtf_system(ops, rho_ext, rho_int)
    ni = ops["M_i"].shape[0]
    B = np.stack([mtf_rhs(ext_mesh, k_ext, d, ni, incident) for d in np.atleast_2d(dirs)], axis=1)
    X = np.linalg.solve(A, B)
    return X.T, ops


def solve_mtf_inplace(ext_mesh, int_mesh, k_ext, k_int, rho_ext, rho_int, dirs, ng=4, chunk=512,
                      incident=0, log=None):
    """Exact discrete MTF solution(s) by dense LU, as solve_mtf, for systems
    whose operators and block matrix do not fit in memory side by side
    (36,488 unknowns: 21.3 GB for the matrix alone).  The matrix of
    mtf_system (same blocks, same printed signs, Sec. 3.3) is allocated once
    in column-major order and filled with the operator rows of each mesh
    `chunk` rows at a time; LAPACK's LU with partial pivoting (getrf) then
    overwrites it, and getrs solves for every right-hand side.
    Returns x [nrhs, n]."""
    import time
    from scipy.linalg import lu_factor, lu_solve
    xe, te = _mesh(*ext_mesh)
    xi, ti = _mesh(*int_mesh)
    ne, ni = xe.shape[0], xi.shape[0]
    n = 2 * ne + 2 * ni
    t0 = time.time()
    A = np.zeros((n, n), dtype=np.complex128, order="F")
    for (xyz, tri, k, off, nv) in ((xe, te, k_ext, 0, ne), (xi, ti, k_int, 2 * ne, ni)):
        for r0 in range(0, nv, chunk):
            rows = np.arange(r0, min(nv, r0 + chunk), dtype=np.int64)
            O = assemble(xyz, tri, k, ng=ng, rows=rows)
            r = off + rows
            A[r, off:off + nv] = -O["K"]
            A[r, off + nv:off + 2 * nv] = O["V"]
            A[nv + r, off:off + nv] = O["D"]
            A[nv + r, off + nv:off + 2 * nv] = O["T"]
            del O
            if log:
                log(f"  {'exterior' if off == 0 else 'interior'} rows {rows[-1] + 1}/{nv}"
                    f" ({time.time() - t0:.0f} s)")
    P_ie = mortar((xi, ti), (xe, te))
    A[0:ne, 2 * ne:2 * ne + ni] = 0.5 * P_ie.T
    A[ne:2 * ne, 2 * ne + ni:] = 0.5 * (rho_ext / rho_int) * P_ie.T
    A[2 * ne:2 * ne + ni, 0:ne] = -0.5 * P_ie
    A[2 * ne + ni:, ne:2 * ne] = -0.5 * (rho_int / rho_ext) * P_ie
    del P_ie
    B = np.stack([mtf_rhs((xe, te), k_ext, d, ni, incident) for d in np.atleast_2d(dirs)], axis=1)
    t1 = time.time()
    if log:
        log(f"  matrix {n} x {n} filled in {t1 - t0:.0f} s; LU ...")
    lu, piv = lu_factor(A, overwrite_a=True, check_finite=False)
    if not np.shares_memory(lu, A):
        raise MemoryError("getrf copied the matrix")
    X = lu_solve((lu, piv), B, check_finite=False)
    if log:
        log(f"  LU and solve {time.time() - t1:.0f} s")
    return np.ascontiguousarray(X.T)


def pmchwt_system(ops, rho_ext, rho_int):
    """The weak-form exterior PMCHWT matrix (Sec. 3.3, Eq. "pmchwt:discrete"),
    with the interior Calderon operator scaled as in Eq.
    "calderon:stf:extint" (V_i by rho_int / rho_ext, D_i by rho_ext / rho_int):
        [ -K_e - hat(K_i)                  V_e + (ri/re) hat(V_i) ]
        [  D_e + (re/ri) hat(D_i)          T_e + hat(T_i)         ]
    hat(X) = P_ei M_i^-1 X M_i^-1 P_ie; unknowns [gamma_D p, gamma_N p] on
    the exterior mesh, right-hand side [f, g]."""
    Oe, Oi, P_ie, M_i = ops["ext"], ops["int"], ops["P_ie"], ops["M_i"]
    P_ei = P_ie.T

    def hat(X):
        return P_ei @ np.linalg.solve(M_i, X @ np.linalg.solve(M_i, P_ie))

    a = rho_int / rho_ext
    return np.block([
        [-Oe["K"] - hat(Oi["K"]), Oe["V"] + a * hat(Oi["V"])],
        [Oe["D"] + hat(Oi["D"]) / a, Oe["T"] + hat(Oi["T"])],
    ])


def pmchwt_rhs(ext_mesh, k_ext, d):
    f, g = plane_wave_rhs(*ext_mesh, k_ext, d)
    return np.concatenate([f, g])


def solve_pmchwt(ext_mesh, int_mesh, k_ext, k_int, rho_ext, rho_int, dirs, ng=4, ops=None):
    """Exact discrete exterior PMCHWT solution(s) by dense LU: (x [nrhs, 2 N_ext], ops)."""
    if ops is None:
        ops = operators(ext_mesh, int_mesh, k_ext, k_int, ng=ng)
    A = pmchwt_system(ops, rho_ext, rho_int)
    B = np.stack([pmchwt_rhs(ext_mesh, k_ext, d) for d in np.atleast_2d(dirs)], axis=1)
    X = np.linalg.solve(A, B)
    return X.T, ops


def high_contrast_neumann_system(ops, rho_ext, rho_int):
    """The weak-form exterior high-contrast Neumann matrix (Sec. 3.3, discrete
    form of Eq. "highcontrast:ext:neu"):
        [ 1/2 M_e - hat(T_i)     -(re/ri) hat(D_i) M_e^-1 V_e ]
        [ M_e                     1/2 M_e - T_e               ]
    hat(X) = P_ei M_i^-1 X M_i^-1 P_ie; unknowns [gamma_N p, mu] on the
    exterior mesh (mu: the single-layer density of the scattered field)."""
    Oe, Oi, P_ie, M_i, M_e = ops["ext"], ops["int"], ops["P_ie"], ops["M_i"], ops["M_e"]
    P_ei = P_ie.T

    def hat(X):
        return P_ei @ np.linalg.solve(M_i, X @ np.linalg.solve(M_i, P_ie))

    c = rho_ext / rho_int
    return np.block([
        [0.5 * M_e - hat(Oi["T"]), -c * hat(Oi["D"]) @ np.linalg.solve(M_e, Oe["V"])],
        [M_e, 0.5 * M_e - Oe["T"]],
    ])


def high_contrast_neumann_rhs(ops, ext_mesh, k_ext, d, rho_ext, rho_int):
    """[(re/ri) hat(D_i) M_e^-1 f; g]: the hypersingular operator acts on the
    Dirichlet trace of the incident wave, whose P1 coefficients are M_e^-1 f."""
    f, g = plane_wave_rhs(*ext_mesh, k_ext, d)
    P_ie, M_i, M_e = ops["P_ie"], ops["M_i"], ops["M_e"]
    hatD = P_ie.T @ np.linalg.solve(M_i, ops["int"]["D"] @ np.linalg.solve(M_i, P_ie))
    return np.concatenate([(rho_ext / rho_int) * hatD @ np.linalg.solve(M_e, f), g])


def solve_high_contrast_neumann(ext_mesh, int_mesh, k_ext, k_int, rho_ext, rho_int, dirs, ng=4, ops=None):
    """Exact discrete solution(s) by dense LU: (x [nrhs, 2 N_ext], ops)."""
    if ops is None:
        ops = operators(ext_mesh, int_mesh, k_ext, k_int, ng=ng)
    A = high_contrast_neumann_system(ops, rho_ext, rho_int)
    B = np.stack([high_contrast_neumann_rhs(ops, ext_mesh, k_ext, d, rho_ext, rho_int)
                  for d in np.atleast_2d(dirs)], axis=1)
    X = np.linalg.solve(A, B)
    return X.T, ops


def projection_error(M_i, M_e, P_ie, norm="fro"):
    """E_int = ||I - M_i^-1 P_ie M_e^-1 P_ei||, E_ext = ||I - M_e^-1 P_ei M_i^-1 P_ie||."""
    P_ei = P_ie.T
    Ei = np.eye(M_i.shape[0]) - np.linalg.solve(M_i, P_ie @ np.linalg.solve(M_e, P_ei))
    Ee = np.eye(M_e.shape[0]) - np.linalg.solve(M_e, P_ei @ np.linalg.solve(M_i, P_ie))
    o = "fro" if norm == "fro" else np.inf
    if norm == "max":
        return np.abs(Ei).max(), np.abs(Ee).max()
    return np.linalg.norm(Ei, o), np.linalg.norm(Ee, o)
