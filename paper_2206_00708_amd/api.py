"""Python face of the bemtx C ABI: same names, argument marshalling only.
Every step of the method runs in the HIP library; torch provides device
buffers and the stream."""
import ctypes

import numpy as np
import torch

from . import _native as N

OK, W_NOCONV = 0, 1
_ERR = {-1: "BEM_E_ARG", -2: "BEM_E_MESH", -3: "BEM_E_MESH_MISMATCH", -4: "BEM_E_STATE",
        -5: "BEM_E_OOM", -6: "BEM_E_DEVICE", -7: "BEM_E_UNSUPPORTED"}
HOST, DEVICE = 0, 1
C128, C64_MIXED = 0, 1


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code < 0:
        raise BemError(code, N.load().bem_last_error().decode())
    return code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_f64(a, device):
    """A contiguous float64 device tensor holding a (tensor or array-like)."""
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


class Context:
    """bem_ctx_create / bem_ctx_destroy on a torch device and stream."""

    def __init__(self, device=0, stream=None, hbm_budget_bytes=0):
        L = N.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(L.bem_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), hbm_budget_bytes, ctypes.byref(h)))
        self._h = h

    def bytes_in_use(self):
        return N.load().bem_ctx_bytes_in_use(self._h)

    def trim(self):
        """bem_ctx_trim: free the assembly scratch kept between problems."""
        _check(N.load().bem_ctx_trim(self._h))

    KERNELS = ("regular_tiles", "gather_tiles", "singular_pairs", "near_scatter", "mtf_dense", "mass_apply",
               "cgs_dots", "cgs_update", "arnoldi_finish", "mass_inverse", "block_gemm", "mass_gemm",
               "krylov_normalize", "field", "mortar")

    def set_strip_tiles(self, tiles=0):
        """bem_ctx_set_strip_tiles: block-pair tiles per assembly strip of the
        meshes created on this context from now on (0: the default)."""
        _check(N.load().bem_ctx_set_strip_tiles(self._h, int(tiles)))

    def set_kernel_timing(self, kernels=()):
        """Time every launch of the named kernels with HIP events (empty: off)."""
        mask = 0
        for k in kernels:
            mask |= 1 << self.KERNELS.index(k)
        _check(N.load().bem_ctx_set_kernel_timing(self._h, mask))

    def kernel_time(self, name):
        """(total milliseconds, launches) of one kernel since timing was enabled."""
        ms = ctypes.c_double(); n = ctypes.c_int64()
        _check(N.load().bem_ctx_kernel_time(self._h, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            N.load().bem_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: the library may already be gone
            pass


class Mesh:
    """bem_mesh_create: xyz float64 [nv,3], tri int32 [nt,3] (host arrays)."""

    def __init__(self, ctx, xyz, tri):
        L = N.load()
        self.ctx = ctx
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(L.bem_mesh_create(ctx._h, self.xyz.ctypes.data, self.xyz.shape[0], self.tri.ctypes.data,
                                 self.tri.shape[0], ctypes.byref(h)))
        self._h = h
        self.nv = self.xyz.shape[0]

    def winding(self, points):
        """bem_mesh_winding: winding numbers (1 inside, 0 outside) at points
        float64 [m,3] (a device tensor, or anything numpy takes)."""
        pts = _dev_f64(points, self.ctx.device).reshape(-1, 3)
        out = torch.empty(pts.shape[0], dtype=torch.float64, device=self.ctx.device)
        _check(N.load().bem_mesh_winding(self._h, _ptr(pts), pts.shape[0], _ptr(out), DEVICE))
        return out

    def close(self):
        # a mesh outlived by its context (an unordered teardown at interpreter
        # exit) is left alone: the context's destruction ended its device state
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):
                N.load().bem_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: the library may already be gone
            pass


class Problem:
    """bem_problem_create and the calls on a transmission problem."""

    def __init__(self, ctx, ext, inte, k_ext, k_int, rho_ext=1.0, rho_int=1.0, precision=C128, singular_gauss=4):
        L = N.load()
        self.ctx, self.ext, self.inte = ctx, ext, inte
        q = N.QuadOpts(singular_gauss)
        h = ctypes.c_void_p()
        _check(L.bem_problem_create(ctx._h, ext._h, inte._h, k_ext, k_int, rho_ext, rho_int, precision,
                                    ctypes.byref(q), ctypes.byref(h)))
        self._h = h
        self.n = 2 * ext.nv + 2 * inte.nv
        self.precision = precision

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self.ctx, "_h", None):   # as for meshes: never after the context
                N.load().bem_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown: the library may already be gone
            pass

    def footprint(self, nrhs=1, maxit=500):
        b = ctypes.c_size_t()
        _check(N.load().bem_problem_footprint(self._h, nrhs, maxit, ctypes.byref(b)))
        return b.value

    def assemble_operators(self, parts=3):
        _check(N.load().bem_assemble_operators(self._h, parts))

    def assemble_projection(self):
        _check(N.load().bem_assemble_projection(self._h))

    def mtf_matvec(self, x, strong=True):
        x = x.to(device=self.ctx.device, dtype=torch.complex128).contiguous()
        y = torch.empty_like(x)
        _check(N.load().bem_mtf_matvec(self._h, _ptr(x), _ptr(y), int(strong), DEVICE))
        return y

    def mtf_matvec_noalloc(self, x, y=None, strong=True):
        """bem_mtf_matvec_noalloc: the same product with the library's static
        work array (no device allocation by the library); asynchronous on
        the context's stream.  x, y: complex128 device tensors of length n."""
        x = x.to(device=self.ctx.device, dtype=torch.complex128).contiguous()
        if y is None:
            y = torch.empty_like(x)
        if y.dtype != torch.complex128 or not y.is_contiguous() or y.numel() != x.numel() or y.device != x.device:
            raise ValueError("y must be a contiguous complex128 tensor like x")
        _check(N.load().bem_mtf_matvec_noalloc(self._h, _ptr(x), _ptr(y), int(strong)))
        return y

    def mtf_matvec_batch(self, x, strong=True):
        """x: [nrhs, n] complex; one product per row (matrix cores for complex64 problems)."""
        x = x.to(device=self.ctx.device, dtype=torch.complex128).contiguous()
        y = torch.empty_like(x)
        _check(N.load().bem_mtf_matvec_batch(self._h, _ptr(x), _ptr(y), x.shape[0], int(strong), DEVICE))
        return y

    def mtf_rhs(self, dirs):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        b = torch.empty((d.shape[0], self.n), dtype=torch.complex128, device=self.ctx.device)
        _check(N.load().bem_mtf_rhs(self._h, d.ctypes.data, d.shape[0], _ptr(b), DEVICE))
        return b

    def solve(self, dirs, tol=1e-6, maxit=1000, ir_max=0, ir_inner_tol=0.0, batch=0):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        out = torch.empty((d.shape[0], self.n), dtype=torch.complex128, device=self.ctx.device)
        opts = N.SolverOpts(tol, maxit, ir_max, ir_inner_tol, batch)
        st = N.Stats()
        code = _check(N.load().bem_solve(self._h, d.ctypes.data, d.shape[0], ctypes.byref(opts), _ptr(out), DEVICE,
                                         ctypes.byref(st)))
        return out, st.as_dict(), code

    def set_incident(self, kind):
        """bem_problem_set_incident: 0 plane waves (dirs are directions), 1 point
        sources (dirs are source positions)."""
        _check(N.load().bem_problem_set_incident(self._h, int(kind)))

    def set_mortar(self, on_device):
        """bem_problem_set_mortar: mortar geometry on the device (True) or the host."""
        _check(N.load().bem_problem_set_mortar(self._h, int(on_device)))

    MASS_AUTO, MASS_DENSE, MASS_SPARSE = 0, 1, 2

    def set_mass_apply(self, mode):
        """bem_problem_set_mass_apply: 0 by size, 1 dense inverse masses, 2 the
        sparse Chebyshev apply; takes effect at the next assemble_projection."""
        _check(N.load().bem_problem_set_mass_apply(self._h, int(mode)))

    def set_graphs(self, on):
        """bem_problem_set_graphs: GMRES steps in captured HIP graphs (True, the
        default) or launched one by one (False); the traces agree bit for bit."""
        _check(N.load().bem_problem_set_graphs(self._h, int(bool(on))))

    def mass_apply_sparse(self):
        """bem_problem_mass_apply: True when the last projection set-up chose the sparse apply."""
        v = ctypes.c_int32()
        _check(N.load().bem_problem_mass_apply(self._h, ctypes.byref(v)))
        return bool(v.value)

    def mortar_ms(self):
        """bem_problem_mortar_ms: wall time of the last projection set-up's mortar step."""
        v = ctypes.c_double()
        _check(N.load().bem_problem_mortar_ms(self._h, ctypes.byref(v)))
        return v.value

    def set_k_int_imag(self, k_int_imag):
        """bem_problem_set_k_int_imag: interior wavenumber k_int + i k_int_imag
        (absorbing interior); assemble again afterwards."""
        _check(N.load().bem_problem_set_k_int_imag(self._h, float(k_int_imag)))

    def field(self, dirs, traces, points, region=None):
        """bem_field: total field [nrhs, m] at points [m,3] from the traces of
        solve() for the plane waves dirs; region [m] is 1 for interior and 0
        for exterior points (default: by the exterior mesh's winding number,
        interior where it exceeds 1/2)."""
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        pts = _dev_f64(points, self.ctx.device).reshape(-1, 3)
        if region is None:
            region = (self.ext.winding(pts) > 0.5).to(torch.int32)
        reg = torch.as_tensor(region, device=self.ctx.device).to(torch.int32).contiguous()
        x = traces.to(device=self.ctx.device, dtype=torch.complex128).contiguous()
        if x.numel() != d.shape[0] * self.n or reg.numel() != pts.shape[0]:
            raise ValueError("traces must be [nrhs, n] and region [m]")
        out = torch.empty((d.shape[0], pts.shape[0]), dtype=torch.complex128, device=self.ctx.device)
        _check(N.load().bem_field(self._h, d.ctypes.data, d.shape[0], _ptr(x), _ptr(pts), _ptr(reg), pts.shape[0],
                                  _ptr(out), DEVICE))
        return out

    def _ext_solve(self, fn, dirs, tol, maxit):
        d = np.ascontiguousarray(np.atleast_2d(dirs), dtype=np.float64)
        out = torch.empty((d.shape[0], 2 * self.ext.nv), dtype=torch.complex128, device=self.ctx.device)
        opts = N.SolverOpts(tol, maxit, 0, 0.0, 0)
        st = N.Stats()
        code = _check(fn(self._h, d.ctypes.data, d.shape[0], ctypes.byref(opts), _ptr(out), DEVICE, ctypes.byref(st)))
        return out, st.as_dict(), code

    def _ext_matvec(self, fn, x, strong):
        xx = x.to(device=self.ctx.device, dtype=torch.complex128).contiguous()
        y = torch.empty_like(xx)
        _check(fn(self._h, _ptr(xx), _ptr(y), int(strong), DEVICE))
        return y

    def solve_pmchwt(self, dirs, tol=1e-6, maxit=1000):
        """bem_solve_pmchwt: exterior PMCHWT traces [nrhs, 2 N_ext] (p, dp/dn+)."""
        return self._ext_solve(N.load().bem_solve_pmchwt, dirs, tol, maxit)

    def pmchwt_matvec(self, x, strong=True):
        """bem_pmchwt_matvec on a complex128 vector of length 2 N_ext."""
        return self._ext_matvec(N.load().bem_pmchwt_matvec, x, strong)

    def solve_hc_neumann(self, dirs, tol=1e-6, maxit=1000):
        """bem_solve_hc_neumann: [nrhs, 2 N_ext] = (dp/dn+, mu) on the exterior mesh."""
        return self._ext_solve(N.load().bem_solve_hc_neumann, dirs, tol, maxit)

    def hc_neumann_matvec(self, x, strong=True):
        """bem_hc_neumann_matvec on a complex128 vector of length 2 N_ext."""
        return self._ext_matvec(N.load().bem_hc_neumann_matvec, x, strong)

    def operator(self, mesh, op):
        nv = self.ext.nv if mesh == 0 else self.inte.nv
        dt = torch.complex128 if self.precision == C128 else torch.complex64
        out = torch.empty((nv, nv), dtype=dt, device=self.ctx.device)
        _check(N.load().bem_copy_operator(self._h, mesh, op.encode(), _ptr(out), DEVICE))
        return out

    def projection(self):
        """P_int,ext as (rowptr int64, col int32, val float64) numpy arrays."""
        L = N.load()
        nnz = ctypes.c_int64()
        _check(L.bem_copy_projection(self._h, None, None, None, ctypes.byref(nnz)))
        rp = np.zeros(self.inte.nv + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        _check(L.bem_copy_projection(self._h, rp.ctypes.data, col.ctypes.data, val.ctypes.data, ctypes.byref(nnz)))
        return rp, col, val


# ---------------------------------------------------------- host-only calls

def check_mesh(xyz, tri):
    """bem_check_mesh: raises BemError(BEM_E_MESH) for an invalid surface mesh."""
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    t = np.ascontiguousarray(tri, dtype=np.int32)
    _check(N.load().bem_check_mesh(x.ctypes.data, x.shape[0], t.ctypes.data, t.shape[0]))


def host_mortar(int_mesh, ext_mesh):
    """bem_host_mortar: P_int,ext as (rowptr, col, val, coverage_defect)."""
    L = N.load()
    xi = np.ascontiguousarray(int_mesh[0], dtype=np.float64); ti = np.ascontiguousarray(int_mesh[1], dtype=np.int32)
    xe = np.ascontiguousarray(ext_mesh[0], dtype=np.float64); te = np.ascontiguousarray(ext_mesh[1], dtype=np.int32)
    nnz = ctypes.c_int64(); dfc = ctypes.c_double()
    args = (xi.ctypes.data, xi.shape[0], ti.ctypes.data, ti.shape[0], xe.ctypes.data, xe.shape[0], te.ctypes.data,
            te.shape[0])
    _check(L.bem_host_mortar(*args, None, None, None, ctypes.byref(nnz), ctypes.byref(dfc)))
    rp = np.zeros(xi.shape[0] + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    _check(L.bem_host_mortar(*args, rp.ctypes.data, col.ctypes.data, val.ctypes.data, ctypes.byref(nnz),
                             ctypes.byref(dfc)))
    return rp, col, val, dfc.value


def tune_table():
    """bem_tune_table: {key: [values]} of the kernel shapes picked by timing."""
    L = N.load()
    n = ctypes.c_size_t()
    _check(L.bem_tune_table(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(L.bem_tune_table(buf, n.value + 1, ctypes.byref(n)))
    out = {}
    for line in buf.value.decode().splitlines():
        f = line.split()
        if f:
            out[f[0]] = [int(v) for v in f[1:]]
    return out


def host_gauss_legendre(n):
    x = np.zeros(n); w = np.zeros(n)
    _check(N.load().bem_host_gauss_legendre(n, x.ctypes.data, w.ctypes.data))
    return x, w


def host_phase_sincos(x):
    """bem_host_phase_sincos: the kernels' sin/cos of the phase, on the host."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    s = np.zeros_like(x); c = np.zeros_like(x)
    _check(N.load().bem_host_phase_sincos(x.size, x.ctypes.data, s.ctypes.data, c.ctypes.data))
    return s, c
