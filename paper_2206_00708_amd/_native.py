"""ctypes declarations of the bemtx C ABI (include/bemtx.h).  Loading fails
loudly when the built library is missing: there is no fallback path."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbemtx.so")

c_status = ctypes.c_int32
vp = ctypes.c_void_p
i32, i64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t


class QuadOpts(ctypes.Structure):
    _fields_ = [("singular_gauss", i32)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("tol", f64), ("maxit", i32), ("ir_max", i32), ("ir_inner_tol", f64), ("batch", i32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", i32), ("ir_steps", i32), ("rel_residual", f64),
                ("t_geometry_ms", f64), ("t_regular_ms", f64), ("t_singular_ms", f64),
                ("t_projection_ms", f64), ("t_matrix_ms", f64), ("t_solve_ms", f64), ("t_iter_ms", f64),
                ("t_assembly_ms", f64), ("graph_steps", i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/bemtx.h
SIGNATURES = {
    "bem_last_error": (ctypes.c_char_p, []),
    "bem_ctx_create": (c_status, [i32, vp, sz, ctypes.POINTER(vp)]),
    "bem_ctx_destroy": (None, [vp]),
    "bem_ctx_bytes_in_use": (sz, [vp]),
    "bem_ctx_trim": (c_status, [vp]),
    "bem_ctx_set_kernel_timing": (c_status, [vp, ctypes.c_uint32]),
    "bem_ctx_kernel_time": (c_status, [vp, ctypes.c_char_p, ctypes.POINTER(f64), ctypes.POINTER(i64)]),
    "bem_mesh_create": (c_status, [vp, vp, i64, vp, i64, ctypes.POINTER(vp)]),
    "bem_mesh_destroy": (None, [vp]),
    "bem_mesh_num_vertices": (i64, [vp]),
    "bem_problem_create": (c_status, [vp, vp, vp, f64, f64, f64, f64, i32, ctypes.POINTER(QuadOpts),
                                      ctypes.POINTER(vp)]),
    "bem_problem_destroy": (None, [vp]),
    "bem_problem_footprint": (c_status, [vp, i32, i32, ctypes.POINTER(sz)]),
    "bem_assemble_operators": (c_status, [vp, i32]),
    "bem_assemble_projection": (c_status, [vp]),
    "bem_mtf_matvec": (c_status, [vp, vp, vp, i32, i32]),
    "bem_mtf_matvec_noalloc": (c_status, [vp, vp, vp, i32]),
    "bem_mtf_matvec_batch": (c_status, [vp, vp, vp, i32, i32, i32]),
    "bem_mtf_rhs": (c_status, [vp, vp, i32, vp, i32]),
    "bem_solve": (c_status, [vp, vp, i32, ctypes.POINTER(SolverOpts), vp, i32, ctypes.POINTER(Stats)]),
    "bem_copy_operator": (c_status, [vp, i32, ctypes.c_char, vp, i32]),
    "bem_copy_projection": (c_status, [vp, vp, vp, vp, ctypes.POINTER(i64)]),
    "bem_field": (c_status, [vp, vp, i32, vp, vp, vp, i64, vp, i32]),
    "bem_problem_set_incident": (c_status, [vp, i32]),
    "bem_problem_set_k_int_imag": (c_status, [vp, f64]),
    "bem_problem_set_mortar": (c_status, [vp, i32]),
    "bem_problem_mortar_ms": (c_status, [vp, ctypes.POINTER(f64)]),
    "bem_problem_set_mass_apply": (c_status, [vp, i32]),
    "bem_problem_mass_apply": (c_status, [vp, ctypes.POINTER(i32)]),
    "bem_problem_set_graphs": (c_status, [vp, i32]),
    "bem_ctx_set_strip_tiles": (c_status, [vp, ctypes.c_int64]),
    "bem_solve_pmchwt": (c_status, [vp, vp, i32, ctypes.POINTER(SolverOpts), vp, i32, ctypes.POINTER(Stats)]),
    "bem_pmchwt_matvec": (c_status, [vp, vp, vp, i32, i32]),
    "bem_solve_hc_neumann": (c_status, [vp, vp, i32, ctypes.POINTER(SolverOpts), vp, i32, ctypes.POINTER(Stats)]),
    "bem_hc_neumann_matvec": (c_status, [vp, vp, vp, i32, i32]),
    "bem_mesh_winding": (c_status, [vp, vp, i64, vp, i32]),
    "bem_tune_table": (c_status, [vp, sz, ctypes.POINTER(sz)]),
    "bem_check_mesh": (c_status, [vp, i64, vp, i64]),
    "bem_host_mortar": (c_status, [vp, i64, vp, i64, vp, i64, vp, i64, vp, vp, vp, ctypes.POINTER(i64),
                                   ctypes.POINTER(f64)]),
    "bem_host_gauss_legendre": (c_status, [i32, vp, vp]),
    "bem_host_phase_sincos": (c_status, [i64, vp, vp, vp]),
}

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"bemtx: HIP library {LIB_PATH} is not built "
                               "(run __graft_entry__.build() or python paper_2206_00708_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
