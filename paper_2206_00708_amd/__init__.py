"""bemtx: nonconforming multiple-traces BEM for acoustic transmission on
MI355X (gfx950).  The compute path is the HIP library libbemtx.so behind the
C ABI of include/bemtx.h; this package only marshals arguments."""
from .api import (Context, Mesh, Problem, BemError, C128, C64_MIXED, HOST, DEVICE, OK, W_NOCONV,  # noqa: F401
                  check_mesh, host_mortar, host_gauss_legendre, host_phase_sincos, tune_table)
