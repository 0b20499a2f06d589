"""MI355X (gfx950) two-phase phase-field step: HIP kernels behind a C ABI.

The hot path -- one RK4 time step of the incompressible two-phase solver
with the energy-based surface tension force of Mirjalili, Khanwale & Mani
(arXiv 2205.05835) -- runs entirely in libtpf.so (HIP, gfx950).  This
package holds the kernels' sources (csrc/), the build script and the ctypes
binding (tpf.py).
"""
from .tpf import (FIELD, FIELDS, Solver, TpfError, lib, make_params, solver_for_case,  # noqa: F401
                  tpf_diag, tpf_params, workspace_bytes)
