"""MI355X-native parareal / L1 / sine-Galerkin solver for quasilinear Caputo subdiffusion.

The solver itself is the HIP library ``libl1pr.so`` (C-ABI in ``include/l1pr.h``); this
package holds its build script, a thin ctypes binding with the same entry-point names
(``solve_serial``, ``solve_parareal``) and the seeded synthetic input generators.
"""
from .solver import (COARSE_L1, COARSE_LEARNED, PararealResult, autotune, check, coarse_apply,
                     fine_apply, make_problem, nmodes, parareal_workspace, solve_parareal,
                     solve_batch, solve_parareal_uneven, solve_serial, solve_serial_noalloc,
                     solve_serial_uneven, workspace_bytes)

__all__ = ["make_problem", "nmodes", "solve_serial", "solve_parareal", "coarse_apply",
           "fine_apply", "workspace_bytes", "parareal_workspace", "PararealResult", "COARSE_L1",
           "COARSE_LEARNED", "solve_serial_uneven", "solve_parareal_uneven", "autotune",
           "solve_batch", "solve_serial_noalloc", "check"]
