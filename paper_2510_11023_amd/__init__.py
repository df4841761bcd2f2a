"""MI355X-native parareal / L1 / sine-Galerkin solver for quasilinear Caputo subdiffusion.

The solver itself is the HIP library ``libl1pr.so`` (C-ABI in ``include/l1pr.h``); this
package holds its build script, a thin ctypes binding with the same entry-point names
(``solve_serial``, ``solve_parareal``) and the seeded synthetic input generators.
"""
from .solver import PararealResult, make_problem, nmodes, solve_parareal, solve_serial, workspace_bytes

__all__ = ["make_problem", "nmodes", "solve_serial", "solve_parareal", "workspace_bytes",
           "PararealResult"]
