"""Python access to the plain serial FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  Shares no code with the
HIP path.  Arrays are float64 numpy arrays (C order).

Problem fields follow ``oracle.h``; see that header for the paper passages each
function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.environ.get("L1PR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build() -> str:
    """Compile ``liboracle.so`` with gcc -O2 (plain C, no BLAS, no threads)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", _SRC, "-o", _LIB, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("modes", ctypes.c_int32),
        ("quad", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("slices", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("T", ctypes.c_double),
        ("d_sel", ctypes.c_int32),
        ("d_param", ctypes.c_double),
        ("f_sel", ctypes.c_int32),
        ("history", ctypes.c_int32),
        ("source_time", ctypes.c_int32),
        ("solver", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Problem)
        L.oracle_validate.argtypes = [pp]
        L.oracle_bweight.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_bweight.restype = ctypes.c_double
        L.oracle_gauss_legendre01.argtypes = [ctypes.c_int32, dp, dp]
        L.oracle_D.argtypes = [pp] + [ctypes.c_double] * 4
        L.oracle_D.restype = ctypes.c_double
        L.oracle_f.argtypes = [pp] + [ctypes.c_double] * 4
        L.oracle_f.restype = ctypes.c_double
        L.oracle_galerkin.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_galerkin_rows.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32), dp, dp]
        L.oracle_step.argtypes = [pp, dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double, dp]
        L.oracle_coarse_G.argtypes = [pp, ctypes.c_int32, dp, dp]
        L.oracle_fine_F.argtypes = [pp, ctypes.c_int32, dp, dp, dp]
        L.oracle_solve_serial.argtypes = [pp, dp, dp, dp]
        L.oracle_soe_nodes.argtypes = [ctypes.c_double, ctypes.c_int32, dp, dp, ctypes.c_int32]
        L.oracle_soe_nodes.restype = ctypes.c_int32
        L.oracle_solve_parareal.argtypes = [pp, dp, dp, ctypes.c_int32, ctypes.c_double, dp, dp,
                                            ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


def problem(dim=1, modes=8, quad=16, steps=16, slices=4, alpha=0.5, T=1.0, d_sel=0,
            d_param=1.0, f_sel=0, history=0, source_time=0, solver=0) -> Problem:
    return Problem(dim, modes, quad, steps, slices, alpha, T, d_sel, d_param, f_sel, history,
                   source_time, solver)


def nmodes(p: Problem) -> int:
    return p.modes if p.dim == 1 else p.modes * p.modes


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed (rc={rc})")


def validate(p: Problem) -> bool:
    return lib().oracle_validate(ctypes.byref(p)) == 0


def bweight(x: float, alpha: float) -> float:
    return lib().oracle_bweight(float(x), float(alpha))


SOE_J0 = 16  # ORACLE_SOE_J0 of oracle.h


def soe_nodes(alpha: float, N: int):
    """(lam, w) of the sum-of-exponentials L1 weights: b_j ~ sum_l w_l exp(-lam_l j) for
    SOE_J0 <= j <= N (merged node lam = 0 first)."""
    lam = np.zeros(512)
    w = np.zeros(512)
    n = lib().oracle_soe_nodes(float(alpha), int(N), _ptr(lam), _ptr(w), 512)
    _check(0 if n > 0 else -1, "soe_nodes")
    return lam[:n].copy(), w[:n].copy()


def gauss_legendre01(Q: int):
    x = np.zeros(Q)
    w = np.zeros(Q)
    lib().oracle_gauss_legendre01(Q, _ptr(x), _ptr(w))
    return x, w


def D(p, x, y, t, u):
    return lib().oracle_D(ctypes.byref(p), x, y, t, u)


def f(p, x, y, t, u):
    return lib().oracle_f(ctypes.byref(p), x, y, t, u)


def galerkin(p, c, tD, tf):
    Md = nmodes(p)
    c = np.ascontiguousarray(c, dtype=np.float64)
    K = np.zeros((Md, Md))
    F = np.zeros(Md)
    _check(lib().oracle_galerkin(ctypes.byref(p), _ptr(c), tD, tf, _ptr(K), _ptr(F)), "galerkin")
    return K, F


def galerkin_rows(p, c, tD, tf, rows):
    """Rows `rows` of K and the whole load F (the same sums as galerkin, row by row)."""
    Md = nmodes(p)
    c = np.ascontiguousarray(c, dtype=np.float64)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    K = np.zeros((len(r), Md))
    F = np.zeros(Md)
    _check(lib().oracle_galerkin_rows(ctypes.byref(p), _ptr(c), tD, tf, len(r),
                                      r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(K),
                                      _ptr(F)), "galerkin_rows")
    return K, F


def step(p, c_prev, tD, tf, hist, tau):
    out = np.zeros(nmodes(p))
    c_prev = np.ascontiguousarray(c_prev, dtype=np.float64)
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    _check(lib().oracle_step(ctypes.byref(p), _ptr(c_prev), tD, tf, _ptr(hist), tau, _ptr(out)),
           "step")
    return out


def coarse_G(p, n, C):
    C = np.ascontiguousarray(C, dtype=np.float64)
    assert C.shape[0] >= n + 1
    out = np.zeros(nmodes(p))
    _check(lib().oracle_coarse_G(ctypes.byref(p), n, _ptr(C), _ptr(out)), "coarse_G")
    return out


def fine_F(p, n, C, want_traj=False):
    C = np.ascontiguousarray(C, dtype=np.float64)
    assert C.shape[0] >= n + 1
    S = p.steps // p.slices
    out = np.zeros(nmodes(p))
    traj = np.zeros((S + 1, nmodes(p))) if want_traj else None
    _check(lib().oracle_fine_F(ctypes.byref(p), n, _ptr(C), _ptr(out), _ptr(traj)), "fine_F")
    return (out, traj) if want_traj else out


def solve_serial(p, u0, want_traj=False):
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    Md = nmodes(p)
    U = np.zeros((p.slices + 1, Md))
    traj = np.zeros((p.steps + 1, Md)) if want_traj else None
    _check(lib().oracle_solve_serial(ctypes.byref(p), _ptr(u0), _ptr(U), _ptr(traj)), "serial")
    return (U, traj) if want_traj else U


def solve_parareal(p, u0, max_iter, tol=0.0, want_iterates=False):
    """Returns (U, iters, incr[:iters], iterates[:iters+1] or None)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    Md = nmodes(p)
    U = np.zeros((p.slices + 1, Md))
    incr = np.zeros(max(max_iter, 1))
    Uit = np.zeros((max_iter + 1, p.slices + 1, Md)) if want_iterates else None
    it = ctypes.c_int32(0)
    _check(lib().oracle_solve_parareal(ctypes.byref(p), _ptr(u0), _ptr(U), max_iter, tol,
                                       _ptr(Uit), _ptr(incr), ctypes.byref(it)), "parareal")
    k = it.value
    return U, k, incr[:k], (Uit[: k + 1] if want_iterates else None)
