"""CPU checks of the C-ABI library: it loads, exports every function that include/l1pr.h
declares, and its host-only entry points (validation, workspace sizing, status strings)
behave.  No compute call is made here (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "l1pr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(l1pr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2510_11023_amd import _lib, build

    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert {"l1pr_solve_serial", "l1pr_solve_parareal"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_host_entry_points(L):
    from paper_2510_11023_amd import make_problem, workloads as W

    p = make_problem(**W.C2)
    assert L.l1pr_validate(ctypes.byref(p)) == 0
    ser = L.l1pr_workspace_bytes(ctypes.byref(p), 32, 0)
    par = L.l1pr_workspace_bytes(ctypes.byref(p), 32, 1)
    # the parareal workspace holds the B*P fine trajectories of S+1 states; with the cosine
    # moments no system matrix goes through device memory, while the quadrature-GEMM assembly
    # adds B*P matrices of M^2 doubles
    assert par > 32 * 64 * 65 * 256 * 8 > ser > 0
    assert par < 32 * 64 * 256 * 256 * 8
    pg = make_problem(assembly=1, **W.C2)
    assert L.l1pr_workspace_bytes(ctypes.byref(pg), 32, 1) - par >= 32 * 64 * 256 * 256 * 8
    # the iterative solve is 2D only; the diagonal solve needs constant D and the moment
    # assembly; solver codes past 2 are invalid
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=1, **W.C2))) == -1
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=1, **W.C3))) == 0
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **W.C3))) == -1
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **W.with_(W.C3, d_sel=0)))) == 0
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **W.with_(W.C2, d_sel=0)))) == 0
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, assembly=1, **W.with_(W.C2, d_sel=0)))) == -1
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=3, **W.with_(W.C2, d_sel=0)))) == -1
    # without a system matrix the diagonal solve takes up to 256 modes per direction in 2D
    big = W.with_(W.C3, d_sel=0, modes=256, quad=384)
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **big))) == 0
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=0, **big))) == -1
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **W.with_(big, modes=257, quad=400)))) == -1
    long1d = W.with_(W.C2, d_sel=0, modes=4096, quad=8192)
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **long1d))) == 0
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=0, **long1d))) == -1
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **W.with_(long1d, modes=4097)))) == -1
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=2, **W.with_(long1d, quad=8193)))) == -1
    # no factorisation workspace for the diagonal solve
    pd, pc = make_problem(solver=2, **W.with_(W.C2, d_sel=0)), make_problem(**W.with_(W.C2, d_sel=0))
    assert L.l1pr_workspace_bytes(ctypes.byref(pd), 32, 1) < L.l1pr_workspace_bytes(ctypes.byref(pc), 32, 1)
    assert L.l1pr_validate(ctypes.byref(make_problem(solver=1, **W.with_(W.C3, quad=95)))) == -1
    bad = make_problem(**W.with_(W.C2, steps=4095))
    assert L.l1pr_validate(ctypes.byref(bad)) == -1
    assert L.l1pr_workspace_bytes(ctypes.byref(bad), 32, 1) == 0
    assert L.l1pr_workspace_bytes(ctypes.byref(p), 0, 1) == 0
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.l1pr_status_string(s)
    # invalid problems are rejected before any device work
    u = ctypes.c_void_p(1)
    assert L.l1pr_solve_serial(ctypes.byref(bad), 1, None, u, u, None, u, 1 << 30, None) == -1
    assert L.l1pr_solve_parareal(ctypes.byref(p), 1, None, u, u, 65, 0.0, 0, None, None, None,
                                 None, None, u, 1 << 30, None) == -1
    # unknown coarse propagator; learned coarse step without a network
    assert L.l1pr_solve_parareal(ctypes.byref(p), 1, None, u, u, 2, 0.0, 2, None, None, None,
                                 None, None, u, 1 << 30, None) == -1
    assert L.l1pr_solve_parareal(ctypes.byref(p), 1, None, u, u, 2, 0.0, 1, None, None, None,
                                 None, None, u, 1 << 30, None) == -1
    assert L.l1pr_check(None, None) == -1


def test_full_history_parareal_workspace_and_limits(L):
    """Full-history parareal keeps the previous iterate's trajectories and the prefix sums
    (B*P*(2S+1)*Mp doubles more); the learned coarse propagator is refused with it."""
    from paper_2510_11023_amd import make_problem, workloads as W

    kw = W.with_(W.C2, modes=48, steps=120, slices=6)
    B, P, S, Mp = 3, 6, 20, 48
    hyb = L.l1pr_workspace_bytes(ctypes.byref(make_problem(**kw)), B, 1)
    full = L.l1pr_workspace_bytes(ctypes.byref(make_problem(**W.with_(kw, history=1))), B, 1)
    extra = B * P * (2 * S + 1) * Mp * 8
    assert extra <= full - hyb <= extra + B * (120 + 130) * 8 + 3 * 256
    u = ctypes.c_void_p(256)
    ph = make_problem(**W.with_(kw, history=1))
    assert L.l1pr_solve_parareal(ctypes.byref(ph), B, None, u, u, 2, 0.0, 1, u, None, None,
                                 None, None, u, 1 << 30, None) == -1


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle, and the binding raises if the library is missing."""
    pkg = os.path.join(ROOT, "paper_2510_11023_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            txt = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in txt and "from oracle" not in txt, fn
    txt = open(os.path.join(pkg, "_lib.py")).read()
    assert "raise ImportError" in txt


def test_profiler_start_stop_without_launches(L):
    """Profiling with and without a kernel filter records nothing until a solver runs (host
    only: no event is created or read)."""
    from paper_2510_11023_amd import _lib

    for names in (None, "chol,history", ",,chol,", ""):
        if names is None:
            L.l1pr_profile_start()
        else:
            L.l1pr_profile_start_only(names.encode())
        assert _lib.profile_stop() == {}


def test_uneven_entry_points_reject_the_diagonal_solve(L):
    """Uneven batches run the factorisation only: with solver = 2 both entry points return
    L1PR_EINVAL from their argument check, before any device call (host buffers stand in for
    the device pointers, which are never touched)."""
    from paper_2510_11023_amd import _lib
    from paper_2510_11023_amd import workloads as W
    from paper_2510_11023_amd.solver import make_problem

    p = make_problem(solver=2, **W.with_(W.C2, d_sel=0, modes=32, quad=48, steps=16, slices=4))
    desc = _lib.Uneven(None, None, None)
    buf = (ctypes.c_double * 64)()
    ptr = ctypes.cast(buf, ctypes.c_void_p)
    assert L.l1pr_solve_serial_uneven(ctypes.byref(p), 1, ctypes.byref(desc), ptr, ptr, ptr, 64,
                                      None) == _lib.EINVAL
    assert L.l1pr_solve_parareal_uneven(ctypes.byref(p), 1, ctypes.byref(desc), ptr, ptr, 1, 0.0,
                                        None, None, None, ptr, 64, None) == _lib.EINVAL
