"""Python entry points with the C-ABI's names: ``solve_serial`` and ``solve_parareal``.

Tensors are torch float64 CUDA (HIP) tensors; the work is enqueued on the current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import Problem


ASSEMBLY_MOMENTS = 0   # stiffness from cosine moments (Toeplitz-plus-Hankel form)
ASSEMBLY_GEMM = 1      # stiffness as the quadrature GEMM dphi^T diag(w D) dphi on FP64 MFMA


def make_problem(dim=1, modes=32, quad=64, steps=256, slices=8, alpha=0.5, T=1.0, d_sel=0,
                 d_param=1.0, f_sel=0, history=0, source_time=0,
                 assembly=ASSEMBLY_MOMENTS, tune=0, solver=0) -> Problem:
    return Problem(dim, modes, quad, steps, slices, alpha, T, d_sel, d_param, f_sel, history,
                   source_time, assembly, tune, solver)


def nmodes(p: Problem) -> int:
    return p.modes if p.dim == 1 else p.modes * p.modes


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _alpha_arg(alpha, B):
    if alpha is None:
        return None, None
    arr = (ctypes.c_double * B)(*[float(a) for a in alpha])
    return arr, ctypes.cast(arr, ctypes.c_void_p)


def _check_u0(p: Problem, u0: torch.Tensor):
    if not (u0.is_cuda and u0.dtype == torch.float64 and u0.is_contiguous()):
        raise ValueError("u0 must be a contiguous float64 device tensor")
    if u0.dim() != 2 or u0.shape[1] != nmodes(p):
        raise ValueError(f"u0 must have shape [batch, {nmodes(p)}]")


def workspace_bytes(p: Problem, batch: int, op: int) -> int:
    return int(_lib.lib().l1pr_workspace_bytes(ctypes.byref(p), batch, op))


def _workspace(p, B, op, device):
    n = workspace_bytes(p, B, op)
    if n == 0:
        raise _lib.L1prError(_lib.EINVAL, "workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=device), n


def solve_serial(p: Problem, u0: torch.Tensor, alpha=None, want_traj: bool = False,
                 workspace: torch.Tensor | None = None):
    """Serial solve of u0.shape[0] instances.  Returns (U [B,P+1,Md], traj [B,N+1,Md] or None)."""
    _check_u0(p, u0)
    B = u0.shape[0]
    Md = nmodes(p)
    U = torch.empty((B, p.slices + 1, Md), dtype=torch.float64, device=u0.device)
    traj = torch.empty((B, p.steps + 1, Md), dtype=torch.float64, device=u0.device) if want_traj else None
    if workspace is None:
        workspace, n = _workspace(p, B, _lib.OP_SERIAL, u0.device)
    else:
        n = workspace.numel() * workspace.element_size()
    keep, aptr = _alpha_arg(alpha, B)
    st = _lib.lib().l1pr_solve_serial(ctypes.byref(p), B, aptr, _ptr(u0), _ptr(U), _ptr(traj),
                                      _ptr(workspace), n, _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_solve_serial")
    return U, traj


def solve_serial_noalloc(p: Problem, u0: torch.Tensor, alpha=None, want_traj: bool = False):
    """solve_serial without a workspace: the library's per-device scratch array is used and
    nothing is allocated on the device beyond the outputs created here (callers that must not
    allocate at all pass their own U and traj to the C entry point)."""
    _check_u0(p, u0)
    B = u0.shape[0]
    Md = nmodes(p)
    U = torch.empty((B, p.slices + 1, Md), dtype=torch.float64, device=u0.device)
    traj = torch.empty((B, p.steps + 1, Md), dtype=torch.float64, device=u0.device) if want_traj else None
    keep, aptr = _alpha_arg(alpha, B)
    st = _lib.lib().l1pr_solve_serial_noalloc(ctypes.byref(p), B, aptr, _ptr(u0), _ptr(U),
                                              _ptr(traj), _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_solve_serial_noalloc")
    return U, traj


@dataclass
class PararealResult:
    U: torch.Tensor
    iters: int
    status: int
    incr: torch.Tensor | None
    iterates: torch.Tensor | None
    # per-instance status on the device: sweeps after which each instance was finished (or
    # that it ran), or a negative status (ENOTCONV, ENONFINITE)
    inst: torch.Tensor | None = None
    workspace: torch.Tensor | None = None


COARSE_L1 = 0
COARSE_LEARNED = 1


def parareal_workspace(p: Problem, batch: int, device, learned: bool = False) -> torch.Tensor:
    n = workspace_bytes(p, batch, _lib.OP_PARAREAL)
    if learned:
        n += int(_lib.lib().l1pr_parareal_learned_extra_bytes(ctypes.byref(p), batch))
    return torch.empty(n, dtype=torch.uint8, device=device)


def _apply(name, p, Z, alpha, workspace):
    if not (Z.is_cuda and Z.dtype == torch.float64 and Z.is_contiguous()):
        raise ValueError("Z must be a contiguous float64 device tensor")
    B = Z.shape[0]
    Md = nmodes(p)
    if tuple(Z.shape[1:]) != (p.slices + 1, Md):
        raise ValueError(f"Z must have shape [batch, {p.slices + 1}, {Md}]")
    out = torch.empty((B, p.slices, Md), dtype=torch.float64, device=Z.device)
    if workspace is None:
        workspace = parareal_workspace(p, B, Z.device)
    keep, aptr = _alpha_arg(alpha, B)
    st = getattr(_lib.lib(), name)(ctypes.byref(p), B, aptr, _ptr(Z), _ptr(out), _ptr(workspace),
                                   workspace.numel(), _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, name)
    return out


def coarse_apply(p: Problem, Z: torch.Tensor, alpha=None, workspace=None) -> torch.Tensor:
    """out[b][n] = G_n(Z_b[0..n]) for every slice n (one coarse L1 step each)."""
    return _apply("l1pr_coarse_apply", p, Z, alpha, workspace)


def fine_apply(p: Problem, Z: torch.Tensor, alpha=None, workspace=None) -> torch.Tensor:
    """out[b][n] = F_n(Z_b[0..n]) for every slice n (the hybrid fine propagator)."""
    return _apply("l1pr_fine_apply", p, Z, alpha, workspace)


def solve_parareal(p: Problem, u0: torch.Tensor, max_iter: int, tol: float = 0.0, alpha=None,
                   want_iterates: bool = False, want_incr: bool = True,
                   workspace: torch.Tensor | None = None, allow_notconv: bool = True,
                   coarse: int = COARSE_L1, mlp_params: torch.Tensor | None = None,
                   want_status: bool = True):
    """Parareal solve.  Returns a PararealResult; iterates is [iters+1, B, P+1, Md].
    tol > 0 stops each instance at its own first sweep whose increment is <= tol (the others
    go on); coarse = COARSE_LEARNED uses the residual network in mlp_params
    (LearnedCoarse.params)."""
    _check_u0(p, u0)
    B = u0.shape[0]
    Md = nmodes(p)
    dev = u0.device
    U = torch.empty((B, p.slices + 1, Md), dtype=torch.float64, device=dev)
    its = torch.empty((max_iter + 1, B, p.slices + 1, Md), dtype=torch.float64, device=dev) \
        if want_iterates else None
    incr = torch.zeros((B, max(max_iter, 1)), dtype=torch.float64, device=dev) if want_incr else None
    inst = torch.empty(B, dtype=torch.int32, device=dev) if want_status else None
    if workspace is None:
        workspace = parareal_workspace(p, B, dev, learned=(coarse == COARSE_LEARNED))
    n = workspace.numel() * workspace.element_size()
    keep, aptr = _alpha_arg(alpha, B)
    it = ctypes.c_int32(0)
    st = _lib.lib().l1pr_solve_parareal(ctypes.byref(p), B, aptr, _ptr(u0), _ptr(U),
                                        int(max_iter), float(tol), int(coarse), _ptr(mlp_params),
                                        _ptr(inst), _ptr(incr), _ptr(its), ctypes.byref(it),
                                        _ptr(workspace), n, _stream())
    if st != _lib.OK and not (allow_notconv and st == _lib.ENOTCONV):
        raise _lib.L1prError(st, "l1pr_solve_parareal")
    k = it.value
    return PararealResult(U=U, iters=k, status=st,
                          incr=None if incr is None else incr[:, :k],
                          iterates=None if its is None else its[: k + 1], inst=inst,
                          workspace=workspace)


def check(workspace: torch.Tensor) -> int:
    """Device status word of the last call on `workspace` (l1pr_check): OK, ENONFINITE or
    EWAIT; waits for the current stream."""
    return int(_lib.lib().l1pr_check(_ptr(workspace), _stream()))


# ---------------------------------------------------------------- uneven batches

def _uneven(modes, spp, alpha, coarse=COARSE_L1, mlp_params=None, mlp_modes=0):
    """Descriptor and the device tensors it points to (kept alive by the caller)."""
    keep = []

    def dev(x, dtype):
        if x is None:
            return None
        t = x if isinstance(x, torch.Tensor) else torch.tensor(list(x), dtype=dtype)
        t = t.to(device="cuda", dtype=dtype).contiguous()
        keep.append(t)
        return ctypes.c_void_p(t.data_ptr())

    d = _lib.Uneven(dev(modes, torch.int32), dev(spp, torch.int32), dev(alpha, torch.float64),
                    int(coarse), _ptr(mlp_params), int(mlp_modes))
    return d, keep


def solve_serial_uneven(p: Problem, u0: torch.Tensor, modes=None, spp=None, alpha=None,
                        workspace=None):
    """Serial (hybrid) solve of an uneven batch: per-instance modes M_b, fine steps per slice
    S_b and order (device arrays or sequences).  Returns U [B][P+1][M]."""
    _check_u0(p, u0)
    B = u0.shape[0]
    ws = workspace if workspace is not None else _workspace(p, B, _lib.OP_SERIAL, u0.device)[0]
    U = torch.empty((B, p.slices + 1, nmodes(p)), dtype=torch.float64, device=u0.device)
    d, keep = _uneven(modes, spp, alpha)
    st = _lib.lib().l1pr_solve_serial_uneven(ctypes.byref(p), B, ctypes.byref(d), _ptr(u0), _ptr(U),
                                             _ptr(ws), ws.numel(), _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_solve_serial_uneven")
    del keep
    return U


def uneven_workspace(p: Problem, batch: int, device, learned: bool = False) -> torch.Tensor:
    return parareal_workspace(p, batch, device, learned=learned)


def solve_parareal_uneven(p: Problem, u0: torch.Tensor, sweeps: int, modes=None, spp=None,
                          alpha=None, conv_tol: float = 0.0, workspace=None, out=None,
                          conv=None, stamps=None, incr=None, coarse: int = COARSE_L1,
                          mlp_params=None, mlp_modes: int = 0):
    """Parareal over an uneven batch with at most `sweeps` sweeps and no host synchronisation;
    an instance is finished at its first sweep whose increment is <= conv_tol.  Returns
    (U, conv, stamps): conv[b] = that sweep (-1 if none), stamps[k] = device wall clock at
    the end of sweep k (k = 0: initial coarse sweep).  coarse = COARSE_LEARNED uses the
    network mlp_params of mlp_modes >= p.modes modes for every instance."""
    _check_u0(p, u0)
    B = u0.shape[0]
    dev = u0.device
    learned = coarse == COARSE_LEARNED
    ws = workspace if workspace is not None else uneven_workspace(p, B, dev, learned=learned)
    U = out if out is not None else torch.empty((B, p.slices + 1, nmodes(p)), dtype=torch.float64,
                                                device=dev)
    conv = conv if conv is not None else torch.empty(B, dtype=torch.int32, device=dev)
    stamps = stamps if stamps is not None else torch.zeros(sweeps + 1, dtype=torch.int64, device=dev)
    d, keep = _uneven(modes, spp, alpha, coarse, mlp_params, mlp_modes)
    st = _lib.lib().l1pr_solve_parareal_uneven(ctypes.byref(p), B, ctypes.byref(d), _ptr(u0),
                                               _ptr(U), sweeps, float(conv_tol), _ptr(conv),
                                               _ptr(stamps), _ptr(incr), _ptr(ws), ws.numel(),
                                               _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_solve_parareal_uneven")
    del keep
    return U, conv, stamps


def autotune(p: Problem, batch: int, workspace=None) -> int:
    """Fastest GEMM variant bits for the fine sweep of `batch` instances (see l1pr_problem.tune)."""
    ws = workspace if workspace is not None else _workspace(p, batch, _lib.OP_PARAREAL, "cuda")[0]
    out = ctypes.c_int32(0)
    st = _lib.lib().l1pr_autotune(ctypes.byref(p), batch, _ptr(ws), ws.numel(), _stream(),
                                  ctypes.byref(out))
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_autotune")
    return int(out.value)


def solve_batch(problems, u0s, parareal_sweeps: int | None = None, workspace=None,
                coarse: int = COARSE_L1, mlp_params=None, mlp_modes: int = 0):
    """Heterogeneous batch: problems[i] (each with its own parameters and alpha) from u0s[i]
    (device float64 [Md_i]).  Serial solutions, or parareal_sweeps plain parareal sweeps.
    Returns a list of slice-end tensors [P_i + 1, Md_i] (views of one output buffer)."""
    n = len(problems)
    if n != len(u0s):
        raise ValueError("one initial vector per problem")
    arr = (Problem * max(n, 1))(*problems)
    sizes = [nmodes(p) for p in problems]
    outs = [(p.slices + 1) * m for p, m in zip(problems, sizes)]
    for u, m in zip(u0s, sizes):
        if not (u.is_cuda and u.dtype == torch.float64 and u.numel() == m):
            raise ValueError("each u0 must be a float64 device vector of the problem's size")
    dev = u0s[0].device if n else torch.device("cuda")
    u0_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64) if n else np.zeros(0, np.int64)
    U_off = np.concatenate([[0], np.cumsum(outs)[:-1]]).astype(np.int64) if n else np.zeros(0, np.int64)
    u0 = torch.cat([u.reshape(-1) for u in u0s]) if n else torch.zeros(1, dtype=torch.float64, device=dev)
    U = torch.empty(max(int(sum(outs)), 1), dtype=torch.float64, device=dev)
    op = _lib.OP_SERIAL if parareal_sweeps is None else _lib.OP_PARAREAL
    nb = int(_lib.lib().l1pr_batch_workspace_bytes(arr, n, op))
    if nb == 0:
        raise _lib.L1prError(_lib.EINVAL, "l1pr_batch_workspace_bytes")
    ws = workspace if workspace is not None else torch.empty(nb, dtype=torch.uint8, device=dev)
    i64 = ctypes.POINTER(ctypes.c_int64)
    st = _lib.lib().l1pr_solve_batch(arr, n, op, int(parareal_sweeps or 0), int(coarse),
                                     _ptr(mlp_params), int(mlp_modes), _ptr(u0),
                                     u0_off.ctypes.data_as(i64), _ptr(U), U_off.ctypes.data_as(i64),
                                     _ptr(ws), ws.numel() * ws.element_size(), _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_solve_batch")
    return [U[o:o + k].view(p.slices + 1, m) for o, k, p, m in zip(U_off, outs, problems, sizes)]


def device_stamp(t: torch.Tensor):
    """Device wall clock into t[0] (int64) when the current stream reaches this point."""
    st = _lib.lib().l1pr_device_stamp(_ptr(t), _stream())
    if st != _lib.OK:
        raise _lib.L1prError(st, "l1pr_device_stamp")


def wall_clock_khz() -> int:
    return int(_lib.lib().l1pr_wall_clock_khz())
