"""ctypes binding of libl1pr.so (include/l1pr.h).

Argument marshalling only: every step of the solver runs in the HIP library.  PyTorch
supplies device memory and the current stream.  The library must be built
(``python -m paper_2510_11023_amd.build``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libl1pr.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, ENONFINITE, ESOLVE, EWAIT = 0, -1, -2, -3, -4, -5, -6, -7
OP_SERIAL, OP_PARAREAL = 0, 1
# bytes of the per-device array that l1pr_solve_serial_noalloc works in (include/l1pr.h)
NOALLOC_SCRATCH_BYTES = 64 << 20


class Problem(ctypes.Structure):
    """Mirror of l1pr_problem."""

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
        ("assembly", ctypes.c_int32),
        ("tune", ctypes.c_int32),
        ("solver", ctypes.c_int32),
    ]


class Uneven(ctypes.Structure):
    """Mirror of l1pr_uneven (device pointers, the coarse propagator and its network)."""

    _fields_ = [("modes", ctypes.c_void_p), ("spp", ctypes.c_void_p), ("alpha", ctypes.c_void_p),
                ("coarse", ctypes.c_int32), ("mlp", ctypes.c_void_p), ("mlp_modes", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    """Mirror of l1pr_kernel_stat."""

    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class MlpInfo(ctypes.Structure):
    """Mirror of l1pr_mlp_info."""

    _fields_ = [("in_", ctypes.c_int32), ("in_padded", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("out", ctypes.c_int32), ("out_padded", ctypes.c_int32),
                ("param_bytes", ctypes.c_size_t), ("state_bytes", ctypes.c_size_t),
                ("flat_count", ctypes.c_int64),
                ("off_in_mean", ctypes.c_size_t), ("off_in_std", ctypes.c_size_t),
                ("off_out_mean", ctypes.c_size_t), ("off_out_std", ctypes.c_size_t),
                ("off_w", ctypes.c_size_t * 4), ("off_b", ctypes.c_size_t * 4),
                ("flat_w", ctypes.c_int64 * 4), ("flat_b", ctypes.c_int64 * 4)]


class L1prError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} (status {status})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2510_11023_amd.build); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        pp = ctypes.POINTER(Problem)
        L.l1pr_workspace_bytes.argtypes = [pp, ctypes.c_int32, ctypes.c_int32]
        L.l1pr_workspace_bytes.restype = ctypes.c_size_t
        L.l1pr_validate.argtypes = [pp]
        L.l1pr_validate.restype = ctypes.c_int
        L.l1pr_solve_serial.argtypes = [pp, ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.l1pr_solve_serial.restype = ctypes.c_int
        L.l1pr_solve_serial_noalloc.argtypes = [pp, ctypes.c_int32, vp, vp, vp, vp, vp]
        L.l1pr_solve_serial_noalloc.restype = ctypes.c_int
        L.l1pr_solve_parareal.argtypes = [pp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32,
                                          ctypes.c_double, ctypes.c_int32, vp, vp, vp, vp,
                                          ctypes.POINTER(ctypes.c_int32), vp, ctypes.c_size_t, vp]
        L.l1pr_solve_parareal.restype = ctypes.c_int
        L.l1pr_check.argtypes = [vp, vp]
        L.l1pr_check.restype = ctypes.c_int
        L.l1pr_parareal_learned_extra_bytes.argtypes = [pp, ctypes.c_int32]
        L.l1pr_parareal_learned_extra_bytes.restype = ctypes.c_size_t
        for name in ("l1pr_coarse_apply", "l1pr_fine_apply"):
            f = getattr(L, name)
            f.argtypes = [pp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_size_t, vp]
            f.restype = ctypes.c_int
        L.l1pr_mlp_layout.argtypes = [ctypes.c_int32, ctypes.POINTER(MlpInfo)]
        L.l1pr_mlp_layout.restype = ctypes.c_int
        L.l1pr_mlp_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.l1pr_mlp_workspace_bytes.restype = ctypes.c_size_t
        L.l1pr_mlp_sync.argtypes = [ctypes.c_int32, vp, vp, vp]
        L.l1pr_mlp_sync.restype = ctypes.c_int
        L.l1pr_mlp_reset_moments.argtypes = [ctypes.c_int32, vp, vp]
        L.l1pr_mlp_reset_moments.restype = ctypes.c_int
        L.l1pr_mlp_stats.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int64, vp, vp]
        L.l1pr_mlp_stats.restype = ctypes.c_int
        L.l1pr_mlp_features.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                        vp, vp, vp]
        L.l1pr_mlp_features.restype = ctypes.c_int
        L.l1pr_mlp_forward.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp,
                                       ctypes.c_size_t, vp]
        L.l1pr_mlp_forward.restype = ctypes.c_int
        L.l1pr_solve_serial_uneven.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32,
                                               ctypes.POINTER(Uneven), vp, vp, vp, ctypes.c_size_t,
                                               vp]
        L.l1pr_solve_serial_uneven.restype = ctypes.c_int
        L.l1pr_solve_parareal_uneven.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32,
                                                 ctypes.POINTER(Uneven), vp, vp, ctypes.c_int32,
                                                 ctypes.c_double, vp, vp, vp, vp, ctypes.c_size_t,
                                                 vp]
        L.l1pr_solve_parareal_uneven.restype = ctypes.c_int
        L.l1pr_batch_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_int32]
        L.l1pr_batch_workspace_bytes.restype = ctypes.c_size_t
        L.l1pr_solve_batch.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32, vp,
                                       ctypes.POINTER(ctypes.c_int64), vp,
                                       ctypes.POINTER(ctypes.c_int64), vp, ctypes.c_size_t, vp]
        L.l1pr_solve_batch.restype = ctypes.c_int
        L.l1pr_device_stamp.argtypes = [vp, vp]
        L.l1pr_device_stamp.restype = ctypes.c_int
        L.l1pr_wall_clock_khz.argtypes = []
        L.l1pr_wall_clock_khz.restype = ctypes.c_int64
        L.l1pr_autotune.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, vp, ctypes.c_size_t,
                                    vp, ctypes.POINTER(ctypes.c_int32)]
        L.l1pr_autotune.restype = ctypes.c_int
        L.l1pr_mlp_infer.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp,
                                     ctypes.c_size_t, vp]
        L.l1pr_mlp_infer.restype = ctypes.c_int
        L.l1pr_mlp_infer_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.l1pr_mlp_infer_workspace_bytes.restype = ctypes.c_size_t
        L.l1pr_mlp_train_step.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_int32,
                                          ctypes.c_float, ctypes.c_int32, vp, vp, vp,
                                          ctypes.c_size_t, vp]
        L.l1pr_mlp_train_step.restype = ctypes.c_int
        L.l1pr_profile_start.argtypes = []
        L.l1pr_profile_start.restype = None
        L.l1pr_profile_start_only.argtypes = [ctypes.c_char_p]
        L.l1pr_profile_start_only.restype = None
        L.l1pr_profile_stop.argtypes = [ctypes.POINTER(KernelStat), ctypes.c_int32]
        L.l1pr_profile_stop.restype = ctypes.c_int32
        L.l1pr_status_string.argtypes = [ctypes.c_int]
        L.l1pr_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().l1pr_status_string(int(status)).decode()


def profile_start(only=None):
    """Bracket every step kernel with HIP events, or only the kernels named in `only` (an
    iterable of names such as "chol", "history")."""
    if only:
        lib().l1pr_profile_start_only(",".join(only).encode())
    else:
        lib().l1pr_profile_start()


def profile_stop():
    """Returns {"kernel/mode/units": (launches, total_ms)} for the launches since profile_start()."""
    cap = 512
    buf = (KernelStat * cap)()
    n = lib().l1pr_profile_stop(buf, cap)
    if n < 0:
        raise L1prError(EHIP, "l1pr_profile_stop")
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(n, cap))}
