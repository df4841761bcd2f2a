"""The serial solve that allocates nothing (l1pr_solve_serial_noalloc, for callers that cannot
allocate device memory) against the serial solve with a caller workspace (l1pr_solve_serial),
through the C-ABI.  Two calls in a row, the second on a smaller input, so that whatever the
first call left in the library's scratch array must not leak into the second.  Both entry
points run the same kernels on the same data, so the results must agree bit for bit (and so
within the 1e-10 parity bar)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_11023_amd import workloads as W  # noqa: E402

TOL = 1e-10


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_11023_amd as l1
    from paper_2510_11023_amd import _lib

    _lib.lib()
    return l1


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def noalloc(p, u0, U, traj):
    from paper_2510_11023_amd import _lib

    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return _lib.lib().l1pr_solve_serial_noalloc(ctypes.byref(p), u0.shape[0], None, ptr(u0),
                                                ptr(U), ptr(traj), stream)


def test_noalloc_matches_workspace_call_twice(gpu):
    # first call: 3 instances, M = 64, with the fine trajectory; second call: 1 instance, a
    # smaller problem (M = 32, fewer steps), no trajectory
    cases = [
        (W.with_(W.C2, modes=64, quad=96, steps=128, slices=8, alpha=0.4), [1, 2, 3], True),
        (W.with_(W.C1, steps=64), None, False),
    ]
    for kw, seeds, want_traj in cases:
        p = gpu.make_problem(**kw)
        if seeds is None:
            u0 = dev(W.u0_sine_mode(kw["modes"])[None, :])
        else:
            u0 = dev(W.u0_batch_1d(kw["modes"], seeds))
        B, M = u0.shape
        U = torch.full((B, kw["slices"] + 1, M), float("nan"), dtype=torch.float64, device="cuda")
        traj = (torch.full((B, kw["steps"] + 1, M), float("nan"), dtype=torch.float64, device="cuda")
                if want_traj else None)
        st = noalloc(p, u0, U, traj)
        assert st == 0, st
        Uw, trw = gpu.solve_serial(p, u0, want_traj=want_traj)
        torch.cuda.synchronize()
        assert rel(U, Uw) <= TOL
        assert torch.equal(U, Uw)
        if want_traj:
            assert torch.equal(traj, trw)


def test_noalloc_rejects_beyond_scratch(gpu):
    from paper_2510_11023_amd import _lib

    # the 1D shape M = 256, N = 4096 with 256 instances needs more than the 64 MiB array
    p = gpu.make_problem(**W.with_(W.C2, alpha=0.3))
    assert gpu.workspace_bytes(p, 256, _lib.OP_SERIAL) > _lib.NOALLOC_SCRATCH_BYTES
    u0 = torch.zeros((256, 256), dtype=torch.float64, device="cuda")
    U = torch.zeros((256, 65, 256), dtype=torch.float64, device="cuda")
    assert noalloc(p, u0, U, None) == _lib.ENOMEM
    assert int(torch.count_nonzero(U)) == 0  # nothing was launched
    # an invalid problem is rejected as by l1pr_solve_serial
    bad = gpu.make_problem(**W.with_(W.C1, alpha=1.5))
    assert noalloc(bad, u0[:1, :32].contiguous(), U, None) == _lib.EINVAL
