"""Status reporting through the C-ABI: the per-instance stop rule of parareal (the flowchart's
test on the increment, applied to each instance), the per-instance status array, the device
status word read by l1pr_check (non-finite states with no host synchronisation, a bounded
device wait that gives up).  Parity of the per-instance stop against the oracle, whose
parareal stops each single instance at its own first sweep that meets the tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_11023_amd import workloads as W  # noqa: E402

TOL = 1e-10


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


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


def test_per_instance_stop_matches_oracle(gpu, orc):
    """Instances with different orders stop at different sweeps: each stops at the oracle's
    own sweep count for that instance, with the oracle's iterate, and its status says so."""
    kw = W.with_(W.C2, modes=32, quad=48, steps=64, slices=16)
    alphas = [0.3, 0.7, 1.0]
    u0 = W.u0_batch_1d(32, [60, 61, 62])
    p = gpu.make_problem(**kw)
    tol = 1e-7
    res = gpu.solve_parareal(p, dev(u0), 16, tol=tol, alpha=alphas)
    torch.cuda.synchronize()
    assert res.status == 0
    inst = res.inst.cpu().numpy()
    U = res.U.cpu().numpy()
    ks = []
    for b, a in enumerate(alphas):
        po = orc.problem(**W.with_(kw, alpha=a))
        Uo, ko, _, _ = orc.solve_parareal(po, u0[b], 16, tol=tol)
        assert inst[b] == ko, (b, inst[b], ko)
        assert rel(U[b], Uo) <= TOL, (b, rel(U[b], Uo))
        ks.append(ko)
    assert res.iters == max(ks)
    assert len(set(ks)) > 1  # the instances really stopped at different sweeps
    # a finished instance holds exactly the iterate of a run with its own sweep count
    for b, a in enumerate(alphas):
        own = gpu.solve_parareal(p, dev(u0[b:b + 1]), ks[b], tol=0.0, alpha=[a])
        assert torch.equal(own.U[0], res.U[b]), b


def test_status_without_stop_test(gpu):
    """tol = 0: every instance runs max_iter sweeps (status = max_iter), or P sweeps (exact)."""
    kw = W.with_(W.C2, modes=16, quad=24, steps=32, slices=8, alpha=0.5)
    p = gpu.make_problem(**kw)
    u0 = dev(W.u0_batch_1d(16, [1, 2]))
    r = gpu.solve_parareal(p, u0, 3, tol=0.0)
    assert r.inst.tolist() == [3, 3] and r.status == 0
    r = gpu.solve_parareal(p, u0, 8, tol=0.0)
    assert r.inst.tolist() == [8, 8]
    assert gpu.check(r.workspace) == 0
    # a tolerance that cannot be met within max_iter < P: ENOTCONV in the call and per instance
    r = gpu.solve_parareal(p, u0, 2, tol=1e-15)
    assert r.status == -4 and r.inst.tolist() == [-4, -4]


def test_nonfinite_reported_without_synchronisation(gpu):
    """A NaN initial coefficient: the serial solve and tol = 0 parareal (no host
    synchronisation) report it through the status word; parareal also per instance, and the
    finite instance of the batch is unaffected."""
    from paper_2510_11023_amd import _lib

    kw = W.with_(W.C2, modes=16, quad=24, steps=32, slices=8, alpha=0.5)
    p = gpu.make_problem(**kw)
    u0 = W.u0_batch_1d(16, [3, 4])
    bad = u0.copy()
    bad[1, 2] = np.nan
    ws = torch.empty(gpu.workspace_bytes(p, 2, _lib.OP_SERIAL), dtype=torch.uint8, device="cuda")
    gpu.solve_serial(p, dev(bad), workspace=ws)
    assert gpu.check(ws) == _lib.ENONFINITE
    gpu.solve_serial(p, dev(u0), workspace=ws)
    assert gpu.check(ws) == _lib.OK  # the next call clears the word
    r = gpu.solve_parareal(p, dev(bad), 4, tol=0.0)
    assert gpu.check(r.workspace) == _lib.ENONFINITE
    assert r.inst.tolist() == [4, _lib.ENONFINITE]
    good = gpu.solve_parareal(p, dev(u0[:1]), 4, tol=0.0).U
    assert torch.equal(r.U[0], good[0])
    # with a stop test the call itself returns ENONFINITE
    with pytest.raises(_lib.L1prError) as ei:
        gpu.solve_parareal(p, dev(bad), 8, tol=1e-9)
    assert ei.value.status == _lib.ENONFINITE


def test_bounded_wait_give_up_is_reported(gpu, monkeypatch):
    """The factor kernel's bounded waits, forced to give up at once from the host (poll limit
    0; every kernel still runs to its end): the status word reports EWAIT, and a parareal call
    with a stop test returns it.  With the default limit the same calls report OK."""
    from paper_2510_11023_amd import _lib

    kw = W.with_(W.C2, modes=32, quad=48, steps=16, slices=4, alpha=0.5)
    p = gpu.make_problem(**kw)
    u0 = dev(W.u0_batch_1d(32, [5]))
    ws = torch.empty(gpu.workspace_bytes(p, 1, _lib.OP_SERIAL), dtype=torch.uint8, device="cuda")
    monkeypatch.setenv("L1PR_TEST_SPIN_LIMIT", "0")
    gpu.solve_serial(p, u0, workspace=ws)
    assert gpu.check(ws) == _lib.EWAIT
    with pytest.raises(_lib.L1prError) as ei:
        gpu.solve_parareal(p, u0, 4, tol=1e-9)
    assert ei.value.status == _lib.EWAIT
    monkeypatch.delenv("L1PR_TEST_SPIN_LIMIT")
    gpu.solve_serial(p, u0, workspace=ws)
    assert gpu.check(ws) == _lib.OK
