"""GPU parity of the sum-of-exponentials history (history = 2, the fast history of the paper's
outlook, Conclusions (i)): the uniform L1 scheme whose history terms at distances >= 16 use
the weights sum_l w_l exp(-lam_l d), carried as exponential sums from step to step.  Against
the oracle's history = 2 at 1e-10 relative (slice ends and every fine state), bit for bit
equal to the exact full history while no step reaches the far part, and within the error
budget of the approximation (1e-11) of the exact full history at the config-2 shape."""
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


CASES = [
    ("1d_a03", W.with_(W.C2, modes=32, quad=48, steps=512, slices=8, alpha=0.3), [1, 2]),
    ("1d_a07_ragged", W.with_(W.C2, modes=40, quad=61, steps=300, slices=5, alpha=0.7, d_sel=3, f_sel=3), [3]),
    ("1d_diag", W.with_(W.C2, modes=24, quad=48, steps=200, slices=4, alpha=0.45, d_sel=0, d_param=0.8), [4]),
    ("2d_a06", dict(W.C3, modes=6, quad=9, steps=96, slices=4), [5]),
]


def _u0(kw, seeds):
    if kw["dim"] == 2:
        return np.stack([W.u0_random_2d(kw["modes"], s) for s in seeds])
    return W.u0_batch_1d(kw["modes"], seeds)


@pytest.mark.parametrize("name,kw,seeds", CASES, ids=[c[0] for c in CASES])
def test_soe_serial_matches_oracle(gpu, orc, name, kw, seeds):
    solver = 2 if kw.get("d_sel", 1) == 0 else 0
    pg = gpu.make_problem(**dict(kw, history=2, solver=solver))
    po = orc.problem(**dict(kw, history=2, solver=solver))
    u0 = _u0(kw, seeds)
    U, tr = gpu.solve_serial(pg, dev(u0), want_traj=True)
    U, tr = U.cpu().numpy(), tr.cpu().numpy()
    for b in range(len(seeds)):
        Uo, tro = orc.solve_serial(po, u0[b], want_traj=True)
        assert rel(U[b], Uo) <= TOL, (name, b, rel(U[b], Uo))
        per = [rel(tr[b][m], tro[m]) for m in range(tro.shape[0]) if np.linalg.norm(tro[m]) > 0]
        assert max(per) <= TOL, (name, b, max(per))


def test_soe_per_instance_alpha(gpu, orc):
    """One batch, three orders (each instance its own node table; at alpha = 1 no far part)."""
    kw = W.with_(W.C2, modes=32, quad=48, steps=256, slices=8)
    alphas = [0.25, 0.6, 1.0]
    u0 = W.u0_batch_1d(32, [7, 8, 9])
    pg = gpu.make_problem(**W.with_(kw, history=2))
    U, _ = gpu.solve_serial(pg, dev(u0), alpha=alphas)
    U = U.cpu().numpy()
    for b, a in enumerate(alphas):
        Uo = orc.solve_serial(orc.problem(**W.with_(kw, alpha=a, history=2)), u0[b])
        assert rel(U[b], Uo) <= TOL, (a, rel(U[b], Uo))


def test_soe_equals_full_history_below_the_near_window(gpu):
    """N = 16 steps: no step reaches distance 16, so history 2 is history 1 bit for bit."""
    kw = W.with_(W.C2, modes=48, quad=72, steps=16, slices=4, alpha=0.35)
    u0 = dev(W.u0_batch_1d(48, [10, 11]))
    U1, t1 = gpu.solve_serial(gpu.make_problem(**W.with_(kw, history=1)), u0, want_traj=True)
    U2, t2 = gpu.solve_serial(gpu.make_problem(**W.with_(kw, history=2)), u0, want_traj=True)
    assert torch.equal(U1, U2) and torch.equal(t1, t2)


@pytest.mark.parametrize("alpha", [0.3, 0.7])
def test_soe_error_budget_at_config2_shape(gpu, alpha):
    """M = 256, Q = 384, N = 4096 (config-2 shape, 4 instances): the approximate history stays
    within 1e-11 of the exact full history."""
    kw = W.with_(W.C2, alpha=alpha)
    u0 = dev(W.u0_batch_1d(256, range(4)))
    U1, _ = gpu.solve_serial(gpu.make_problem(**W.with_(kw, history=1)), u0)
    U2, _ = gpu.solve_serial(gpu.make_problem(**W.with_(kw, history=2)), u0)
    gap = rel(U2.cpu().numpy(), U1.cpu().numpy())
    assert gap <= 1e-11, gap


def test_soe_rejected_by_parareal(gpu):
    from paper_2510_11023_amd import _lib

    p = gpu.make_problem(**W.with_(W.C2, modes=16, quad=24, steps=64, slices=4, history=2))
    with pytest.raises(_lib.L1prError) as ei:
        gpu.solve_parareal(p, dev(W.u0_batch_1d(16, [0])), 2)
    assert ei.value.status == _lib.EINVAL
