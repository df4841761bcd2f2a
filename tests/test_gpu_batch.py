"""GPU: the heterogeneous batch call (l1pr_solve_batch).  Problems that differ in modes, steps,
order, quadrature, dimension and history run as groups in one call; every problem's result
equals its own single-problem run bit for bit, and the oracle to 1e-10."""
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


def base1d(**kw):
    return W.with_(W.C2, quad=64, slices=4, T=1.0, **kw)


# (problem keywords, seed); the comment names the group each lands in
PROBLEMS = [
    (base1d(modes=24, steps=16, alpha=0.3), 1),          # uneven, padded 32
    (base1d(modes=30, steps=24, alpha=0.6), 2),          # uneven, padded 32
    (dict(W.C3, modes=4, quad=8, steps=8, slices=4, alpha=0.5), 3),   # 2D
    (base1d(modes=40, steps=12, alpha=0.5), 4),          # uneven, padded 48
    (base1d(modes=32, steps=16, alpha=0.8), 5),          # uneven, padded 32
    (W.with_(base1d(modes=24, steps=16, alpha=0.4), quad=80), 6),   # its own quadrature
    (dict(W.C3, modes=4, quad=8, steps=8, slices=4, alpha=0.7), 7),   # 2D, same group as above
]


def u0_of(kw, seed):
    if kw["dim"] == 2:
        return W.u0_random_2d(kw["modes"], seed)
    return W.u0_random_1d(kw["modes"], seed)


def test_batch_serial_equals_single_runs_and_oracle(gpu, orc):
    full = (base1d(modes=16, steps=8, alpha=0.5, history=1), 8)  # full history: its own group
    probs = PROBLEMS + [full]
    ps = [gpu.make_problem(**kw) for kw, _ in probs]
    u0s = [torch.tensor(u0_of(kw, s), device="cuda") for kw, s in probs]
    outs = gpu.solve_batch(ps, u0s)
    for (kw, s), p, u, U in zip(probs, ps, u0s, outs):
        own, _ = gpu.solve_serial(p, u[None])
        assert torch.equal(U, own[0]), kw
        ref = orc.solve_serial(orc.problem(**kw), u0_of(kw, s))
        assert rel(U.cpu().numpy(), ref) <= TOL, (kw, rel(U.cpu().numpy(), ref))


def test_batch_parareal_equals_single_runs(gpu):
    ps = [gpu.make_problem(**kw) for kw, _ in PROBLEMS]
    u0s = [torch.tensor(u0_of(kw, s), device="cuda") for kw, s in PROBLEMS]
    outs = gpu.solve_batch(ps, u0s, parareal_sweeps=2)
    for (kw, s), p, u, U in zip(PROBLEMS, ps, u0s, outs):
        own = gpu.solve_parareal(p, u[None], 2, tol=0.0).U
        assert torch.equal(U, own[0]), kw


def test_batch_constant_d_diagonal_groups(gpu, orc):
    """Problems with the diagonal solve (solver = 2) never join an uneven group (which runs
    the factorisation only): each size runs as its own plain group, equal to its single run
    and to the oracle."""
    probs = [(base1d(modes=24, steps=16, alpha=0.3, d_sel=0, d_param=0.7), 1),
             (base1d(modes=30, steps=16, alpha=0.6, d_sel=0, d_param=0.7), 2),
             (base1d(modes=30, steps=16, alpha=0.6, d_sel=0, d_param=0.7), 3),
             (dict(W.C3, modes=4, quad=8, steps=8, slices=4, d_sel=0, d_param=0.7), 4)]
    ps = [gpu.make_problem(solver=2, **kw) for kw, _ in probs] + [gpu.make_problem(**PROBLEMS[0][0])]
    u0s = [torch.tensor(u0_of(kw, s), device="cuda") for kw, s in probs + [PROBLEMS[0]]]
    outs = gpu.solve_batch(ps, u0s)
    for i, (p, u, U) in enumerate(zip(ps, u0s, outs)):
        own, _ = gpu.solve_serial(p, u[None])
        assert torch.equal(U, own[0]), i
    for (kw, s), U in zip(probs, outs):
        ref = orc.solve_serial(orc.problem(solver=2, **kw), u0_of(kw, s))
        assert rel(U.cpu().numpy(), ref) <= TOL, (kw, rel(U.cpu().numpy(), ref))


def test_batch_rejects_before_launching(gpu):
    from paper_2510_11023_amd import _lib

    kw, s = PROBLEMS[0]
    good = gpu.make_problem(**kw)
    hist = gpu.make_problem(**W.with_(kw, history=1))
    u = torch.tensor(u0_of(kw, s), device="cuda")
    with pytest.raises(_lib.L1prError):
        gpu.solve_batch([good, hist], [u, u.clone()], parareal_sweeps=1)
    bad = gpu.make_problem(**W.with_(kw, alpha=1.5))
    with pytest.raises(_lib.L1prError):
        gpu.solve_batch([good, bad], [u, u.clone()])
