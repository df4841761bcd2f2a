"""GPU tests of the 2D step solve by preconditioned conjugate gradients (solver = 1): the
stiffness applied separably at the Gauss points, the constant-coefficient sine operator as
preconditioner, stop at ||r|| <= 1e-14 ||rhs||.

Bars: serial trajectories and parareal iterates against the oracle's direct solves at 1e-10
relative L2; at full size (64 x 64 modes, 96 x 96 points) the step equation on sampled rows
with the oracle's own rows of K; parareal exact bit for bit against the GPU serial solve with
the same solver; an instance's result independent of its batch; agreement with the GPU's
Cholesky path."""
import math

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


def c3(**kw):
    base = dict(W.C3)
    base.update(kw)
    return base


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def u0_2d(M, seeds):
    return np.stack([W.u0_random_2d(M, s) for s in seeds])


CASES = {
    "M4_Q8": c3(modes=4, quad=8, steps=16, slices=4),
    "ragged_M5_Q9": c3(modes=5, quad=9, steps=12, slices=3, alpha=0.35),
    "mms_M3": c3(modes=3, quad=8, steps=16, slices=4, d_sel=1, f_sel=1, alpha=0.5),
    "full_history_M4": c3(modes=4, quad=8, steps=12, slices=3, history=1),
    "M18_Q27": c3(modes=18, quad=27, steps=4, slices=2),
    "M24_Q36_a09": c3(modes=24, quad=36, steps=6, slices=2, alpha=0.9),
}


@pytest.mark.parametrize("name", list(CASES))
def test_cg_serial_matches_oracle(gpu, orc, name):
    kw = CASES[name]
    print(f"[cg2d] {name}", flush=True)
    pg, po = gpu.make_problem(solver=1, **kw), orc.problem(**kw)
    u0 = u0_2d(kw["modes"], [3, 4])
    U, tr = gpu.solve_serial(pg, dev(u0), want_traj=True)
    U, tr = U.cpu().numpy(), tr.cpu().numpy()
    for b in range(2):
        Uo, tro = orc.solve_serial(po, u0[b], want_traj=True)
        assert rel(U[b], Uo) <= TOL, (name, b, rel(U[b], Uo))
        per = [rel(tr[b][m], tro[m]) for m in range(tro.shape[0])]
        assert max(per) <= TOL, (name, b, max(per))


def test_cg_parareal_exact_and_matches_oracle(gpu, orc):
    kw = c3(modes=6, quad=10, steps=12, slices=3, alpha=0.45)
    pg, po = gpu.make_problem(solver=1, **kw), orc.problem(**kw)
    u0 = u0_2d(6, [7])
    Us, _ = gpu.solve_serial(pg, dev(u0))
    r = gpu.solve_parareal(pg, dev(u0), 3, tol=0.0, want_iterates=True)
    _, ko, _, ito = orc.solve_parareal(po, u0[0], 3, want_iterates=True)
    its = r.iterates.cpu().numpy()
    for k in range(4):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k
        assert rel(its[k, 0], ito[k]) <= TOL, (k, rel(its[k, 0], ito[k]))
    assert torch.equal(r.U, Us)


def test_cg_batch_independent_and_close_to_cholesky(gpu):
    kw = c3(modes=20, quad=30, steps=6, slices=2, alpha=0.7)
    u0 = u0_2d(20, [8, 9, 10])
    pc, pd = gpu.make_problem(solver=1, **kw), gpu.make_problem(**kw)
    U3, _ = gpu.solve_serial(pc, dev(u0))
    for b in range(3):
        U1, _ = gpu.solve_serial(pc, dev(u0[b:b + 1]))
        assert torch.equal(U1[0], U3[b]), b
    Ud, _ = gpu.solve_serial(pd, dev(u0))
    assert rel(U3.cpu().numpy(), Ud.cpu().numpy()) <= 1e-12


def test_cg_full_size_first_step_rows_match_oracle(gpu, orc):
    """One config-3 step at full size (4096 coefficients, 96 x 96 points) by conjugate
    gradients: on sampled rows the GPU state c1 satisfies c1 + tau K(c0) c1 = c0 + tau F(c0)
    with the oracle's rows of K and F."""
    T = 1.0 / 2048
    kw = c3(steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(solver=1, **kw), orc.problem(**kw)
    c0 = W.u0_random_2d(kw["modes"], 0)
    _, tr = gpu.solve_serial(pg, dev(c0[None]), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    Md = kw["modes"] ** 2
    rows = sorted({0, 1, 63, 64, Md - 1, *np.random.default_rng(18).choice(Md, 11, replace=False).tolist()})
    Kr, F = orc.galerkin_rows(po, c0, 0.0, 0.0, rows)
    for i, k in enumerate(rows):
        lhs = c1[k] + tau * (Kr[i] @ c1)
        rhs = c0[k] + tau * F[k]
        scale = abs(c1[k]) + tau * (np.abs(Kr[i]) @ np.abs(c1)) + abs(c0[k]) + tau * abs(F[k])
        assert abs(lhs - rhs) <= TOL * scale, (k, abs(lhs - rhs) / scale)


def test_cg_full_size_parareal_exact(gpu):
    kw = c3(steps=16, slices=4, T=16.0 / 2048)
    pg = gpu.make_problem(solver=1, **kw)
    u0 = dev(W.u0_random_2d(kw["modes"], 1)[None])
    Us, _ = gpu.solve_serial(pg, u0)
    r = gpu.solve_parareal(pg, u0, 4, tol=0.0, want_iterates=True)
    for k in range(5):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k
    assert torch.equal(r.U, Us)
