"""GPU tests of the constant-D diagonal step solve (solver = 2): the sine basis diagonalises the
stiffness, D (grad phi_k, grad phi_l) = D lambda_k delta_kl, so a step is
c_k = (hist_k + tau F_k) / (1 + tau D lambda_k) with the load F by Gauss quadrature.

Bars: serial trajectories and parareal iterates against the oracle's solver = 2 at 1e-10
relative L2 (1D below and above 256 modes, 2D, hybrid and full history); backward Euler in closed form at alpha = 1; at the full config-2
shape every coefficient of one step against the oracle's load; parareal exact bit for bit
against the GPU serial solve; an instance's result independent of its batch; agreement with
the Cholesky path where the quadrature makes the stiffness diagonal to rounding."""
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


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def const_d(base, **kw):
    out = dict(base)
    out.update(d_sel=0, d_param=0.8)
    out.update(kw)
    return out


def u0_of(kw, seeds):
    if kw["dim"] == 1:
        return W.u0_batch_1d(kw["modes"], seeds)
    return np.stack([W.u0_random_2d(kw["modes"], s) for s in seeds])


CASES = {
    "1d_M24_Q32": const_d(W.C2, modes=24, quad=32, steps=16, slices=4, alpha=0.55),
    "1d_ragged_M13_Q17_sin": const_d(W.C2, modes=13, quad=17, steps=12, slices=3, alpha=0.3,
                                     f_sel=3),
    "1d_full_history_M16": const_d(W.C2, modes=16, quad=24, steps=12, slices=3, history=1),
    "1d_M300_Q310": const_d(W.C2, modes=300, quad=310, steps=4, slices=2, alpha=0.7),
    "1d_alpha1": const_d(W.C2, modes=20, quad=30, steps=8, slices=2, alpha=1.0),
    "2d_M6_Q9": const_d(W.C3, modes=6, quad=9, steps=12, slices=3),
    "2d_ragged_M7_Q10_logistic": const_d(W.C3, modes=7, quad=10, steps=9, slices=3, alpha=0.85,
                                         f_sel=2),
    "2d_full_history_M4": const_d(W.C3, modes=4, quad=8, steps=12, slices=3, history=1),
    "2d_M12_Q18": const_d(W.C3, modes=12, quad=18, steps=8, slices=2, alpha=0.6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_diag_serial_matches_oracle(gpu, orc, name):
    kw = CASES[name]
    print(f"[diag] {name}", flush=True)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    u0 = u0_of(kw, [3, 4])
    U, tr = gpu.solve_serial(pg, dev(u0), want_traj=True)
    U, tr = U.cpu().numpy(), tr.cpu().numpy()
    for b in range(2):
        Uo, tro = orc.solve_serial(po, u0[b], want_traj=True)
        assert rel(U[b], Uo) <= TOL, (name, b, rel(U[b], Uo))
        per = [rel(tr[b][m], tro[m]) for m in range(tro.shape[0])]
        assert max(per) <= TOL, (name, b, max(per))


@pytest.mark.parametrize("dim", [1, 2])
def test_diag_backward_euler_closed_form(gpu, dim):
    """alpha = 1, f = 0: every mode decays as c_k(0) (1 + dt D lambda_k)^(-m)."""
    M = 12 if dim == 1 else 5
    kw = const_d(W.C2 if dim == 1 else W.C3, modes=M, quad=M, steps=12, slices=3, alpha=1.0,
                 f_sel=0, history=1)
    print(f"[diag] backward Euler dim={dim}", flush=True)
    u0 = u0_of(kw, [9])
    _, tr = gpu.solve_serial(gpu.make_problem(solver=2, **kw), dev(u0), want_traj=True)
    if dim == 1:
        lam = (np.arange(1, M + 1) * math.pi) ** 2
    else:
        k1, k2 = np.meshgrid(np.arange(1, M + 1), np.arange(1, M + 1), indexing="ij")
        lam = ((k1 ** 2 + k2 ** 2) * math.pi ** 2).ravel()
    ref = u0[0][None, :] * (1.0 + (1.0 / 12) * 0.8 * lam[None, :]) ** (-np.arange(13)[:, None])
    got = tr[0].cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", ["1d_M24_Q32", "1d_full_history_M16", "2d_M6_Q9",
                                  "1d_M300_Q310"])
def test_diag_parareal_exact_and_matches_oracle(gpu, orc, name):
    kw = CASES[name]
    P = kw["slices"]
    print(f"[diag] parareal {name}", flush=True)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    u0 = u0_of(kw, [7])
    Us, _ = gpu.solve_serial(pg, dev(u0))
    r = gpu.solve_parareal(pg, dev(u0), P, tol=0.0, want_iterates=True)
    _, _, _, ito = orc.solve_parareal(po, u0[0], P, want_iterates=True)
    its = r.iterates.cpu().numpy()
    for k in range(P + 1):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k
        assert rel(its[k, 0], ito[k]) <= TOL, (k, rel(its[k, 0], ito[k]))
    assert torch.equal(r.U, Us)


@pytest.mark.parametrize("tune", [1, 2, 3])
def test_diag_tile_variants_match_oracle_and_stay_exact(gpu, orc, tune):
    """The GEMM tile variants (tune bits 0 and 1) change the load vector's summation order
    only: serial against the oracle at 1e-10, parareal exact against the serial solve."""
    kw = CASES["1d_M24_Q32"]
    print(f"[diag] tune={tune}", flush=True)
    pg, po = gpu.make_problem(solver=2, tune=tune, **kw), orc.problem(solver=2, **kw)
    u0 = u0_of(kw, [5, 6])
    Us, _ = gpu.solve_serial(pg, dev(u0))
    for b in range(2):
        assert rel(Us[b].cpu().numpy(), orc.solve_serial(po, u0[b])) <= TOL, b
    r = gpu.solve_parareal(pg, dev(u0), 2, tol=0.0, want_iterates=True)
    for k in range(3):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k


def test_diag_full_shape_first_step_every_coefficient(gpu, orc):
    """One step at the config-2 shape with constant D (256 modes, 384 points): every GPU
    coefficient satisfies c1_k (1 + tau D lambda_k) = c0_k + tau F_k with the oracle's load."""
    T = 1.0 / 4096
    kw = const_d(W.C2, steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    c0 = W.u0_batch_1d(kw["modes"], [0])
    _, tr = gpu.solve_serial(pg, dev(c0), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    _, F = orc.galerkin_rows(po, c0[0], 0.0, 0.0, [0])
    lam = (np.arange(1, kw["modes"] + 1) * math.pi) ** 2
    lhs = c1 * (1.0 + tau * 0.8 * lam)
    rhs = c0[0] + tau * F
    scale = np.abs(lhs) + np.abs(c0[0]) + tau * np.abs(F)
    assert np.max(np.abs(lhs - rhs) / scale) <= TOL


def test_diag_2d_128_modes_first_step_every_coefficient(gpu, orc):
    """2D with 128 x 128 modes (16384 coefficients, beyond the factorisation paths), 144 x 144
    points: every coefficient of one step against the oracle's load, and parareal exact."""
    T = 1.0 / 2048
    kw = const_d(W.C3, modes=128, quad=144, steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    c0 = W.u0_random_2d(128, 2)
    _, tr = gpu.solve_serial(pg, dev(c0[None]), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    _, F = orc.galerkin_rows(po, c0, 0.0, 0.0, [0])
    k1, k2 = np.meshgrid(np.arange(1, 129), np.arange(1, 129), indexing="ij")
    lam = ((k1 ** 2 + k2 ** 2) * math.pi ** 2).ravel()
    lhs = c1 * (1.0 + tau * 0.8 * lam)
    rhs = c0 + tau * F
    scale = np.abs(lhs) + np.abs(c0) + tau * np.abs(F)
    assert np.max(np.abs(lhs - rhs) / scale) <= TOL
    kp = const_d(W.C3, modes=128, quad=144, steps=8, slices=4, T=8.0 / 2048)
    pp = gpu.make_problem(solver=2, **kp)
    u0 = dev(np.stack([W.u0_random_2d(128, s) for s in (3, 4)]))
    Us, _ = gpu.solve_serial(pp, u0)
    r = gpu.solve_parareal(pp, u0, 4, tol=0.0, want_iterates=True)
    for k in range(5):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k


def test_diag_1d_4096_modes_first_step_every_coefficient(gpu, orc):
    """1D with 4096 modes and 4608 points (beyond the factorisation paths): every coefficient
    of one step against the oracle's load; parareal exact at 2048 modes."""
    T = 1.0 / 4096
    kw = const_d(W.C2, modes=4096, quad=4608, steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    c0 = W.u0_batch_1d(4096, [1])
    _, tr = gpu.solve_serial(pg, dev(c0), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    _, F = orc.galerkin_rows(po, c0[0], 0.0, 0.0, [0])
    lam = (np.arange(1, 4097) * math.pi) ** 2
    lhs = c1 * (1.0 + tau * 0.8 * lam)
    rhs = c0[0] + tau * F
    scale = np.abs(lhs) + np.abs(c0[0]) + tau * np.abs(F)
    assert np.max(np.abs(lhs - rhs) / scale) <= TOL
    kp = const_d(W.C2, modes=2048, quad=2304, steps=8, slices=4, T=8.0 / 4096)
    pp = gpu.make_problem(solver=2, **kp)
    u0 = dev(W.u0_batch_1d(2048, [2, 3]))
    Us, _ = gpu.solve_serial(pp, u0)
    r = gpu.solve_parareal(pp, u0, 4, tol=0.0, want_iterates=True)
    for k in range(5):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k


def test_diag_2d_256_modes_first_step_every_coefficient(gpu, orc):
    """2D at the largest shape the diagonal solve accepts and the bench times (256 x 256
    modes, 384 x 384 points): every coefficient of one step against the oracle's load."""
    T = 1.0 / 2048
    kw = const_d(W.C3, modes=256, quad=384, steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    c0 = W.u0_random_2d(256, 2)
    _, tr = gpu.solve_serial(pg, dev(c0[None]), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    _, F = orc.galerkin_rows(po, c0, 0.0, 0.0, [0])
    k1, k2 = np.meshgrid(np.arange(1, 257), np.arange(1, 257), indexing="ij")
    lam = ((k1 ** 2 + k2 ** 2) * math.pi ** 2).ravel()
    lhs = c1 * (1.0 + tau * 0.8 * lam)
    rhs = c0 + tau * F
    scale = np.abs(lhs) + np.abs(c0) + tau * np.abs(F)
    assert np.max(np.abs(lhs - rhs) / scale) <= TOL


def test_diag_1d_largest_shape_first_step_every_coefficient(gpu, orc):
    """1D at the largest shape the diagonal solve accepts (4096 modes, 8192 points): one step
    against the oracle's load, within 1e-10 relative L2 over all coefficients.  Coefficient by
    coefficient the bound is 1e-9: each F_k is an 8192-term sum whose terms cancel for high
    modes, so its rounding relative to |F_k| grows with the number of terms (the GPU's blocked
    sum and the oracle's sequential one differ by 1.0e-10 at the worst coefficient here)."""
    T = 1.0 / 4096
    kw = const_d(W.C2, modes=4096, quad=8192, steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(solver=2, **kw), orc.problem(solver=2, **kw)
    c0 = W.u0_batch_1d(4096, [2])
    _, tr = gpu.solve_serial(pg, dev(c0), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    _, F = orc.galerkin_rows(po, c0[0], 0.0, 0.0, [0])
    lam = (np.arange(1, 4097) * math.pi) ** 2
    lhs = c1 * (1.0 + tau * 0.8 * lam)
    rhs = c0[0] + tau * F
    assert rel(lhs, rhs) <= TOL
    scale = np.abs(lhs) + np.abs(c0[0]) + tau * np.abs(F)
    assert np.max(np.abs(lhs - rhs) / scale) <= 10 * TOL


def test_diag_full_shape_parareal_exact(gpu):
    """Config-2 shape with constant D, 32 instances, 64 slices of 4 steps: parareal iterates
    equal the serial solution bit for bit on the converged slices."""
    kw = const_d(W.C2, steps=256, slices=64, T=256.0 / 4096)
    pg = gpu.make_problem(solver=2, **kw)
    u0 = dev(W.u0_batch_1d(kw["modes"], range(32)))
    Us, _ = gpu.solve_serial(pg, u0)
    r = gpu.solve_parareal(pg, u0, 6, tol=0.0, want_iterates=True)
    for k in range(7):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k


def test_diag_batch_independent_and_close_to_cholesky(gpu):
    """At Q = 4M the quadrature stiffness is diagonal to rounding: the diagonal solve and the
    Cholesky path agree to 1e-11; an instance's result does not depend on its batch."""
    for kw in (const_d(W.C2, modes=40, quad=160, steps=12, slices=3, alpha=0.6),
               const_d(W.C3, modes=8, quad=32, steps=6, slices=2, alpha=0.6)):
        print(f"[diag] batch/cholesky dim={kw['dim']}", flush=True)
        u0 = u0_of(kw, [8, 9, 10])
        pd, pc = gpu.make_problem(solver=2, **kw), gpu.make_problem(**kw)
        U3, _ = gpu.solve_serial(pd, dev(u0))
        for b in range(3):
            U1, _ = gpu.solve_serial(pd, dev(u0[b:b + 1]))
            assert torch.equal(U1[0], U3[b]), b
        Uc, _ = gpu.solve_serial(pc, dev(u0))
        assert rel(U3.cpu().numpy(), Uc.cpu().numpy()) <= 1e-11
