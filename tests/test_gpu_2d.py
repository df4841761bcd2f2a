"""GPU parity of the 2D (tensor sine basis) path against the oracle: the separable products
(lagged state, D, f, load vector, cosine moments) on FP64 MFMA, the stiffness from the 2D
moments, the register-resident factorisation (padded size <= 256) and the device-memory
factorisation (larger).  Tolerance 1e-10 relative L2, as for 1D."""
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


CASES = {
    # register path (padded M^2 <= 256)
    "c3_small_M4_Q8": c3(modes=4, quad=8, steps=16, slices=4),
    "ragged_M5_Q9": c3(modes=5, quad=9, steps=12, slices=3, alpha=0.35),
    "M16_Q20": c3(modes=16, quad=20, steps=4, slices=2),
    "mms_M3": c3(modes=3, quad=8, steps=16, slices=4, d_sel=1, f_sel=1, alpha=0.5),
    "full_history_M4": c3(modes=4, quad=8, steps=12, slices=3, history=1),
    # device-memory factorisation (padded M^2 = 336 > 256)
    "devmem_M18_Q20": c3(modes=18, quad=20, steps=4, slices=2),
}


def u0_2d(M, seeds):
    return np.stack([W.u0_random_2d(M, s) for s in seeds])


@pytest.mark.parametrize("name", list(CASES))
def test_serial_2d_matches_oracle(gpu, orc, name):
    kw = CASES[name]
    pg, po = gpu.make_problem(**kw), orc.problem(**kw)
    u0 = u0_2d(kw["modes"], [3, 4])
    U, _ = gpu.solve_serial(pg, torch.tensor(u0, device="cuda"))
    U = U.cpu().numpy()
    for b in range(2):
        ref = orc.solve_serial(po, u0[b])
        assert rel(U[b], ref) <= TOL, (name, b, rel(U[b], ref))


@pytest.mark.parametrize("name", ["c3_small_M4_Q8", "ragged_M5_Q9", "devmem_M18_Q20"])
def test_parareal_2d_exact_and_matches_oracle(gpu, orc, name):
    kw = CASES[name]
    pg, po = gpu.make_problem(**kw), orc.problem(**kw)
    u0 = u0_2d(kw["modes"], [7])
    u0d = torch.tensor(u0, device="cuda")
    Us, _ = gpu.solve_serial(pg, u0d)
    P = kw["slices"]
    r = gpu.solve_parareal(pg, u0d, P, tol=0.0, want_iterates=True)
    for k in range(P + 1):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), (name, k)
    ref = orc.solve_parareal(po, u0[0], 1)[0]  # after one sweep
    assert rel(r.iterates[1][0].cpu().numpy(), ref) <= TOL


def test_2d_coarse_and_fine_apply(gpu, orc):
    kw = CASES["ragged_M5_Q9"]
    pg, po = gpu.make_problem(**kw), orc.problem(**kw)
    P, Md = kw["slices"], kw["modes"] ** 2
    rng = np.random.default_rng(2)
    Z = rng.normal(size=(1, P + 1, Md)) * 0.3
    G = gpu.coarse_apply(pg, torch.tensor(Z, device="cuda")).cpu().numpy()
    F = gpu.fine_apply(pg, torch.tensor(Z, device="cuda")).cpu().numpy()
    for n in range(P):
        assert rel(G[0, n], orc.coarse_G(po, n, Z[0, : n + 1])) <= TOL
        assert rel(F[0, n], orc.fine_F(po, n, Z[0, : n + 1])) <= TOL


# ------------------------------------------------- full size (config 3: 64 x 64 modes), sampled

def test_full_size_first_step_rows_match_oracle(gpu, orc):
    """One step of the config-3 step size at full size (4096 coefficients, 96 x 96 points)
    through the blocked factorisation: on sampled rows, the GPU state c1 satisfies the step's
    equation c1 + tau K(c0) c1 = c0 + tau F(c0) with the oracle's own rows of K and load F."""
    import math

    T = 1.0 / 2048  # one step of N = 2048 on (0, 1)
    kw = c3(steps=1, slices=1, T=T)
    pg, po = gpu.make_problem(**kw), orc.problem(**kw)
    c0 = W.u0_random_2d(kw["modes"], 0)
    _, tr = gpu.solve_serial(pg, torch.tensor(c0[None], device="cuda"), want_traj=True)
    c1 = tr[0, 1].cpu().numpy()
    tau = T ** kw["alpha"] * math.gamma(2.0 - kw["alpha"])
    Md = kw["modes"] ** 2
    rows = sorted({0, 1, 63, 64, Md - 1, *np.random.default_rng(17).choice(Md, 11, replace=False).tolist()})
    Kr, F = orc.galerkin_rows(po, c0, 0.0, 0.0, rows)
    for i, k in enumerate(rows):
        lhs = c1[k] + tau * (Kr[i] @ c1)
        rhs = c0[k] + tau * F[k]
        scale = abs(c1[k]) + tau * (np.abs(Kr[i]) @ np.abs(c1)) + abs(c0[k]) + tau * abs(F[k])
        assert abs(lhs - rhs) <= TOL * scale, (k, abs(lhs - rhs) / scale)


def test_full_size_parareal_exact(gpu):
    """Full mode count (64 x 64), short horizon: the first k+1 slice ends of iterate k equal the
    serial solution bit for bit, and all of them after P sweeps."""
    kw = c3(steps=16, slices=4, T=16.0 / 2048)
    pg = gpu.make_problem(**kw)
    u0 = torch.tensor(W.u0_random_2d(kw["modes"], 1)[None], device="cuda")
    Us, _ = gpu.solve_serial(pg, u0)
    r = gpu.solve_parareal(pg, u0, 4, tol=0.0, want_iterates=True)
    for k in range(5):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k
    assert torch.equal(r.U, Us)
