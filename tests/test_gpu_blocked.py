"""GPU parity of the blocked device-memory factorisation (systems with more than 256
coefficients): diagonal blocks factored in registers and inverted, panel GEMMs with the
triangular inverse, MFMA trailing updates, blocked back substitution.  Against the oracle at
1e-10 relative L2, in 1D (quadrature-GEMM assembly) and 2D (moment assembly), with ragged
last blocks and both block widths; plus bitwise independence from the batch and parareal
exactness, which need every unit's arithmetic to be independent of the launch."""
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


# (name, problem keywords, tune bits, seeds); padded sizes and block splits in the names
CASES = [
    # 1D, quadrature-GEMM assembly: Mp 400 = 256 + 144, cond(I + tau K) about 7e4.  The blocks
    # are applied through explicit triangular inverses; one step of iterative refinement per
    # solve brings the error back to that of a backward-stable solve.
    ("1d_M400_nb256", W.with_(W.C2, modes=400, quad=420, steps=64, slices=2, alpha=0.9), 0, [21]),
    # 1D: Mp 304 = 128 + 128 + 48
    ("1d_M300_nb128", W.with_(W.C2, modes=300, quad=330, steps=48, slices=3, alpha=0.9), 4, [23]),
    # 1D at cond(A) about 1e6: eight steps of dt = 1/8 (Mp 400 = 256 + 144)
    ("1d_M400_N8_cond1e6", W.with_(W.C2, modes=400, quad=420, steps=8, slices=2, alpha=0.5), 0, [24]),
    # 1D: Mp 272 = 256 + 16 (a one-tile last block)
    ("1d_M272_nb256", W.with_(W.C2, modes=272, quad=300, steps=48, slices=3, alpha=0.9), 0, [25]),
    # 2D: Mp 576 = 256 + 256 + 64
    ("2d_M24_nb256", dict(W.C3, modes=24, quad=30, steps=4, slices=2), 0, [3, 4]),
    # 2D: Mp 336 = 128 + 128 + 80
    ("2d_M18_nb128", dict(W.C3, modes=18, quad=20, steps=4, slices=2, alpha=0.45), 4, [5]),
    # 2D with the 64 x 64 trailing-update tiles (tune bit 3): Mp 576 = 256 + 256 + 64
    ("2d_M24_trail64", dict(W.C3, modes=24, quad=30, steps=4, slices=2), 8, [7]),
    # 2D full history through the blocked path
    ("2d_M17_full", dict(W.C3, modes=17, quad=20, steps=6, slices=2, history=1), 0, [6]),
]


def u0_for(kw, seeds):
    if kw["dim"] == 2:
        return np.stack([W.u0_random_2d(kw["modes"], s) for s in seeds])
    return W.u0_batch_1d(kw["modes"], seeds)


@pytest.mark.parametrize("name,kw,tune,seeds", CASES, ids=[c[0] for c in CASES])
def test_blocked_serial_matches_oracle(gpu, orc, name, kw, tune, seeds):
    assembly = 1 if kw["dim"] == 1 else 0
    pg = gpu.make_problem(assembly=assembly, tune=tune, **kw)
    po = orc.problem(**kw)
    u0 = u0_for(kw, seeds)
    U, tr = gpu.solve_serial(pg, dev(u0), want_traj=True)
    U, tr = U.cpu().numpy(), tr.cpu().numpy()
    for b in range(len(seeds)):
        Uo, tro = orc.solve_serial(po, u0[b], want_traj=True)
        assert rel(U[b], Uo) <= TOL, (name, b, rel(U[b], Uo))
        per = [rel(tr[b][m], tro[m]) for m in range(tro.shape[0])]
        assert max(per) <= TOL, (name, b, max(per))


def test_blocked_batch_independent_bitwise(gpu):
    kw = dict(W.C3, modes=20, quad=24, steps=4, slices=2)
    p = gpu.make_problem(**kw)
    u0 = u0_for(kw, [8, 9, 10])
    U3, _ = gpu.solve_serial(p, dev(u0))
    for b in range(3):
        U1, _ = gpu.solve_serial(p, dev(u0[b:b + 1]))
        assert torch.equal(U1[0], U3[b]), b


@pytest.mark.parametrize("dim", [1, 2])
def test_blocked_parareal_exact_after_P_sweeps(gpu, dim):
    if dim == 2:
        kw = dict(W.C3, modes=18, quad=20, steps=6, slices=3)
    else:
        kw = W.with_(W.C2, modes=280, quad=300, steps=6, slices=3, alpha=0.5)
    p = gpu.make_problem(assembly=1 if dim == 1 else 0, **kw)
    u0 = dev(u0_for(kw, [11]))
    Us, _ = gpu.solve_serial(p, u0)
    P = kw["slices"]
    r = gpu.solve_parareal(p, u0, P, tol=0.0, want_iterates=True)
    for k in range(P + 1):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k
    assert torch.equal(r.U, Us)


def test_autotune_blocked_variants(gpu, orc):
    """The autotuner chooses among the blocked factorisation's variants (block width, trailing
    tiles); the chosen problem still matches the oracle and parareal stays exact."""
    kw = dict(W.C3, modes=18, quad=20, steps=6, slices=3)
    p = gpu.make_problem(**kw)
    t = gpu.autotune(p, 2)
    assert t in (0, 4, 8, 12), t
    p.tune = t
    u0 = u0_for(kw, [12, 13])
    Us, _ = gpu.solve_serial(p, dev(u0))
    for b in range(2):
        assert rel(Us[b].cpu().numpy(), orc.solve_serial(orc.problem(**kw), u0[b])) <= TOL
    r = gpu.solve_parareal(p, dev(u0), kw["slices"], tol=0.0)
    assert torch.equal(r.U, Us)
