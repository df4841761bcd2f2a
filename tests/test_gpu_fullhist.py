"""GPU tests of full-history parareal (history = 1): the fine propagator of slice n takes its
L1 history over the whole fine grid, from the previous iterate's fine trajectories for the
steps before nS.

Bars: every iterate matches the oracle's full-history parareal to 1e-10 relative L2 (same
seeded inputs); after k sweeps the first k+1 slice ends equal the GPU's full-history serial
solution bit for bit, and all of them after P sweeps.  Cases cover the register path (1D and
2D), the evaluation path and the blocked factorisation (Mp > 256), one step per slice, slices
longer than the prefix kernel's step chunk, and step counts that leave ragged row blocks.
"""
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


def u0_for(kw, seeds):
    if kw["dim"] == 2:
        return np.stack([W.u0_random_2d(kw["modes"], s) for s in seeds])
    return W.u0_batch_1d(kw["modes"], seeds)


H = dict(history=1)
CASES = [
    # S = 10: row blocks of 4 plus a ragged pair, one partial step chunk
    ("1d_S10", W.with_(W.C2, modes=48, quad=72, steps=60, slices=6, alpha=0.35, **H), [14, 15]),
    # S = 40: two step chunks (the second partial)
    ("1d_S40", W.with_(W.C2, modes=20, quad=32, steps=200, slices=5, alpha=0.6, **H), [16]),
    # S = 1: every earlier state comes from the previous iterate
    ("1d_S1", W.with_(W.C2, modes=16, quad=24, steps=8, slices=8, alpha=0.5, **H), [17]),
    # Mp = 288 > 256: evaluation kernel and blocked factorisation (T = 0.1 keeps cond(A) ~ 1e4)
    ("1d_M280_eval", W.with_(W.C2, modes=280, quad=300, steps=12, slices=3, alpha=0.5, T=0.1, **H), [18]),
    # 2D, register path (Mp = 48)
    ("2d_M6", dict(W.C3, modes=6, quad=10, steps=12, slices=3, **H), [19]),
    # 2D, blocked path (Mp = 304)
    ("2d_M17_blk", dict(W.C3, modes=17, quad=20, steps=6, slices=2, **H), [20]),
]


@pytest.mark.parametrize("name,kw,seeds", CASES, ids=[c[0] for c in CASES])
def test_full_history_parareal_matches_oracle_and_is_exact(gpu, orc, name, kw, seeds):
    print(f"[fullhist] {name}", flush=True)
    P = kw["slices"]
    p = gpu.make_problem(**kw)
    u0 = u0_for(kw, seeds)
    Us, _ = gpu.solve_serial(p, dev(u0))
    r = gpu.solve_parareal(p, dev(u0), P, tol=0.0, want_iterates=True)
    assert r.iters == P
    its = r.iterates.cpu().numpy()
    # bitwise exactness against the GPU's own full-history serial solution
    for k in range(P + 1):
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), (name, k)
    assert torch.equal(r.U, Us), name
    # every iterate against the oracle's full-history parareal
    po = orc.problem(**kw)
    for b in range(len(seeds)):
        _, ko, _, ito = orc.solve_parareal(po, u0[b], P, want_iterates=True)
        assert ko == P
        for k in range(P + 1):
            e = rel(its[k, b], ito[k])
            assert e <= TOL, (name, b, k, e)


SERIAL_CASES = [
    # N past the serial solve's 64-step prefix blocks, with a ragged last block
    ("1d_N200", W.with_(W.C2, modes=40, quad=60, steps=200, slices=5, alpha=0.45, **H), [24, 25]),
    ("1d_M280_N130", W.with_(W.C2, modes=280, quad=300, steps=130, slices=2, alpha=0.6, T=0.1, **H), [26]),
    ("2d_M6_N140", dict(W.C3, modes=6, quad=10, steps=140, slices=2, alpha=0.3, **H), [27]),
]


@pytest.mark.parametrize("name,kw,seeds", SERIAL_CASES, ids=[c[0] for c in SERIAL_CASES])
def test_full_history_serial_blocks_match_oracle(gpu, orc, name, kw, seeds):
    """The full-history serial solve sums each step's history as a per-block prefix (formed
    before the block's first step) plus the rows since the block began; slice ends and the
    whole trajectory match the oracle's direct sum to 1e-10."""
    print(f"[fullhist serial] {name}", flush=True)
    p = gpu.make_problem(**kw)
    u0 = u0_for(kw, seeds)
    U, tr = gpu.solve_serial(p, dev(u0), want_traj=True)
    U, tr = U.cpu().numpy(), tr.cpu().numpy()
    po = orc.problem(**kw)
    for b in range(len(seeds)):
        Uo, tro = orc.solve_serial(po, u0[b], want_traj=True)
        assert rel(U[b], Uo) <= TOL, (name, b, rel(U[b], Uo))
        per = [rel(tr[b][m], tro[m]) for m in range(tro.shape[0])]
        assert max(per) <= TOL, (name, b, max(per))


def test_full_history_fixed_point_is_not_the_hybrid_one(gpu):
    """The two variants converge to different discrete solutions (uniform L1 with full
    history vs the paper's hybrid propagator); each parareal reaches its own."""
    kw = W.with_(W.C2, modes=32, quad=48, steps=64, slices=8, alpha=0.4)
    u0 = dev(W.u0_batch_1d(32, [21, 22]))
    ph, pf = gpu.make_problem(**kw), gpu.make_problem(**W.with_(kw, history=1))
    Uh, _ = gpu.solve_serial(ph, u0)
    Uf, _ = gpu.solve_serial(pf, u0)
    rf = gpu.solve_parareal(pf, u0, 8, tol=0.0)
    rh = gpu.solve_parareal(ph, u0, 8, tol=0.0)
    assert torch.equal(rf.U, Uf) and torch.equal(rh.U, Uh)
    assert rel(Uf.cpu().numpy(), Uh.cpu().numpy()) > 1e-6


def test_full_history_parareal_tolerance_stop(gpu, orc):
    """With tol > 0 the run stops at the first sweep whose increment is below it, the same
    sweep as the oracle's, with the same result to 1e-10."""
    kw = W.with_(W.C2, modes=24, quad=36, steps=96, slices=12, alpha=0.7, history=1)
    u0 = W.u0_batch_1d(24, [23])
    p = gpu.make_problem(**kw)
    r = gpu.solve_parareal(p, dev(u0), 12, tol=1e-6)
    Uo, ko, incr_o, _ = orc.solve_parareal(orc.problem(**kw), u0[0], 12, tol=1e-6)
    assert r.iters == ko < 12, (r.iters, ko)
    assert rel(r.U.cpu().numpy()[0], Uo) <= TOL
    assert rel(r.incr.cpu().numpy()[0], incr_o[: r.iters]) <= 1e-6
