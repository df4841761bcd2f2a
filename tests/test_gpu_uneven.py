"""GPU tests of uneven batches (instances with their own modes, steps per slice and order
under one problem), the GEMM-variant autotuner and graph capture of a whole parareal run.

An uneven batch must reproduce each instance's own run bit for bit (same padded mode count,
same quadrature), match the oracle to 1e-10 relative L2, and keep parareal's exactness.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_11023_amd import workloads as W  # noqa: E402


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


# bucket Mp = 48: instances with M in 33..48, Q = 96 for all; P = 8 slices, S_b in 1..6
BASE = dict(dim=1, modes=48, quad=96, steps=8 * 6, slices=8, alpha=0.5, T=1.0, d_sel=1,
            d_param=1.0, f_sel=1, history=0, source_time=0)
MODES = [48, 40, 33, 45, 48]
SPP = [6, 3, 1, 5, 4]
ALPHA = [0.5, 0.3, 0.9, 1.0, 0.65]


def u0_for(M, Mb_list, seed0=10):
    u0 = np.zeros((len(Mb_list), M))
    for b, mb in enumerate(Mb_list):
        u0[b, :mb] = W.u0_random_1d(mb, seed0 + b)
    return u0


def own_problem(gpu, b, **extra):
    kw = dict(BASE, modes=MODES[b], steps=BASE["slices"] * SPP[b], alpha=ALPHA[b])
    kw.update(extra)
    return gpu.make_problem(**kw), kw


def test_uneven_serial_equals_own_runs_bitwise_and_oracle(gpu, orc):
    p = gpu.make_problem(**BASE)
    u0 = u0_for(BASE["modes"], MODES)
    U = gpu.solve_serial_uneven(p, torch.tensor(u0, device="cuda"), MODES, SPP, ALPHA).cpu().numpy()
    for b in range(len(MODES)):
        pb, kw = own_problem(gpu, b)
        Ub, _ = gpu.solve_serial(pb, torch.tensor(u0[b:b + 1, :MODES[b]], device="cuda"))
        Ub = Ub.cpu().numpy()[0]
        assert np.array_equal(U[b, :, :MODES[b]], Ub), b
        assert not np.any(U[b, :, MODES[b]:]), b
        ref = orc.solve_serial(orc.problem(**kw), u0[b, :MODES[b]])
        assert rel(Ub, ref) <= 1e-10, (b, rel(Ub, ref))


def test_uneven_parareal_equals_own_runs_and_is_exact(gpu):
    p = gpu.make_problem(**BASE)
    u0 = torch.tensor(u0_for(BASE["modes"], MODES), device="cuda")
    Us = gpu.solve_serial_uneven(p, u0, MODES, SPP, ALPHA)
    for k in (0, 1, 3, BASE["slices"]):
        U, conv, stamps = gpu.solve_parareal_uneven(p, u0, k, MODES, SPP, ALPHA)
        # exactness: the first k+1 slice ends equal the serial solution bit for bit
        assert torch.equal(U[:, : k + 1], Us[:, : k + 1]), k
        for b in (0, 2):
            pb, _ = own_problem(gpu, b)
            r = gpu.solve_parareal(pb, u0[b:b + 1, :MODES[b]].contiguous(), k, tol=0.0)
            assert torch.equal(U[b, :, :MODES[b]], r.U[0]), (k, b)


def test_uneven_convergence_flags_and_stamps(gpu):
    p = gpu.make_problem(**BASE)
    u0 = torch.tensor(u0_for(BASE["modes"], MODES), device="cuda")
    sweeps, tol = 6, 1e-9
    B = len(MODES)
    incr = torch.zeros((B, sweeps), dtype=torch.float64, device="cuda")
    U, conv, stamps = gpu.solve_parareal_uneven(p, u0, sweeps, MODES, SPP, ALPHA, conv_tol=tol,
                                                incr=incr)
    inc, cv, st = incr.cpu().numpy(), conv.cpu().numpy(), stamps.cpu().numpy()
    for b in range(B):
        hit = [k + 1 for k in range(sweeps) if inc[b, k] <= tol]
        assert cv[b] == (hit[0] if hit else -1), (b, cv[b], inc[b])
    assert np.all(np.diff(st) >= 0) and st[-1] > st[0]


def test_autotune_bits_and_exactness(gpu):
    kw = W.with_(W.C4, modes=96, quad=144, steps=8 * 4, slices=8)
    p = gpu.make_problem(**kw)
    t = gpu.autotune(p, 4)
    assert 0 <= t <= 3
    for tune in range(4):
        q = gpu.make_problem(**W.with_(kw, tune=tune))
        u0 = torch.tensor(W.u0_batch_1d(96, [1, 2, 3, 4]), device="cuda")
        Us, _ = gpu.solve_serial(q, u0)
        r = gpu.solve_parareal(q, u0, 3, tol=0.0, want_iterates=True)
        for k in range(4):
            assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), (tune, k)
        if tune:
            U0, _ = gpu.solve_serial(p, u0)
            assert rel(Us.cpu().numpy(), U0.cpu().numpy()) <= 1e-12


def test_graph_captured_uneven_parareal_replays(gpu):
    """The whole uneven parareal run captured as one HIP graph; every replay (with eager work
    in between) equals the eager result bit for bit."""
    p = gpu.make_problem(**BASE)
    B = len(MODES)
    u0 = torch.tensor(u0_for(BASE["modes"], MODES), device="cuda")
    modes = torch.tensor(MODES, dtype=torch.int32, device="cuda")
    spp = torch.tensor(SPP, dtype=torch.int32, device="cuda")
    alpha = torch.tensor(ALPHA, dtype=torch.float64, device="cuda")
    from paper_2510_11023_amd import solver

    ws = solver._workspace(p, B, 1, "cuda")[0]
    out = torch.empty((B, BASE["slices"] + 1, BASE["modes"]), dtype=torch.float64, device="cuda")
    conv = torch.empty(B, dtype=torch.int32, device="cuda")
    stamps = torch.zeros(5, dtype=torch.int64, device="cuda")
    eager, _, _ = gpu.solve_parareal_uneven(p, u0, 4, modes, spp, alpha, conv_tol=1e-9, workspace=ws)
    eager = eager.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        gpu.solve_parareal_uneven(p, u0, 4, modes, spp, alpha, conv_tol=1e-9, workspace=ws,
                                  out=out, conv=conv, stamps=stamps)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.solve_parareal_uneven(p, u0, 4, modes, spp, alpha, conv_tol=1e-9, workspace=ws,
                                  out=out, conv=conv, stamps=stamps)
    for rep in range(3):
        out.zero_()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        assert float(junk) == float(junk)


# ------------------------------------------------------- learned coarse step, uneven batches

def _net(gpu, modes, seed=3, train_kw=None):
    """A residual network for `modes` modes: statistics and one epoch on the plain coarse/fine
    pairs of a uniform problem (its quality does not matter here, only that it corrects)."""
    from paper_2510_11023_amd.learned import LearnedCoarse, training_data

    model = LearnedCoarse(modes, seed=seed)
    kw = dict(BASE, modes=modes, quad=2 * modes)
    if train_kw:
        kw.update(train_kw)
    pg = gpu.make_problem(**kw)
    u0 = torch.tensor(W.u0_batch_1d(modes, range(16)), device="cuda")
    x, t = training_data(pg, u0, list(W.alphas_uniform(16, seed=seed)), model)
    model.set_stats(x, t)
    model.train(x, t, epochs=1, batch=64, lr=1e-3, seed=1)
    return model


def test_learned_uneven_exact_and_equals_own_runs(gpu):
    p = gpu.make_problem(**BASE)
    u0 = torch.tensor(u0_for(BASE["modes"], MODES), device="cuda")
    model = _net(gpu, BASE["modes"])
    L = dict(coarse=gpu.COARSE_LEARNED, mlp_params=model.params, mlp_modes=BASE["modes"])
    Us = gpu.solve_serial_uneven(p, u0, MODES, SPP, ALPHA)
    plain0, _, _ = gpu.solve_parareal_uneven(p, u0, 0, MODES, SPP, ALPHA)
    for k in (0, 1, 3, BASE["slices"]):
        U, conv, _ = gpu.solve_parareal_uneven(p, u0, k, MODES, SPP, ALPHA, **L)
        assert torch.equal(U[:, : k + 1], Us[:, : k + 1]), k
        if k == 0:
            assert not torch.equal(U, plain0)  # the correction is applied
        # instances with the group's own mode count reproduce their own learned runs
        for b in (0, 4):
            pb, _ = own_problem(gpu, b)
            r = gpu.solve_parareal(pb, u0[b:b + 1, :MODES[b]].contiguous(), k, tol=0.0,
                                   coarse=gpu.COARSE_LEARNED, mlp_params=model.params)
            assert torch.equal(U[b, :, :MODES[b]], r.U[0]), (k, b)
        # coefficients above an instance's own modes stay exactly zero
        for b in range(len(MODES)):
            assert not torch.any(U[b, :, MODES[b]:]), (k, b)


def test_learned_uneven_falls_back_to_plain(gpu):
    """A network with a non-finite output: every unit keeps the plain coarse value, bit for bit."""
    from paper_2510_11023_amd.learned import LearnedCoarse

    p = gpu.make_problem(**BASE)
    u0 = torch.tensor(u0_for(BASE["modes"], MODES), device="cuda")
    model = LearnedCoarse(BASE["modes"], seed=2)
    bad = model.masters()
    bad[model.info.flat_b[3]] = np.nan
    model.set_masters(bad)
    a, ca, _ = gpu.solve_parareal_uneven(p, u0, 3, MODES, SPP, ALPHA, conv_tol=1e-9,
                                         coarse=gpu.COARSE_LEARNED, mlp_params=model.params,
                                         mlp_modes=BASE["modes"])
    b, cb, _ = gpu.solve_parareal_uneven(p, u0, 3, MODES, SPP, ALPHA, conv_tol=1e-9)
    assert torch.equal(a, b) and torch.equal(ca, cb)


def test_learned_network_wider_than_the_batch(gpu):
    """One network of 64 modes serves a batch of at most 48 (zero-padded inputs): the uneven
    call stays exact, and the batch call running the same network over one of its problems
    gives that instance's result bit for bit."""
    p = gpu.make_problem(**BASE)
    u0 = torch.tensor(u0_for(BASE["modes"], MODES), device="cuda")
    model = _net(gpu, 64, seed=4)
    L = dict(coarse=gpu.COARSE_LEARNED, mlp_params=model.params, mlp_modes=64)
    Us = gpu.solve_serial_uneven(p, u0, MODES, SPP, ALPHA)
    U, _, _ = gpu.solve_parareal_uneven(p, u0, 2, MODES, SPP, ALPHA, **L)
    assert torch.equal(U[:, :3], Us[:, :3])
    b = 1
    kw = dict(BASE, modes=MODES[b], steps=BASE["slices"] * SPP[b], alpha=ALPHA[b])
    out = gpu.solve_batch([gpu.make_problem(**kw)], [u0[b, :MODES[b]].contiguous()],
                          parareal_sweeps=2, **L)
    assert torch.equal(out[0], U[b, :, :MODES[b]])
    from paper_2510_11023_amd import _lib

    with pytest.raises(_lib.L1prError):  # a network narrower than the batch's modes
        gpu.solve_parareal_uneven(p, u0, 1, MODES, SPP, ALPHA, coarse=gpu.COARSE_LEARNED,
                                  mlp_params=model.params, mlp_modes=32)
