"""GPU parity: the HIP library (through its C-ABI) against the CPU oracle.

Bar (FP64 path): relative L2 error <= 1e-10 on slice ends, trajectories and parareal
iterates, on the same seeded inputs.  GPU self-consistency checks are bitwise: parareal
reproduces the GPU serial solution exactly, runs are deterministic, and an instance's
result does not depend on the rest of its batch.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_11023_amd as l1
    from paper_2510_11023_amd import _lib

    _lib.lib()
    return l1


def both(gpu, orc, assembly=0, **kw):
    return gpu.make_problem(assembly=assembly, **kw), orc.problem(**kw)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run_serial(gpu, p, u0, alpha=None):
    U, traj = gpu.solve_serial(p, dev(u0), alpha=alpha, want_traj=True)
    torch.cuda.synchronize()
    return U.cpu().numpy(), traj.cpu().numpy()


from paper_2510_11023_amd import workloads as W  # noqa: E402


# ------------------------------------------------------------------ serial parity

SERIAL_CASES = [
    # name, problem kwargs, seeds
    ("config1", dict(W.C1), None),
    ("small_c2_a03", W.with_(W.C2, modes=64, quad=96, steps=128, slices=8, alpha=0.3), [0, 1, 2]),
    ("small_c2_a07", W.with_(W.C2, modes=64, quad=96, steps=96, slices=8, alpha=0.7), [3, 4]),
    ("small_c2_a10", W.with_(W.C2, modes=64, quad=96, steps=64, slices=8, alpha=1.0), [5]),
    ("ragged_M40_Q61", W.with_(W.C2, modes=40, quad=61, steps=40, slices=5, alpha=0.45), [6, 7]),
    ("ragged_M70_Q100", W.with_(W.C2, modes=70, quad=100, steps=36, slices=4, alpha=0.55, d_sel=3, f_sel=3), [8]),
    ("M1", W.with_(W.C2, modes=1, quad=3, steps=20, slices=4, alpha=0.5), [9]),
    ("one_slice", W.with_(W.C2, modes=16, quad=24, steps=24, slices=1, alpha=0.6, d_sel=1, f_sel=3), [10]),
    ("one_step_per_slice", W.with_(W.C2, modes=16, quad=24, steps=12, slices=12, alpha=0.6, d_sel=4, f_sel=4), [11]),
    ("paper_model", W.with_(W.C2, modes=32, quad=48, steps=64, slices=8, alpha=0.5, d_sel=4, f_sel=4), [12]),
    ("const_D_mms_new_time", W.with_(W.C2, modes=8, quad=16, steps=32, slices=4, alpha=0.4, d_sel=0, d_param=0.7, f_sel=5, source_time=1), [13]),
    ("full_history", W.with_(W.C2, modes=48, quad=72, steps=60, slices=6, alpha=0.35, history=1), [14, 15]),
    ("tiles_M96", W.with_(W.C2, modes=96, quad=144, steps=32, slices=4, alpha=0.8), [16]),
    ("tiles_M128", W.with_(W.C2, modes=128, quad=192, steps=16, slices=4, alpha=0.5), [17]),
]


def _u0(kw, seeds):
    if seeds is None:
        return W.u0_sine_mode(kw["modes"])[None, :]
    return W.u0_batch_1d(kw["modes"], seeds)


GEMM_CASES = [c for c in SERIAL_CASES if c[0] in (
    "config1", "small_c2_a03", "ragged_M40_Q61", "M1", "full_history", "tiles_M128")]
# beyond the register path: the blocked device-memory factorisation with one step of
# iterative refinement per solve (cond(I + tau K) about 4e4 here)
GEMM_CASES += [("beyond_register_path_M272", W.with_(W.C2, modes=272, quad=300, steps=48, slices=3, alpha=0.9), [18])]


def _serial_case(gpu, orc, name, kw, seeds, assembly):
    pg, po = both(gpu, orc, assembly=assembly, **kw)
    u0 = _u0(kw, seeds)
    Ug, trg = run_serial(gpu, pg, u0)
    for b in range(u0.shape[0]):
        Uo, tro = orc.solve_serial(po, u0[b], want_traj=True)
        assert rel(Ug[b], Uo) <= TOL, (name, b, rel(Ug[b], Uo))
        assert rel(trg[b], tro) <= TOL, (name, b, rel(trg[b], tro))
        # each fine state, not only the aggregate
        per = [rel(trg[b][m], tro[m]) for m in range(tro.shape[0]) if np.linalg.norm(tro[m]) > 0]
        assert max(per) <= TOL, (name, b, max(per))


@pytest.mark.parametrize("name,kw,seeds", SERIAL_CASES, ids=[c[0] for c in SERIAL_CASES])
def test_serial_matches_oracle(gpu, orc, name, kw, seeds):
    """Default path: cosine-moment stiffness inside the register-resident step kernel."""
    _serial_case(gpu, orc, name, kw, seeds, assembly=0)


@pytest.mark.parametrize("name,kw,seeds", GEMM_CASES, ids=[c[0] for c in GEMM_CASES])
def test_serial_gemm_assembly_matches_oracle(gpu, orc, name, kw, seeds):
    """Quadrature-GEMM stiffness on MFMA (register Cholesky for M <= 256, the blocked
    device-memory Cholesky beyond)."""
    _serial_case(gpu, orc, name, kw, seeds, assembly=1)


def test_serial_per_instance_alpha(gpu, orc):
    kw = W.with_(W.C2, modes=48, quad=72, steps=64, slices=8)
    alphas = [0.25, 0.6, 1.0]
    u0 = W.u0_batch_1d(48, [20, 21, 22])
    pg = gpu.make_problem(**kw)
    Ug, _ = run_serial(gpu, pg, u0, alpha=alphas)
    for b, a in enumerate(alphas):
        Uo = orc.solve_serial(orc.problem(**W.with_(kw, alpha=a)), u0[b])
        assert rel(Ug[b], Uo) <= TOL


# ---------------------------------------------------------------- parareal parity

PARA_CASES = [
    ("config1", dict(W.C1), None, [1, 3, 8]),
    ("small_c2_a03", W.with_(W.C2, modes=64, quad=96, steps=128, slices=8, alpha=0.3), [0, 1], [2, 8]),
    ("small_c2_a10", W.with_(W.C2, modes=64, quad=96, steps=64, slices=8, alpha=1.0), [2], [3]),
    ("ragged", W.with_(W.C2, modes=40, quad=61, steps=40, slices=5, alpha=0.45, d_sel=3, f_sel=3), [3, 4], [2, 5]),
    ("S1", W.with_(W.C2, modes=16, quad=24, steps=6, slices=6, alpha=0.6), [5], [2]),
    ("P1", W.with_(W.C2, modes=16, quad=24, steps=10, slices=1, alpha=0.6), [6], [1]),
]


@pytest.mark.parametrize("assembly", [0, 1])
@pytest.mark.parametrize("name,kw,seeds,iters", PARA_CASES, ids=[c[0] for c in PARA_CASES])
def test_parareal_iterates_match_oracle(gpu, orc, name, kw, seeds, iters, assembly):
    pg, po = both(gpu, orc, assembly=assembly, **kw)
    u0 = _u0(kw, seeds)
    for K in iters:
        res = gpu.solve_parareal(pg, dev(u0), K, tol=0.0, want_iterates=True)
        torch.cuda.synchronize()
        assert res.iters == min(K, kw["slices"])
        its = res.iterates.cpu().numpy()
        inc = res.incr.cpu().numpy()
        for b in range(u0.shape[0]):
            Uo, ko, inco, itso = orc.solve_parareal(po, u0[b], K, tol=0.0, want_iterates=True)
            assert ko == res.iters
            for k in range(ko + 1):
                assert rel(its[k, b], itso[k]) <= TOL, (name, K, b, k, rel(its[k, b], itso[k]))
            assert rel(res.U.cpu().numpy()[b], Uo) <= TOL
            # increments are differences of nearly equal iterates: compare absolutely
            assert np.allclose(inc[b], inco, rtol=1e-6, atol=1e-11)


def test_parareal_tolerance_stop(gpu, orc):
    kw = W.with_(W.C2, modes=32, quad=48, steps=64, slices=16, alpha=0.5)
    pg, po = both(gpu, orc, **kw)
    u0 = W.u0_batch_1d(32, [30])
    res = gpu.solve_parareal(pg, dev(u0), 16, tol=1e-7)
    _, ko, _, _ = orc.solve_parareal(po, u0[0], 16, tol=1e-7)
    assert res.iters == ko
    assert res.status == 0


def test_parareal_notconv_status(gpu):
    kw = W.with_(W.C2, modes=32, quad=48, steps=64, slices=16, alpha=0.5)
    pg = gpu.make_problem(**kw)
    u0 = W.u0_batch_1d(32, [31])
    res = gpu.solve_parareal(pg, dev(u0), 2, tol=1e-14)
    assert res.iters == 2 and res.status == -4


# ------------------------------------------------------------ GPU self-consistency

@pytest.mark.parametrize("assembly,modes", [(0, 64), (1, 64), (1, 272)])
def test_parareal_exact_after_P_sweeps_bitwise(gpu, assembly, modes):
    """After k sweeps the first k+1 slice ends equal the GPU serial solution bit for bit
    (finite termination of parareal, Section 3.2)."""
    kw = W.with_(W.C2, modes=modes, quad=modes * 3 // 2, steps=80, slices=10, alpha=0.3)
    pg = gpu.make_problem(assembly=assembly, **kw)
    u0 = dev(W.u0_batch_1d(modes, [40, 41, 42]))
    Us, _ = gpu.solve_serial(pg, u0)
    res = gpu.solve_parareal(pg, u0, 10, tol=0.0, want_iterates=True)
    torch.cuda.synchronize()
    its = res.iterates
    for k in range(res.iters + 1):
        assert torch.equal(its[k][:, : k + 1], Us[:, : k + 1]), k
    assert torch.equal(res.U, Us)


def test_deterministic_and_batch_independent(gpu):
    kw = W.with_(W.C2, modes=48, quad=72, steps=48, slices=6, alpha=0.4)
    pg = gpu.make_problem(**kw)
    u0 = W.u0_batch_1d(48, [50, 51, 52, 53])
    Ua, _ = gpu.solve_serial(pg, dev(u0))
    Ub, _ = gpu.solve_serial(pg, dev(u0))
    assert torch.equal(Ua, Ub)
    U1, _ = gpu.solve_serial(pg, dev(u0[2:3]))
    assert torch.equal(U1[0], Ua[2])
    Ra = gpu.solve_parareal(pg, dev(u0), 3).U
    Rb = gpu.solve_parareal(pg, dev(u0[1:2]), 3).U
    assert torch.equal(Ra[1], Rb[0])


@pytest.mark.parametrize("tune", [0, 1, 2, 3])
def test_batch_independent_across_gemm_tiles(gpu, tune):
    """The batched GEMMs tile 32 units x 32 columns (or 16 x 16 split-K tiles, tune bits 0 and
    1): 37 instances make 37 serial units and 222 fine units per sweep, several unit tiles with
    a partial last one, and Mp = 48, Qp = 80 and 97 moments leave partial column tiles and
    reduction chunks.
    Every instance's result must equal its own single-instance run bit for bit, in the serial
    solve and in a parareal sweep."""
    kw = W.with_(W.C2, modes=40, quad=66, steps=36, slices=6, alpha=0.45)
    print(f"[parity] gemm tiles tune={tune}", flush=True)
    pg = gpu.make_problem(tune=tune, **kw)
    u0 = W.u0_batch_1d(40, range(70, 107))
    Ua, _ = gpu.solve_serial(pg, dev(u0))
    Ra = gpu.solve_parareal(pg, dev(u0), 2, tol=0.0).U
    for b in (0, 17, 31, 32, 36):
        U1, _ = gpu.solve_serial(pg, dev(u0[b:b + 1]))
        assert torch.equal(U1[0], Ua[b]), b
        R1 = gpu.solve_parareal(pg, dev(u0[b:b + 1]), 2, tol=0.0).U
        assert torch.equal(R1[0], Ra[b]), b


def test_invalid_arguments_rejected(gpu):
    from paper_2510_11023_amd import _lib

    u0 = dev(W.u0_batch_1d(8, [0]))
    for bad in (dict(alpha=0.0), dict(alpha=1.2), dict(steps=10, slices=4), dict(quad=4),
                dict(d_sel=0, d_param=-1.0), dict(f_sel=9), dict(T=-1.0)):
        kw = W.with_(W.C2, modes=8, quad=16, steps=16, slices=4)
        kw.update(bad)
        p = gpu.make_problem(**kw)
        with pytest.raises(Exception):
            gpu.solve_serial(p, u0)
    p = gpu.make_problem(**W.with_(W.C2, modes=8, quad=16, steps=16, slices=4))
    with pytest.raises(_lib.L1prError):
        gpu.solve_parareal(p, u0, 5)          # max_iter > P
    with pytest.raises(_lib.L1prError):
        gpu.solve_serial(p, u0, alpha=[1.5])  # bad per-instance alpha
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.L1prError) as ei:
        gpu.solve_serial(p, u0, workspace=ws)
    assert ei.value.status == _lib.ENOMEM


# ------------------------------------------------- full size (config 2), sampled

@pytest.fixture(scope="module", params=[0, 1], ids=["moments", "gemm"])
def c2_full(gpu, request):
    kw = W.with_(W.C2, alpha=0.3)
    pg = gpu.make_problem(assembly=request.param, **kw)
    u0 = W.u0_batch_1d(256, range(W.C2_BATCH))
    U, _ = gpu.solve_serial(pg, dev(u0))
    torch.cuda.synchronize()
    return kw, u0, U.cpu().numpy(), request.param


def test_full_size_serial_sampled_slices(gpu, orc, c2_full):
    """Full config-2 size (B = 32, M = 256, Q = 384, N = 4096, P = 64): the oracle's fine
    propagator on the GPU's slice ends C_0..C_n reproduces the GPU's C_{n+1} for sampled
    (instance, slice) pairs."""
    kw, u0, U, asm = c2_full
    po = orc.problem(**kw)
    for b, n in ((0, 0), (17, 1), (31, 63)):
        ref = orc.fine_F(po, n, U[b, : n + 1])
        assert rel(U[b, n + 1], ref) <= TOL, (b, n, rel(U[b, n + 1], ref))


@pytest.fixture(scope="module", params=[0.7, 1.0], ids=["a07", "a10"])
def c2_full_alpha(gpu, request):
    kw = W.with_(W.C2, alpha=request.param)
    pg = gpu.make_problem(**kw)
    u0 = W.u0_batch_1d(256, range(W.C2_BATCH))
    U, _ = gpu.solve_serial(pg, dev(u0))
    torch.cuda.synchronize()
    return kw, U.cpu().numpy()


def test_full_size_serial_sampled_slices_other_alpha(gpu, orc, c2_full_alpha):
    """The other two config-2 groups (alpha = 0.7 and 1.0) at full size: the oracle's fine
    propagator on the GPU's slice ends reproduces sampled slice ends, first, middle and last
    slice."""
    kw, U = c2_full_alpha
    po = orc.problem(**kw)
    for b, n in ((3, 0), (20, 31), (30, 63)):
        ref = orc.fine_F(po, n, U[b, : n + 1])
        assert rel(U[b, n + 1], ref) <= TOL, (kw["alpha"], b, n, rel(U[b, n + 1], ref))


def test_full_size_parareal_prefix_exact(gpu, c2_full):
    kw, u0, U, asm = c2_full
    pg = gpu.make_problem(assembly=asm, **kw)
    res = gpu.solve_parareal(pg, dev(u0), 3, tol=0.0, want_iterates=True)
    torch.cuda.synchronize()
    its = res.iterates.cpu().numpy()
    for k in range(4):
        assert np.array_equal(its[k][:, : k + 1], U[:, : k + 1])
    # the iterates approach the serial solution
    errs = [rel(its[k], U) for k in range(4)]
    assert errs[3] < errs[0]


def test_full_size_concurrent_groups_equal_sequential(gpu):
    """The benchmark's schedule: independent alpha groups at the full config-2 size, each on a
    stream and a workspace of its own, give exactly the results they give one after another."""
    B, alphas, k = 32, (0.3, 1.0), 3
    u0 = dev(W.u0_batch_1d(256, range(B)))
    probs = {a: gpu.make_problem(**W.with_(W.C2, alpha=a)) for a in alphas}
    ws = [torch.empty(gpu.workspace_bytes(probs[a], B, 1), dtype=torch.uint8, device="cuda")
          for a in alphas]
    seq = {a: gpu.solve_parareal(probs[a], u0, k, tol=0.0, want_incr=False, workspace=ws[0]).U
           for a in alphas}
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in alphas]
    cur = torch.cuda.current_stream()
    conc = {}
    for a, s, w in zip(alphas, streams, ws):
        s.wait_stream(cur)
        with torch.cuda.stream(s):
            conc[a] = gpu.solve_parareal(probs[a], u0, k, tol=0.0, want_incr=False, workspace=w).U
    for s in streams:
        cur.wait_stream(s)
    torch.cuda.synchronize()
    for a in alphas:
        assert torch.equal(conc[a], seq[a]), a
