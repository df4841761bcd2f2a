"""GPU runs of the paper's own model problem (its numerical examples): D = 1 + u,
f = sin(pi x) e^-t, u0 = x^4 (1-x)^4, alpha = 0.5, with 2^8 coarse intervals of 2^5 fine
steps and 16 sine modes.  Serial solve and parareal iterates against the oracle at 1e-10
relative L2; the tolerance-stopped run (the paper's 1e-10 stop test) ends within a few
sweeps at the serial solution."""
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


def test_paper_model_matches_oracle(gpu, orc):
    kw = dict(W.PAPER)
    u0 = W.u0_paper_1d(kw["modes"])
    p = gpu.make_problem(**kw)
    ud = torch.tensor(u0[None], dtype=torch.float64, device="cuda")
    Us, _ = gpu.solve_serial(p, ud)
    po = orc.problem(**kw)
    Uo = orc.solve_serial(po, u0)
    assert rel(Us.cpu().numpy()[0], Uo) <= TOL
    r = gpu.solve_parareal(p, ud, 4, tol=0.0, want_iterates=True)
    _, ko, _, ito = orc.solve_parareal(po, u0, 4, want_iterates=True)
    its = r.iterates.cpu().numpy()[:, 0]
    for k in range(ko + 1):
        assert rel(its[k], ito[k]) <= TOL, (k, rel(its[k], ito[k]))
        assert torch.equal(r.iterates[k][:, : k + 1], Us[:, : k + 1]), k


def test_paper_model_tolerance_stop(gpu):
    kw = dict(W.PAPER)
    p = gpu.make_problem(**kw)
    ud = torch.tensor(W.u0_paper_1d(kw["modes"])[None], dtype=torch.float64, device="cuda")
    Us, _ = gpu.solve_serial(p, ud)
    r = gpu.solve_parareal(p, ud, kw["slices"], tol=1e-10)
    assert r.status == 0 and r.iters < 20, (r.status, r.iters)
    assert rel(r.U.cpu().numpy(), Us.cpu().numpy()) < 1e-9
