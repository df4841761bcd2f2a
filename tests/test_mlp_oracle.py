"""Pins of the numpy reference of the learned propagator's network (CPU).

The BF16 rounding is checked against torch's bfloat16 conversion, the activation derivative
and the whole backward pass against central finite differences (float64, rounding off), and
the first Adam step against its closed form.
"""
import numpy as np
import pytest

from oracle import mlp as om


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 4000),
                        np.array([0.0, -0.0, 1.0, 3.0, 1.00390625, 1.01171875, 65504.0, -2.5e-38,
                                  np.inf, -np.inf], dtype=np.float32)])
    ref = torch.tensor(x).to(torch.bfloat16).float().numpy()
    got = om.bf16(x)
    assert np.array_equal(got, ref)
    assert np.isnan(om.bf16(np.array([np.nan], dtype=np.float32))[0])


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (om.silu(z + h) - om.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - om.silu_grad(z))) < 1e-8


def _tiny_net(rng, nin=6, inp=8, hidden=5, out=3, outp=4):
    ws = [rng.normal(size=(hidden, inp)) * 0.5, rng.normal(size=(hidden, hidden)) * 0.5,
          rng.normal(size=(hidden, hidden)) * 0.5, rng.normal(size=(outp, hidden)) * 0.5]
    ws[0][:, nin:] = 0.0
    ws[3][out:, :] = 0.0
    bs = [rng.normal(size=hidden) * 0.1, rng.normal(size=hidden) * 0.1,
          rng.normal(size=hidden) * 0.1, np.concatenate([rng.normal(size=out) * 0.1, [0.0] * (outp - out)])]
    norms = (rng.normal(size=nin), 1 + rng.random(nin), rng.normal(size=out), 1 + rng.random(out))
    return ws, bs, norms


def test_backward_matches_finite_differences():
    """The chain rule of the reference (transposes, activation derivative, bias sums, the
    normalised-output loss) against central differences of the float64 loss."""
    rng = np.random.default_rng(1)
    nin, inp, out = 6, 8, 3
    ws, bs, norms = _tiny_net(rng, nin, inp, 5, out, 4)
    x = rng.normal(size=(7, nin))
    t = rng.normal(size=(7, out))
    loss, gW, gb = om.loss_and_grads(ws, bs, norms, x, t, inp, out, exact=True)
    h = 1e-6
    for l in range(4):
        for (i, j) in [(0, 0), (1, 2), (2, 4)]:
            if l == 3 and i >= out:
                continue
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][i, j] += h
            wm[l][i, j] -= h
            fd = (om.loss_and_grads(wp, bs, norms, x, t, inp, out, exact=True)[0]
                  - om.loss_and_grads(wm, bs, norms, x, t, inp, out, exact=True)[0]) / (2 * h)
            assert abs(fd - gW[l][i, j]) < 1e-7 * max(1.0, abs(fd)), (l, i, j, fd, gW[l][i, j])
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][1] += h
        bm[l][1] -= h
        fd = (om.loss_and_grads(ws, bp, norms, x, t, inp, out, exact=True)[0]
              - om.loss_and_grads(ws, bm, norms, x, t, inp, out, exact=True)[0]) / (2 * h)
        assert abs(fd - gb[l][1]) < 1e-7 * max(1.0, abs(fd))


def test_first_adam_step_closed_form():
    """Adam's first step: m_hat = g, v_hat = g^2, so w moves by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.ones(4)
    w1, m, v = om.adam(w, np.zeros(4), np.zeros(4), g, 0.01, 1)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
