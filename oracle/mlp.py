"""Plain numpy reference of the learned coarse propagator's network (test infrastructure).

Definition (shared with the HIP library only through this description):
  x = (x_raw - in_mean) / in_std, rounded to BF16 (round to nearest even), padded with zeros;
  z_l = W_l h_{l-1} + b_l  (BF16 weights and inputs, exact products, sums rounded to FP32),
  h_l = BF16(silu(z_l)),  silu(z) = z / (1 + exp(-z)),  l = 1, 2, 3;
  o = W_4 h_3 + b_4 (FP32): the normalised residual; r = o * out_std + out_mean.
Inside parareal the same network is evaluated in FP64 (the BF16 weights are exact in FP64;
inputs, activations and sums in FP64): forward(..., exact=True).
Normalisation: per-column input mean/std; per-mode output mean and one common output scale
(the root mean square of the per-mode standard deviations).
Loss: mean over rows and the M real outputs of (o - (t - out_mean) / out_std)^2.
Backward as the library forms it: dO = BF16(2 (o - tn) / (n M)); dW_l = dZ_l^T h_{l-1};
db_l = column sums of dZ_l; dZ_{l-1} = BF16((dZ_l W_l) * silu'(z_{l-1})).
Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias correction) on FP32 masters.

Sums are taken in float64 and rounded once, so the reference is the exactly rounded value
of each stage; the library's FP32 accumulation order differs from it by rounding.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round float32 values to the nearest BF16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (rounded & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def _mm(a, b, exact=False):
    """float64 product rounded to float32 (kept in float64 when exact)."""
    r = a.astype(np.float64) @ b.astype(np.float64)
    return r if exact else r.astype(np.float32)


def _ident(x):
    return np.asarray(x, dtype=np.float64)


def forward(ws, bs, norms, x_raw, in_padded, keep=False, exact=False):
    """ws: BF16-valued weights [out][in_padded] (float32 arrays); bs: FP32 biases.
    Returns o [n][out_padded] (and the intermediates when keep).  exact=True evaluates in
    float64 throughout (the inference form used inside parareal)."""
    rnd = _ident if exact else bf16
    ft = np.float64 if exact else np.float32
    in_mean, in_std, out_mean, out_std = norms
    n, nin = x_raw.shape
    xn = ((x_raw.astype(ft) - in_mean) / in_std).astype(ft)
    X0 = np.zeros((n, in_padded), dtype=ft)
    X0[:, :nin] = rnd(xn)
    h = X0
    Zs, Hs = [], [X0]
    for l in range(3):
        z = (_mm(h, ws[l].T, exact) + bs[l]).astype(ft)
        h = rnd(silu(z))
        Zs.append(z)
        Hs.append(h)
    o = (_mm(h, ws[3].T, exact) + bs[3]).astype(ft)
    if keep:
        return o, Zs, Hs
    return o


def loss_and_grads(ws, bs, norms, x_raw, t_raw, in_padded, out, exact=False):
    """Mean squared error of the normalised output and the gradients.  exact=True skips every
    BF16/FP32 rounding (float64 throughout), for derivative checks."""
    rnd = _ident if exact else bf16
    ft = np.float64 if exact else np.float32
    in_mean, in_std, out_mean, out_std = norms
    o, Zs, Hs = forward(ws, bs, norms, x_raw, in_padded, keep=True, exact=exact)
    n = x_raw.shape[0]
    tn = np.zeros_like(o)
    tn[:, :out] = ((t_raw.astype(ft) - out_mean) / out_std).astype(ft)
    d = np.zeros_like(o)
    d[:, :out] = o[:, :out] - tn[:, :out]
    loss = float((d[:, :out].astype(np.float64) ** 2).sum() / (n * out))
    dO = rnd((2.0 * d / (n * out)).astype(ft))
    gW = [None] * 4
    gb = [None] * 4
    gW[3] = _mm(dO.T, Hs[3], exact)
    gb[3] = dO.astype(np.float64).sum(axis=0).astype(ft)
    dz = rnd((_mm(dO, ws[3], exact) * silu_grad(Zs[2])).astype(ft))
    for l in (2, 1, 0):
        gW[l] = _mm(dz.T, Hs[l], exact)
        gb[l] = dz.astype(np.float64).sum(axis=0).astype(ft)
        if l > 0:
            dz = rnd((_mm(dz, ws[l], exact) * silu_grad(Zs[l - 1])).astype(ft))
    return loss, gW, gb


def adam(w, m, v, g, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def correction(ws, bs, norms, G, alpha, n, P, in_padded, out):
    """Denormalised residual r for coarse values G [B][M] at slice n, the network evaluated in
    float64 as inside parareal."""
    B, M = G.shape
    x = np.zeros((B, M + 2), dtype=np.float64)
    x[:, :M] = G
    x[:, M] = np.asarray(alpha, dtype=np.float64)
    x[:, M + 1] = n / P
    o = forward(ws, bs, norms, x, in_padded, exact=True)
    in_mean, in_std, out_mean, out_std = norms
    return o[:, :out] * out_std.astype(np.float64) + out_mean.astype(np.float64)
