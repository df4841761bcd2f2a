"""Learned coarse propagator: residual MLP G_L,n = G_n + r(G_n, alpha, n/P).

Training pairs come from the solver itself: serial (fine) solutions C* of seeded instances,
x = [G_n(C*_0..C*_n) ; alpha ; n/P] and target t = C*_{n+1} - G_n(C*_0..C*_n), and optionally
the states that plain parareal visits on its way there: for its iterates U^k (k < sweeps),
x = [G_n(U^k_0..U^k_n) ; alpha ; n/P] and t = F_n(U^k_0..U^k_n) - G_n(U^k_0..U^k_n), the very
difference a sweep adds to the coarse value.  Parareal contracts by how well G follows F near
the iterates, not only on the converged trajectory.  Every
arithmetic step (serial solves, coarse steps, features, statistics, forward/backward, Adam)
runs in the HIP library; this module allocates buffers, draws the seeded initial weights and
the per-epoch sample order on the host, and sequences the calls.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from .solver import _ptr, _stream, coarse_apply, fine_apply, solve_parareal, solve_serial


def _check(st, what):
    if st != _lib.OK:
        raise _lib.L1prError(st, what)


def mlp_info(modes: int) -> _lib.MlpInfo:
    info = _lib.MlpInfo()
    _check(_lib.lib().l1pr_mlp_layout(modes, ctypes.byref(info)), "l1pr_mlp_layout")
    return info


def glorot_init(modes: int, seed: int) -> np.ndarray:
    """Flat FP32 initial parameters [W1 b1 W2 b2 W3 b3 W4 b4]: Glorot-uniform weights (the
    output layer scaled by 0.1 so the initial correction is small), zero biases, zero padding."""
    info = mlp_info(modes)
    rng = np.random.default_rng(seed)
    flat = np.zeros(info.flat_count, dtype=np.float32)
    shapes = [(info.hidden, info.in_padded, info.in_), (info.hidden, info.hidden, info.hidden),
              (info.hidden, info.hidden, info.hidden), (info.out_padded, info.hidden, info.hidden)]
    for l, (rows, ld, fan_in) in enumerate(shapes):
        fan_out = info.out if l == 3 else rows
        a = math.sqrt(6.0 / (fan_in + fan_out)) * (0.1 if l == 3 else 1.0)
        w = np.zeros((rows, ld), dtype=np.float32)
        real_rows = info.out if l == 3 else rows
        w[:real_rows, :fan_in] = rng.uniform(-a, a, size=(real_rows, fan_in)).astype(np.float32)
        flat[info.flat_w[l]: info.flat_w[l] + rows * ld] = w.reshape(-1)
    return flat


class LearnedCoarse:
    """Parameters and optimiser state of the residual network for M modes (device tensors)."""

    def __init__(self, modes: int, device="cuda", seed: int = 0):
        self.modes = modes
        self.info = mlp_info(modes)
        self.device = torch.device(device)
        self.params = torch.zeros(self.info.param_bytes, dtype=torch.uint8, device=self.device)
        self.state = torch.zeros(3 * self.info.flat_count, dtype=torch.float32, device=self.device)
        self.set_masters(glorot_init(modes, seed))
        self.step = 0

    # -- parameter access -------------------------------------------------------------
    def set_masters(self, flat: np.ndarray):
        self.state[: self.info.flat_count] = torch.from_numpy(flat.astype(np.float32)).to(self.device)
        _check(_lib.lib().l1pr_mlp_reset_moments(self.modes, _ptr(self.state), _stream()), "reset")
        _check(_lib.lib().l1pr_mlp_sync(self.modes, _ptr(self.state), _ptr(self.params), _stream()),
               "sync")

    def masters(self) -> np.ndarray:
        return self.state[: self.info.flat_count].cpu().numpy()

    def norms(self):
        """(in_mean, in_std, out_mean, out_std) as numpy arrays (unpadded)."""
        def view(off, n):
            return self.params[off: off + 4 * n].view(torch.float32).cpu().numpy()[:n]
        i = self.info
        return (view(i.off_in_mean, i.in_), view(i.off_in_std, i.in_),
                view(i.off_out_mean, i.out), view(i.off_out_std, i.out))

    def param_arrays(self):
        """BF16 weights (as float32 values, [out][in_padded]) and FP32 biases."""
        i = self.info
        ws, bs = [], []
        shapes = [(i.hidden, i.in_padded), (i.hidden, i.hidden), (i.hidden, i.hidden),
                  (i.out_padded, i.hidden)]
        for l, (r, c) in enumerate(shapes):
            w = self.params[i.off_w[l]: i.off_w[l] + 2 * r * c].view(torch.bfloat16).float()
            ws.append(w.reshape(r, c).cpu().numpy())
            bs.append(self.params[i.off_b[l]: i.off_b[l] + 4 * r].view(torch.float32).cpu().numpy())
        return ws, bs

    # -- data -------------------------------------------------------------------------
    def features(self, p, Z: torch.Tensor, G: torch.Tensor, alpha: torch.Tensor):
        """x [B*P][M+2], t [B*P][M] from slice ends Z and coarse values G (device FP64)."""
        B, P = Z.shape[0], p.slices
        x = torch.empty((B * P, self.modes + 2), dtype=torch.float32, device=self.device)
        t = torch.empty((B * P, self.modes), dtype=torch.float32, device=self.device)
        _check(_lib.lib().l1pr_mlp_features(self.modes, B, P, _ptr(alpha), _ptr(Z), _ptr(G), _ptr(x),
                                            _ptr(t), _stream()), "features")
        return x, t

    def set_stats(self, x: torch.Tensor, t: torch.Tensor):
        _check(_lib.lib().l1pr_mlp_stats(self.modes, _ptr(x), _ptr(t), x.shape[0], _ptr(self.params),
                                         _stream()), "stats")

    # -- compute ----------------------------------------------------------------------
    def forward(self, x: torch.Tensor) -> torch.Tensor:
        n = x.shape[0]
        ws = torch.empty(_lib.lib().l1pr_mlp_workspace_bytes(self.modes, n, 0), dtype=torch.uint8,
                         device=self.device)
        y = torch.empty((n, self.modes), dtype=torch.float32, device=self.device)
        _check(_lib.lib().l1pr_mlp_forward(self.modes, _ptr(self.params), _ptr(x), n, _ptr(y),
                                           _ptr(ws), ws.numel(), _stream()), "forward")
        return y

    def infer(self, x: torch.Tensor) -> torch.Tensor:
        """The network as parareal evaluates it (FP64; x [n][M+2] FP64)."""
        n = x.shape[0]
        ws = torch.empty(_lib.lib().l1pr_mlp_infer_workspace_bytes(self.modes, n), dtype=torch.uint8,
                         device=self.device)
        y = torch.empty((n, self.modes), dtype=torch.float64, device=self.device)
        _check(_lib.lib().l1pr_mlp_infer(self.modes, _ptr(self.params), _ptr(x), n, _ptr(y),
                                         _ptr(ws), ws.numel(), _stream()), "infer")
        return y

    def train_step(self, x, t, idx, lr, ws, loss=None, grad=None):
        self.step += 1
        n = idx.shape[0] if idx is not None else x.shape[0]
        _check(_lib.lib().l1pr_mlp_train_step(self.modes, _ptr(self.params), _ptr(self.state), _ptr(x),
                                              _ptr(t), _ptr(idx), n, float(lr), self.step, _ptr(loss),
                                              _ptr(grad), _ptr(ws), ws.numel(), _stream()),
               "train_step")

    def train(self, x, t, epochs: int, batch: int = 1024, lr: float = 1e-3, seed: int = 0,
              lr_final: float | None = None, log=None):
        """Mini-batch Adam over a seeded shuffle per epoch; cosine decay of the rate to
        lr_final.  Returns the mean loss of each epoch."""
        N = x.shape[0]
        ws = torch.empty(_lib.lib().l1pr_mlp_workspace_bytes(self.modes, batch, 1),
                         dtype=torch.uint8, device=self.device)
        nb = N // batch
        losses = torch.zeros(epochs * nb, dtype=torch.float32, device=self.device)
        total = epochs * nb
        lr_final = lr * 0.05 if lr_final is None else lr_final
        it = 0
        for ep in range(epochs):
            perm = np.random.default_rng(seed + 7919 * ep).permutation(N).astype(np.int32)
            idx = torch.from_numpy(perm).to(self.device)
            for bi in range(nb):
                rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * it / max(total, 1)))
                self.train_step(x, t, idx[bi * batch:(bi + 1) * batch], rate, ws, loss=losses[it:it + 1])
                it += 1
            if log:
                log(f"epoch {ep}: loss {losses[ep * nb:(ep + 1) * nb].mean().item():.4e}")
        return losses.view(epochs, nb).mean(dim=1).cpu().numpy()


def training_data(p, u0: torch.Tensor, alphas, model: LearnedCoarse, chunk: int = 1024,
                  sweeps: int = 0):
    """Training pairs: the serial solutions of the instances (per-instance alpha) with the plain
    coarse step on every slice, then, for k < sweeps, the plain parareal iterates U^k with
    F_n(U^k) - G_n(U^k) as target.  Returns (x, t): per chunk of instances, the serial pairs,
    then those of U^0, U^1, ...; rows b*P + n within each block."""
    xs, ts = [], []
    B = u0.shape[0]
    for b0 in range(0, B, chunk):
        b1 = min(B, b0 + chunk)
        al = [float(a) for a in alphas[b0:b1]]
        ad = torch.tensor(al, dtype=torch.float64, device=u0.device)
        Z, _ = solve_serial(p, u0[b0:b1], alpha=al)
        G = coarse_apply(p, Z, alpha=al)
        x, t = model.features(p, Z, G, ad)
        xs.append(x)
        ts.append(t)
        del Z, G
        if sweeps > 0:
            its = solve_parareal(p, u0[b0:b1], sweeps, tol=0.0, alpha=al, want_iterates=True,
                                 want_incr=False).iterates
            for k in range(min(sweeps, its.shape[0])):
                U = its[k].contiguous()
                G = coarse_apply(p, U, alpha=al)
                F = fine_apply(p, U, alpha=al)
                Zf = torch.cat([U[:, :1], F], dim=1).contiguous()  # row n+1 = F_n(U)
                x, t = model.features(p, Zf, G, ad)
                xs.append(x)
                ts.append(t)
                del U, G, F, Zf
            del its
    return torch.cat(xs), torch.cat(ts)


def _pad_modes(X: torch.Tensor, modes: int) -> torch.Tensor:
    """[..., M] -> [..., modes] with zero coefficients appended (the modes a problem does not
    carry; its coarse and fine values are exactly zero there)."""
    M = X.shape[-1]
    if M == modes:
        return X.contiguous()
    out = torch.zeros(X.shape[:-1] + (modes,), dtype=X.dtype, device=X.device)
    out[..., :M] = X
    return out


def training_data_padded(p, u0: torch.Tensor, alphas, model: LearnedCoarse, sweeps: int = 0):
    """training_data for a problem with fewer modes than the network: the slice ends, coarse
    and fine values of the problem are padded with zero coefficients up to model.modes before
    the features are formed, so one network can serve batches of several mode counts
    (uneven batches).  Same row order as training_data."""
    xs, ts = [], []
    al = [float(a) for a in alphas]
    ad = torch.tensor(al, dtype=torch.float64, device=u0.device)
    Z, _ = solve_serial(p, u0, alpha=al)
    G = coarse_apply(p, Z, alpha=al)
    x, t = model.features(p, _pad_modes(Z, model.modes), _pad_modes(G, model.modes), ad)
    xs.append(x)
    ts.append(t)
    if sweeps > 0:
        its = solve_parareal(p, u0, sweeps, tol=0.0, alpha=al, want_iterates=True,
                             want_incr=False).iterates
        for k in range(min(sweeps, its.shape[0])):
            U = its[k].contiguous()
            G = coarse_apply(p, U, alpha=al)
            F = fine_apply(p, U, alpha=al)
            Zf = torch.cat([U[:, :1], F], dim=1)
            x, t = model.features(p, _pad_modes(Zf, model.modes), _pad_modes(G, model.modes), ad)
            xs.append(x)
            ts.append(t)
    return torch.cat(xs), torch.cat(ts)
