"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds none of the method's arithmetic: it only draws problem parameters and
initial sine coefficients.  Every workload is synthetic (the paper uses no dataset).

Coefficients are in the orthonormal basis sqrt(2) sin(k pi x) (2D: 2 sin sin); N(m, v)
below takes v as the variance.
"""
from __future__ import annotations

import math

import numpy as np

# Problem parameters as plain dicts (field names of l1pr_problem).
# config 1: 1D manufactured solution, alpha = 0.5, M = 32, Q = 64, N = 256, P = 8
C1 = dict(dim=1, modes=32, quad=64, steps=256, slices=8, alpha=0.5, T=1.0, d_sel=1, d_param=1.0,
          f_sel=1, history=0, source_time=0)
# config 2: 1D, D = 1 + 1/(1+u^2), f = 0.1 u (1-u), M = 256, Q = 384, N = 4096, P = 64, B = 32,
# one batched run per alpha in {0.3, 0.7, 1.0}
C2 = dict(dim=1, modes=256, quad=384, steps=4096, slices=64, alpha=0.3, T=1.0, d_sel=2,
          d_param=1.0, f_sel=2, history=0, source_time=0)
C2_ALPHAS = (0.3, 0.7, 1.0)
C2_BATCH = 32
# config 3: 2D, 64x64 modes, 96x96 quadrature, alpha = 0.6, D = 1 + exp(-u^2)/2, f = sin u
C3 = dict(dim=2, modes=64, quad=96, steps=2048, slices=128, alpha=0.6, T=1.0, d_sel=3,
          d_param=1.0, f_sel=3, history=0, source_time=0)
# config 4: learned coarse propagator, 1D, M = 128 (Q = 192), N = 2048, P = 64, alpha ~ U(0.2, 1);
# D, f and the u0 law as in config 2; 4096 training instances, 64 held-out instances
C4 = dict(dim=1, modes=128, quad=192, steps=2048, slices=64, alpha=0.5, T=1.0, d_sel=2,
          d_param=1.0, f_sel=2, history=0, source_time=0)
C4_TRAIN_SEEDS = range(0, 4096)
C4_EVAL_SEEDS = range(100000, 100064)
C4_TRAIN_ALPHA_SEED = 4242
C4_EVAL_ALPHA_SEED = 2424
# training pairs also from the first plain parareal iterates U^0 .. U^2 of each training instance
C4_TRAIN_SWEEPS = 3


# config 5: uneven batch of 256 instances, P = 64 slices, each with its own modes
# M ~ U{64..256}, fine steps per slice S ~ U{8..64} (N = 64 S) and alpha ~ U(0.2, 1);
# D = 1 + sin^2(u)/2 and the manufactured source of config 1 (with the instance's alpha),
# u0 = sin(pi x).  Instances are grouped by padded mode count roundup16(M); a group uses
# Q = 2 roundup16(M) Gauss points.
C5 = dict(dim=1, slices=64, alpha=0.5, T=1.0, d_sel=1, d_param=1.0, f_sel=1, history=0,
          source_time=0)
C5_COUNT = 256
C5_SEED = 5


# the paper's model problem (its numerical examples): D = 1 + u, f = sin(pi x) e^-t,
# u0 = x^4 (1-x)^4, alpha = 0.5, on (0, 1); T = 1 (not stated there).  Its error-vs-iteration
# run uses 2^8 coarse intervals of 2^5 fine steps and 2^4 spatial unknowns (here: 16 sine
# modes, 24 Gauss points)
PAPER = dict(dim=1, modes=16, quad=24, steps=256 * 32, slices=256, alpha=0.5, T=1.0, d_sel=4,
             d_param=1.0, f_sel=4, history=0, source_time=0)


def c5_instances(count: int = C5_COUNT, seed: int = C5_SEED):
    """(modes, steps per slice, alpha) arrays of the uneven batch."""
    rng = np.random.default_rng(seed)
    modes = rng.integers(64, 257, size=count)
    spp = rng.integers(8, 65, size=count)
    alpha = rng.uniform(0.2, 1.0, size=count)
    return modes, spp, alpha


def with_(base: dict, **kw) -> dict:
    d = dict(base)
    d.update(kw)
    return d


def u0_sine_mode(M: int) -> np.ndarray:
    """Coefficients of u0 = sin(pi x): sqrt(2) sin(pi x) / sqrt(2)."""
    c = np.zeros(M)
    c[0] = 1.0 / math.sqrt(2.0)
    return c


def u0_paper_1d(M: int) -> np.ndarray:
    """Sine coefficients of u0 = x^4 (1-x)^4, k = 1..M, in closed form.  Integrating by parts
    (p(0) = p(1) = p''(0) = p''(1) = 0, p(1-x) = p(x)), sqrt(2) int_0^1 p(x) sin(k pi x) dx
    = sqrt(2) (1 - (-1)^k) (p''''(0)/a^5 - p^(6)(0)/a^7 + p^(8)(0)/a^9), a = k pi, with
    p''''(0) = 24, p^(6)(0) = 4320, p^(8)(0) = 40320; zero for even k."""
    c = np.zeros(M)
    for k in range(1, M + 1, 2):
        a = k * math.pi
        c[k - 1] = 2.0 * math.sqrt(2.0) * (24.0 / a ** 5 - 4320.0 / a ** 7 + 40320.0 / a ** 9)
    return c


def u0_random_1d(M: int, seed: int) -> np.ndarray:
    """c_k ~ N(0, k^-3), k = 1..M."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, M + 1, dtype=np.float64)
    return rng.normal(0.0, 1.0, size=M) * k ** -1.5


def u0_random_2d(M: int, seed: int) -> np.ndarray:
    """c_{k1 k2} ~ N(0, (k1^2 + k2^2)^-1.5), lexicographic (k1-1)*M + (k2-1)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, M + 1, dtype=np.float64)
    var = (k[:, None] ** 2 + k[None, :] ** 2) ** -1.5
    return (rng.normal(0.0, 1.0, size=(M, M)) * np.sqrt(var)).reshape(-1)


def u0_batch_1d(M: int, seeds) -> np.ndarray:
    return np.stack([u0_random_1d(M, s) for s in seeds])


def alphas_uniform(n: int, seed: int, lo: float = 0.2, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n)
