"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds none of the method's arithmetic.  It only draws random
numbers (numpy PCG64 via ``default_rng``) and assembles inputs from them; the
one step that needs the DCT tensor product (making a tensor of given tubal
rank from two Gaussian factors) takes the product as a callable, so the oracle
side passes the oracle's product and the GPU side passes the library's.

Workload recipes (shapes and distributions of the paper's experiments):

* ``tsvt_case``    one tensor = t-product of N(0,1) factors n1 x r x n3 and
                   r x n2 x n3, plus N(0, noise_var) noise (the small FP64
                   t-SVT case is 64 x 64 x 16, r = 5, noise_var = 0.01, tau 1).
* ``completion_case``  t-product of N(0,1) factors of tubal rank r, min-max
                   scaled to [0, 1]; observed set = Bernoulli(sr) mask; B is
                   the tensor on the observed set and 0 elsewhere; tau decays
                   geometrically from tau0 to tau1 over L iterations with
                   beta_l = 1/tau_l.  Multispectral-shaped: 256 x 256 x 31,
                   r = 10, sr = 0.3.  Video-shaped: 144 x 176 x 100, r = 15,
                   sr = 0.2.
* ``batch_shapes`` uneven batch: n1, n2 uniform integers in [32, 512], n3 in
                   [8, 128], rank floor(min(n1, n2)/10), tau = 0.1(sqrt n1 +
                   sqrt n2) (the noise bulk edge for N(0, 0.01) noise).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

TProd = Callable[[np.ndarray, np.ndarray], np.ndarray]

SEED_BASE = 1000  # configuration i uses seed SEED_BASE + i
JOB_SEED_STRIDE = 10000  # job j of configuration i uses seed JOB_SEED_STRIDE*i + j


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def gaussian(g: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    return np.asfortranarray(g.standard_normal(shape) * scale)


def gaussian_factors(g: np.random.Generator, n1: int, n2: int, n3: int, r: int):
    """Two N(0,1) spatial factors of shapes n1 x r x n3 and r x n2 x n3."""
    return gaussian(g, (n1, r, n3)), gaussian(g, (r, n2, n3))


def bernoulli_mask(g: np.random.Generator, shape, sr: float) -> np.ndarray:
    return np.asfortranarray((g.random(shape) < sr).astype(np.uint8))


def minmax01(T: np.ndarray) -> np.ndarray:
    lo, hi = float(T.min()), float(T.max())
    return np.asfortranarray((T - lo) / (hi - lo)) if hi > lo else np.zeros_like(T, order="F")


def geometric_taus(tau0: float, tau1: float, L: int) -> np.ndarray:
    if L == 1:
        return np.array([tau0], dtype=np.float64)
    l = np.arange(L, dtype=np.float64)
    return tau0 * (tau1 / tau0) ** (l / (L - 1))


@dataclass
class TsvtCase:
    Z: np.ndarray
    tau: float
    seed: int


def tsvt_case(tprod: TProd, n1: int, n2: int, n3: int, r: int, noise_var: float, tau: float, seed: int) -> TsvtCase:
    g = rng(seed)
    F1, F2 = gaussian_factors(g, n1, n2, n3, r)
    E = gaussian(g, (n1, n2, n3), np.sqrt(noise_var))
    Z = np.asfortranarray(tprod(F1, F2) + E)
    return TsvtCase(Z=Z, tau=float(tau), seed=seed)


@dataclass
class CompletionCase:
    T: np.ndarray  # ground truth in [0, 1]
    mask: np.ndarray  # uint8, 1 = observed
    B: np.ndarray  # T on the observed set, 0 elsewhere
    taus: np.ndarray
    betas: np.ndarray
    seed: int


def completion_case(tprod: TProd, n1: int, n2: int, n3: int, r: int, sr: float, L: int, seed: int,
                    tau0: float = 10.0, tau1: float = 0.1) -> CompletionCase:
    g = rng(seed)
    F1, F2 = gaussian_factors(g, n1, n2, n3, r)
    T = minmax01(tprod(F1, F2))
    mask = bernoulli_mask(g, (n1, n2, n3), sr)
    B = np.asfortranarray(np.where(mask != 0, T, 0.0))
    taus = geometric_taus(tau0, tau1, L)
    return CompletionCase(T=T, mask=mask, B=B, taus=taus, betas=1.0 / taus, seed=seed)


@dataclass
class BatchShape:
    n1: int
    n2: int
    n3: int
    r: int
    tau: float
    seed: int


def batch_shapes(count: int, seed: int, lo: int = 32, hi: int = 512, n3lo: int = 8, n3hi: int = 128,
                 cfg_index: int = 4) -> List[BatchShape]:
    g = rng(seed)
    out = []
    for j in range(count):
        n1 = int(g.integers(lo, hi + 1))
        n2 = int(g.integers(lo, hi + 1))
        n3 = int(g.integers(n3lo, n3hi + 1))
        r = max(1, min(n1, n2) // 10)
        out.append(BatchShape(n1, n2, n3, r, 0.1 * (np.sqrt(n1) + np.sqrt(n2)), JOB_SEED_STRIDE * cfg_index + j))
    return out


def batch_tensor(tprod: TProd, s: BatchShape, noise_var: float = 0.01) -> np.ndarray:
    return tsvt_case(tprod, s.n1, s.n2, s.n3, s.r, noise_var, s.tau, s.seed).Z


def poisson_arrivals(g: np.random.Generator, qps: float, count: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    return np.cumsum(g.exponential(1.0 / qps, size=count))
