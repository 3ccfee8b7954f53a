"""Seeded synthetic inputs for the HOSCF workloads.

This module only draws and assembles inputs (tensors, initial factors, loss
weights); it contains none of the method's arithmetic, so both the HIP path and
the independent FP64 oracle can be fed from it.

Recipe (every workload):
  * Gaussian noise is drawn slab by slab along mode 1; slab i uses its own
    PCG64 stream seeded with SeedSequence([seed, 0, i]) so slabs can be drawn
    in parallel and the result does not depend on the thread count.
  * Planted factors use SeedSequence([seed, 1]); initial factors use
    SeedSequence([seed + 1000]); loss weights use SeedSequence([seed, 3]).
  * Every entry is assembled in FP64 and rounded once to the storage dtype.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence, Tuple

import numpy as np

_SLAB_ROWS_TARGET = 1 << 22  # entries per generation slab


def _rng(*key) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def unit_gaussian(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal(n)
    return v / math.sqrt(float(v @ v))


def _outer_rows(vecs: Sequence[np.ndarray]) -> np.ndarray:
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gaussian_plus_cp(dims: Sequence[int], weights: Sequence[float],
                     factors: Sequence[Sequence[np.ndarray]], seed: int,
                     noise_std: float = 1.0, dtype=np.float32,
                     out: Optional[np.ndarray] = None) -> np.ndarray:
    """noise_std * N(0,1) + sum_r weights[r] * a_r1 o ... o a_rN, assembled in
    FP64 slab by slab along mode 1 and rounded once to ``dtype``."""
    dims = [int(d) for d in dims]
    T = out if out is not None else np.empty(dims, dtype=dtype)
    rest = int(np.prod(dims[1:]))
    step = max(1, _SLAB_ROWS_TARGET // max(rest, 1))
    tails = [_outer_rows(f[1:]) for f in factors]

    def fill(s: int):
        e = min(dims[0], s + step)
        slab = np.empty([e - s] + dims[1:], dtype=np.float64)
        if noise_std != 0.0:
            slab[...] = _rng(seed, 0, s // step).standard_normal(slab.shape) * noise_std
        else:
            slab[...] = 0.0
        for w, f, tail in zip(weights, factors, tails):
            slab += w * np.multiply.outer(f[0][s:e], tail)
        T[s:e] = slab.astype(T.dtype)

    starts = list(range(0, dims[0], step))
    if len(starts) > 1:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, starts))
    else:
        for s in starts:
            fill(s)
    return T


def init_factors(dims: Sequence[int], seed: int, uniform: bool = False) -> np.ndarray:
    """Stacked initial factors [x_1; ...; x_N] (FP64): N(0,1) entries
    normalised per block (uniform on each sphere), or U[0,1] entries
    normalised per block when ``uniform`` (the paper's experiments)."""
    rng = _rng(seed + 1000)
    out = []
    for d in dims:
        v = rng.random(d) if uniform else rng.standard_normal(d)
        out.append(v / math.sqrt(float(v @ v)))
    return np.concatenate(out)


def planted_rank_one(dims: Sequence[int], lam: float, seed: int, dtype=np.float32,
                     noise_std: float = 1.0) -> Tuple[np.ndarray, List[np.ndarray]]:
    """N(0,1) noise + lam * a_1 o ... o a_N with unit Gaussian planted factors."""
    rng = _rng(seed, 1)
    fac = [unit_gaussian(rng, d) for d in dims]
    T = gaussian_plus_cp(dims, [lam], [fac], seed, noise_std=noise_std, dtype=dtype)
    return T, fac


def planted_cp(dims: Sequence[int], lams: Sequence[float], seed: int, dtype=np.float32,
               noise_std: float = 1.0) -> Tuple[np.ndarray, List[List[np.ndarray]]]:
    """N(0,1) noise + sum_r lams[r] * a_r1 o ... o a_rN with unit Gaussian
    planted factors (drawn term by term, mode by mode)."""
    rng = _rng(seed, 1)
    fac = [[unit_gaussian(rng, d) for d in dims] for _ in lams]
    T = gaussian_plus_cp(dims, list(lams), fac, seed, noise_std=noise_std, dtype=dtype)
    return T, fac


def planted_lambda(dims: Sequence[int], factor: float = 3.0) -> float:
    """factor * E||noise||_F / sqrt(max dim) with E||noise||_F read as
    sqrt(prod dims)."""
    return factor * math.sqrt(float(np.prod(dims))) / math.sqrt(max(dims))


# --- the workloads --------------------------------------------------------

def small_planted(seed: int = 1, n: int = 64, order: int = 3, lam: float = 10.0,
                  dtype=np.float64):
    """Order-3 n^3 FP64 N(0,1) plus lam * a o b o c (unit Gaussian a, b, c)."""
    return planted_rank_one([n] * order, lam, seed, dtype=dtype)


def large_planted(dims: Sequence[int], seed: int, dtype=np.float32):
    """N(0,1) noise plus planted rank-one with lambda = 3 sqrt(prod I)/sqrt(max I)."""
    return planted_rank_one(dims, planted_lambda(dims), seed, dtype=dtype)


def cp_plus_noise(dims: Sequence[int], rank: int, noise_frac: float, seed: int,
                  dtype=np.float32):
    """Rank-R CP tensor with iid N(0,1) (unnormalised) factors and unit
    weights, plus Gaussian noise scaled so ||noise||_F = noise_frac * ||T_cp||_F
    (||T_cp||_F^2 in closed form: sum_{r,s} prod_n <a_rn, a_sn>)."""
    rng = _rng(seed, 1)
    fac = [[rng.standard_normal(d) for d in dims] for _ in range(rank)]
    gram = np.ones((rank, rank))
    for n in range(len(dims)):
        A = np.stack([fac[r][n] for r in range(rank)])
        gram *= A @ A.T
    cp_norm = math.sqrt(float(gram.sum()))
    noise_std = noise_frac * cp_norm / math.sqrt(float(np.prod(dims)))
    T = gaussian_plus_cp(dims, [1.0] * rank, fac, seed, noise_std=noise_std, dtype=dtype)
    return T, fac, noise_std


def batched_planted(count: int, seed: int, lo: int = 8, hi: int = 96, order: int = 3,
                    lam_lo: float = 1.0, lam_hi: float = 20.0, dtype=np.float32):
    """``count`` order-3 tensors with dims uniform in {lo..hi} per mode,
    N(0,1) plus lambda * a o b o c with lambda ~ U[lam_lo, lam_hi]."""
    rng = _rng(seed, 2)
    shapes = rng.integers(lo, hi + 1, size=(count, order))
    lams = rng.uniform(lam_lo, lam_hi, size=count)
    tensors = []
    for b in range(count):
        dims = [int(v) for v in shapes[b]]
        T, _ = planted_rank_one(dims, float(lams[b]), seed * 1_000_003 + b, dtype=dtype)
        tensors.append(T)
    return tensors, shapes, lams


def batched_inits(shapes, rank: int, seed: int) -> List[List[np.ndarray]]:
    """x0[b][r]: stacked Gaussian unit factors per tensor and deflation term."""
    return [[init_factors([int(d) for d in shapes[b]], seed * 7919 + b * 131 + r)
             for r in range(rank)] for b in range(len(shapes))]


def loss_weights(dims: Sequence[int], seed: int) -> List[np.ndarray]:
    rng = _rng(seed, 3)
    return [rng.standard_normal(d) for d in dims]


def exp_tensor(n: int = 30, order: int = 3) -> np.ndarray:
    """Example 2 'EXP': A[i_1..i_d] = sum_j (-1)^(j+1) j exp(-i_j), 1-based."""
    idx = np.arange(1, n + 1, dtype=np.float64)
    T = np.zeros([n] * order)
    for j in range(1, order + 1):
        shape = [1] * order
        shape[j - 1] = n
        T = T + ((-1) ** (j + 1)) * j * np.exp(-idx).reshape(shape)
    return T


def arcsin_tensor(n: int = 20, order: int = 4) -> np.ndarray:
    """Example 2 'ARCSIN', read as sum_j arcsin((-1)^(i_j) * j / i_j) when
    i_j >= j for all j, else 0 (1-based indices)."""
    idx = np.arange(1, n + 1, dtype=np.float64)
    T = np.zeros([n] * order)
    mask = np.ones([n] * order, dtype=bool)
    for j in range(1, order + 1):
        shape = [1] * order
        shape[j - 1] = n
        with np.errstate(invalid="ignore"):
            term = np.where(idx >= j, np.arcsin(np.clip(((-1.0) ** idx) * j / idx, -1, 1)), 0.0)
        T = T + term.reshape(shape)
        mask &= (idx >= j).reshape(shape)
    return np.where(mask, T, 0.0)
