"""Seeded synthetic inputs: random fields, temperature ladders and the named
workloads.  This module holds no arithmetic of the method itself; it only
draws disorder realizations and lays out temperature sets, so that the HIP
path, the oracle and the benchmark all consume identical arrays.

The paper draws the field as h_i = rand(+-1), one instance shared by all
replicas (Sec. 3.1, step 2); the continuous (Gaussian) variant and the
workload sizes below are synthetic stand-ins with the shapes the paper
studies (L in {8, 16, 32, 64}, Sec. 1 and Sec. 7).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


def bimodal_fields(L: int, key) -> np.ndarray:
    """h_i = +-1 with probability 1/2 each, float32, natural site order."""
    rng = np.random.default_rng(key)
    return np.where(rng.random(L ** 3) < 0.5, -1.0, 1.0).astype(np.float32)


def gaussian_fields(L: int, key) -> np.ndarray:
    """h_i ~ N(0, 1), float32, natural site order."""
    rng = np.random.default_rng(key)
    return rng.standard_normal(L ** 3, dtype=np.float32)


def linear_temps(R: int, lo: float, hi: float) -> np.ndarray:
    if R == 1:
        return np.array([lo], dtype=np.float64)
    return np.linspace(lo, hi, R, dtype=np.float64)


def geometric_temps(R: int, lo: float, hi: float) -> np.ndarray:
    if R == 1:
        return np.array([lo], dtype=np.float64)
    return lo * (hi / lo) ** (np.arange(R, dtype=np.float64) / (R - 1))


def random_spins(R: int, L: int, key) -> np.ndarray:
    rng = np.random.default_rng(key)
    return np.where(rng.random((R, L ** 3)) < 0.5, -1, 1).astype(np.int8)


@dataclasses.dataclass(frozen=True)
class Realization:
    """One disorder realization with its replica ladder and run length."""
    L: int
    R: int
    J: float
    h: float
    fields: np.ndarray
    temps: np.ndarray
    seed: int = 0
    realization: int = 0
    sweeps: int = 0
    every: int = 10
    R_cap: int = 0
    adapt: Optional[dict] = None

    @property
    def attempts_per_sweep(self) -> int:
        return self.R * self.L ** 3


def plain_l8() -> Realization:
    """L=8, J=1, bimodal fields h=1.0, R=16 linear in [1.5, 5.0], 1000 sweeps,
    exchange every 10, seed 0."""
    return Realization(L=8, R=16, J=1.0, h=1.0, fields=bimodal_fields(8, [0, 0]),
                       temps=linear_temps(16, 1.5, 5.0), seed=0, sweeps=1000, every=10)


def paper_scale_l32(sweeps: int = 10_000) -> Realization:
    """L=32, Gaussian fields h=2.0, R=64 geometric in [1, 6], 10^4 sweeps."""
    return Realization(L=32, R=64, J=1.0, h=2.0, fields=gaussian_fields(32, [0, 1]),
                       temps=geometric_temps(64, 1.0, 6.0), seed=0, sweeps=sweeps, every=10)


def adaptive_l64(sweeps: int = 20_000, trials: int = 4, trial_sweeps: int = 2000) -> Realization:
    """L=64, bimodal fields h=2.25, R=128 linear in [1, 6]; 4 trial runs of 2000
    sweeps insert temperatures where the adjacent rate is < 0.2 (cap 192,
    at most 16 per trial), then 2x10^4 sweeps."""
    return Realization(L=64, R=128, J=1.0, h=2.25, fields=bimodal_fields(64, [0, 2]),
                       temps=linear_temps(128, 1.0, 6.0), seed=0, sweeps=sweeps, every=10,
                       R_cap=192,
                       adapt=dict(trials=trials, sweeps_per_trial=trial_sweeps, every=10,
                                  rate_threshold=0.2, max_insert_per_trial=16, R_cap=192))


def hbm_streaming_l64(n: int = 16, R: int = 128, sweeps: int = 200) -> list:
    """The L=64 kernel on more data than the 256 MB on-package cache holds:
    n realizations of L=64 with R replicas each (n R L^3 bytes of spins,
    512 MiB at the defaults), +-1 fields h=2.25, T linear in [1, 6], run as
    one batch so every half-sweep streams all of them through HBM."""
    return [Realization(L=64, R=R, J=1.0, h=2.25, fields=bimodal_fields(64, [8, q]),
                        temps=linear_temps(R, 1.0, 6.0), seed=0, realization=q, sweeps=sweeps, every=10)
            for q in range(n)]


def batched_mix(n: int = 256, sweeps: int = 5000) -> list:
    """n independent realizations, L uniform over {8, 16, 32} with R = 16/32/64,
    even ids bimodal, odd ids Gaussian, h ~ U[1.0, 2.5], T geometric in [1, 6]."""
    rng = np.random.default_rng(4)
    Ls = rng.choice([8, 16, 32], size=n)
    hs = rng.uniform(1.0, 2.5, size=n)
    out = []
    for rho in range(n):
        L = int(Ls[rho])
        R = {8: 16, 16: 32, 32: 64}[L]
        f = bimodal_fields(L, [4, rho]) if rho % 2 == 0 else gaussian_fields(L, [4, rho])
        out.append(Realization(L=L, R=R, J=1.0, h=float(hs[rho]), fields=f,
                               temps=geometric_temps(R, 1.0, 6.0), seed=0, realization=rho,
                               sweeps=sweeps, every=10))
    return out


def served_stream(n: int = 2000, rate: float = 50.0, sweeps: int = 2000, trial_sweeps: int = 500):
    """Poisson arrivals of realization requests: L in {8,16,32,64} with
    probabilities {.4,.3,.2,.1}, R0 = min(2L, 128), Gaussian fields with
    h ~ U[1.5, 2.5], T linear in [1, 6]; one adaptive trial then the run."""
    arr = np.cumsum(np.random.default_rng(5).exponential(1.0 / rate, size=n))
    rng = np.random.default_rng(6)
    Ls = rng.choice([8, 16, 32, 64], size=n, p=[0.4, 0.3, 0.2, 0.1])
    hs = rng.uniform(1.5, 2.5, size=n)
    reqs = []
    for q in range(n):
        L = int(Ls[q])
        R0 = min(2 * L, 128)
        R_cap = int(np.ceil(1.5 * R0))
        reqs.append((float(arr[q]), Realization(
            L=L, R=R0, J=1.0, h=float(hs[q]), fields=gaussian_fields(L, [5, q]),
            temps=linear_temps(R0, 1.0, 6.0), seed=0, realization=q, sweeps=sweeps, every=10,
            R_cap=R_cap,
            adapt=dict(trials=1, sweeps_per_trial=trial_sweeps, every=10, rate_threshold=0.2,
                       max_insert_per_trial=R_cap - R0, R_cap=R_cap))))
    return reqs
